// Cluster locating on 8-bit codes with adaptive operand precision (paper
// Sec. 3.1 vector space division, Sec. 3.3-3.4 sub-space features and the
// regressor, Sec. 4.1 the distance module's CL pass with partial distances
// summed over slices, Sec. 4.2 MSB-first operand bits).
//
//  k_clq       query codes per slice (zero-padded to one MFMA K) and their
//              squared norms at the search's two widths
//  k_clcn      the centroids' squared norms per slice at the two widths
//  k_clbits    per (query, slice): d' to every sub-space centre, C1, the
//              regressor, one bit per sub-space (low width or 8 bits)
//  k_coarse_int  integer coarse distances on the int8 MFMA: per slice the
//              dot products at both widths, the width of each centroid
//              slice's sub-space selects one, partial distances summed
//              over the slices; written as order keys for top-nprobe
#include "device_common.h"

namespace amp {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

struct ClArgs {
  const uint32_t* tab;  // exact decision table of the CL predictor, or null (direct evaluation)
  const float* Q;
  int nq, d, nlist, S, P, PW, w, ec;
  float o;
  int lo, hi;  // operand widths of the two classes (slot 0: low, slot 1: high)
  int8_t* clq;
  int32_t* clqn;
  uint32_t* clmask;
  int32_t* clcn;
  const int8_t* clc;
  const uint16_t* clasg;
  const int8_t* clz;
  const int32_t* clr;
  const int32_t* cln;
  float* keys;
  int32_t* out_d;
  uint8_t* out_bits;
};

// 8-bit signed code: x - o rounded to FP32, scaled by 2^-ec (exact), rounded
// half to even, clamped to [-128, 127]
__device__ __forceinline__ int cl_code(float x, float o, int ec) {
  const float v = rintf(ldexpf(__fsub_rn(x, o), -ec));
  return (int)__builtin_amdgcn_fmed3f(v, -128.f, 127.f);
}
// b-bit MSB-first operand: the low 8 - b bits cleared (floor)
__device__ __forceinline__ int cl_trunc(int v, int b) { return v - (v & ((1 << (8 - b)) - 1)); }
// the same on four packed codes
__device__ __forceinline__ uint32_t cl_bytemask(int b) {
  const uint32_t m = (0xFFu << (8 - b)) & 0xFFu;
  return m * 0x01010101u;
}

template <int KP>
__global__ __launch_bounds__(256) void k_clq(ClArgs a) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)a.nq * a.S) return;
  const int64_t q = id / a.S;
  const int s = (int)(id % a.S);
  const float* x = a.Q + q * a.d + (int64_t)s * a.w;
  uint32_t* dst = reinterpret_cast<uint32_t*>(a.clq + id * KP);
  int nlo = 0, nhi = 0;
#pragma unroll
  for (int t0 = 0; t0 < KP; t0 += 4) {
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = t0 + j;
      const int v = t < a.w ? cl_code(x[t], a.o, a.ec) : 0;
      const int vl = cl_trunc(v, a.lo), vh = cl_trunc(v, a.hi);
      nlo += vl * vl;
      nhi += vh * vh;
      word |= ((uint32_t)v & 0xFFu) << (8 * j);
    }
    dst[t0 / 4] = word;
  }
  a.clqn[id * 2] = nlo;
  a.clqn[id * 2 + 1] = nhi;
}

template <int KP>
__global__ __launch_bounds__(256) void k_clcn(ClArgs a) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)a.nlist * a.S) return;
  const int8_t* c = a.clc + id * KP;
  int nlo = 0, nhi = 0;
  for (int t = 0; t < a.w; ++t) {
    const int v = c[t];
    const int vl = cl_trunc(v, a.lo), vh = cl_trunc(v, a.hi);
    nlo += vl * vl;
    nhi += vh * vh;
  }
  a.clcn[id * 2] = nlo;
  a.clcn[id * 2 + 1] = nhi;
}

__device__ __forceinline__ int64_t cl_mitchell_q8(int64_t x) {
  uint64_t y = (uint64_t)x + 1;
  int k = 63 - __clzll((long long)y);
  return 256 * (int64_t)k + (int64_t)((y << 8) >> k) - 256;
}

// the 10-bit feature of one raw feature value
__device__ __forceinline__ int32_t cl_feature(int64_t x, const ModelArgs& ma, int f) {
  const int64_t v = ((cl_mitchell_q8(x) - ma.feat_lo[f]) * ma.feat_mul[f]) >> 16;
  return (int32_t)(v < 0 ? 0 : (v > 1023 ? 1023 : v));
}

// regressor score of one feature vector (the support vectors are the same
// across the wave: scalar loads); u and sv lie in [0, 1023]: exact 24-bit
// products, |u - sv|^2 < 2^23
__device__ __forceinline__ int64_t cl_score(const int32_t (&uf)[5], const ModelArgs& ma, const int32_t* s_table) {
  const uint32_t gm = (uint32_t)ma.g_mul;
  auto term = [&](int i) -> int64_t {
    const int32_t* sv = ma.sv + 5 * i;
    const int e0 = uf[0] - sv[0], e1 = uf[1] - sv[1], e2 = uf[2] - sv[2], e3 = uf[3] - sv[3], e4 = uf[4] - sv[4];
    const uint32_t dist2 = (uint32_t)(__mul24(e0, e0) + __mul24(e1, e1) + __mul24(e2, e2) + __mul24(e3, e3) +
                                      __mul24(e4, e4));
    const uint32_t idx = __umulhi(dist2, gm);
    const int32_t K = s_table[idx < (uint32_t)(kTableN - 1) ? idx : (uint32_t)(kTableN - 1)];
    return (int64_t)ma.beta[i] * K;
  };
  int64_t y0 = 0, y1 = 0;
  int i = 0;
  for (; i + 1 < ma.n_sv; i += 2) {
    y0 += term(i);
    y1 += term(i + 1);
  }
  if (i < ma.n_sv) y0 += term(i);
  return ma.beta0 + y0 + y1;
}

// Exact decision table of the CL predictor: for slice s, nearest sub-space
// C1 and sub-space u the features r1, n1 (of C1) and r2, n2 (of u) are
// fixed, so the width is a function of the 10-bit d' feature alone.  One
// wave per (s, C1, u) evaluates the regressor at all 1024 values: bit ud of
// the 32-word row is 1 where the low width is chosen.
__global__ __launch_bounds__(256) void k_cltab(ClArgs a, ModelArgs ma, uint32_t* tab) {
  __shared__ int32_t s_table[kTableN];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < kTableN; i += 256) s_table[i] = ma.table[i];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;  // (s * P + c1) * P + u
  if (row >= (int64_t)a.S * a.P * a.P) return;
  const int u = (int)(row % a.P), c1 = (int)((row / a.P) % a.P), s = (int)(row / ((int64_t)a.P * a.P));
  int32_t uf[5];
  uf[1] = cl_feature(a.clr[(int64_t)s * a.P + c1], ma, 1);
  uf[2] = cl_feature(a.clr[(int64_t)s * a.P + u], ma, 2);
  uf[3] = cl_feature(a.cln[(int64_t)s * a.P + c1], ma, 3);
  uf[4] = cl_feature(a.cln[(int64_t)s * a.P + u], ma, 4);
#pragma unroll 1
  for (int j = 0; j < 16; ++j) {
    uf[0] = j * 64 + lane;
    const bool low = cl_score(uf, ma, s_table) <= ma.theta[0];
    const uint64_t m = __ballot(low);
    if (lane == 0) {
      tab[row * 32 + 2 * j] = (uint32_t)m;
      tab[row * 32 + 2 * j + 1] = (uint32_t)(m >> 32);
    }
  }
}

// One wave per (query, slice); lanes over the sub-spaces (P <= 1024).
template <int KP>
__global__ __launch_bounds__(256) void k_clbits(ClArgs a, ModelArgs ma) {
  __shared__ int32_t s_table[kTableN];
  __shared__ int32_t s_v[4][64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < kTableN; i += 256) s_table[i] = ma.table[i];
  const int64_t item = (int64_t)blockIdx.x * 4 + wave;
  const bool on = item < (int64_t)a.nq * a.S;
  s_v[wave][lane] = (on && lane < a.w) ? (int)a.clq[item * KP + lane] : 0;
  __syncthreads();
  if (!on) return;
  const int s = (int)(item % a.S);
  const int nj = (a.P + 63) >> 6;
  // d' of every sub-space (exact: below 64 * 255^2 < 2^22)
  int32_t d2v[16];
  uint64_t best = ~0ull;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    d2v[j] = 0;
    const int u = j * 64 + lane;
    if (j < nj && u < a.P) {
      const int8_t* z = a.clz + ((int64_t)s * a.P + u) * KP;
      int acc = 0;
      for (int t = 0; t < a.w; ++t) {
        const int df = s_v[wave][t] - (int)z[t];
        acc += df * df;
      }
      d2v[j] = acc;
      const uint64_t key = ((uint64_t)acc << 10) | (uint64_t)u;  // ties: lower index
      best = key < best ? key : best;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(best, off);
    best = o < best ? o : best;
  }
  const int c1 = (int)(best & 1023u);
  const int64_t rowbase = ((int64_t)s * a.P + c1) * a.P;
  int32_t uf[5];
  if (!a.tab) {
    uf[1] = cl_feature(a.clr[(int64_t)s * a.P + c1], ma, 1);
    uf[3] = cl_feature(a.cln[(int64_t)s * a.P + c1], ma, 3);
  }
#pragma unroll 1
  for (int j = 0; j < nj; ++j) {
    const int u = j * 64 + lane;
    bool low = false;
    if (u < a.P) {
      const int32_t ud = cl_feature(d2v[j], ma, 0);
      if (a.tab) {
        // the exact decision table: one bit read
        low = (a.tab[(rowbase + u) * 32 + (ud >> 5)] >> (ud & 31)) & 1u;
      } else {
        uf[0] = ud;
        uf[2] = cl_feature(a.clr[(int64_t)s * a.P + u], ma, 2);
        uf[4] = cl_feature(a.cln[(int64_t)s * a.P + u], ma, 4);
        low = cl_score(uf, ma, s_table) <= ma.theta[0];
      }
      if (a.out_bits) a.out_bits[item * a.P + u] = (uint8_t)(low ? a.lo : a.hi);
    }
    const uint64_t m = __ballot(low);
    if (lane == 0) {
      a.clmask[item * a.PW + 2 * j] = (uint32_t)m;
      if (2 * j + 1 < a.PW) a.clmask[item * a.PW + 2 * j + 1] = (uint32_t)(m >> 32);
    }
  }
}

// 64 x 64 (query, centroid) tile per workgroup, each wave a 32 x 32 quarter
// of 2 x 2 int8 MFMA 16x16 tiles; one K pass (32 or 64 bytes) per slice.
template <int KP, bool ADAPT, bool IP>
__global__ __launch_bounds__(256) void k_coarse_int(ClArgs a) {
  __shared__ uint32_t s_mask[ADAPT ? 64 * 32 : 1];
  __shared__ int32_t s_qn[64][2], s_cn[64][2];
  __shared__ uint16_t s_asg[64];
  const int q0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const uint32_t mlo = cl_bytemask(a.lo), mhi = cl_bytemask(a.hi);
  int64_t arow[2], brow[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    // rows beyond the matrix read a valid row; their outputs are not written
    const int qr = q0 + wr + 16 * t + (lane & 15), cr = c0 + wc + 16 * t + (lane & 15);
    arow[t] = qr < a.nq ? qr : a.nq - 1;
    brow[t] = cr < a.nlist ? cr : a.nlist - 1;
  }
  int acc[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
  for (int s = 0; s < a.S; ++s) {
    __syncthreads();  // the previous slice's tables are no longer read
    if (ADAPT)
      for (int idx = tid; idx < 64 * a.PW; idx += 256) {
        const int r = idx / a.PW, wv = idx % a.PW, qq = q0 + r;
        s_mask[r * a.PW + wv] = qq < a.nq ? a.clmask[((int64_t)qq * a.S + s) * a.PW + wv] : 0u;
      }
    if (!IP && tid < 64) {
      const int64_t qq = q0 + tid < a.nq ? q0 + tid : a.nq - 1;
      s_qn[tid][0] = a.clqn[(qq * a.S + s) * 2];
      s_qn[tid][1] = a.clqn[(qq * a.S + s) * 2 + 1];
    } else if (!IP && tid < 128) {
      const int64_t cc = c0 + tid - 64 < a.nlist ? c0 + tid - 64 : a.nlist - 1;
      s_cn[tid - 64][0] = a.clcn[(cc * a.S + s) * 2];
      s_cn[tid - 64][1] = a.clcn[(cc * a.S + s) * 2 + 1];
    } else if (ADAPT && tid >= 128 && tid < 192) {
      const int64_t cc = c0 + tid - 128 < a.nlist ? c0 + tid - 128 : a.nlist - 1;
      s_asg[tid - 128] = a.clasg[cc * a.S + s];
    }
    __syncthreads();
    v4i phi[2][2], plo[2][2];
    if constexpr (KP == 32) {
      u32x2 A[2], B[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        A[t] = *reinterpret_cast<const u32x2*>(a.clq + (arow[t] * a.S + s) * KP + g * 8);
        B[t] = *reinterpret_cast<const u32x2*>(a.clc + (brow[t] * a.S + s) * KP + g * 8);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const u32x2 ah = A[i] & mhi, bh = B[j] & mhi;
          phi[i][j] = __builtin_amdgcn_mfma_i32_16x16x32_i8(__builtin_bit_cast(long, ah), __builtin_bit_cast(long, bh),
                                                            (v4i){0, 0, 0, 0}, 0, 0, 0);
          if constexpr (ADAPT) {
            const u32x2 al = A[i] & mlo, bl = B[j] & mlo;
            plo[i][j] = __builtin_amdgcn_mfma_i32_16x16x32_i8(__builtin_bit_cast(long, al),
                                                              __builtin_bit_cast(long, bl), (v4i){0, 0, 0, 0}, 0, 0, 0);
          }
        }
    } else {
      u32x4 A[2], B[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        A[t] = *reinterpret_cast<const u32x4*>(a.clq + (arow[t] * a.S + s) * KP + g * 16);
        B[t] = *reinterpret_cast<const u32x4*>(a.clc + (brow[t] * a.S + s) * KP + g * 16);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const u32x4 ah = A[i] & mhi, bh = B[j] & mhi;
          phi[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(v4i, ah), __builtin_bit_cast(v4i, bh),
                                                            (v4i){0, 0, 0, 0}, 0, 0, 0);
          if constexpr (ADAPT) {
            const u32x4 al = A[i] & mlo, bl = B[j] & mlo;
            plo[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(v4i, al),
                                                              __builtin_bit_cast(v4i, bl), (v4i){0, 0, 0, 0}, 0, 0, 0);
          }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int cl = wc + 16 * j + (lane & 15);
        int sub = 0;
        if constexpr (ADAPT) sub = s_asg[cl];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ql = wr + 16 * i + 4 * g + r;
          int low = 0;
          if constexpr (ADAPT) low = (s_mask[ql * a.PW + (sub >> 5)] >> (sub & 31)) & 1;
          const int dot = low ? plo[i][j][r] : phi[i][j][r];
          const int slot = low ? 0 : 1;
          acc[i][j][r] += IP ? -dot : s_qn[ql][slot] + s_cn[cl][slot] - 2 * dot;
        }
      }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = q0 + wr + 16 * i + 4 * g + r, c = c0 + wc + 16 * j + (lane & 15);
        if (q < a.nq && c < a.nlist) {
          const int D = acc[i][j][r];
          // order keys as non-negative float bit patterns (inner product:
          // offset by 2^30; |D| < 2^25)
          a.keys[(int64_t)q * a.nlist + c] = __int_as_float(IP ? D + (1 << 30) : D);
          if (a.out_d) a.out_d[(int64_t)q * a.nlist + c] = D;
        }
      }
}

template <int KP>
hipError_t launch_cl_kp(const ClArgs& a, bool adaptive, bool ip, const ModelArgs& clma, hipStream_t st) {
  const int64_t items = (int64_t)a.nq * a.S;
  hipLaunchKernelGGL(k_clq<KP>, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_clcn<KP>, dim3((unsigned)(((int64_t)a.nlist * a.S + 255) / 256)), dim3(256), 0, st, a);
  if (adaptive) hipLaunchKernelGGL(k_clbits<KP>, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st, a, clma);
  const dim3 grid((a.nlist + 63) / 64, (a.nq + 63) / 64);
  if (adaptive) {
    if (ip) hipLaunchKernelGGL((k_coarse_int<KP, true, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_coarse_int<KP, true, false>), grid, dim3(256), 0, st, a);
  } else {
    if (ip) hipLaunchKernelGGL((k_coarse_int<KP, false, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_coarse_int<KP, false, false>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cltab(const amp_index* ix, const ModelArgs& clma, uint32_t* tab, hipStream_t st) {
  const DeviceIndex& dv = ix->dev;
  ClArgs a{};
  a.S = ix->cl_S;
  a.P = ix->cl_P;
  a.clr = dv.clr;
  a.cln = dv.cln;
  const int64_t rows = (int64_t)a.S * a.P * a.P;
  hipLaunchKernelGGL(k_cltab, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, a, clma, tab);
  return hipGetLastError();
}

hipError_t launch_cl(const amp_index* ix, const Workspace& ws, const float* queries, const SearchDims& sd,
                     const ModelArgs& clma, float* keys, hipStream_t st) {
  const DeviceIndex& dv = ix->dev;
  ClArgs a{};
  a.tab = sd.cl_tab;
  a.Q = queries;
  a.nq = sd.nq;
  a.d = sd.d;
  a.nlist = sd.nlist;
  a.S = sd.cl_S;
  a.P = sd.cl_P;
  a.PW = sd.cl_pw;
  a.w = sd.cl_w;
  a.ec = sd.cl_ec;
  a.o = sd.cl_o;
  a.lo = sd.cl_lo;
  a.hi = sd.cl_hi;
  a.clq = ws.clq;
  a.clqn = ws.clqn;
  a.clmask = ws.clmask;
  a.clcn = ws.clcn;
  a.clc = dv.clc;
  a.clasg = dv.clasg;
  a.clz = dv.clz;
  a.clr = dv.clr;
  a.cln = dv.cln;
  a.keys = keys;
  a.out_d = sd.out_cl_dist;
  a.out_bits = sd.out_cl_bits;
  const bool adaptive = sd.cl_policy == AMP_CL_ADAPTIVE, ip = sd.metric == AMP_IP;
  return sd.cl_kp == 32 ? launch_cl_kp<32>(a, adaptive, ip, clma, st) : launch_cl_kp<64>(a, adaptive, ip, clma, st);
}

}  // namespace amp
