// HIP kernels (gfx950) of the cluster-adaptive IVF-PQ search.
//
// Stage map (paper Sec. 2.1 and Sec. 4.1):
//   k_sqnorm / k_coarse  CL distances on FP32 MFMA (16x16x4) with norm epilogue
//   k_topn*              CL selection: nprobe smallest by (distance, list id)
//   k_pairs              RC on the operand grid, PPM features and the fixed-point
//                        RBF regressor -> LUT width per (query, probed list)
//   k_qhist/qscan/qscatter  work queue: pairs grouped by (lane class, list)
//   k_scan<...>          persistent: LC on BF16 MFMA (exact on the grid),
//                        per-pair quantisation, packed-lane DC scan, pruning
//                        against the query's running threshold (TSM forwarding)
//   k_merge              TS: per-query top-k by (distance, id)
#include "scan_kernels.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace amp {

// ------------------------------------------------------------------ resets
// the per-search resets of the search workspace in one launch (fills by
// kernel, not memsets: a captured search graph holds no memset node):
// bucket counters, unit counters, flags and work counters to 0, bounds to
// "none", candidate counts to 0
struct ResetArgs {
  uint32_t* cnt;
  size_t ncnt;
  uint32_t* counters;
  size_t ncounters;
  uint32_t* flags;   // [4]
  uint64_t* work;    // [4]
  uint64_t* tau;     // [nq]
  uint32_t* ccount;  // [nq]
  int32_t* ipmask;   // [nq] or null
  size_t nq;
};
__global__ void k_reset(ResetArgs r) {
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, st = (size_t)gridDim.x * blockDim.x;
  for (size_t i = i0; i < r.ncnt; i += st) r.cnt[i] = 0;
  for (size_t i = i0; i < r.ncounters; i += st) r.counters[i] = 0;
  for (size_t i = i0; i < r.nq; i += st) {
    r.tau[i] = ~0ull;
    r.ccount[i] = 0;
    if (r.ipmask) r.ipmask[i] = 0;
  }
  if (i0 < 4) {
    r.flags[i0] = 0;
    r.work[i0] = 0;
  }
}

// per-query sizes handed over in device memory: each k into [1, kmax] and
// nprobe into [1, npmax] (flag 32 if one was outside), copied into the
// workspace's per-query arrays
__global__ void k_sizes(const int32_t* __restrict__ kin, const int32_t* __restrict__ npin, int32_t* __restrict__ kout,
                        int32_t* __restrict__ npout, int nq, int kmax, int npmax, int32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int kv = kin[i], nv = npin[i];
  const int kc = kv < 1 ? 1 : (kv > kmax ? kmax : kv);
  const int nc = nv < 1 ? 1 : (nv > npmax ? npmax : nv);
  if (kc != kv || nc != nv) atomicOr(&flags[0], 32);
  kout[i] = kc;
  npout[i] = nc;
}

// status word of a search from its error flags (the host-mode mapping):
// 16 / 8 internal errors, 32 a clamped size, 4 unit table and 2 candidate
// overflow
__global__ void k_status(const int32_t* __restrict__ flags, int32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const int32_t f = flags[0];
  int32_t s = AMP_OK;
  if (f & (16 | 8)) s = AMP_EDEVICE;
  else if (f & 32) s = AMP_EINVAL;
  else if (f) s = AMP_EOVERFLOW;
  *out = s;
}

// ------------------------------------------------------------------ CL
// squared norm of each row, FP32: one wave per row, lane-strided partial sums
// combined by a butterfly (a fixed order for a given d)
__global__ void k_sqnorm(const float* __restrict__ X, int rows, int d, float* __restrict__ out) {
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= rows) return;
  const float* x = X + (size_t)r * d;
  float s = 0.f;
  for (int t = lane; t < d; t += 64) s = fmaf(x[t], x[t], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[r] = s;
}

// D[q][c] = (|q|^2 + |c|^2) - 2 q.c (L2) or -q.c (IP).  64x64 tile per
// workgroup, each wave a 32x32 quarter of 2x2 MFMA 16x16x4 FP32 tiles; K in
// chunks of KC staged through LDS, the next chunk's loads issued before the
// current chunk's products (16-byte loads when d is a multiple of 4 and the
// rows 16-byte aligned).  The products run in k order whatever the chunk, so
// the sums do not depend on it.
constexpr int CL_T = 64, CL_K = 32;
template <int KC, bool VEC>
__global__ __launch_bounds__(256) void k_coarse(const float* __restrict__ Q, const float* __restrict__ C,
                                                const float* __restrict__ qn, const float* __restrict__ cn,
                                                float* __restrict__ D, int nq, int nlist, int d, int metric) {
  __shared__ float Qs[CL_T][KC + 1];
  __shared__ float Cs[CL_T][KC + 1];
  const int q0 = blockIdx.y * CL_T, c0 = blockIdx.x * CL_T;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  constexpr int NV = CL_T * KC / 4 / 256;  // 16-byte loads per thread and tile
  float4 qa[NV], ca[NV];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int f = tid + 256 * u, r = f / (KC / 4), gk = k0 + 4 * (f % (KC / 4));
      if (VEC) {
        qa[u] = (q0 + r < nq && gk < d) ? *reinterpret_cast<const float4*>(Q + (size_t)(q0 + r) * d + gk)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        ca[u] = (c0 + r < nlist && gk < d) ? *reinterpret_cast<const float4*>(C + (size_t)(c0 + r) * d + gk)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        float* qv = &qa[u].x;
        float* cv = &ca[u].x;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          qv[e] = (q0 + r < nq && gk + e < d) ? Q[(size_t)(q0 + r) * d + gk + e] : 0.f;
          cv[e] = (c0 + r < nlist && gk + e < d) ? C[(size_t)(c0 + r) * d + gk + e] : 0.f;
        }
      }
    }
  };
  f4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  load(0);
  for (int k0 = 0; k0 < d; k0 += KC) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int f = tid + 256 * u, r = f / (KC / 4), kk = 4 * (f % (KC / 4));
      Qs[r][kk] = qa[u].x; Qs[r][kk + 1] = qa[u].y; Qs[r][kk + 2] = qa[u].z; Qs[r][kk + 3] = qa[u].w;
      Cs[r][kk] = ca[u].x; Cs[r][kk + 1] = ca[u].y; Cs[r][kk + 2] = ca[u].z; Cs[r][kk + 3] = ca[u].w;
    }
    __syncthreads();
    if (k0 + KC < d) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      float a0 = Qs[wr + (lane & 15)][kk + (lane >> 4)];
      float a1 = Qs[wr + 16 + (lane & 15)][kk + (lane >> 4)];
      float b0 = Cs[wc + (lane & 15)][kk + (lane >> 4)];
      float b1 = Cs[wc + 16 + (lane & 15)][kk + (lane >> 4)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        int qi = q0 + wr + 16 * i + 4 * (lane >> 4) + r;
        int ci = c0 + wc + 16 * j + (lane & 15);
        if (qi < nq && ci < nlist) {
          float dot = acc[i][j][r];
          D[(size_t)qi * nlist + ci] = metric == AMP_L2 ? (qn[qi] + cn[ci]) - 2.f * dot : -dot;
        }
      }
}

// CL under L1: D = sum_t |q_t - c_t| (no dense product to put on MFMA):
// 64 x 64 (query, centroid) tile per workgroup staged through LDS, each
// thread 16 sums
__global__ __launch_bounds__(256) void k_coarse_l1(const float* __restrict__ Q, const float* __restrict__ C,
                                                   float* __restrict__ D, int nq, int nlist, int d) {
  __shared__ float Qs[CL_T][CL_K + 1];
  __shared__ float Cs[CL_T][CL_K + 1];
  const int q0 = blockIdx.y * CL_T, c0 = blockIdx.x * CL_T;
  const int tid = threadIdx.x, tq = tid >> 4, tc = tid & 15;
  float acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = 0; k0 < d; k0 += CL_K) {
    for (int i = tid; i < CL_T * CL_K; i += 256) {
      const int r = i / CL_K, kk = i % CL_K, gk = k0 + kk;
      Qs[r][kk] = (q0 + r < nq && gk < d) ? Q[(size_t)(q0 + r) * d + gk] : 0.f;
      Cs[r][kk] = (c0 + r < nlist && gk < d) ? C[(size_t)(c0 + r) * d + gk] : 0.f;
    }
    __syncthreads();
    for (int kk = 0; kk < CL_K; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += fabsf(Qs[tq + 16 * i][kk] - Cs[tc + 16 * j][kk]);
    __syncthreads();
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int qi = q0 + tq + 16 * i, ci = c0 + tc + 16 * j;
      if (qi < nq && ci < nlist) D[(size_t)qi * nlist + ci] = acc[i][j];
    }
}

// grid codebook as int16 [M][256][8] (zero-padded), for the L1 LUT build
__global__ void k_prep_cbi(const float* __restrict__ cb, int M, int dsub, int grid_e, int grid_kind,
                           int16_t* __restrict__ cbi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * kKsub * 8) return;
  const int t = i & 7, e = i >> 3;
  cbi[i] = t < dsub ? (int16_t)grid_val(cb[(size_t)e * dsub + t], grid_e, grid_kind) : (int16_t)0;
}

// bfloat16 bit patterns to FP32 (exact: the pattern is the top half)
__global__ void k_bf16_widen(const uint16_t* __restrict__ in, float* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = __uint_as_float((uint32_t)in[i] << 16);
}

// ------------------------------------------------------------------ index build
// squared norms of n rows of dd floats with leading dimension ld (a wave per row)
__global__ void k_sqnorm_ld(const float* __restrict__ X, int64_t n, int dd, int ld, float* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  float s = 0.f;
  for (int t = lane; t < dd; t += 64) {
    const float v = X[r * ld + t];
    s = fmaf(v, v, s);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[r] = s;
}

// nearest of k centroids (squared L2 in FP32, ties to the lower index) for n
// rows of dd floats (leading dimension ld) and its distance.  64 rows per
// workgroup; centroids in tiles of 64 on FP32 MFMA 16x16x4 (the coarse
// distance kernel's tiling); each tile's distances go through LDS and the
// row's thread keeps the running minimum.
__global__ __launch_bounds__(256) void k_assign(const float* __restrict__ X, const float* __restrict__ xn,
                                                int64_t n, int dd, int ld, const float* __restrict__ C,
                                                const float* __restrict__ cn, int k, int32_t* __restrict__ out_a,
                                                float* __restrict__ out_d) {
  __shared__ float Xs[CL_T][CL_K + 1];
  __shared__ float Cs[CL_T][CL_K + 1];
  __shared__ float Ds[CL_T][CL_T + 1];
  const int64_t r0 = (int64_t)blockIdx.x * CL_T;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  float best = 3.4e38f;
  int besti = 0;
  for (int c0 = 0; c0 < k; c0 += CL_T) {
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < dd; k0 += CL_K) {
      for (int i = tid; i < CL_T * CL_K; i += 256) {
        const int r = i / CL_K, kk = i % CL_K, gk = k0 + kk;
        Xs[r][kk] = (r0 + r < n && gk < dd) ? X[(r0 + r) * ld + gk] : 0.f;
        Cs[r][kk] = (c0 + r < k && gk < dd) ? C[(size_t)(c0 + r) * dd + gk] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < CL_K; kk += 4) {
        const float a0 = Xs[wr + (lane & 15)][kk + (lane >> 4)];
        const float a1 = Xs[wr + 16 + (lane & 15)][kk + (lane >> 4)];
        const float b0 = Cs[wc + (lane & 15)][kk + (lane >> 4)];
        const float b1 = Cs[wc + 16 + (lane & 15)][kk + (lane >> 4)];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int q = 0; q < 4; ++q) {
          const int rr = wr + 16 * i + 4 * (lane >> 4) + q, cc = wc + 16 * j + (lane & 15);
          Ds[rr][cc] = c0 + cc < k ? cn[c0 + cc] - 2.f * acc[i][j][q] : 3.4e38f;
        }
    __syncthreads();
    if (tid < CL_T)
      for (int c = 0; c < CL_T && c0 + c < k; ++c) {
        const float v = Ds[tid][c];
        if (v < best) {
          best = v;
          besti = c0 + c;
        }
      }
    __syncthreads();
  }
  if (tid < CL_T && r0 + tid < n) {
    out_a[r0 + tid] = besti;
    if (out_d) out_d[r0 + tid] = best + xn[r0 + tid];
  }
}

// residual rows x - c_a of a chunk
__global__ void k_residual(const float* __restrict__ X, const int32_t* __restrict__ a, const float* __restrict__ C,
                           int64_t n, int d, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  const int64_t r = i / d;
  const int t = (int)(i - r * d);
  out[i] = X[i] - C[(size_t)a[r] * d + t];
}

// ------------------------------------------------------------------ sorting
// ascending bitonic sort of n (power of two) 64-bit keys in LDS by the block
__device__ void block_bitonic_u64(uint64_t* keys, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        int pos = 2 * i - (i & (stride - 1));
        int oth = pos + stride;
        bool asc = (pos & size) == 0;
        uint64_t a = keys[pos], b = keys[oth];
        if ((a > b) == asc) {
          keys[pos] = b;
          keys[oth] = a;
        }
      }
      __syncthreads();
    }
  }
}

// the kk-th smallest (1-based, kk <= n) of n 64-bit keys in LDS, by radix
// select: passes over 8-bit digits, most significant first, each
// counting the digits of the keys that share the digits chosen so far and
// choosing the digit whose count range holds the remaining rank.  hist: 256
// counters in LDS; sel: two words in LDS.  Every thread of the block returns
// the key.
__device__ uint64_t block_select_u64(const uint64_t* keys, int n, int kk, uint32_t* hist, uint32_t* sel) {
  const int tid = threadIdx.x, lane = tid & 63;
  // the digits above the highest bit where the smallest and largest keys
  // differ are common to every key: the passes start below them
  uint64_t lo = ~0ull, hi = 0;
  for (int i = tid; i < n; i += blockDim.x) {
    const uint64_t k = keys[i];
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  uint64_t* mm = reinterpret_cast<uint64_t*>(hist);  // two words a wave (at most 16 waves)
  if (lane == 0) {
    mm[2 * (tid >> 6)] = lo;
    mm[2 * (tid >> 6) + 1] = hi;
  }
  __syncthreads();
  lo = mm[0];
  hi = mm[1];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
    lo = mm[2 * w] < lo ? mm[2 * w] : lo;
    hi = mm[2 * w + 1] > hi ? mm[2 * w + 1] : hi;
  }
  __syncthreads();  // hist is cleared by the first pass
  if (lo == hi) return lo;
  const int top = (63 - __builtin_clzll(lo ^ hi)) & ~7;
  uint64_t mask = top >= 56 ? 0ull : ~((1ull << (top + 8)) - 1);
  uint64_t prefix = lo & mask;
  uint32_t rank = (uint32_t)kk;
  for (int shift = top; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      const uint64_t k = keys[i];
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      // four bins a lane, inclusive scan over the wave
      const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
      const uint32_t own = h0 + h1 + h2 + h3;
      uint32_t inc = own;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
      }
      const uint32_t below = inc - own;
      if (below < rank && rank <= inc) {
        uint32_t c = below, dg = 4 * lane;
        if (c + h0 < rank) {
          c += h0;
          ++dg;
          if (c + h1 < rank) {
            c += h1;
            ++dg;
            if (c + h2 < rank) {
              c += h2;
              ++dg;
            }
          }
        }
        sel[0] = dg;
        sel[1] = c;
      }
    }
    __syncthreads();
    prefix |= (uint64_t)sel[0] << shift;
    mask |= 255ull << shift;
    rank -= sel[1];
    __syncthreads();  // sel and hist are rewritten by the next pass
  }
  return prefix;
}

// same with a secondary signed 64-bit tie-breaker
__device__ void block_bitonic_u64_i64(uint64_t* keys, int64_t* vals, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        int pos = 2 * i - (i & (stride - 1));
        int oth = pos + stride;
        bool asc = (pos & size) == 0;
        uint64_t a = keys[pos], b = keys[oth];
        int64_t va = vals[pos], vb = vals[oth];
        bool gt = (a > b) || (a == b && va > vb);
        if (gt == asc) {
          keys[pos] = b;
          keys[oth] = a;
          vals[pos] = vb;
          vals[oth] = va;
        }
      }
      __syncthreads();
    }
  }
}

// CL selection: the nprobe smallest (distance, list) of each query.
// General case: a workgroup per query, bitonic sort of all nlist keys in LDS.
__global__ __launch_bounds__(256) void k_topn(const float* __restrict__ D, int nlist, int np2,
                                              const int32_t* __restrict__ npq, int npconst, int npmax,
                                              int32_t* __restrict__ probes) {
  extern __shared__ uint64_t keys[];
  const int q = blockIdx.x;
  const float* row = D + (size_t)q * nlist;
  for (int i = threadIdx.x; i < np2; i += blockDim.x)
    keys[i] = i < nlist ? (((uint64_t)fkey(row[i]) << 32) | (uint32_t)i) : ~0ull;
  __syncthreads();
  block_bitonic_u64(keys, np2);
  const int np = npq ? npq[q] : npconst;
  for (int r = threadIdx.x; r < npmax; r += blockDim.x)
    probes[(size_t)q * npmax + r] = r < np ? (int32_t)(keys[r] & 0xFFFFFFFFu) : -1;
}

// nlist <= 256 * PER (larger rows or nprobe > 64): a workgroup per query
// holds the row in registers (key j * 256 + thread).  The nprobe-th smallest
// order key x is found bit by bit: the count of keys below a candidate is
// the sum over the four waves of ballot bit counts, exchanged through LDS
// (two alternating slots: one barrier per bit).  The keys up to x, with
// their list ids, are gathered in LDS (any order); up to 512 of them each
// take the output row of their rank by (key, list id) among them, more are
// padded to a power of two and sorted.  The first nprobe are the probes,
// the same as a sort of the whole row.
template <int PER>
__global__ __launch_bounds__(256) void k_topn_wg(const float* __restrict__ D, int nlist,
                                                 const int32_t* __restrict__ npq, int npconst, int npmax,
                                                 int32_t* __restrict__ probes) {
  extern __shared__ uint64_t sel[];  // room for the next power of two >= nlist
  __shared__ int s_cnt[2][4];
  __shared__ int s_n;
  const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float* row = D + (size_t)q * nlist;
  uint32_t key[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = j * 256 + tid;
    key[j] = i < nlist ? fkey(row[i]) : 0xFFFFFFFFu;
  }
  const int k = npq ? npq[q] : npconst;
  if (tid == 0) s_n = 0;
  uint32_t x = 0;  // largest value with fewer than k keys below it: the k-th smallest
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t t = x | (1u << bit);
    int c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) c += __popcll(__ballot(key[j] < t));
    if (lane == 0) s_cnt[bit & 1][wv] = c;
    __syncthreads();
    if (s_cnt[bit & 1][0] + s_cnt[bit & 1][1] + s_cnt[bit & 1][2] + s_cnt[bit & 1][3] < k) x = t;
  }
  // gather the keys <= x (at least k of them; ties at x all come along)
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = j * 256 + tid;
    const bool take = i < nlist && key[j] <= x;
    const uint64_t bal = __ballot(take);
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(&s_n, __popcll(bal));
    base = __shfl(base, 0);
    if (take) sel[base + __popcll(bal & ((1ull << lane) - 1))] = ((uint64_t)key[j] << 32) | (uint32_t)i;
  }
  __syncthreads();
  const int n = s_n;
  if (n <= 512) {  // uniform over the workgroup
    // (key, list id) are distinct: each selected key's output row is the
    // count of selected keys below it (no sort, no barrier)
    for (int t = tid; t < n; t += 256) {
      const uint64_t v = sel[t];
      int rank = 0;
      for (int j = 0; j < n; ++j) rank += sel[j] < v;
      if (rank < npmax) probes[(size_t)q * npmax + rank] = rank < k ? (int32_t)(v & 0xFFFFFFFFu) : -1;
    }
    for (int r = n + tid; r < npmax; r += 256) probes[(size_t)q * npmax + r] = -1;
    return;
  }
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = n + tid; i < n2; i += 256) sel[i] = ~0ull;
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < (n2 >> 1); i += 256) {
        const int pos = 2 * i - (i & (stride - 1));
        const bool asc = (pos & size) == 0;
        const uint64_t u = sel[pos], v = sel[pos + stride];
        if ((u > v) == asc) {
          sel[pos] = v;
          sel[pos + stride] = u;
        }
      }
      __syncthreads();
    }
  for (int r = tid; r < npmax; r += 256)
    probes[(size_t)q * npmax + r] = r < k ? (int32_t)(sel[r] & 0xFFFFFFFFu) : -1;
}

// nlist <= 64 * PER and nprobe <= 64: one wave per query, no sort of the
// whole row.  Lane l holds keys l, l + 64, ...  The nprobe-th smallest
// order key is found bit by bit (count of keys below a candidate, summed
// over the wave); the keys below it, and the equal ones with the lowest list
// ids, are compacted and sorted by (key, list) across the lanes.
template <int PER>
__global__ __launch_bounds__(256) void k_topn_wave(const float* __restrict__ D, int nlist, int nq,
                                                   const int32_t* __restrict__ npq, int npconst, int npmax,
                                                   int32_t* __restrict__ probes) {
  __shared__ uint64_t s_sel[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = blockIdx.x * 4 + wv;
  const bool on = q < nq;  // no early return: the workgroup synchronises below
  uint32_t key[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = j * 64 + lane;
    key[j] = on && i < nlist ? fkey(D[(size_t)q * nlist + i]) : 0xFFFFFFFFu;
  }
  const int k = on ? (npq ? npq[q] : npconst) : 0;
  // wave-wide count of keys below t: one ballot per key slot and a bit
  // count of the mask (no cross-lane shuffles)
  auto count_below = [&](uint32_t t) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) c += __popcll(__ballot(key[j] < t));
    return c;
  };
  uint32_t x = 0;  // largest value with fewer than k keys below it: the k-th smallest
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t t = x | (1u << bit);
    if (count_below(t) < k) x = t;
  }
  int need_eq = k - count_below(x);  // keys equal to x to take, lowest list id first
  s_sel[wv][lane] = ~0ull;
  __syncthreads();
  int base = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {  // list ids ascend with (j, lane)
    const bool eq = key[j] == x;
    const uint64_t meq = __ballot(eq);
    const int eq_rank = __popcll(meq & ((1ull << lane) - 1));
    const bool sel = on && (key[j] < x || (eq && eq_rank < need_eq));
    need_eq -= __popcll(meq) < need_eq ? __popcll(meq) : need_eq;
    const uint64_t msel = __ballot(sel);
    if (sel) {
      const int pos = base + __popcll(msel & ((1ull << lane) - 1));
      s_sel[wv][pos] = ((uint64_t)key[j] << 32) | (uint32_t)(j * 64 + lane);
    }
    base += __popcll(msel);
  }
  __syncthreads();
  uint64_t v = s_sel[wv][lane];
  for (int kb = 2; kb <= 64; kb <<= 1)
    for (int jb = kb >> 1; jb > 0; jb >>= 1) {
      const uint64_t o = __shfl_xor(v, jb);
      const bool keep_min = ((lane & kb) == 0) == ((lane & jb) == 0);
      v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
    }
  if (on && lane < npmax) probes[(size_t)q * npmax + lane] = lane < k ? (int32_t)(v & 0xFFFFFFFFu) : -1;
}

// ------------------------------------------------------------------ PPM
struct PairArgs {
  const float* Q;
  const float* C;
  const int16_t* qi16;    // inner product: queries and centroids on the grid (d' = |qi - ci|^2)
  const int16_t* ci16;
  int64_t* dot_out;       // adaptive inner product: qi.ci of every pair (read in the same pass), or null
  int32_t* ipmask;        // with dot_out: the widths each query's pairs use
  const int32_t* probes;
  const int32_t* radq;
  const int64_t* offsets;
  const uint8_t* xbits;
  uint8_t* pbits;
  int nq, d, npmax, grid_e, grid_kind, metric, policy, fixed_bits, lane_sel_M;
  int lg_npp;  // log2 of the pair slots per query (power of two >= npmax)
  int lg_T;    // log2 of the threads per pair (small batches: several share the work)
  uint32_t allowed;
  int64_t margin;
};

__device__ __forceinline__ int64_t mitchell_q8(int64_t x) {
  uint64_t y = (uint64_t)x + 1;
  int k = 63 - __clzll((long long)y);
  return 256 * (int64_t)k + (int64_t)((y << 8) >> k) - 256;
}

__device__ __forceinline__ int pick_bits(int64_t y, const int64_t* theta, uint32_t allowed, int64_t margin) {
  int last = 16;
  for (int b = 4; b <= 16; b += 4) {
    if (!(allowed & (1u << b))) continue;
    last = b;
    if (b == 16 || y + margin <= theta[b / 4 - 1]) return b;
  }
  return last;
}

// 256 threads per workgroup: 256 / (npp T) queries, npp (power of two >=
// npmax) pair slots per query, T threads per pair (T > 1 only for batches too
// small to fill the chip: the T threads split the residual norm and the
// support-vector sum, then combine them across their lanes)
__global__ __launch_bounds__(256) void k_pairs(PairArgs a, ModelArgs ma) {
  __shared__ unsigned long long s_best[256];
  __shared__ int64_t s_dq2[256];
  __shared__ int32_t s_dot[256];
  __shared__ int32_t s_wmask[256];  // widths of each query slot's pairs (with dot_out)
  __shared__ int32_t s_table[kTableN];
  const int lg = a.lg_npp, lt = a.lg_T, T = 1 << lt;
  const int t = threadIdx.x & (T - 1);
  const int slot = threadIdx.x >> (lg + lt), r = (threadIdx.x >> lt) & ((1 << lg) - 1);
  const int q = blockIdx.x * (256 >> (lg + lt)) + slot;
  const bool adaptive = a.policy == AMP_POLICY_ADAPTIVE;
  if (adaptive)
    for (int i = threadIdx.x; i < kTableN; i += blockDim.x) s_table[i] = ma.table[i];
  if ((threadIdx.x & ((1 << (lg + lt)) - 1)) == 0) {
    s_best[slot] = ~0ull;
    s_wmask[slot] = 0;
  }
  __syncthreads();
  const bool valid = q < a.nq && r < a.npmax;
  const int p = valid ? a.probes[(size_t)q * a.npmax + r] : -1;
  // d' = |grid residual|^2 of pair (qq, pp): the part of lane t of tn
  // (four coordinates per step, d % 4 == 0)
  // (inner product: also the part of qi.ci, into dot)
  auto dq2_part = [&](int qq, int pp, int t0, int tn, int& dot) -> int64_t {
    int64_t s2 = 0;
    const bool l2 = a.metric != AMP_IP;  // L2 and L1: d' of the grid residual
    if (!l2 && a.qi16) {
      // inner product: both sides already on the grid
      auto acc2 = [&](uint32_t x, uint32_t c) {
        const int x0 = (int)(int16_t)(x & 0xFFFFu), x1 = (int)(int16_t)(x >> 16);
        const int c0 = (int)(int16_t)(c & 0xFFFFu), c1 = (int)(int16_t)(c >> 16);
        const int v0 = x0 - c0, v1 = x1 - c1;
        s2 += (int64_t)(v0 * v0 + v1 * v1);
        dot += x0 * c0 + x1 * c1;
      };
      if ((a.d & 7) == 0) {
        // eight coordinates per 16-byte read (rows 16-byte aligned)
        const u32x4* xq = reinterpret_cast<const u32x4*>(a.qi16 + (size_t)qq * a.d);
        const u32x4* xc = reinterpret_cast<const u32x4*>(a.ci16 + (size_t)pp * a.d);
        for (int i = t0; i < (a.d >> 3); i += tn) {
          const u32x4 x = xq[i], c = xc[i];
          acc2(x[0], c[0]);
          acc2(x[1], c[1]);
          acc2(x[2], c[2]);
          acc2(x[3], c[3]);
        }
        return s2;
      }
      const u32x2* xq = reinterpret_cast<const u32x2*>(a.qi16 + (size_t)qq * a.d);
      const u32x2* xc = reinterpret_cast<const u32x2*>(a.ci16 + (size_t)pp * a.d);
      for (int i = t0; i < (a.d >> 2); i += tn) {
        const u32x2 x = xq[i], c = xc[i];
        const int x0 = (int)(int16_t)(x[0] & 0xFFFFu), x1 = (int)(int16_t)(x[0] >> 16);
        const int x2 = (int)(int16_t)(x[1] & 0xFFFFu), x3 = (int)(int16_t)(x[1] >> 16);
        const int c0 = (int)(int16_t)(c[0] & 0xFFFFu), c1 = (int)(int16_t)(c[0] >> 16);
        const int c2 = (int)(int16_t)(c[1] & 0xFFFFu), c3 = (int)(int16_t)(c[1] >> 16);
        const int v0 = x0 - c0, v1 = x1 - c1, v2 = x2 - c2, v3 = x3 - c3;
        s2 += (int64_t)(v0 * v0 + v1 * v1) + (int64_t)(v2 * v2 + v3 * v3);
        dot += x0 * c0 + x1 * c1 + x2 * c2 + x3 * c3;
      }
      return s2;
    }
    const float4* qv = reinterpret_cast<const float4*>(a.Q + (size_t)qq * a.d);
    const float4* cv = reinterpret_cast<const float4*>(a.C + (size_t)pp * a.d);
    for (int i = t0; i < (a.d >> 2); i += tn) {
      const float4 x = qv[i], c = cv[i];
      int v0, v1, v2, v3;
      if (l2) {
        v0 = grid_val(x.x - c.x, a.grid_e, a.grid_kind);
        v1 = grid_val(x.y - c.y, a.grid_e, a.grid_kind);
        v2 = grid_val(x.z - c.z, a.grid_e, a.grid_kind);
        v3 = grid_val(x.w - c.w, a.grid_e, a.grid_kind);
      } else {
        v0 = grid_val(x.x, a.grid_e, a.grid_kind) - grid_val(c.x, a.grid_e, a.grid_kind);
        v1 = grid_val(x.y, a.grid_e, a.grid_kind) - grid_val(c.y, a.grid_e, a.grid_kind);
        v2 = grid_val(x.z, a.grid_e, a.grid_kind) - grid_val(c.z, a.grid_e, a.grid_kind);
        v3 = grid_val(x.w, a.grid_e, a.grid_kind) - grid_val(c.w, a.grid_e, a.grid_kind);
      }
      s2 += (int64_t)(v0 * v0 + v1 * v1) + (int64_t)(v2 * v2 + v3 * v3);
    }
    return s2;
  };
  int64_t dq2 = 0;
  int dot = 0;  // (inner product with dot_out)
  if (adaptive && T == 1) {
    // a thread per pair: the rows are read by sixteen lanes per pair, sixteen
    // pairs of the workgroup at a time (coalesced 128-byte segments), and the
    // norms handed over through LDS; the thread of a pair slot is its index
    const int l16 = threadIdx.x & 15, grp = threadIdx.x >> 4;
    for (int e0 = 0; e0 < 256; e0 += 16) {
      const int e = e0 + grp;
      const int qs = blockIdx.x * (256 >> lg) + (e >> lg), rs = e & ((1 << lg) - 1);
      const int pp = qs < a.nq && rs < a.npmax ? a.probes[(size_t)qs * a.npmax + rs] : -1;
      int dp = 0;
      int64_t s2 = pp >= 0 ? dq2_part(qs, pp, l16, 16, dp) : 0;
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        s2 += __shfl_xor(s2, o, 16);
        dp += __shfl_xor(dp, o, 16);
      }
      if (l16 == 0) {
        s_dq2[e] = s2;
        s_dot[e] = dp;
      }
    }
    __syncthreads();
    dq2 = s_dq2[threadIdx.x];
    dot = s_dot[threadIdx.x];
  } else if (adaptive && p >= 0) {
    dq2 = dq2_part(q, p, t, T, dot);
  }
  // the T threads of a pair are adjacent lanes of one wave (T <= 64)
  if (T > 1)
    for (int o = 1; o < T; o <<= 1) {
      dq2 += __shfl_xor(dq2, o);
      dot += __shfl_xor(dot, o);
    }
  if (adaptive && p >= 0 && t == 0)
    atomicMin(&s_best[slot], (unsigned long long)((uint64_t)dq2 << 13 | (uint64_t)p));
  __syncthreads();
  if (valid) {
    uint8_t bits = 0;
    if (p >= 0) {
      if (a.policy == AMP_POLICY_FP32) {
        bits = 32;
      } else if (a.policy == AMP_POLICY_FIXED) {
        bits = (uint8_t)a.fixed_bits;
      } else if (a.policy == AMP_POLICY_EXPLICIT) {
        bits = a.xbits[(size_t)q * a.npmax + r];
      } else {
        const int c1 = (int)(s_best[slot] & 8191ull);
        int64_t x[5];
        x[0] = dq2;
        x[1] = a.radq[c1];
        x[2] = a.radq[p];
        x[3] = a.offsets[c1 + 1] - a.offsets[c1];
        x[4] = a.offsets[p + 1] - a.offsets[p];
        int32_t u[5];
        for (int f = 0; f < 5; ++f) {
          int64_t v = ((mitchell_q8(x[f]) - ma.feat_lo[f]) * ma.feat_mul[f]) >> 16;
          u[f] = (int32_t)(v < 0 ? 0 : (v > 1023 ? 1023 : v));
        }
        // integer sum: the split over threads does not change the result
        // u and sv lie in [0, 1023] (sv checked when the model is set): the
        // squared differences are exact 24-bit products (full-rate multiplies)
        // and |u - sv|^2 < 2^23; g_mul < 2^32, so the table index is the high
        // word of one 32 x 32-bit product
        const uint32_t gm = (uint32_t)ma.g_mul;
        auto term = [&](int i) -> int64_t {
          const int32_t* sv = ma.sv + 5 * i;
          const int d0 = u[0] - sv[0], d1 = u[1] - sv[1], d2 = u[2] - sv[2], d3 = u[3] - sv[3], d4 = u[4] - sv[4];
          const uint32_t dist2 = (uint32_t)(__mul24(d0, d0) + __mul24(d1, d1) + __mul24(d2, d2) + __mul24(d3, d3) +
                                            __mul24(d4, d4));
          const uint32_t idx = __umulhi(dist2, gm);
          const int32_t K = s_table[idx < (uint32_t)(kTableN - 1) ? idx : (uint32_t)(kTableN - 1)];
          return (int64_t)ma.beta[i] * K;
        };
        // two independent chains (an integer sum: the order does not matter)
        int64_t y = 0, y1 = 0;
        if (T == 1) {
          // a thread per pair: the support-vector index is the same across the
          // wave, so sv and beta are read through scalar loads
          int i = 0;
          for (; i + 1 < ma.n_sv; i += 2) {
            y += term(i);
            y1 += term(i + 1);
          }
          if (i < ma.n_sv) y += term(i);
        } else {
          int i = t;
          for (; i + T < ma.n_sv; i += 2 * T) {
            y += term(i);
            y1 += term(i + T);
          }
          if (i < ma.n_sv) y += term(i);
        }
        y += y1;
        for (int o = 1; o < T; o <<= 1) y += __shfl_xor(y, o);
        bits = (uint8_t)pick_bits(ma.beta0 + y, ma.theta, a.allowed, a.margin);
      }
    }
    if (t == 0) a.pbits[(size_t)q * a.npmax + r] = bits;
    if (a.dot_out && p >= 0 && t == 0) {
      // the pair's list term for its base (k_iptab subtracts it from the sum
      // of the query's row minima) and its width in the query slot's mask
      a.dot_out[(size_t)q * a.npmax + r] = dot;
      atomicOr(&s_wmask[slot], 1 << ((bits >> 2) - 1));
    }
  }
  if (a.dot_out) {
    // one atomic per query for the widths its tables are needed at
    __syncthreads();
    if ((threadIdx.x & ((1 << (lg + lt)) - 1)) == 0 && q < a.nq && s_wmask[slot])
      atomicOr(&a.ipmask[q], s_wmask[slot]);
  }
}

// ------------------------------------------------------------------ queue
// Buckets are class-major.  Phase 1 holds the rank-0 pair of every query,
// phase 2 every active pair.  One atomic per pair on its (class, list)
// counter gives its rank inside the bucket; the scatter and the work-unit
// table are then written without atomics.  Counters are indexed by list id
// (the most-probed lists stay spread over memory channels), offsets and
// units by the list's position in the launch order lorder (largest first).
struct QueueArgs {
  const int32_t* probes;
  const uint8_t* pbits;
  const int32_t* kq;      // per-query k, or null (kconst)
  int kconst;
  const int64_t* offsets;
  const int32_t* lorder;  // bucket position -> list (largest list first)
  const int32_t* lpos;    // list -> bucket position
  int32_t* cnt;       // [2][kQSub][NB] by (sub-counter, class, list id)
  int32_t* rank;      // [2][nq*npmax]
  int64_t* pairoff;   // [2][NB+1] by (class, launch position)
  int64_t* unitoff;   // [2][NB+1] by (class, launch position)
  int32_t* sorted;    // [2][nq*npmax]
  int4* units;        // [2][max_units]: {list, first pair, pair count, chunk}
  int32_t* flags;
  int nq, npmax, nlist, M, ncls, wpr;
  int gran;               // quantiser granularity (lane classes of 4-bit pairs)
  int64_t chunk[2], max_units;  // list chunk of a work unit in phase 1, phase 2
  int ph0, ph1;           // queue phases built by this launch: [ph0, ph1) of {0 bound, 1 full scan}
  const int64_t* pbase;   // lower bound of every pair's estimates (integer: exact base; FP32 policy,
                          // inner product: the key of its in-order FP32 bound), or null: every pair
                          // joins phase 2
  int fkeys;              // pbase holds FP32 keys (FP32 policy)
  const uint64_t* tau;    // the queries' phase-1 bounds (with pbase)
  uint64_t* work;         // phase-2 work counters (pairs dropped here count as skipped), or null
};

// a pair joins the full scan unless its lower bound already exceeds its
// query's phase-1 bound (then no vector of its list can reach the top-k)
__device__ __forceinline__ bool pair_live(const QueueArgs& a, size_t i) {
  if (!a.pbase) return true;
  const uint64_t key = a.fkeys ? (uint64_t)a.pbase[i] : ikey(a.pbase[i]);
  return key <= a.tau[i / a.npmax];
}

__device__ __forceinline__ int pair_class(int bits, int M, int gran) {
  if (bits == 32) return 0;
  if (bits == 4 && gran == 0 && M <= 2184) return 0;  // 4-bit entries, sums widened (lane_class)
  uint64_t top = (uint64_t)M * ((1ull << bits) - 1);
  return top <= 0xFFull ? 0 : (top <= 0xFFFFull ? 1 : 2);
}
// pairs of a work unit: WPR LUT words of 32 / lane_bits(class) fields
__device__ __forceinline__ int class_pairs(int cls, int wpr, bool fp32, int gran) {
  return fp32 ? wpr : (cls == 0 && !gran ? unit_pairs(4, wpr) : wpr * (4 >> cls));
}

// sub-counter of a pair: the pairs of a much-probed list spread over kQSub
// counters (in different cache lines), so their atomics do not queue on one
__device__ __forceinline__ int pair_sub(size_t i) {
  return (int)(((uint32_t)i * 0x9E3779B1u) >> 28) & (kQSub - 1);
}

// the phase-1 bound of a query comes from its nearest probes: rank 0, and
// each further rank while the lists of the ranks before it hold fewer than k
// vectors (so that the bound covers k distinct vectors whenever the probed
// lists hold that many)
__device__ __forceinline__ bool in_phase1(const QueueArgs& a, size_t i) {
  const size_t q = i / a.npmax;
  const int r = (int)(i - q * a.npmax);
  if (r == 0) return true;
  const int kk = a.kq ? a.kq[q] : a.kconst;
  int64_t cum = 0;
  for (int j = 0; j < r; ++j) {
    const int p = a.probes[q * a.npmax + j];
    cum += a.offsets[p + 1] - a.offsets[p];
    if (cum >= kk) return false;
  }
  return true;
}

__global__ void k_qhist(QueueArgs a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)a.nq * a.npmax;
  if (i >= n) return;
  const int p = a.probes[i];
  if (p < 0) return;
  const int cls = pair_class(a.pbits[i], a.M, a.gran);
  const int NB = a.ncls * a.nlist;
  const size_t b = (size_t)pair_sub(i) * NB + cls * a.nlist + p;
  if (a.ph1 > 1) {
    if (pair_live(a, i)) a.rank[n + i] = atomicAdd(&a.cnt[(size_t)kQSub * NB + b], 1);
    else if (a.work) atomicAdd((unsigned long long*)&a.work[2], 1ull);
  }
  if (a.ph0 == 0 && in_phase1(a, i)) a.rank[i] = atomicAdd(&a.cnt[b], 1);
}

// per (phase, class, list) bucket: its pair total from the sub-counters
// (which become offsets inside the bucket) and its unit count, stored at the
// bucket's launch position (pairoff / unitoff hold counts until k_qscan)
__global__ void k_qtot(QueueArgs a, int fp32) {
  const int NB = a.ncls * a.nlist;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (a.ph1 - a.ph0) * NB) return;
  const int ph = a.ph0 + i / NB, b = i % NB, cls = b / a.nlist, p = b % a.nlist;
  int32_t* cnt = a.cnt + (size_t)ph * kQSub * NB;
  int x[kQSub];
#pragma unroll
  for (int u = 0; u < kQSub; ++u) x[u] = cnt[(size_t)u * NB + b];
  int c = 0;
#pragma unroll
  for (int u = 0; u < kQSub; ++u) {
    const int xu = x[u];
    x[u] = c;
    c += xu;
  }
#pragma unroll
  for (int u = 0; u < kQSub; ++u) cnt[(size_t)u * NB + b] = x[u];
  const int64_t n = a.offsets[p + 1] - a.offsets[p];
  const int64_t nch = (n + a.chunk[ph] - 1) / a.chunk[ph];
  const int G = class_pairs(cls, a.wpr, fp32, a.gran);
  const int pos = cls * a.nlist + a.lpos[p];
  a.pairoff[(size_t)ph * (NB + 1) + pos] = c;
  a.unitoff[(size_t)ph * (NB + 1) + pos] = ((c + G - 1) / G) * nch;
}

// inclusive scan of one int64 over a 1024-thread workgroup (wave scans, then
// a scan of the 16 wave totals)
__device__ __forceinline__ int64_t block_scan_1024(int64_t v, int64_t* s_w) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  if (lane == 63) s_w[wv] = v;
  __syncthreads();
  if (wv == 0) {
    int64_t t = lane < 16 ? s_w[lane] : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int64_t o = __shfl_up(t, off);
      if (lane >= off) t += o;
    }
    if (lane < 16) s_w[lane] = t;
  }
  __syncthreads();
  const int64_t r = v + (wv ? s_w[wv - 1] : 0);
  __syncthreads();  // s_w is reused by the next scan
  return r;
}

// exclusive scans of the pair and unit counts in launch order, one
// workgroup of 1024 threads, each a contiguous run of positions
__global__ __launch_bounds__(1024) void k_qscan(QueueArgs a, int fp32) {
  __shared__ int64_t s_w[16];
  const int NB = a.ncls * a.nlist;
  const int per = (NB + 1023) / 1024;
  for (int ph = a.ph0; ph < a.ph1; ++ph) {
    int64_t* po = a.pairoff + (size_t)ph * (NB + 1);
    int64_t* uo = a.unitoff + (size_t)ph * (NB + 1);
    const int b0 = threadIdx.x * per;
    int64_t sp = 0, su = 0;
    for (int b = b0; b < b0 + per && b < NB; ++b) {
      sp += po[b];
      su += uo[b];
    }
    const int64_t ip = block_scan_1024(sp, s_w), iu = block_scan_1024(su, s_w);
    int64_t xp = ip - sp, xu = iu - su;  // exclusive
    if (threadIdx.x == 1023) {
      po[NB] = ip;
      uo[NB] = iu;
    }
    for (int b = b0; b < b0 + per && b < NB; ++b) {
      const int64_t cp = po[b], cu = uo[b];
      po[b] = xp;
      uo[b] = xu;
      xp += cp;
      xu += cu;
    }
  }
}

__global__ void k_qscatter(QueueArgs a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)a.nq * a.npmax;
  if (i >= n) return;
  const int p = a.probes[i];
  if (p < 0) return;
  const int cls = pair_class(a.pbits[i], a.M, a.gran);
  const int b = cls * a.nlist + a.lpos[p];
  const int NB = a.ncls * a.nlist;
  const size_t bs = (size_t)pair_sub(i) * NB + cls * a.nlist + p;  // sub-counter offset
  if (a.ph1 > 1 && pair_live(a, i))
    a.sorted[n + a.pairoff[(NB + 1) + b] + a.cnt[(size_t)kQSub * NB + bs] + a.rank[n + i]] = (int32_t)i;
  if (a.ph0 == 0 && in_phase1(a, i)) a.sorted[a.pairoff[b] + a.cnt[bs] + a.rank[i]] = (int32_t)i;
}

// grid-stride over (phase, unit): find the unit's bucket by binary search of
// the unit offsets and write its descriptor
__global__ void k_qunits(QueueArgs a, int fp32) {
  const int NB = a.ncls * a.nlist;
  for (int ph = a.ph0; ph < a.ph1; ++ph) {
    const int64_t* po = a.pairoff + (size_t)ph * (NB + 1);
    const int64_t* uo = a.unitoff + (size_t)ph * (NB + 1);
    const int64_t total = uo[NB];
    if (total > a.max_units) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.flags[0], 4);
      continue;
    }
    int4* units = a.units + (size_t)ph * a.max_units;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
         u += (int64_t)gridDim.x * blockDim.x) {
      int lo = 0, hi = NB;  // uo[lo] <= u < uo[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (uo[mid] <= u) lo = mid; else hi = mid;
      }
      const int b = lo, cls = b / a.nlist, p = a.lorder[b % a.nlist];
      const int64_t n = a.offsets[p + 1] - a.offsets[p];
      const int64_t nch = (n + a.chunk[ph] - 1) / a.chunk[ph];
      const int G = class_pairs(cls, a.wpr, fp32, a.gran);
      const int64_t local = u - uo[b], grp = local / nch, ch = local % nch;
      const int64_t left = (po[b + 1] - po[b]) - grp * G;
      units[u] = make_int4(p, (int)(po[b] + grp * G), (int)(left < G ? left : G), (int)ch);
    }
  }
}

// ------------------------------------------------------------------ bound
// tau[q] = the k-th smallest key of the query's phase-1 bound buffer (every
// entry is the estimate of a distinct vector, so it bounds the query's k-th
// smallest estimate from above), or no bound with fewer than k entries; the
// buffer is emptied for phase 2.  Queries with at most 64 entries: one wave
// each (register bitonic sort); the rest: k_tau, a workgroup each (radix
// select).
__global__ __launch_bounds__(256) void k_tau_wave(uint32_t* ccount, const uint64_t* ckey, uint64_t* tau,
                                                  const int32_t* kq, int kconst, int nq, size_t capq,
                                                  int32_t* any_retry) {
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q == 0 && lane < 2) any_retry[lane] = 0;  // no phase-2 re-run requested yet (two rounds)
  if (q >= nq) return;
  const uint32_t cnt = ccount[q];
  const int n = (int)(cnt < capq ? cnt : capq);
  if (n > 64) return;
  uint64_t key = lane < n ? ckey[(size_t)q * capq + lane] : ~0ull;
  for (int kb = 2; kb <= 64; kb <<= 1)
    for (int jb = kb >> 1; jb > 0; jb >>= 1) {
      const uint64_t o = __shfl_xor(key, jb);
      const bool keep_min = ((lane & kb) == 0) == ((lane & jb) == 0);
      key = keep_min ? (o < key ? o : key) : (o > key ? o : key);
    }
  const int kk = kq ? kq[q] : kconst;
  const uint64_t kth = __shfl(key, kk <= 64 ? kk - 1 : 63);
  if (lane == 0) {
    tau[q] = n >= kk ? kth : ~0ull;
    ccount[q] = 0;
  }
}

__global__ __launch_bounds__(256) void k_tau(uint32_t* ccount, const uint64_t* ckey, uint64_t* tau,
                                             const int32_t* kq, int kconst, int nq, size_t capq) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + capq * 8);  // [256]
  uint32_t* sel = hist + 256;                                     // [2]
  int* s_n = reinterpret_cast<int*>(sel + 2);
  int* s_q = s_n + 1;  // [blockDim.x]
  // the workgroup's queries q = blockIdx.x + i * gridDim.x, a thread each:
  // the entry counts are read side by side, and only the queries with more
  // than 64 entries are sorted
  for (int64_t base = blockIdx.x; base < nq; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + (int64_t)threadIdx.x * gridDim.x;
    bool big = false;
    if (q < nq) {
      const uint32_t c = ccount[q];
      big = (c < capq ? c : capq) > 64;  // (the others: k_tau_wave)
    }
    if (threadIdx.x == 0) *s_n = 0;
    __syncthreads();
    if (big) s_q[atomicAdd(s_n, 1)] = (int)q;
    __syncthreads();
    const int nb = *s_n;
    for (int t = 0; t < nb; ++t) {
      const int qq = s_q[t];
      const uint32_t cnt = ccount[qq];
      const int n = (int)(cnt < capq ? cnt : capq);
      const int kk = kq ? kq[qq] : kconst;
      if (n < kk) {  // uniform over the workgroup
        if (threadIdx.x == 0) {
          tau[qq] = ~0ull;
          ccount[qq] = 0;
        }
        continue;
      }
      for (int i = threadIdx.x; i < n; i += blockDim.x) keys[i] = ckey[(size_t)qq * capq + i];
      __syncthreads();
      const uint64_t kth = block_select_u64(keys, n, kk, hist, sel);
      if (threadIdx.x == 0) {
        tau[qq] = kth;
        ccount[qq] = 0;
      }
      // (the select ends on a barrier: the LDS is free for the next query)
    }
    __syncthreads();  // every thread has read the list before it is reset
  }
}

// after phase 2: a query whose candidates overflowed the buffer takes the
// k-th smallest (distance, id) of the candidates kept (distinct vectors, each
// within its old bound) as a tighter bound and is marked for a re-run of
// phase 2; the others are unmarked.  Block 0 also rewinds the phase-2 unit counters.
__global__ __launch_bounds__(256) void k_retry(uint32_t* ccount, const uint64_t* ckey, const int64_t* cid,
                                               uint64_t* tau, int64_t* tau_id, const int32_t* kq, int kconst, int nq,
                                               size_t capq, uint8_t* retry, int32_t* any_retry, uint32_t* counters,
                                               int ncounters) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
  int64_t* vals = reinterpret_cast<int64_t*>(lds + capq * 8);
  int* s_n = reinterpret_cast<int*>(lds + capq * 16);
  int* s_q = s_n + 1;  // [blockDim.x]
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < ncounters; i += blockDim.x) counters[i] = 0;
  // the workgroup's queries q = blockIdx.x + i * gridDim.x, a thread each:
  // the candidate counts are read side by side (no chain of dependent
  // loads), and only the overflowed queries go on to the sort
  for (int64_t base = blockIdx.x; base < nq; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + (int64_t)threadIdx.x * gridDim.x;
    bool over = false;
    if (q < nq) {
      over = ccount[q] > capq;
      if (!over) retry[q] = 0;
    }
    if (threadIdx.x == 0) *s_n = 0;
    __syncthreads();
    if (over) s_q[atomicAdd(s_n, 1)] = (int)q;
    __syncthreads();
    const int n = *s_n;
    for (int t = 0; t < n; ++t) {
      const int qq = s_q[t];
      for (size_t i = threadIdx.x; i < capq; i += blockDim.x) {
        keys[i] = ckey[(size_t)qq * capq + i];
        vals[i] = cid[(size_t)qq * capq + i];
      }
      __syncthreads();
      block_bitonic_u64_i64(keys, vals, (int)capq);
      const int kk = kq ? kq[qq] : kconst;
      if (threadIdx.x == 0) {
        tau[qq] = keys[kk - 1];
        tau_id[qq] = vals[kk - 1];
        ccount[qq] = 0;
        retry[qq] = 1;
        *any_retry = 1;
      }
      __syncthreads();  // the LDS is reused by the next query
    }
    __syncthreads();  // every thread has read the list before it is reset
  }
}

// ------------------------------------------------------------------ TS
struct MergeArgs {
  const uint32_t* ccount;
  const uint64_t* ckey;
  const int64_t* cid;
  const int32_t* kq;
  int32_t* flags;
  int64_t* out_ids;
  float* out_dist;
  int64_t* out_qdist;
  int kconst, kmax, fp32;
  float h2;
  size_t capq;
};

// output row r of query q from its sorted candidate r (n candidates)
__device__ __forceinline__ void merge_emit(const MergeArgs& a, int q, int r, int n, int kk, uint64_t key,
                                           int64_t id) {
  const size_t o = (size_t)q * a.kmax + r;
  if (r < kk && r < n) {
    a.out_ids[o] = id;
    if (a.fp32) {
      a.out_dist[o] = fkey_val((uint32_t)key);
      if (a.out_qdist) a.out_qdist[o] = -1;
    } else {
      const int64_t D = ikey_val(key);
      a.out_dist[o] = __ll2float_rn(D) * a.h2;
      if (a.out_qdist) a.out_qdist[o] = D;
    }
  } else {
    a.out_ids[o] = -1;
    a.out_dist[o] = __builtin_inff();
    if (a.out_qdist) a.out_qdist[o] = INT64_MAX;
  }
}

// queries with at most 64 candidates: one wave per query, a register bitonic
// sort of (key, id) across the lanes
__global__ __launch_bounds__(256) void k_merge_wave(MergeArgs a, int nq) {
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  const uint32_t cnt = a.ccount[q];
  if (cnt > a.capq && lane == 0) atomicOr(&a.flags[0], 2);
  const int n = (int)(cnt < a.capq ? cnt : a.capq);
  if (n > 64) return;  // the workgroup kernel takes it
  uint64_t key = lane < n ? a.ckey[(size_t)q * a.capq + lane] : ~0ull;
  int64_t id = lane < n ? a.cid[(size_t)q * a.capq + lane] : INT64_MAX;
  for (int kb = 2; kb <= 64; kb <<= 1)
    for (int jb = kb >> 1; jb > 0; jb >>= 1) {
      const uint64_t ok = __shfl_xor(key, jb);
      const int64_t oid = __shfl_xor(id, jb);
      const bool other_less = ok < key || (ok == key && oid < id);
      const bool other_more = ok > key || (ok == key && oid > id);
      const bool keep_min = ((lane & kb) == 0) == ((lane & jb) == 0);
      if (keep_min ? other_less : other_more) {
        key = ok;
        id = oid;
      }
    }
  const int kk = a.kq ? a.kq[q] : a.kconst;
  for (int r = lane; r < a.kmax; r += 64) merge_emit(a, q, r, n, kk, key, id);
}

// queries with more than 64 candidates and more than k: a workgroup per
// query (strided over the queries).  A radix select finds the k-th smallest
// key; the candidates up to it, when at most kMergeSel, take their output
// rows from their rank (key, id, position) among themselves.  The other
// queries (at most k candidates, or more than kMergeSel up to the k-th key)
// are left to k_merge_full, marked by id -2 in their first output row.
constexpr int kMergeSel = 256;

__global__ __launch_bounds__(256) void k_merge(MergeArgs a, int nq) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
  uint64_t* skey = reinterpret_cast<uint64_t*>(lds + a.capq * 8);  // [kMergeSel]
  int64_t* sval = reinterpret_cast<int64_t*>(skey + kMergeSel);    // [kMergeSel]
  int32_t* sidx = reinterpret_cast<int32_t*>(sval + kMergeSel);    // [kMergeSel]
  uint32_t* hist = reinterpret_cast<uint32_t*>(sidx + kMergeSel);  // [256]
  uint32_t* sel = hist + 256;                                       // [2]
  uint32_t* s_cnt = sel + 2;
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint32_t cnt = a.ccount[q];
    if (cnt > a.capq && threadIdx.x == 0) atomicOr(&a.flags[0], 2);
    const int n = (int)(cnt < a.capq ? cnt : a.capq);
    if (n <= 64) continue;  // uniform over the workgroup
    const int kk = a.kq ? a.kq[q] : a.kconst;
    if (kk >= n) {
      if (threadIdx.x == 0) a.out_ids[(size_t)q * a.kmax] = -2;
      continue;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) keys[i] = a.ckey[(size_t)q * a.capq + i];
    if (threadIdx.x == 0) *s_cnt = 0;
    __syncthreads();
    const uint64_t v = block_select_u64(keys, n, kk, hist, sel);
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      if (keys[i] <= v) {
        const uint32_t j = atomicAdd(s_cnt, 1u);
        if (j < (uint32_t)kMergeSel) {
          skey[j] = keys[i];
          sval[j] = a.cid[(size_t)q * a.capq + i];
          sidx[j] = i;
        }
      }
    __syncthreads();
    const int ns = (int)*s_cnt;
    if (ns > kMergeSel) {  // uniform over the workgroup
      if (threadIdx.x == 0) a.out_ids[(size_t)q * a.kmax] = -2;
    } else {
      for (int t = threadIdx.x; t < ns; t += blockDim.x) {
        const uint64_t kt = skey[t];
        const int64_t it = sval[t];
        const int xt = sidx[t];
        int rank = 0;
        for (int j = 0; j < ns; ++j) {
          const uint64_t kj = skey[j];
          const int64_t ij = sval[j];
          rank += kj < kt || (kj == kt && (ij < it || (ij == it && sidx[j] < xt)));
        }
        if (rank < kk) merge_emit(a, q, rank, n, kk, kt, it);
      }
      for (int r = kk + threadIdx.x; r < a.kmax; r += blockDim.x) merge_emit(a, q, r, n, kk, ~0ull, INT64_MAX);
    }
    __syncthreads();  // the LDS is reused by the next query
  }
}

// the queries k_merge left (id -2 in the first output row): a workgroup per
// query (strided over the queries), every candidate sorted by (key, id) in
// LDS (bitonic over the next power of two)
__global__ __launch_bounds__(256) void k_merge_full(MergeArgs a, int nq) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
  int64_t* vals = reinterpret_cast<int64_t*>(lds + a.capq * 8);
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint32_t cnt = a.ccount[q];
    const int n = (int)(cnt < a.capq ? cnt : a.capq);
    if (n <= 64 || a.out_ids[(size_t)q * a.kmax] != -2) continue;  // uniform over the workgroup
    __syncthreads();  // every thread has read the mark before it is overwritten
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = threadIdx.x; i < np2; i += blockDim.x) {
      keys[i] = i < n ? a.ckey[(size_t)q * a.capq + i] : ~0ull;
      vals[i] = i < n ? a.cid[(size_t)q * a.capq + i] : INT64_MAX;
    }
    __syncthreads();
    block_bitonic_u64_i64(keys, vals, np2);
    const int kk = a.kq ? a.kq[q] : a.kconst;
    for (int r = threadIdx.x; r < a.kmax; r += blockDim.x)
      merge_emit(a, q, r, n, kk, r < n ? keys[r] : ~0ull, r < n ? vals[r] : INT64_MAX);
    __syncthreads();  // the LDS is reused by the next query
  }
}

// ------------------------------------------------------------------ index prep
// MFMA B fragments of the grid codebook: for m-pair mp, codeword tile jt and
// lane l (group kg = l/16, codeword j = 16 jt + l%16):
//   kg even: cbi[m][j][0..dsub) zero-padded to 8;  kg odd: digits of
//   cc = |cbi[m][j]|^2 (base 256, most significant first) then 65536, 256, 1
// bsw: BF16 (all groups); bsw16: FP16 dims (odd groups zero).
__global__ void k_prep_bsw(const float* __restrict__ cb, int M, int dsub, int grid_e, int grid_kind,
                           u32x4* __restrict__ bsw, u32x4* __restrict__ bsw16, u32x2* __restrict__ bsw8) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = (M / 2) * 16 * 64;
  if (idx >= total) return;
  const int lane = idx & 63, jt = (idx >> 6) & 15, mp = idx >> 10;
  const int kg = lane >> 4, j = jt * 16 + (lane & 15);
  const int m = 2 * mp + (kg >> 1);
  const float* c = cb + ((size_t)m * kKsub + j) * dsub;
  float v[8];
  int ci[kMaxDsub];
  int cc = 0;
  for (int t = 0; t < kMaxDsub; ++t) {
    ci[t] = t < dsub ? grid_val(c[t], grid_e, grid_kind) : 0;
    cc += ci[t] * ci[t];
  }
  uint32_t h[4] = {0, 0, 0, 0}, f8[2] = {0, 0};
  if ((kg & 1) == 0) {
    for (int t = 0; t < 8; ++t) v[t] = (float)ci[t];
    for (int t = 0; t < 4; ++t) h[t] = f16_bits(v[2 * t]) | (f16_bits(v[2 * t + 1]) << 16);
    // e4m3 bytes (exact on the e4m3 grid; the FP8 build is only offered there)
    f8[0] = f8_bits4(v[0], v[1], v[2], v[3]);
    f8[1] = f8_bits4(v[4], v[5], v[6], v[7]);
  } else {
    v[0] = (float)(cc >> 16);
    v[1] = (float)((cc >> 8) & 255);
    v[2] = (float)(cc & 255);
    v[3] = 65536.f;
    v[4] = 256.f;
    v[5] = 1.f;
    v[6] = 0.f;
    v[7] = 0.f;
  }
  u32x4 o;
  for (int t = 0; t < 4; ++t) o[t] = bf16_bits(v[2 * t]) | (bf16_bits(v[2 * t + 1]) << 16);
  bsw[idx] = o;
  bsw16[idx] = (u32x4){h[0], h[1], h[2], h[3]};
  bsw8[idx] = (u32x2){f8[0], f8[1]};
}

// ------------------------------------------------------------------ inner-product tables
// queries on the operand grid (inner product)
__global__ void k_qgrid(const float* __restrict__ Q, int16_t* __restrict__ qi, size_t n, int grid_e, int grid_kind) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    qi[i] = (int16_t)grid_val(Q[i], grid_e, grid_kind);
}

// inner product, FP32 policy: each query's dot products q_m . c_mj in FP32
// (the FMA chain of the scan's FP32 entries, in the same order)
__global__ void k_iptab_f32(BaseArgs b) {
  const size_t n = (size_t)b.nq * b.M * kKsub;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t q = i / ((size_t)b.M * kKsub);
    const int e = (int)(i - q * b.M * kKsub), m = e >> 8;
    const float* r = b.Q + q * b.d + m * b.dsub;
    const float* c = b.codebook + (size_t)e * b.dsub;
    float dot = 0.f;
#pragma unroll
    for (int t = 0; t < kMaxDsub; ++t)
      if (t < b.dsub) dot = fmaf(r[t], c[t], dot);
    b.iptab[i] = __float_as_int(dot);
  }
}

// inner product: qi.ci of each pair (exact integers; k_iptab subtracts it
// from the sum of the query's row minima: the pair's base), for the
// policies whose predictor pass does not compute it.  A workgroup per query,
// sixteen lanes per probed list (sixteen lists per step); the widths the
// query's pairs use (the tables k_ipq builds) are gathered in the workgroup
// and set with one atomic.
__global__ __launch_bounds__(256) void k_ipbase(BaseArgs b) {
  __shared__ int s_mask;
  const size_t q = blockIdx.x;
  const int tid = threadIdx.x, r = tid & 15, grp = tid >> 4;
  if (tid == 0) s_mask = 0;
  __syncthreads();
  const u32x2* qv = reinterpret_cast<const u32x2*>(b.qi16 + q * b.d);
  const int d4 = b.d >> 2;
  int mask = 0;
  for (int j0 = 0; j0 < b.npmax; j0 += 16) {
    const int j = j0 + grp;
    const size_t i = q * b.npmax + j;
    const int p = j < b.npmax ? b.probes[i] : -1;
    int acc = 0;
    if (p >= 0) {
      const u32x2* cv = reinterpret_cast<const u32x2*>(b.ci16 + (size_t)p * b.d);
      for (int t4 = r; t4 < d4; t4 += 16) {
        const u32x2 x = qv[t4], c = cv[t4];
        acc += (int)(int16_t)(x[0] & 0xFFFFu) * (int)(int16_t)(c[0] & 0xFFFFu) +
               (int)(int16_t)(x[0] >> 16) * (int)(int16_t)(c[0] >> 16) +
               (int)(int16_t)(x[1] & 0xFFFFu) * (int)(int16_t)(c[1] & 0xFFFFu) +
               (int)(int16_t)(x[1] >> 16) * (int)(int16_t)(c[1] >> 16);
      }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (p >= 0 && r == 0) {
      b.pbase[i] = acc;  // qi.ci: k_iptab turns it into the base once the query's minima are known
      mask |= 1 << ((b.pbits[i] >> 2) - 1);
    }
  }
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (tid == 0 && s_mask) atomicOr(&b.ipmask[q], s_mask);
}

// inner product, FP32 policy: the largest dot product of each (query,
// subspace) row of the query's FP32 table (a wave per row)
__global__ __launch_bounds__(256) void k_ipmax_f32(BaseArgs b) {
  const int lane = threadIdx.x & 63;
  const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (size_t)b.nq * b.M) return;
  const float* t = reinterpret_cast<const float*>(b.iptab) + row * kKsub;
  float mx = fmaxf(fmaxf(t[lane], t[lane + 64]), fmaxf(t[lane + 128], t[lane + 192]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if (lane == 0) reinterpret_cast<float*>(b.iplo)[row] = mx;
}

// inner product, FP32 policy: the key of each pair's lower bound, computed
// with the scan's own FP32 arithmetic (a wave per pair): the pair's base
// term bf = sum over the subspaces (in order) of the FMA chain of -q_t c_t,
// then the in-order sum over the subspaces of the smallest LUT entry,
// bf - max_j dot_0j for subspace 0 and 0 - max_j dot_mj for the others
// (rounding is monotone, so these are the rows' smallest entries)
__global__ __launch_bounds__(256) void k_ipbase_f32(BaseArgs b) {
  const int lane = threadIdx.x & 63;
  const size_t i = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= (size_t)b.nq * b.npmax) return;
  const int p = b.probes[i];
  if (p < 0) return;
  const size_t q = i / b.npmax;
  const float* r = b.Q + q * b.d;
  const float* c = b.C + (size_t)p * b.d;
  float bf = 0.f;
  for (int m0 = 0; m0 < b.M; m0 += 64) {
    const int m = m0 + lane;
    float sq = 0.f;
    if (m < b.M)
      for (int t = 0; t < b.dsub; ++t) sq = fmaf(-r[m * b.dsub + t], c[m * b.dsub + t], sq);
    const int nm = b.M - m0 < 64 ? b.M - m0 : 64;
    for (int k = 0; k < nm; ++k) bf += __shfl(sq, k);  // in subspace order, the same on every lane
  }
  const float* mx = reinterpret_cast<const float*>(b.iplo) + q * b.M;
  float sb = 0.f;
  for (int m = 0; m < b.M; ++m) sb += (m == 0 ? bf : 0.f) - mx[m];
  if (lane == 0) b.pbase[i] = (int64_t)fkey(sb);
}

// LUT export (test hook), inner product: a pair's LUT is its query's table
// at its width (a workgroup per pair)
__global__ void k_export_ip(BaseArgs b, uint16_t* exq, int32_t* exs, int64_t* exb, int32_t* ext) {
  const size_t i = blockIdx.x;
  const int p = b.probes[i];
  if (p < 0) return;
  const size_t q = i / b.npmax;
  const int wi = (b.pbits[i] >> 2) - 1;
  const size_t tsz = (size_t)b.M * kKsub;
  if (threadIdx.x == 0) {
    exs[i] = b.ipsh[q * 4 + wi];
    exb[i] = b.pbase[i];
  }
  const uint16_t* slot = b.iptq + (q * 4 + wi) * tsz;
  const bool by = ip_bytes(b.gran, wi, b.M);
  for (size_t e = threadIdx.x; e < tsz; e += blockDim.x) {
    exq[i * tsz + e] = by ? reinterpret_cast<const uint8_t*>(slot)[e] : slot[e];
    if (ext) ext[i * tsz + e] = b.iptab[q * tsz + e];
  }
}

// inner product, integer policies: each query's table quantised at every
// width its pairs use: shift s from the query's span (smallest with
// (span + hf(s)) >> s <= 2^b - 1), entries (T - min_m + hf(s)) >> s as
// uint16, or as bytes in the first half of the table's slot (width 4 with
// one width per pair: ip_bytes); eight entries per thread, read once and
// written at every width the query needs
__global__ void k_ipq(BaseArgs b) {
  const size_t per = (size_t)b.M * kKsub / 8;
  const size_t n = (size_t)b.nq * per;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t q = i / per;
    const int mask = b.ipmask[q];
    if (!mask) continue;
    const size_t e0 = (i - q * per) * 8;
    const int m = (int)(e0 >> 8);
    const int lo = b.iplo[q * b.M + m];
    const int32_t* T = b.iptab + q * b.M * kKsub + e0;
    const u32x4 t0 = *reinterpret_cast<const u32x4*>(T), t1 = *reinterpret_cast<const u32x4*>(T + 4);
    const int tv[8] = {(int)t0[0], (int)t0[1], (int)t0[2], (int)t0[3], (int)t1[0], (int)t1[1], (int)t1[2], (int)t1[3]};
    for (int wi = 0; wi < 4; ++wi) {
      if (!(mask & (1 << wi))) continue;
      const size_t qw = q * 4 + wi;
      const int sh = quant_shift(b.ipspan[q], b.gran ? b.M : 1, 4 * (wi + 1));
      const int off = (sh ? 1 << (sh - 1) : 0) - lo;
      if (e0 == 0) b.ipsh[qw] = sh;
      uint32_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = (uint32_t)((tv[k] + off) >> sh);
      uint16_t* slot = b.iptq + qw * ((size_t)b.M * kKsub);
      if (ip_bytes(b.gran, wi, b.M)) {
        *reinterpret_cast<u32x2*>(reinterpret_cast<uint8_t*>(slot) + e0) =
            (u32x2){v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24), v[4] | (v[5] << 8) | (v[6] << 16) | (v[7] << 24)};
      } else {
        *reinterpret_cast<u32x4*>(slot + e0) =
            (u32x4){v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16)};
      }
    }
  }
}

// ------------------------------------------------------------------ host launchers
template <typename K>
static void* kaddr(K k) { return reinterpret_cast<void*>(k); }

hipError_t launch_prep_index(const amp_index* ix, hipStream_t st) {
  const DeviceIndex& dv = ix->dev;
  hipLaunchKernelGGL(k_sqnorm, dim3((ix->nlist + 3) / 4), dim3(256), 0, st, dv.centroids, ix->nlist,
                     ix->d, dv.cnorm);
  const int total = (ix->M / 2) * 16 * 64;
  hipLaunchKernelGGL(k_prep_cbi, dim3((ix->M * kKsub * 8 + 255) / 256), dim3(256), 0, st, dv.codebook, ix->M,
                     ix->dsub, ix->grid_e, ix->grid_kind, dv.cbi16);
  const size_t nc = (size_t)ix->nlist * ix->d;
  hipLaunchKernelGGL(k_qgrid, dim3((unsigned)std::min<size_t>((nc + 255) / 256, 65536)), dim3(256), 0, st,
                     dv.centroids, dv.ci16, nc, ix->grid_e, ix->grid_kind);
  hipLaunchKernelGGL(k_prep_bsw, dim3((total + 255) / 256), dim3(256), 0, st, dv.codebook, ix->M, ix->dsub,
                     ix->grid_e, ix->grid_kind, reinterpret_cast<u32x4*>(dv.bsw),
                     reinterpret_cast<u32x4*>(dv.bsw16), reinterpret_cast<u32x2*>(dv.bsw8));
  return hipGetLastError();
}

// dynamic LDS of a scan launch (lw_bits -1: the mixed-class kernel), the
// layout the kernel computes for itself
static size_t scan_lds_bytes(int lw_bits, int phase, int M, int d, int wpr, int nt) {
  const bool fp = lw_bits == 0;
  const int cw = lw_bits < 0 ? wpr : class_wpr(lw_bits, wpr);
  return (size_t)scan_lds_layout(unit_pairs(lw_bits, wpr), cw, M, d, fp, phase, nt).total;
}

int scan_wpr(int M, bool fp32, int lut_dtype, bool narrow) {
  return narrow ? 1 : kernel_wpr(scan_mt(fp32 ? 0 : 8, M, dt_of(lut_dtype)));
}

static int g_num_cu = 0;

// lwb < 0: every integer lane class in one launch (k_scan_mix).  A LUT tile
// so large that one 256-thread workgroup fills a CU's LDS leaves one wave
// per SIMD to hide the LDS and code-load latencies: the generic variant then
// runs 512-thread workgroups (two waves per SIMD on the same LUT;
// AMP_SCAN_WG512=0 keeps 256).
static hipError_t launch_scan(int lwb, int ph, int dt, int wpr, const ScanArgs& sa, hipStream_t st) {
  const bool mix = lwb < 0;
  auto pick = [&](int nt) {
    return ph == 1 ? pick_scan_ph1(lwb, sa.M, dt, wpr, nt)
                   : (ph == 2 ? pick_scan_ph2(lwb, sa.M, dt, wpr, nt) : pick_scan_ph3(lwb, sa.M, dt, wpr, nt));
  };
  ScanFn fn = pick(kThreads);
  int nt = kThreads;
  // the queue packed units for `wpr` words per row: the variant must agree
  const int mt = scan_mt(mix ? 8 : lwb, sa.M, dt);
  if (!fn || variant_wpr(mt, scan_nr(mt, wpr)) != wpr) return hipErrorInvalidValue;
  size_t lds = scan_lds_bytes(lwb, ph, sa.M, sa.d, wpr, nt);
  hipError_t e = hipFuncSetAttribute(kaddr(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kaddr(fn), nt, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  static const bool wg512 = [] {
    const char* v = getenv("AMP_SCAN_WG512");
    return !(v && v[0] == '0');
  }();
  if (per_cu == 1 && wg512) {
    ScanFn f2 = pick(2 * kThreads);
    if (f2) {
      const size_t l2 = scan_lds_bytes(lwb, ph, sa.M, sa.d, wpr, 2 * kThreads);
      int pc2 = 0;
      if ((e = hipFuncSetAttribute(kaddr(f2), hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2)) != hipSuccess)
        return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc2, kaddr(f2), 2 * kThreads, l2)) != hipSuccess)
        return e;
      if (pc2 >= 1) {
        fn = f2;
        nt = 2 * kThreads;
        lds = l2;
        per_cu = pc2;
      }
    }
  }
  if (!g_num_cu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  // phase 3 (the re-run) usually has nothing to do: one workgroup per CU
  hipLaunchKernelGGL(fn, dim3(g_num_cu * (ph == 3 ? 1 : per_cu)), dim3(nt), lds, st, sa);
  return hipGetLastError();
}

hipError_t launch_assign(const float* X, int64_t n, int dd, int ld, const float* C, int k, float* xn, float* cn,
                         int32_t* out_a, float* out_d, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sqnorm_ld, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, n, dd, ld, xn);
  hipLaunchKernelGGL(k_sqnorm_ld, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, st, C, (int64_t)k, dd, dd, cn);
  hipLaunchKernelGGL(k_assign, dim3((unsigned)((n + CL_T - 1) / CL_T)), dim3(256), 0, st, X, xn, n, dd, ld, C, cn, k,
                     out_a, out_d);
  return hipGetLastError();
}

hipError_t launch_residual(const float* X, const int32_t* a, const float* C, int64_t n, int d, float* out,
                           hipStream_t st) {
  const int64_t total = n * d;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X, a, C, n, d, out);
  return hipGetLastError();
}

hipError_t launch_search(const amp_index* ix, const Workspace& ws, const float* queries_in, const SearchDims& sd,
                         const ModelArgs& ma, const ModelArgs& clma, int64_t* out_ids, float* out_dist,
                         int64_t* out_qdist,
                         float* out_coarse, hipStream_t st, hipEvent_t* ev) {
  const DeviceIndex& dv = ix->dev;
  const bool fp32 = sd.policy == AMP_POLICY_FP32;
  const int ncls = fp32 ? 1 : kNCls;
  const int NB = ncls * sd.nlist;
  const size_t npairs = (size_t)sd.nq * sd.npmax;
  auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], st); };
  mark(0);
  // resets, one launch (before anything that may raise a flag)
  {
    ResetArgs ra;
    ra.cnt = reinterpret_cast<uint32_t*>(ws.cnt);
    ra.ncnt = (size_t)2 * kQSub * NB;
    ra.counters = ws.counters;
    ra.ncounters = (size_t)2 * (kNCls + 1) * kQueueSlot;
    ra.flags = reinterpret_cast<uint32_t*>(ws.flags);
    ra.work = ws.work;
    ra.tau = ws.tau;
    ra.ccount = ws.ccount;
    ra.ipmask = sd.metric == AMP_IP ? ws.ipmask : nullptr;
    ra.nq = (size_t)sd.nq;
    hipLaunchKernelGGL(k_reset, dim3(256), dim3(256), 0, st, ra);
  }
  // device-resident per-query sizes: checked, clamped and copied in
  if (sd.k_dev) {
    hipLaunchKernelGGL(k_sizes, dim3((sd.nq + 255) / 256), dim3(256), 0, st, sd.k_dev, sd.np_dev, ws.kq, ws.npq,
                       sd.nq, sd.kmax, sd.npmax, ws.flags);
  }
  // BF16 query rows are widened first (exact)
  const float* queries = queries_in;
  if (sd.q_bf16) {
    const size_t nel = (size_t)sd.nq * sd.d;
    hipLaunchKernelGGL(k_bf16_widen, dim3((unsigned)std::min<size_t>((nel + 255) / 256, 65536)), dim3(256), 0, st,
                       sd.q_bf16, sd.q_conv, nel);
    queries = sd.q_conv;
  }
  // CL
  float* coarse = out_coarse ? out_coarse : ws.coarse;
  if (sd.cl_policy != AMP_CL_FP32) {
    // integer cluster locating on 8-bit codes (fixed or adaptive operand
    // widths): order keys of the exact integer distances
    const hipError_t e = launch_cl(ix, ws, queries, sd, clma, ws.coarse, st);
    if (e != hipSuccess) return e;
    coarse = ws.coarse;
  } else if (sd.metric == AMP_L1) {
    hipLaunchKernelGGL(k_coarse_l1, dim3((sd.nlist + CL_T - 1) / CL_T, (sd.nq + CL_T - 1) / CL_T), dim3(256), 0,
                       st, queries, dv.centroids, coarse, sd.nq, sd.nlist, sd.d);
  } else {
    hipLaunchKernelGGL(k_sqnorm, dim3((sd.nq + 3) / 4), dim3(256), 0, st, queries, sd.nq, sd.d, ws.qnorm);
    const dim3 g((sd.nlist + CL_T - 1) / CL_T, (sd.nq + CL_T - 1) / CL_T);
    const bool vec = sd.d % 4 == 0 && ((reinterpret_cast<uintptr_t>(queries) | reinterpret_cast<uintptr_t>(dv.centroids)) & 15) == 0;
    // (64-wide K chunks measured the same as 32 at 4096 x 2048 x 768)
    if (vec)
      hipLaunchKernelGGL((k_coarse<CL_K, true>), g, dim3(256), 0, st, queries, dv.centroids, ws.qnorm, dv.cnorm, coarse,
                         sd.nq, sd.nlist, sd.d, sd.metric);
    else
      hipLaunchKernelGGL((k_coarse<CL_K, false>), g, dim3(256), 0, st, queries, dv.centroids, ws.qnorm, dv.cnorm,
                         coarse, sd.nq, sd.nlist, sd.d, sd.metric);
  }
  mark(1);
  int np2 = 1;
  while (np2 < sd.nlist) np2 <<= 1;
  if (sd.npmax <= 64 && sd.nlist <= 1024) {
    const dim3 g((sd.nq + 3) / 4), b(256);
    const int32_t* npq = ws.npq ? ws.npq : nullptr;
    if (sd.nlist <= 64)
      hipLaunchKernelGGL(k_topn_wave<1>, g, b, 0, st, coarse, sd.nlist, sd.nq, npq, sd.npconst, sd.npmax, ws.probes);
    else if (sd.nlist <= 128)
      hipLaunchKernelGGL(k_topn_wave<2>, g, b, 0, st, coarse, sd.nlist, sd.nq, npq, sd.npconst, sd.npmax, ws.probes);
    else if (sd.nlist <= 256)
      hipLaunchKernelGGL(k_topn_wave<4>, g, b, 0, st, coarse, sd.nlist, sd.nq, npq, sd.npconst, sd.npmax, ws.probes);
    else if (sd.nlist <= 512)
      hipLaunchKernelGGL(k_topn_wave<8>, g, b, 0, st, coarse, sd.nlist, sd.nq, npq, sd.npconst, sd.npmax, ws.probes);
    else
      hipLaunchKernelGGL(k_topn_wave<16>, g, b, 0, st, coarse, sd.nlist, sd.nq, npq, sd.npconst, sd.npmax, ws.probes);
  } else if (sd.nlist <= 4096) {
    const int32_t* npq = ws.npq ? ws.npq : nullptr;
    const size_t lds = np2 * sizeof(uint64_t);
    if (sd.nlist <= 1024)
      hipLaunchKernelGGL(k_topn_wg<4>, dim3(sd.nq), dim3(256), lds, st, coarse, sd.nlist, npq, sd.npconst, sd.npmax,
                         ws.probes);
    else if (sd.nlist <= 2048)
      hipLaunchKernelGGL(k_topn_wg<8>, dim3(sd.nq), dim3(256), lds, st, coarse, sd.nlist, npq, sd.npconst, sd.npmax,
                         ws.probes);
    else
      hipLaunchKernelGGL(k_topn_wg<16>, dim3(sd.nq), dim3(256), lds, st, coarse, sd.nlist, npq, sd.npconst,
                         sd.npmax, ws.probes);
  } else {
    hipLaunchKernelGGL(k_topn, dim3(sd.nq), dim3(256), np2 * sizeof(uint64_t), st, coarse, sd.nlist, np2,
                       ws.npq ? ws.npq : nullptr, sd.npconst, sd.npmax, ws.probes);
  }
  mark(2);
  const bool ipm = sd.metric == AMP_IP;
  // inner product, integer policies: the queries on the grid (predictor,
  // table build, pair bases)
  if (ipm && !fp32) {
    const size_t nel = (size_t)sd.nq * sd.d;
    hipLaunchKernelGGL(k_qgrid, dim3((unsigned)std::min<size_t>((nel + 255) / 256, 65536)), dim3(256), 0, st, queries,
                       ws.qi16, nel, sd.grid_e, sd.grid_kind);
  }
  // PPM
  PairArgs pa;
  pa.Q = queries;
  pa.C = dv.centroids;
  pa.qi16 = (ipm && !fp32) ? ws.qi16 : nullptr;
  pa.ci16 = dv.ci16;
  const bool pdot = ipm && !fp32 && sd.policy == AMP_POLICY_ADAPTIVE;
  pa.dot_out = pdot ? ws.pbase : nullptr;
  pa.ipmask = pdot ? ws.ipmask : nullptr;
  pa.probes = ws.probes;
  pa.radq = dv.radq;
  pa.offsets = dv.offsets;
  pa.xbits = ws.xbits;
  pa.pbits = ws.pbits;
  pa.nq = sd.nq;
  pa.d = sd.d;
  pa.npmax = sd.npmax;
  pa.grid_e = sd.grid_e;
  pa.grid_kind = sd.grid_kind;
  pa.metric = sd.metric;
  pa.policy = sd.policy;
  pa.fixed_bits = sd.fixed_bits;
  pa.lane_sel_M = sd.M;
  pa.allowed = sd.allowed_mask;
  pa.margin = sd.margin;
  pa.lg_npp = 0;
  while ((1 << pa.lg_npp) < sd.npmax) ++pa.lg_npp;
  // threads per pair: more for batches too small to fill the chip (about
  // 2^17 threads), at most 64 and at most one query per workgroup
  pa.lg_T = 0;
  while (pa.lg_T < 6 && pa.lg_npp + pa.lg_T < 8 && ((int64_t)sd.nq << (pa.lg_npp + pa.lg_T + 1)) <= (1 << 17))
    ++pa.lg_T;
  const int qpb = 256 >> (pa.lg_npp + pa.lg_T);
  hipLaunchKernelGGL(k_pairs, dim3((sd.nq + qpb - 1) / qpb), dim3(256), 0, st, pa, ma);
  mark(3);
  // exact bases of the pairs (integer policies): the full scan's queue is
  // built after the phase-1 bound and leaves out the pairs whose base exceeds
  // it.  (The FP32 policy tests its bound inside the scan, after its LUT.)
  const bool early = (!fp32 || ipm) && !sd.noskip;
  const int dt = dt_of(sd.lut_dtype);
  hipError_t err = hipSuccess;
  {
    BaseArgs ba;
    ba.Q = queries;
    ba.C = dv.centroids;
    ba.bsw = reinterpret_cast<const u32x4*>(dv.bsw);
    ba.bsw16 = reinterpret_cast<const u32x4*>(dv.bsw16);
    ba.bsw8 = reinterpret_cast<const u32x2*>(dv.bsw8);
    ba.cbi16 = dv.cbi16;
    ba.ci16 = dv.ci16;
    ba.probes = ws.probes;
    ba.pbase = ws.pbase;
    ba.qi16 = ws.qi16;
    ba.iptab = ws.iptab;
    ba.iplo = ws.iplo;
    ba.ipspan = ws.ipspan;
    ba.iplsum = ws.iplsum;
    ba.iptq = ws.iptq;
    ba.ipsh = ws.ipsh;
    ba.ipmask = ws.ipmask;
    ba.pbits = ws.pbits;
    ba.codebook = dv.codebook;
    ba.nq = sd.nq;
    ba.d = sd.d;
    ba.M = sd.M;
    ba.dsub = sd.dsub;
    ba.npmax = sd.npmax;
    ba.grid_e = sd.grid_e;
    ba.grid_kind = sd.grid_kind;
    ba.metric = sd.metric;
    ba.gran = sd.gran;
    if (ipm && fp32) {
      // the queries' FP32 dot-product tables, their row maxima, the pairs'
      // FP32 lower bounds
      const size_t n = (size_t)sd.nq * sd.M * kKsub;
      hipLaunchKernelGGL(k_iptab_f32, dim3((unsigned)std::min<size_t>((n + 255) / 256, 1 << 20)), dim3(256), 0, st,
                         ba);
      hipLaunchKernelGGL(k_ipmax_f32, dim3((unsigned)(((size_t)sd.nq * sd.M + 3) / 4)), dim3(256), 0, st, ba);
      hipLaunchKernelGGL(k_ipbase_f32, dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, st, ba);
    } else if (ipm) {
      // the pairs' qi.ci and the widths each query needs, then the queries'
      // tables with their minima (and the pair bases), then the quantised tables
      const size_t tlds = base_lds_layout(kTabQ, sd.M, sd.d).total;
      auto fn = dt == DT_F16 ? k_iptab<DT_F16> : (dt == DT_F8 ? k_iptab<DT_F8> : k_iptab<DT_BF16>);
      if ((err = hipFuncSetAttribute(kaddr(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)tlds)) != hipSuccess)
        return err;
      // (adaptive: the predictor pass wrote qi.ci and the width masks)
      if (sd.policy != AMP_POLICY_ADAPTIVE)
        hipLaunchKernelGGL(k_ipbase, dim3((unsigned)sd.nq), dim3(256), 0, st, ba);
      hipLaunchKernelGGL(fn, dim3((sd.nq + kTabQ - 1) / kTabQ), dim3(kThreads), tlds, st, ba);
      const size_t nq8 = (size_t)sd.nq * sd.M * kKsub / 8;
      hipLaunchKernelGGL(k_ipq, dim3((unsigned)std::min<size_t>((nq8 + 255) / 256, 1 << 20)), dim3(256), 0, st, ba);
    } else if (early) {
      // L2 / L1: every pair's LUT minima, as many pairs per workgroup as
      // fit 64 KB of residual rows (128 at most): they share the B fragments
      int G = 128;
      while (G > 8 && (size_t)G * ri_stride(sd.d) * 2 > 65536) G >>= 1;
      ba.G = G;
      const size_t blds = base_lds_layout(G, sd.M, sd.d).total;
      auto fn = dt == DT_F16 ? k_base<DT_F16> : (dt == DT_F8 ? k_base<DT_F8> : k_base<DT_BF16>);
      if ((err = hipFuncSetAttribute(kaddr(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)blds)) != hipSuccess)
        return err;
      hipLaunchKernelGGL(fn, dim3((unsigned)((npairs + G - 1) / G)), dim3(kThreads), blds, st, ba);
    }
  }
  mark(4);
  // queue
  QueueArgs qa;
  qa.probes = ws.probes;
  qa.pbits = ws.pbits;
  qa.kq = ws.kq;
  qa.kconst = sd.kconst;
  qa.offsets = dv.offsets;
  qa.lorder = dv.lorder;
  qa.lpos = dv.lpos;
  qa.cnt = ws.cnt;
  qa.rank = ws.rank;
  qa.pairoff = ws.pairoff;
  qa.unitoff = ws.unitoff;
  qa.sorted = ws.sorted;
  qa.units = ws.units;
  qa.flags = ws.flags;
  qa.nq = sd.nq;
  qa.npmax = sd.npmax;
  qa.nlist = sd.nlist;
  qa.M = sd.M;
  qa.ncls = ncls;
  qa.gran = sd.gran;
  qa.wpr = sd.wpr;
  qa.chunk[0] = sd.chunk1;
  qa.chunk[1] = sd.chunk;
  qa.max_units = sd.max_units;
  qa.pbase = nullptr;
  qa.fkeys = 0;
  qa.tau = ws.tau;
  qa.work = nullptr;
  const int qb = (int)((npairs + 255) / 256);
  // one build of the queue phases [ph0, ph1)
  auto build_queue = [&](int ph0, int ph1) {
    QueueArgs q = qa;
    q.ph0 = ph0;
    q.ph1 = ph1;
    if (ph1 > 1 && early) {
      q.pbase = ws.pbase;
      q.fkeys = fp32 ? 1 : 0;
      q.work = sd.want_work ? ws.work : nullptr;
    }
    hipLaunchKernelGGL(k_qhist, dim3(qb), dim3(256), 0, st, q);
    hipLaunchKernelGGL(k_qtot, dim3(((ph1 - ph0) * NB + 255) / 256), dim3(256), 0, st, q, fp32 ? 1 : 0);
    hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, st, q, fp32 ? 1 : 0);
    hipLaunchKernelGGL(k_qscatter, dim3(qb), dim3(256), 0, st, q);
    hipLaunchKernelGGL(k_qunits, dim3(512), dim3(256), 0, st, q, fp32 ? 1 : 0);
  };
  build_queue(0, early ? 1 : 2);
  mark(5);
  // LC + DC, phase 1 then phase 2
  ScanArgs sa;
  sa.Q = queries;
  sa.C = dv.centroids;
  sa.codebook = dv.codebook;
  sa.bsw = reinterpret_cast<const u32x4*>(dv.bsw);
  sa.bsw16 = reinterpret_cast<const u32x4*>(dv.bsw16);
  sa.bsw8 = reinterpret_cast<const u32x2*>(dv.bsw8);
  sa.cbi16 = dv.cbi16;
  sa.codes = dv.codes;
  sa.ids = dv.ids;
  sa.offsets = dv.offsets;
  sa.kq = ws.kq;
  sa.pbits = ws.pbits;
  sa.tau = ws.tau;
  sa.ccount = ws.ccount;
  sa.ckey = ws.ckey;
  sa.cid = ws.cid;
  sa.flags = ws.flags;
  sa.nq = sd.nq;
  sa.d = sd.d;
  sa.M = sd.M;
  sa.dsub = sd.dsub;
  sa.nlist = sd.nlist;
  sa.npmax = sd.npmax;
  sa.grid_e = sd.grid_e;
  sa.grid_kind = sd.grid_kind;
  sa.metric = sd.metric;
  sa.gran = sd.gran;
  sa.noskip = sd.noskip;
  sa.kconst = sd.kconst;
  sa.kmax = sd.kmax;
  sa.chunk = sd.chunk;  // per phase below
  sa.capq = sd.capq;
  sa.retry = nullptr;
  sa.tau_id = nullptr;
  sa.any_retry = nullptr;
  sa.work = nullptr;
  sa.steal = sd.queue;
  sa.iptab = ws.iptab;
  sa.iptq = ws.iptq;
  sa.ipsh = ws.ipsh;
  sa.pbase_g = ws.pbase;
  sa.tab_out = nullptr;
  // the lane classes run one after another on the caller's stream, each a
  // persistent kernel over its own unit range.  (Running them concurrently
  // on separate streams was measured slower on the mid-size workload: scan
  // phase 2 took 1.86 ms against 1.50 ms serially.)
  for (int ph = 1; ph <= 2; ++ph) {
    sa.sorted = ws.sorted + (ph == 2 ? npairs : 0);
    sa.unitoff = ws.unitoff + (ph == 2 ? (NB + 1) : 0);
    sa.units = ws.units + (ph == 2 ? sd.max_units : 0);
    sa.chunk = ph == 2 ? sd.chunk : sd.chunk1;
    int sa_lwb;
    if (fp32 || sd.policy == AMP_POLICY_FIXED) {
      // one lane class holds every pair: its own kernel
      const int c = fp32 ? 0 : lane_class(sd.M, sd.fixed_bits, sd.gran);
      sa.cls = c;
      sa.counter = ws.counters + ((ph - 1) * (kNCls + 1) + c) * kQueueSlot;
      sa_lwb = fp32 ? 0 : lane_bits(c, sd.gran);
    } else {
      sa.cls = -1;
      sa.counter = ws.counters + ((ph - 1) * (kNCls + 1) + kNCls) * kQueueSlot;
      sa_lwb = -1;
    }
    ScanArgs sp = sa;
    sp.work = (ph == 2 && sd.want_work) ? ws.work : nullptr;
    if ((err = launch_scan(sa_lwb, ph, dt, sd.wpr, sp, st)) != hipSuccess) return err;
    if (ph == 1) {
      // phase-1 minima -> per-query bound, buffer emptied for the candidates
      hipLaunchKernelGGL(k_tau_wave, dim3((sd.nq + 3) / 4), dim3(256), 0, st, ws.ccount, ws.ckey, ws.tau, ws.kq,
                         sd.kconst, sd.nq, sd.capq, ws.flags + 1);
      // keys + digit counts + selection + list of the queries to select in
      const size_t tlds = sd.capq * 8 + 4 * (256 + 2 + 1 + 256);
      err = hipFuncSetAttribute(kaddr(k_tau), hipFuncAttributeMaxDynamicSharedMemorySize, (int)tlds);
      if (err != hipSuccess) return err;
      hipLaunchKernelGGL(k_tau, dim3(sd.nq < 1024 ? sd.nq : 1024), dim3(256), tlds, st, ws.ccount, ws.ckey, ws.tau,
                         ws.kq, sd.kconst, sd.nq, sd.capq);
      if (early) build_queue(1, 2);  // the full scan's queue: live pairs only
    }
    mark(5 + ph);
    if (ph == 2) {
      // (timed with the merge stage: the phase-2 stage is its scan alone)
      // up to two re-runs of phase 2 for queries whose candidates overflowed,
      // each with a tighter bound (the scan kernels return at once when no
      // query takes part); each re-run shrinks a query's candidate count by
      // about k / capq
      const size_t rlds = sd.capq * 16 + 4 * (1 + 256);  // sort rows + overflowed-query list
      err = hipFuncSetAttribute(kaddr(k_retry), hipFuncAttributeMaxDynamicSharedMemorySize, (int)rlds);
      if (err != hipSuccess) return err;
      ScanArgs sr = sa;
      sr.retry = ws.retry;
      sr.tau_id = ws.tau_id;
      for (int rr = 0; rr < sd.reruns; ++rr) {
        sr.any_retry = ws.flags + 1 + rr;  // one flag per round
        hipLaunchKernelGGL(k_retry, dim3(sd.nq < 256 ? sd.nq : 256), dim3(256), rlds, st, ws.ccount, ws.ckey,
                           ws.cid, ws.tau, ws.tau_id, ws.kq, sd.kconst, sd.nq, sd.capq, ws.retry,
                           ws.flags + 1 + rr, ws.counters + (kNCls + 1) * kQueueSlot,
                           (kNCls + 1) * kQueueSlot);
        // phase 3: the phase-2 scan's re-run (its own kernel symbol)
        if ((err = launch_scan(sa_lwb, 3, dt, sd.wpr, sr, st)) != hipSuccess) return err;
      }
    }
  }
  // TS
  MergeArgs ma2;
  ma2.ccount = ws.ccount;
  ma2.ckey = ws.ckey;
  ma2.cid = ws.cid;
  ma2.kq = ws.kq;
  ma2.flags = ws.flags;
  ma2.out_ids = out_ids;
  ma2.out_dist = out_dist;
  ma2.out_qdist = out_qdist;
  ma2.kconst = sd.kconst;
  ma2.kmax = sd.kmax;
  ma2.fp32 = fp32 ? 1 : 0;
  ma2.h2 = ldexpf(1.f, sd.metric == AMP_L1 ? sd.grid_e : 2 * sd.grid_e);  // L1 estimates are in units of h
  ma2.capq = sd.capq;
  const size_t mlds = sd.capq * 8 + kMergeSel * 20 + 4 * (256 + 3);
  err = hipFuncSetAttribute(kaddr(k_merge), hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds);
  if (err != hipSuccess) return err;
  const size_t flds = sd.capq * 16;
  err = hipFuncSetAttribute(kaddr(k_merge_full), hipFuncAttributeMaxDynamicSharedMemorySize, (int)flds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_merge_wave, dim3((sd.nq + 3) / 4), dim3(256), 0, st, ma2, sd.nq);
  hipLaunchKernelGGL(k_merge, dim3(sd.nq < 1024 ? sd.nq : 1024), dim3(256), mlds, st, ma2, sd.nq);
  hipLaunchKernelGGL(k_merge_full, dim3(sd.nq < 512 ? sd.nq : 512), dim3(256), flds, st, ma2, sd.nq);
  if (sd.lut_export) {
    // test hook: every pair's LUT as the search builds it
    const amp_lut_export* ex = sd.lut_export;
    BaseArgs eb{};
    eb.Q = queries;
    eb.C = dv.centroids;
    eb.bsw = reinterpret_cast<const u32x4*>(dv.bsw);
    eb.bsw16 = reinterpret_cast<const u32x4*>(dv.bsw16);
    eb.bsw8 = reinterpret_cast<const u32x2*>(dv.bsw8);
    eb.probes = ws.probes;
    eb.pbase = ws.pbase;
    eb.iptab = ws.iptab;
    eb.iptq = ws.iptq;
    eb.ipsh = ws.ipsh;
    eb.pbits = ws.pbits;
    eb.nq = sd.nq;
    eb.d = sd.d;
    eb.M = sd.M;
    eb.dsub = sd.dsub;
    eb.npmax = sd.npmax;
    eb.grid_e = sd.grid_e;
    eb.grid_kind = sd.grid_kind;
    eb.metric = sd.metric;
    eb.gran = sd.gran;
    if (ipm) {
      hipLaunchKernelGGL(k_export_ip, dim3((unsigned)npairs), dim3(256), 0, st, eb, ex->q, ex->shift, ex->base, ex->t);
    } else {
      const size_t elds = base_lds_layout(kBaseExport, sd.M, sd.d).total;
      auto fn = dt == DT_F16 ? k_export<DT_F16> : (dt == DT_F8 ? k_export<DT_F8> : k_export<DT_BF16>);
      if ((err = hipFuncSetAttribute(kaddr(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)elds)) != hipSuccess)
        return err;
      hipLaunchKernelGGL(fn, dim3((unsigned)((npairs + kBaseExport - 1) / kBaseExport)), dim3(kThreads), elds, st, eb,
                         ex->q, ex->shift, ex->base, ex->t);
    }
  }
  if (sd.out_status) hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, st, ws.flags, sd.out_status);
  mark(8);
  return hipGetLastError();
}

}  // namespace amp
