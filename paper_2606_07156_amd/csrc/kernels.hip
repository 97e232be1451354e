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
#include "amp_internal.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace amp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ helpers
// order-preserving keys: integers (sign flip) and floats (IEEE total order)
__device__ __forceinline__ uint64_t ikey(int64_t v) { return (uint64_t)v ^ 0x8000000000000000ull; }
__device__ __forceinline__ int64_t ikey_val(uint64_t k) { return (int64_t)(k ^ 0x8000000000000000ull); }
__device__ __forceinline__ uint32_t fkey(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fkey_val(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

// nearest E4M3 value of an integer: 3 mantissa bits, ties to even, saturating
// at 448 (OCP 8-bit floating point specification, E4M3 "fn" encoding)
__device__ __forceinline__ int e4m3_int(int v) {
  int a = v < 0 ? -v : v;
  if (a >= 16) {
    int E = 31 - __clz(a);
    int sh = E - 3;
    int q = a >> sh;
    int rem = a & ((1 << sh) - 1);
    int half = 1 << (sh - 1);
    if (rem > half || (rem == half && (q & 1))) q++;
    a = q << sh;
  }
  a = a > 448 ? 448 : a;
  return v < 0 ? -a : a;
}

// operand grid: round half to even of r * 2^-e, then saturate (9-bit grid) or
// round to the e4m3-representable integers
__device__ __forceinline__ int grid_val(float r, int e, int kind) {
  const float x = rintf(ldexpf(r, -e));
  if (kind == AMP_GRID_U9) return (int)__builtin_amdgcn_fmed3f(x, -255.f, 255.f);
  return e4m3_int((int)__builtin_amdgcn_fmed3f(x, -65536.f, 65536.f));
}

__device__ __forceinline__ uint32_t bf16_bits(float v) {  // exact inputs only
  return __float_as_uint(v) >> 16;
}

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
  size_t nq;
};
__global__ void k_reset(ResetArgs r) {
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, st = (size_t)gridDim.x * blockDim.x;
  for (size_t i = i0; i < r.ncnt; i += st) r.cnt[i] = 0;
  for (size_t i = i0; i < r.ncounters; i += st) r.counters[i] = 0;
  for (size_t i = i0; i < r.nq; i += st) {
    r.tau[i] = ~0ull;
    r.ccount[i] = 0;
  }
  if (i0 < 4) {
    r.flags[i0] = 0;
    r.work[i0] = 0;
  }
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
// workgroup, each wave a 32x32 quarter of 2x2 MFMA 16x16x4 FP32 tiles.
constexpr int CL_T = 64, CL_K = 32;
__global__ __launch_bounds__(256) void k_coarse(const float* __restrict__ Q, const float* __restrict__ C,
                                                const float* __restrict__ qn, const float* __restrict__ cn,
                                                float* __restrict__ D, int nq, int nlist, int d, int metric) {
  __shared__ float Qs[CL_T][CL_K + 1];
  __shared__ float Cs[CL_T][CL_K + 1];
  const int q0 = blockIdx.y * CL_T, c0 = blockIdx.x * CL_T;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < d; k0 += CL_K) {
    for (int i = tid; i < CL_T * CL_K; i += 256) {
      int r = i / CL_K, kk = i % CL_K, gk = k0 + kk;
      Qs[r][kk] = (q0 + r < nq && gk < d) ? Q[(size_t)(q0 + r) * d + gk] : 0.f;
      Cs[r][kk] = (c0 + r < nlist && gk < d) ? C[(size_t)(c0 + r) * d + gk] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < CL_K; kk += 4) {
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
// their list ids, are gathered in LDS (any order), padded to a power of two
// and sorted by (key, list id); the first nprobe are the probes, the same as
// a sort of the whole row.
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
  __shared__ int32_t s_table[kTableN];
  const int lg = a.lg_npp, lt = a.lg_T, T = 1 << lt;
  const int t = threadIdx.x & (T - 1);
  const int slot = threadIdx.x >> (lg + lt), r = (threadIdx.x >> lt) & ((1 << lg) - 1);
  const int q = blockIdx.x * (256 >> (lg + lt)) + slot;
  const bool adaptive = a.policy == AMP_POLICY_ADAPTIVE;
  if (adaptive)
    for (int i = threadIdx.x; i < kTableN; i += blockDim.x) s_table[i] = ma.table[i];
  if ((threadIdx.x & ((1 << (lg + lt)) - 1)) == 0) s_best[slot] = ~0ull;
  __syncthreads();
  const bool valid = q < a.nq && r < a.npmax;
  const int p = valid ? a.probes[(size_t)q * a.npmax + r] : -1;
  int64_t dq2 = 0;
  if (adaptive && p >= 0) {
    // d' = |grid residual|^2, four coordinates per step (d % 4 == 0)
    const float4* qv = reinterpret_cast<const float4*>(a.Q + (size_t)q * a.d);
    const float4* cv = reinterpret_cast<const float4*>(a.C + (size_t)p * a.d);
    const bool l2 = a.metric != AMP_IP;  // L2 and L1: d' of the grid residual
    for (int i = t; i < (a.d >> 2); i += T) {
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
      dq2 += (int64_t)(v0 * v0 + v1 * v1) + (int64_t)(v2 * v2 + v3 * v3);
    }
  }
  // the T threads of a pair are adjacent lanes of one wave (T <= 64)
  for (int o = 1; o < T; o <<= 1) dq2 += __shfl_xor(dq2, o);
  if (adaptive && p >= 0 && t == 0)
    atomicMin(&s_best[slot], (unsigned long long)((uint64_t)dq2 << 13 | (uint64_t)p));
  __syncthreads();
  if (!valid) return;
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
  int64_t chunk[2], max_units;  // list chunk of a work unit in phase 1, phase 2
};

__device__ __forceinline__ int pair_class(int bits, int M) {
  if (bits == 32) return 0;
  uint64_t top = (uint64_t)M * ((1ull << bits) - 1);
  return top <= 0xFFull ? 0 : (top <= 0xFFFFull ? 1 : 2);
}
__device__ __forceinline__ int class_pairs(int cls, int wpr, bool fp32) {
  return fp32 ? wpr : wpr * (4 >> cls);
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
  const int cls = pair_class(a.pbits[i], a.M);
  const int NB = a.ncls * a.nlist;
  const size_t b = (size_t)pair_sub(i) * NB + cls * a.nlist + p;
  a.rank[n + i] = atomicAdd(&a.cnt[(size_t)kQSub * NB + b], 1);
  if (in_phase1(a, i)) a.rank[i] = atomicAdd(&a.cnt[b], 1);
}

// per (phase, class, list) bucket: its pair total from the sub-counters
// (which become offsets inside the bucket) and its unit count, stored at the
// bucket's launch position (pairoff / unitoff hold counts until k_qscan)
__global__ void k_qtot(QueueArgs a, int fp32) {
  const int NB = a.ncls * a.nlist;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * NB) return;
  const int ph = i / NB, b = i % NB, cls = b / a.nlist, p = b % a.nlist;
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
  const int G = class_pairs(cls, a.wpr, fp32);
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
  for (int ph = 0; ph < 2; ++ph) {
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
  const int cls = pair_class(a.pbits[i], a.M);
  const int b = cls * a.nlist + a.lpos[p];
  const int NB = a.ncls * a.nlist;
  const size_t bs = (size_t)pair_sub(i) * NB + cls * a.nlist + p;  // sub-counter offset
  a.sorted[n + a.pairoff[(NB + 1) + b] + a.cnt[(size_t)kQSub * NB + bs] + a.rank[n + i]] = (int32_t)i;
  if (in_phase1(a, i)) a.sorted[a.pairoff[b] + a.cnt[bs] + a.rank[i]] = (int32_t)i;
}

// grid-stride over (phase, unit): find the unit's bucket by binary search of
// the unit offsets and write its descriptor
__global__ void k_qunits(QueueArgs a, int fp32) {
  const int NB = a.ncls * a.nlist;
  for (int ph = 0; ph < 2; ++ph) {
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
      const int G = class_pairs(cls, a.wpr, fp32);
      const int64_t local = u - uo[b], grp = local / nch, ch = local % nch;
      const int64_t left = (po[b + 1] - po[b]) - grp * G;
      units[u] = make_int4(p, (int)(po[b] + grp * G), (int)(left < G ? left : G), (int)ch);
    }
  }
}

// ------------------------------------------------------------------ scan
struct ScanArgs {
  const float* Q;
  const float* C;
  const float* codebook;   // FP32 policy
  const u32x4* bsw;        // integer policy MFMA B fragments (BF16, with aug slots)
  const u32x4* bsw16;      // FP16 dims fragments
  const int16_t* cbi16;    // [M][256][8] grid codebook (L1 LUT build)
  const uint8_t* codes;
  const int64_t* ids;
  const int64_t* offsets;
  const int32_t* kq;
  const uint8_t* pbits;
  const int32_t* sorted;   // this phase's sorted pairs
  const int64_t* unitoff;  // this phase's unit offsets (NB+1)
  const int4* units;       // this phase's unit table
  uint32_t* counter;       // this phase/class unit counter
  uint64_t* tau;
  uint32_t* ccount;
  uint64_t* ckey;
  int64_t* cid;
  int32_t* flags;
  const uint8_t* retry;     // phase 3 (re-run of phase 2): queries taking part
  const int64_t* tau_id;    // phase 3: id of the bound's (distance, id) key
  const int32_t* any_retry; // phase 3: non-zero if any query takes part
  uint64_t* work;           // phase 2 work counters (code bytes scanned, live pairs, dead pairs) or null
  int nq, d, M, dsub, nlist, npmax, grid_e, grid_kind, metric, kconst, kmax, cls;
  int steal;                // unit queue: 0 one counter, 1 per-XCD ranges with stealing
  int64_t chunk;
  size_t capq;
};

// Unit fetch of the persistent scan kernels (called by one thread of the
// workgroup; returns a unit number of the launch order, `total` once the
// queue is drained).  steal = 0: one counter over the cost-sorted order.
// steal = 1: the order is cut into kXcd contiguous ranges, range x served
// by the workgroups of XCD x (workgroups are dispatched to the XCDs in turn,
// so blockIdx mod kXcd is the XCD), which keeps the units of one list
// (adjacent in the order) on one XCD's L2; a workgroup whose range is used
// up takes units from the next ranges in ring order (work stealing).  Every
// counter sits in its own 128-byte line; the counters only grow, so a
// drained range stays drained and every workgroup ends after at most kXcd
// failed attempts.
struct UnitQueue {
  uint32_t* ctr;
  int64_t total;
  int steal, home, vic;
  __device__ __forceinline__ UnitQueue(uint32_t* c, int64_t t, int s)
      : ctr(c), total(t), steal(s), home((int)(blockIdx.x % kXcd)), vic(0) {}
  __device__ __forceinline__ int64_t next() {
    if (!steal) return (int64_t)atomicAdd(ctr, 1u);
    for (; vic < kXcd; ++vic) {
      const int x = (home + vic) % kXcd;
      const int64_t lo = total * x / kXcd, hi = total * (x + 1) / kXcd;
      if (lo >= hi) continue;
      const int64_t u = lo + (int64_t)atomicAdd(ctr + x * kCtrStride, 1u);
      if (u < hi) return u;
    }
    return total;
  }
};

// words per LUT row for a subspace count: the LUT of one work unit takes
// M * 256 * WPR * 4 bytes of LDS
__host__ __device__ constexpr int wpr_for(int M) { return M <= 16 ? 4 : (M <= 32 ? 2 : 1); }
// words per LUT row of a scan kernel variant: the variants specialised for a
// subspace count MT pack wpr_for(MT) words, the generic one (MT = 0) one word.
// The work-unit queue packs pairs into units with the same figure, so both
// sides take it from here.
__host__ __device__ constexpr int kernel_wpr(int MT) { return MT ? wpr_for(MT) : 1; }
// a variant specialised for MT may also run with one-word rows (NR = 1:
// sparse batches, a few pairs per list), keeping its codes in registers
__host__ __device__ constexpr int variant_wpr(int MT, int NR) { return NR ? 1 : kernel_wpr(MT); }

// row stride (int16 elements) of the integer residuals in LDS: each row is
// padded by 32 bytes, so the eight rows that the LC A-operand build reads at
// once (d a multiple of 64 puts them all in one bank otherwise) fall in
// distinct banks, as do the two subspaces of an m-pair
__host__ __device__ constexpr int ri_stride(int d) { return d + 16; }

// LDS carve-up of one scan workgroup (all offsets in bytes, 16-aligned)
struct ScanLds {
  int lut, ri, rr, lo, hi, pq, pb, ps, pbase, psig, lmin, ctl, total;
};
__host__ __device__ inline ScanLds scan_lds_layout(int G, int wpr, int M, int d, bool fp32, int phase) {
  ScanLds L;
  int o = 0;
  auto take = [&](int bytes) { int r = o; o += (bytes + 15) & ~15; return r; };
  L.lut = take(M * kKsub * wpr * 4);
  L.ri = take(G * (fp32 ? d * 4 : ri_stride(d) * 2));
  L.rr = take(G * M * 4);
  L.lo = take(G * M * 4);
  L.hi = take(G * M * 4);
  L.pq = take(G * 4);
  L.pb = take(G * 4);
  L.ps = take(G * 4);
  L.pbase = take(G * 8);
  L.psig = take(G * 4);
  // phase 1 keeps per-thread minima after the scan: reuse the LUT space
  L.lmin = L.lut;
  if (phase == 1 && G * kThreadsP2 * 4 > M * kKsub * wpr * 4) L.lmin = take(G * kThreadsP2 * 4);
  // unit-claim control words: kept in the dynamic LDS too, so that the LUT
  // starts at LDS address 0 and row addresses fold into instruction offsets
  L.ctl = take(64);  // unit index, class, re-run vote, live vote, unit descriptor, 3 work counters
  L.total = o;
  return L;
}

template <int LWB>  // lane bits 8/16/32, 0 = FP32 LUT
struct Lane {
  static constexpr int W = LWB ? 32 / LWB : 1;
  static constexpr uint32_t MASK = LWB == 32 || LWB == 0 ? 0xFFFFFFFFu : ((1u << LWB) - 1);
};

// where pair g of a work unit sits in a LUT row: word and field.  The 8-bit
// class with four words per row interleaves the pairs (word 2 h + t holds
// pairs 8 t + 4 h + 0..3) so that a lane of the LUT build writes its two
// words with one 8-byte store; every other layout is word g / W, field g % W.
template <int LWB, int WPR>
struct PairSlot {
  static constexpr bool IL = LWB == 8 && WPR == 4;
  static constexpr int W = Lane<LWB>::W;
  __host__ __device__ static constexpr int word(int g) { return IL ? (((g >> 2) & 1) << 1) | (g >> 3) : g / W; }
  __host__ __device__ static constexpr int field(int g) { return IL ? (g & 3) : g % W; }
  __host__ __device__ static constexpr int pair(int w, int f) {
    return IL ? ((w & 1) << 3) | ((w >> 1) << 2) | f : w * W + f;
  }
};

// LDS-address-space views: the scan kernels declare no static LDS, so their
// dynamic block (the LUT first) starts at LDS address 0 and a row address is
// a plain constant offset plus the scaled code byte
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
typedef __attribute__((address_space(3))) const u32x2 lds_u32x2;
typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;

template <int WPR>
__device__ __forceinline__ void lut_row_load(lds_u32* lut, int row, uint32_t* w) {
  if constexpr (WPR == 4) {
    u32x4 x = *reinterpret_cast<lds_u32x4*>(lut + row);
    w[0] = x[0]; w[1] = x[1]; w[2] = x[2]; w[3] = x[3];
  } else if constexpr (WPR == 2) {
    u32x2 x = *reinterpret_cast<lds_u32x2*>(lut + row);
    w[0] = x[0]; w[1] = x[1];
  } else {
    w[0] = lut[row];
  }
}

// min / max over each 16-lane row of a wave: after row shifts by 1, 2, 4, 8
// (lanes without a source keep their value) lane 15 of the row holds it
template <bool MAX, int K>
__device__ __forceinline__ int row16_step(int v) {
  const int o = __builtin_amdgcn_update_dpp(v, v, 0x110 + K, 0xF, 0xF, false);  // row_shr:K
  return MAX ? (o > v ? o : v) : (o < v ? o : v);
}
template <bool MAX>
__device__ __forceinline__ int row16_reduce(int v) {
  return row16_step<MAX, 8>(row16_step<MAX, 4>(row16_step<MAX, 2>(row16_step<MAX, 1>(v))));
}

// LC matrix dtypes of the integer LUT build.  (An FP8 e4m3 variant is not
// offered: the 16x16x32 FP8 MFMA of gfx950 does not return the exact sum of
// e4m3-grid products of the magnitudes the grid allows.)
enum { DT_BF16 = 1, DT_F16 = 2 };

__device__ __forceinline__ uint32_t f16_bits(float v) {  // exact inputs only
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
}
// One m-pair of the integer LUT of a work unit.  Rows of the A operand are
// (subspace slot ms, pair g) = ms*8 + g; K holds [dims m0 | aug m0 | dims m1 |
// aug m1], 8 slots each.  The aug slots carry |cbi|^2 (digits in B, powers
// of two in A) and |ri|^2 + off (digits in A, powers of two in B).
//  * DT_BF16: one BF16 MFMA 16x16x32 with everything scaled by 2^-s in A
//    gives exactly 2^-s (T + off) (every partial sum is an integer multiple of
//    2^-s below 2^(24-s));
//  * DT_F16: the aug terms on BF16 MFMA, then the dot products (-2 ri, or
//    -ri for inner product) on an FP16 MFMA accumulating into the same FP32
//    registers: T + off exactly, scaled by 2^-s afterwards.
// Inner product: dims coefficient -1 and no |ri|^2, |cbi|^2 terms.
// PASS 1: off = 0, s = 0, record min/max over the codewords (integer
// compares of the exact values);
// PASS 2: quantise (truncation of the exact non-negative value) and pack.
// The pass is a template argument so that the 16 x NGT products of an m-pair
// are independent straight-line code the compiler can overlap.
template <int LWB, int WPR, int DT, int PASS, bool IP>
__device__ __forceinline__ void lut_mpair(const ScanArgs& a, char* lds, const ScanLds& L, int M, int np_u,
                                          int mp, const u32x4 (&B)[16], const u32x4 (&Bd)[16]) {
  constexpr int pass = PASS;
  constexpr int W = Lane<LWB>::W;
  constexpr int G = WPR * W;
  constexpr int NGT = (G + 7) / 8;
  const int lane = threadIdx.x & 63;
  const int16_t* ri = reinterpret_cast<const int16_t*>(lds + L.ri);
  const int32_t* rr = reinterpret_cast<const int32_t*>(lds + L.rr);
  int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
  int32_t* hi = reinterpret_cast<int32_t*>(lds + L.hi);
  const int32_t* ps = reinterpret_cast<const int32_t*>(lds + L.ps);
  uint32_t* lut = reinterpret_cast<uint32_t*>(lds + L.lut);
  const int row = lane & 15, kg = lane >> 4;
  const int ms_row = row >> 3;
  const int dsub = a.dsub;
  const int rs = ri_stride(a.d);
  constexpr bool ip = IP;  // metric as a compile-time flag: no per-value select
  bf16x8 A[NGT];
  u32x4 Ad[NGT];
#pragma unroll
  for (int gt = 0; gt < NGT; ++gt) {
    const int g = gt * 8 + (row & 7);
    const int m = 2 * mp + ms_row;
    uint32_t pk[4] = {0, 0, 0, 0}, pd[4] = {0, 0, 0, 0};
    if (g < np_u && (kg >> 1) == ms_row) {
      const int s = pass == 1 ? 0 : ps[g];
      const float sc = DT == DT_BF16 ? ldexpf(1.f, -s) : 1.f;
      if ((kg & 1) == 0) {
        const int coef = ip ? -1 : -2;
        // the subspace's grid residual: one 16-byte read when d_sub = 8
        // (rows and subspaces 16-byte aligned), else element by element
        int rv[8];
        if (dsub == 8 && (a.d & 7) == 0) {
          const u32x4 w = *reinterpret_cast<const u32x4*>(ri + g * rs + m * 8);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            rv[2 * t] = (int)(int16_t)(w[t] & 0xFFFFu);
            rv[2 * t + 1] = (int)(int16_t)(w[t] >> 16);
          }
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t) rv[t] = t < dsub ? (int)ri[g * rs + m * dsub + t] : 0;
        }
        if constexpr (DT == DT_BF16) {
          float v[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) v[t] = t < dsub ? (float)(coef * rv[t]) * sc : 0.f;
#pragma unroll
          for (int t = 0; t < 4; ++t) pk[t] = bf16_bits(v[2 * t]) | (bf16_bits(v[2 * t + 1]) << 16);
        } else {
          float v[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) v[t] = t < dsub ? (float)(coef * rv[t]) : 0.f;
#pragma unroll
          for (int t = 0; t < 4; ++t) pd[t] = f16_bits(v[2 * t]) | (f16_bits(v[2 * t + 1]) << 16);
        }
      } else {
        int32_t X = ip ? 0 : rr[g * M + m];
        if (pass == 2) X += lo[g * M + m];  // lo holds off = hf(s) - min after pass 1
        const float sg = X < 0 ? -1.f : 1.f;
        const uint32_t ax = (uint32_t)(X < 0 ? -X : X);
        const float cm = ip ? 0.f : sc;
        float v[8];
        v[0] = 65536.f * cm;
        v[1] = 256.f * cm;
        v[2] = cm;
        v[3] = sg * (float)(ax >> 16) * sc;
        v[4] = sg * (float)((ax >> 8) & 255u) * sc;
        v[5] = sg * (float)(ax & 255u) * sc;
        v[6] = 0.f;
        v[7] = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) pk[t] = bf16_bits(v[2 * t]) | (bf16_bits(v[2 * t + 1]) << 16);
      }
    }
    u32x4 u = {pk[0], pk[1], pk[2], pk[3]};
    A[gt] = __builtin_bit_cast(bf16x8, u);
    Ad[gt] = (u32x4){pd[0], pd[1], pd[2], pd[3]};
  }
  // D rows of this lane: (ms = kg>>1, g = gt*8 + 4*(kg&1) + i), column j
  const int m_out = 2 * mp + (kg >> 1);
  float rsc[NGT][4];  // 2^-s of each row (used after a non-BF16 build)
#pragma unroll
  for (int gt = 0; gt < NGT; ++gt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int g = gt * 8 + 4 * (kg & 1) + i;
      rsc[gt][i] = (DT == DT_BF16 || pass == 1 || g >= np_u) ? 1.f : ldexpf(1.f, -ps[g]);
    }
  int mn[NGT][4], mx[NGT][4];
  uint32_t wv8[NGT];  // packed words of the interleaved 8-bit layout
#pragma unroll
  for (int gt = 0; gt < NGT; ++gt)
#pragma unroll
    for (int i = 0; i < 4; ++i) { mn[gt][i] = 0x7FFFFFFF; mx[gt][i] = -0x7FFFFFFF - 1; }
#pragma unroll
  for (int jt = 0; jt < 16; ++jt) {
    const bf16x8 Bf = __builtin_bit_cast(bf16x8, B[jt]);
    const u32x4 Bdj = Bd[jt];
    const int j = jt * 16 + (lane & 15);
#pragma unroll
    for (int gt = 0; gt < NGT; ++gt) {
      f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[gt], Bf, (f4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      if constexpr (DT == DT_F16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, Ad[gt]),
                                                     __builtin_bit_cast(f16x8, Bdj), acc, 0, 0, 0);
      }
      const int g0 = gt * 8 + 4 * (kg & 1);
      if constexpr (PASS == 1) {
        // exact integers: for L2 (T >= 0) the float bit patterns order as
        // integers; inner product values may be negative and are converted
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t = ip ? (int)acc[i] : __float_as_int(acc[i]);
          mn[gt][i] = t < mn[gt][i] ? t : mn[gt][i];
          mx[gt][i] = t > mx[gt][i] ? t : mx[gt][i];
        }
      } else if (g0 < G) {
        uint32_t qv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float vv = DT == DT_BF16 ? acc[i] : acc[i] * rsc[gt][i];  // power-of-two scale: exact
          qv[i] = (uint32_t)vv;  // exact and >= 0: truncation = floor
        }
        uint32_t* dst = lut + (size_t)(m_out * kKsub + j) * WPR;
        if constexpr (PairSlot<LWB, WPR>::IL) {
          wv8[gt] = qv[0] | (qv[1] << 8) | (qv[2] << 16) | (qv[3] << 24);
          if (gt == NGT - 1)  // words 2 h, 2 h + 1 (h = kg & 1): one 8-byte store
            *reinterpret_cast<u32x2*>(dst + 2 * (kg & 1)) = (u32x2){wv8[0], wv8[1]};
        } else if constexpr (LWB == 8) {
          dst[g0 >> 2] = qv[0] | (qv[1] << 8) | (qv[2] << 16) | (qv[3] << 24);
        } else if constexpr (LWB == 16) {
          const int w0 = g0 >> 1;
          if (w0 + 1 < WPR)
            *reinterpret_cast<u32x2*>(dst + w0) = (u32x2){qv[0] | (qv[1] << 16), qv[2] | (qv[3] << 16)};
          else if (w0 < WPR)
            dst[w0] = qv[0] | (qv[1] << 16);
        } else if constexpr (WPR == 4) {
          *reinterpret_cast<u32x4*>(dst) = (u32x4){qv[0], qv[1], qv[2], qv[3]};  // g0 == 0 here
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (g0 + i < WPR) dst[g0 + i] = qv[i];
        }
      }
    }
  }
  if constexpr (PASS == 1) {
#pragma unroll
    for (int gt = 0; gt < NGT; ++gt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int a0 = row16_reduce<false>(mn[gt][i]), b0 = row16_reduce<true>(mx[gt][i]);
        if (!ip) {
          a0 = (int)__int_as_float(a0);
          b0 = (int)__int_as_float(b0);
        }
        const int g = gt * 8 + 4 * (kg & 1) + i;
        if ((lane & 15) == 15 && g < np_u) {
          lo[g * M + m_out] = a0;
          hi[g * M + m_out] = b0;
        }
      }
  }
}

// FP32 LUT entries are built by thread (m, j) = (kMPar i + tid / 256, tid % 256)
// (threads past kMPar * 256 do not take part)
constexpr int kMPar = kThreads / kKsub;  // subspaces built side by side
template <int WPR, int MT>
struct Owned {
  // codewords of the FP32 LUT entries a thread owns
  static constexpr int NM = MT ? MT / kMPar : 1;
  float c[NM][kMaxDsub];
};

// One work unit (G pairs of one list, lane class LWB; 0 = FP32 LUT): RC, LC,
// quantisation, DC scan, and the phase's bound or candidate forwarding.
// L may be the layout of a larger tile (the mixed-class kernel).
template <int LWB, int MT, int PHASE, int DT, int NR, typename Own, typename Fetch>
__device__ __forceinline__ void scan_unit(const ScanArgs& a, char* lds, const ScanLds& L, const Own& own,
                                          const int4 unit, Fetch&& fetch_next) {
  constexpr int WPR = variant_wpr(MT, NR);
  constexpr bool FP = LWB == 0;
  constexpr int W = Lane<LWB>::W;
  constexpr int G = WPR * W;
  constexpr uint32_t MASK = Lane<LWB>::MASK;
  constexpr bool CRES = FP && MT != 0 && MT <= 16;  // FP32 codewords stay in registers
  const int M = MT ? MT : a.M;
  int32_t* pq = reinterpret_cast<int32_t*>(lds + L.pq);
  int32_t* pb = reinterpret_cast<int32_t*>(lds + L.pb);
  int32_t* ps = reinterpret_cast<int32_t*>(lds + L.ps);
  int64_t* pbase = reinterpret_cast<int64_t*>(lds + L.pbase);
  uint32_t* psig = reinterpret_cast<uint32_t*>(lds + L.psig);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int own_j = tid % kKsub, own_m0 = tid / kKsub;
  const bool owner = tid < kMPar * kKsub;
    const int p = unit.x;
    int np_u = unit.z;
    if (np_u > G) {  // a unit never holds more pairs than the tile (guarded, flagged)
      if (tid == 0) atomicOr(&a.flags[0], 8);
      np_u = G;
    }
    const int64_t L0 = a.offsets[p];
    const int64_t n_list = a.offsets[p + 1] - L0;
    const int64_t v0 = (int64_t)unit.w * a.chunk;
    const int64_t v1 = v0 + a.chunk < n_list ? v0 + a.chunk : n_list;
    if (tid < G) {
      if (tid < np_u) {
        const int pid = a.sorted[unit.y + tid];
        pq[tid] = pid / a.npmax;
        pb[tid] = a.pbits[pid];
      } else {
        pq[tid] = -1;
        pb[tid] = 16;
      }
    }
    if (PHASE == 3) {
      // re-run: a unit with no pair of a re-run query is skipped whole (the
      // vote goes through a control word of the dynamic LDS: the scan
      // kernels use no static LDS)
      int& s_part = *reinterpret_cast<int*>(lds + L.ctl + 8);
      if (tid == 0) s_part = 0;
      __syncthreads();
      if (tid < np_u && a.retry[pq[tid]]) s_part = 1;
      __syncthreads();
      if (!s_part) {
        fetch_next();
        return;
      }
    }
    __syncthreads();
    // ---- RC: residuals (FP32, then onto the grid for integer policies)
    // (inner product: the query itself, on the grid for integer policies)
    // four coordinates per thread and step (d is a multiple of 4, query rows
    // and centroids 16-byte aligned); (pair, quad) advanced without division
    const bool ip = a.metric == AMP_IP;
    const bool l1 = a.metric == AMP_L1;
    {
      const int d4 = a.d >> 2;
      const int gstep = kThreads / d4, tstep = kThreads - gstep * d4;
      int g = tid / d4, t4 = tid - g * d4;
      const float4* C4 = reinterpret_cast<const float4*>(a.C + (size_t)p * a.d);
      while (g < np_u) {
        const float4 qv = reinterpret_cast<const float4*>(a.Q + (size_t)pq[g] * a.d)[t4];
        float4 r = qv;
        if (!ip) {
          const float4 cv = C4[t4];
          r.x = qv.x - cv.x;
          r.y = qv.y - cv.y;
          r.z = qv.z - cv.z;
          r.w = qv.w - cv.w;
        }
        if constexpr (FP) {
          reinterpret_cast<float4*>(lds + L.ri)[g * d4 + t4] = r;
        } else {
          const uint32_t v0 = (uint32_t)grid_val(r.x, a.grid_e, a.grid_kind) & 0xFFFFu;
          const uint32_t v1 = (uint32_t)grid_val(r.y, a.grid_e, a.grid_kind) & 0xFFFFu;
          const uint32_t v2 = (uint32_t)grid_val(r.z, a.grid_e, a.grid_kind) & 0xFFFFu;
          const uint32_t v3 = (uint32_t)grid_val(r.w, a.grid_e, a.grid_kind) & 0xFFFFu;
          reinterpret_cast<u32x2*>(lds + L.ri)[g * (ri_stride(a.d) >> 2) + t4] = (u32x2){v0 | (v1 << 16), v2 | (v3 << 16)};
        }
        g += gstep;
        t4 += tstep;
        if (t4 >= d4) {
          t4 -= d4;
          ++g;
        }
      }
    }
    __syncthreads();
    // ---- per-pair pruning threshold in the lane domain (phases 2, 3): a
    // pair whose base already exceeds its query's bound is dead (pb = -1)
    auto pair_threshold = [&](int g) -> bool {
      uint32_t sig = 0;
      bool live = false;
      if (g < np_u && (PHASE != 3 || a.retry[pq[g]])) {
        const uint64_t tk = a.tau[pq[g]];
        live = true;
        if (tk == ~0ull) {
          sig = 0xFFFFFFFFu;
        } else if constexpr (FP) {
          sig = (uint32_t)tk;
          // the pair's lower bound (sum of its row minima) already above
          if (PHASE >= 2 && fkey(reinterpret_cast<const float*>(lds + L.pbase)[g]) > sig) live = false;
        } else {
          const int64_t t = ikey_val(tk);
          if (t < pbase[g]) {
            live = false;
          } else {
            const int64_t dd = (t - pbase[g]) >> ps[g];
            sig = dd > (int64_t)MASK ? MASK : (uint32_t)dd;
          }
        }
      }
      psig[g] = live ? sig : 0;
      pb[g] = live ? pb[g] : -1;  // -1: no candidate can pass
      return live;
    };
    auto thresholds = [&] {
      if (PHASE >= 2 && tid < G) pair_threshold(tid);
    };
    // ---- LC
    if constexpr (FP) {
      // T[m][j] = (|r_m|^2 + |c_mj|^2) - 2 r_m.c_mj in FP32 (one FMA chain per entry)
      const float* r32 = reinterpret_cast<const float*>(lds + L.ri);
      float* rr32 = reinterpret_cast<float*>(lds + L.rr);
      for (int e = tid; e < np_u * M; e += kThreads) {
        const int g = e / M, m = e % M;
        const float* r = r32 + g * a.d + m * a.dsub;
        float sq = 0.f;
        if (ip) {  // partial -q.c of this subspace
          const float* c = a.C + (size_t)p * a.d + m * a.dsub;
#pragma unroll
          for (int t = 0; t < kMaxDsub; ++t)
            if (t < a.dsub) sq = fmaf(-r[t], c[t], sq);
        } else {
#pragma unroll
          for (int t = 0; t < kMaxDsub; ++t)
            if (t < a.dsub) sq = fmaf(r[t], r[t], sq);
        }
        rr32[e] = sq;
      }
      __syncthreads();
      if (tid < G) {
        ps[tid] = 0;
        pbase[tid] = 0;
      }
      float* lut = reinterpret_cast<float*>(lds + L.lut);
      // the metric is a compile-time tag of the entry code (0 L2, 1 IP, 2 L1)
      auto entry = [&](auto mtag, int m, const float (&c)[kMaxDsub]) {
        constexpr int MM = decltype(mtag)::value;
        const int e = m * kKsub + own_j;
        float cc = 0.f;
        if constexpr (MM == 0) {
#pragma unroll
          for (int t = 0; t < kMaxDsub; ++t) cc = fmaf(c[t], c[t], cc);
        }
        float out[WPR];
#pragma unroll
        for (int g = 0; g < WPR; ++g) {
          float sv = 0.f;
          if (g < np_u) {
            const float* r = r32 + g * a.d + m * a.dsub;
            if constexpr (MM == 2) {
              float ad = 0.f;
#pragma unroll
              for (int t = 0; t < kMaxDsub; ++t)
                if (t < a.dsub) ad += fabsf(r[t] - c[t]);
              sv = ad;
            } else {
              float dot = 0.f;
#pragma unroll
              for (int t = 0; t < kMaxDsub; ++t)
                if (t < a.dsub) dot = fmaf(r[t], c[t], dot);
              if constexpr (MM == 1) {
                // inner product: the pair's base -q.c (sum of the subspace
                // partials) is folded into subspace 0's entries
                float bf = 0.f;
                if (m == 0)
                  for (int mm = 0; mm < M; ++mm) bf += rr32[g * M + mm];
                sv = bf - dot;
              } else {
                sv = fmaf(-2.f, dot, rr32[g * M + m] + cc);
              }
            }
          }
          out[g] = sv;
        }
        float* dst = lut + (size_t)e * WPR;
#pragma unroll
        for (int g = 0; g < WPR; ++g) dst[g] = out[g];
      };
      auto fill = [&](auto mtag) {
        if constexpr (CRES) {
          if (owner) {
#pragma unroll
            for (int i = 0; i < MT / kMPar; ++i) entry(mtag, kMPar * i + own_m0, own.c[i]);
          }
        } else if (owner) {
          for (int m = own_m0; m < M; m += kMPar) {
            float c[kMaxDsub];
#pragma unroll
            for (int t = 0; t < kMaxDsub; ++t)
              c[t] = t < a.dsub ? a.codebook[((size_t)m * kKsub + own_j) * a.dsub + t] : 0.f;
            entry(mtag, m, c);
          }
        }
      };
      if (l1) fill(std::integral_constant<int, 2>{});
      else if (ip) fill(std::integral_constant<int, 1>{});
      else fill(std::integral_constant<int, 0>{});
    } else {
      int32_t* rr = reinterpret_cast<int32_t*>(lds + L.rr);
      const int16_t* ri = reinterpret_cast<const int16_t*>(lds + L.ri);
      const bool vec8 = a.dsub == 8 && (a.d & 7) == 0;  // 16-byte aligned subspace rows
      for (int e = tid; e < np_u * M; e += kThreads) {
        const int g = e / M, m = e % M;
        int32_t sacc = 0;
        if (vec8 && !ip) {
          // |ri|^2 of the subspace from one 16-byte read
          const u32x4 w = *reinterpret_cast<const u32x4*>(ri + g * ri_stride(a.d) + m * 8);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int lo16 = (int)(int16_t)(w[t] & 0xFFFFu), hi16 = (int)(int16_t)(w[t] >> 16);
            sacc += lo16 * lo16 + hi16 * hi16;
          }
        } else {
          for (int t = 0; t < a.dsub; ++t) {
            const int v = ri[g * ri_stride(a.d) + m * a.dsub + t];
            // L2: |ri|^2 of the subspace; IP: qi.ci of the subspace (base term)
            sacc += ip ? v * grid_val(a.C[(size_t)p * a.d + m * a.dsub + t], a.grid_e, a.grid_kind) : v * v;
          }
        }
        rr[e] = sacc;
      }
      __syncthreads();
      // the 16 B fragments of an m-pair are issued together, then consumed
      auto build = [&](auto pass_tag, auto ip_tag) {
        constexpr int PASS = decltype(pass_tag)::value;
        constexpr bool IPM = decltype(ip_tag)::value;
        for (int mp = wave; mp < M / 2; mp += kThreads / 64) {
          u32x4 Bt[16], Bd[16];
#pragma unroll
          for (int jt = 0; jt < 16; ++jt) {
            const size_t fi = ((size_t)mp * 16 + jt) * 64 + lane;
            Bt[jt] = a.bsw[fi];
            if constexpr (DT == DT_F16) Bd[jt] = a.bsw16[fi];
            else Bd[jt] = (u32x4){0u, 0u, 0u, 0u};
          }
          lut_mpair<LWB, WPR, DT, PASS, IPM>(a, lds, L, M, np_u, mp, Bt, Bd);
        }
      };
      using P1 = std::integral_constant<int, 1>;
      using P2 = std::integral_constant<int, 2>;
      using IPt = std::integral_constant<bool, true>;
      using L2t = std::integral_constant<bool, false>;
      // L1: T[m][j] = sum_t |ri_t - cbi_t| on the VALU (not a product, no
      // MFMA), exact integers.  Pass 1: a thread per (pair, subspace) row
      // finds its min / max over the 256 codewords; pass 2: a thread per
      // (subspace, codeword) entry quantises it for every pair of the unit
      // and packs the row words as the MFMA build does.
      auto build_l1 = [&](int pass) {
        int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
        int32_t* hi = reinterpret_cast<int32_t*>(lds + L.hi);
        if (pass == 1) {
          for (int e = tid; e < np_u * M; e += kThreads) {
            const int g = e / M, m = e % M;
            int rv[kMaxDsub];
#pragma unroll
            for (int t = 0; t < kMaxDsub; ++t) rv[t] = t < a.dsub ? (int)ri[g * ri_stride(a.d) + m * a.dsub + t] : 0;
            int mn = 0x7FFFFFFF, mx = 0;
            const int16_t* cb = a.cbi16 + (size_t)m * kKsub * 8;
            for (int j = 0; j < kKsub; ++j) {
              int v = 0;
#pragma unroll
              for (int t = 0; t < kMaxDsub; ++t) v += abs(rv[t] - (int)cb[j * 8 + t]);
              mn = v < mn ? v : mn;
              mx = v > mx ? v : mx;
            }
            lo[e] = mn;
            hi[e] = mx;
          }
        } else {
          uint32_t* lut = reinterpret_cast<uint32_t*>(lds + L.lut);
          for (int e = tid; e < M * kKsub; e += kThreads) {
            const int m = e / kKsub, j = e % kKsub;
            int cv[kMaxDsub];
#pragma unroll
            for (int t = 0; t < kMaxDsub; ++t) cv[t] = a.cbi16[((size_t)m * kKsub + j) * 8 + t];
            uint32_t wds[WPR];
#pragma unroll
            for (int w = 0; w < WPR; ++w) wds[w] = 0;
#pragma unroll
            for (int w = 0; w < WPR; ++w)
#pragma unroll
              for (int f = 0; f < W; ++f) {
                const int g = PairSlot<LWB, WPR>::pair(w, f);
                if (g < np_u) {
                  int v = 0;
#pragma unroll
                  for (int t = 0; t < kMaxDsub; ++t)
                    if (t < a.dsub) v += abs((int)ri[g * ri_stride(a.d) + m * a.dsub + t] - cv[t]);
                  const uint32_t qv = (uint32_t)((v + lo[g * M + m]) >> ps[g]);  // lo: hf(s) - min here
                  wds[w] |= LWB == 32 ? qv : (qv << (f * LWB));
                }
              }
            uint32_t* dst = lut + (size_t)(m * kKsub + j) * WPR;
#pragma unroll
            for (int w = 0; w < WPR; ++w) dst[w] = wds[w];
          }
        }
      };
      if (l1) build_l1(1);
      else if (ip) build(P1{}, IPt{});
      else build(P1{}, L2t{});
      if (tid == 0) *reinterpret_cast<int*>(lds + L.ctl + 12) = 0;  // live-pair count of the unit
      __syncthreads();
      {
        // per pair g: shift s, base = sum of the subspace minima (inner
        // product: minus qi.ci); sixteen threads (a 16-lane row) per pair
        const int32_t* lo = reinterpret_cast<const int32_t*>(lds + L.lo);
        const int32_t* hi = reinterpret_cast<const int32_t*>(lds + L.hi);
        const int32_t* rrp = reinterpret_cast<const int32_t*>(lds + L.rr);
        const int g = tid >> 4, r = tid & 15;
        int32_t span = 0;
        int64_t bsum = 0;
        if (g < np_u)
          for (int m = r; m < M; m += 16) {
            const int32_t l = lo[g * M + m], h = hi[g * M + m];
            span = h - l > span ? h - l : span;
            bsum += l - (ip ? rrp[g * M + m] : 0);
          }
        span = row16_reduce<true>(span);
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) bsum += __shfl_xor(bsum, off, 16);
        if (r == 15 && g < G) {
          if (g < np_u) {
            const int64_t top = (1ll << pb[g]) - 1, R = span;
            int sh = 0;
            while (((R + (sh ? (1ll << (sh - 1)) : 0)) >> sh) > top) ++sh;
            ps[g] = sh;
            pbase[g] = bsum;
          }
          // phases 2, 3: the bases are known before pass 2, the pair's
          // threshold too (same lane, no barrier); live pairs are counted
          if (PHASE >= 2 && pair_threshold(g))
            atomicAdd(reinterpret_cast<int*>(lds + L.ctl + 12), 1);
        }
      }
      __syncthreads();
      if constexpr (PHASE >= 2) {
        // a unit whose pairs are all dead skips pass 2 and the scan (the
        // count goes through a control word, zeroed before pass 1 ended)
        const int nlive = *reinterpret_cast<int*>(lds + L.ctl + 12);
        if (PHASE == 2 && tid == 0 && a.work) {
          // work counters (code bytes of the pairs scanned, live and skipped
          // pairs): kept by the workgroup, added to the totals at its end
          uint64_t* wc = reinterpret_cast<uint64_t*>(lds + L.ctl + 32);
          wc[0] += (uint64_t)(nlive * (v1 - v0) * M);
          wc[1] += (uint64_t)nlive;
          wc[2] += (uint64_t)(np_u - nlive);
        }
        if (!nlive) {
          fetch_next();
          return;
        }
      }
      {
        // lo -> the offset hf(s) - lo that pass 2 adds before the shift
        int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
        for (int e = tid; e < np_u * M; e += kThreads) {
          const int g = e / M, sh = ps[g];
          lo[e] = (sh ? (1 << (sh - 1)) : 0) - lo[e];
        }
      }
      __syncthreads();
      if (l1) build_l1(2);
      else if (ip) build(P2{}, IPt{});
      else build(P2{}, L2t{});
      __syncthreads();
    }
    if constexpr (FP) {  // (integer LUTs: right after the shifts, before pass 2)
      if constexpr (PHASE >= 2) {
        // lower bound of each pair's FP32 sums: its row minima summed in the
        // scan's subspace order (FP32 addition is monotone, so no vector's
        // in-order sum is below it); sixteen threads per subspace, WPR pairs
        // per 16-byte LUT row
        __syncthreads();  // the LUT entries are written
        const float* lutf = reinterpret_cast<const float*>(lds + L.lut);
        float* rmin = reinterpret_cast<float*>(lds + L.lo);  // [G][M]
        for (int m0 = 0; m0 < M; m0 += kThreads / 16) {
          const int m = m0 + (tid >> 4), jb = (tid & 15) * 16;
          float mn[WPR];
#pragma unroll
          for (int g = 0; g < WPR; ++g) mn[g] = __builtin_inff();
          if (m < M)
            for (int j = jb; j < jb + 16; ++j) {
#pragma unroll
              for (int g = 0; g < WPR; ++g) mn[g] = fminf(mn[g], lutf[(m * kKsub + j) * WPR + g]);
            }
#pragma unroll
          for (int g = 0; g < WPR; ++g) {
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) mn[g] = fminf(mn[g], __shfl_xor(mn[g], o, 16));
            if (m < M && (tid & 15) == 0 && g < np_u) rmin[g * M + m] = mn[g];
          }
        }
        __syncthreads();
        if (tid < np_u) {
          float sb = 0.f;
          for (int m = 0; m < M; ++m) sb += rmin[tid * M + m];
          reinterpret_cast<float*>(lds + L.pbase)[tid] = sb;
        }
        __syncthreads();
        thresholds();
        int& s_live = *reinterpret_cast<int*>(lds + L.ctl + 12);
        if (tid == 0) s_live = 0;
        __syncthreads();
        if (tid < np_u && pb[tid] >= 0) atomicAdd(&s_live, 1);
        __syncthreads();
        const int nlive = s_live;
        if (PHASE == 2 && tid == 0 && a.work) {
          uint64_t* wc = reinterpret_cast<uint64_t*>(lds + L.ctl + 32);
          wc[0] += (uint64_t)(nlive * (v1 - v0) * M);
          wc[1] += (uint64_t)nlive;
          wc[2] += (uint64_t)(np_u - nlive);
        }
        if (!nlive) {
          fetch_next();
          return;
        }
      } else {
        __syncthreads();  // the LUT entries are written
      }
    }
    // ---- DC scan: one vector per thread, codes of the next vector prefetched
    uint32_t sig[G];
    bool live[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      sig[g] = psig[g];
      live[g] = PHASE >= 2 ? pb[g] >= 0 : g < np_u;
    }
    uint32_t lmin[G];
#pragma unroll
    for (int g = 0; g < G; ++g) lmin[g] = 0xFFFFFFFFu;
    // packed thresholds of the 8-bit lane class: fields 0,2 and 1,3 of each
    // word in 16-bit halves with guard bit 8; dead pairs never hit
    uint32_t sig_e[WPR], sig_o[WPR], msk_e[WPR], msk_o[WPR];
    if constexpr (PHASE >= 2 && LWB == 8) {
#pragma unroll
      for (int w = 0; w < WPR; ++w) {
        uint32_t se = 0, so = 0, me = 0, mo = 0;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int g = PairSlot<LWB, WPR>::pair(w, f);
          const uint32_t sg = live[g] ? (sig[g] > 255u ? 255u : sig[g]) : 255u;
          const uint32_t gb = live[g] ? 0x100u : 0u;
          if (f & 1) { so |= (sg | 0x100u) << (16 * (f >> 1)); mo |= gb << (16 * (f >> 1)); }
          else { se |= (sg | 0x100u) << (16 * (f >> 1)); me |= gb << (16 * (f >> 1)); }
        }
        sig_e[w] = se; sig_o[w] = so; msk_e[w] = me; msk_o[w] = mo;
      }
    }
    lds_u32* lut = reinterpret_cast<lds_u32*>((uintptr_t)L.lut);  // LDS address (see lds_u32)
    constexpr int MQ = MT ? MT / 4 : 1;  // code dwords per vector held in registers
    // vectors per thread and step: one-word rows (a few pairs per list, the
    // streaming case) make a vector cheap to scan, so four are kept in flight
    // to cover HBM latency; wide rows are compute-bound at one
    constexpr int PV = (NR && MT != 0) ? 4 : 1;
    uint32_t cw_next[PV][MQ];
    if constexpr (MT != 0) {
#pragma unroll
      for (int pv = 0; pv < PV; ++pv) {
        const int64_t v = v0 + tid + pv * kThreads;
        if (v < v1) {
          const uint32_t* cp = reinterpret_cast<const uint32_t*>(a.codes + (size_t)(L0 + v) * MT);
#pragma unroll
          for (int i = 0; i < MQ; ++i) cw_next[pv][i] = cp[i];
        }
      }
    }
    fetch_next();  // the next unit's descriptor, read while this one scans
    for (int64_t vb = v0; vb < v1; vb += kThreads * PV) {
      uint32_t cwg[PV][MQ];
#pragma unroll
      for (int pv = 0; pv < PV; ++pv)
#pragma unroll
        for (int i = 0; i < MQ; ++i) cwg[pv][i] = cw_next[pv][i];
      if constexpr (MT != 0) {
#pragma unroll
        for (int pv = 0; pv < PV; ++pv) {
          const int64_t vn = vb + tid + (PV + pv) * kThreads;
          if (vn < v1) {
            const uint32_t* cp = reinterpret_cast<const uint32_t*>(a.codes + (size_t)(L0 + vn) * MT);
#pragma unroll
            for (int i = 0; i < MQ; ++i) cw_next[pv][i] = cp[i];
          }
        }
      }
#pragma unroll
      for (int pv = 0; pv < PV; ++pv) {
      const int64_t v = vb + tid + pv * kThreads;
      uint32_t cw[MQ];
#pragma unroll
      for (int i = 0; i < MQ; ++i) cw[i] = cwg[pv][i];
      if (v < v1) {
        uint32_t acc[WPR];
        float accf[WPR];
#pragma unroll
        for (int w = 0; w < WPR; ++w) { acc[w] = 0; accf[w] = 0.f; }
        const uint32_t* cpg = reinterpret_cast<const uint32_t*>(a.codes + (size_t)(L0 + v) * M);
        for (int m4 = 0; m4 < M; m4 += 4) {
          uint32_t c4;
          if constexpr (MT != 0) c4 = cw[m4 >> 2];
          else c4 = cpg[m4 >> 2];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int rowi = ((m4 + i) * kKsub + ((c4 >> (8 * i)) & 255u)) * WPR;
            uint32_t x[WPR];
            lut_row_load<WPR>(lut, rowi, x);
#pragma unroll
            for (int w = 0; w < WPR; ++w) {
              if constexpr (FP) accf[w] += __uint_as_float(x[w]);
              else acc[w] += x[w];
            }
          }
        }
        auto emit = [&](int g, uint32_t S) {
          const int q = pq[g];
          uint64_t key;
          if constexpr (FP) key = (uint64_t)S;
          else key = ikey(pbase[g] + ((int64_t)S << ps[g]));
          const int64_t id = a.ids[L0 + v];
          // re-run: the bound is a (distance, id) key, ties past its id go
          if (PHASE == 3 && key == a.tau[q] && id > a.tau_id[q]) return;
          const uint32_t pos = atomicAdd(&a.ccount[q], 1u);
          if (pos < a.capq) {
            a.ckey[(size_t)q * a.capq + pos] = key;
            a.cid[(size_t)q * a.capq + pos] = id;
          }
        };
        if constexpr (PHASE >= 2 && LWB == 8) {
          // four 8-bit sums per word: test all four against their thresholds
          // at once in two 16-bit-lane halves (guard bit 8 survives iff S <= sigma)
#pragma unroll
          for (int w = 0; w < WPR; ++w) {
            const uint32_t e = acc[w] & 0x00FF00FFu, o = (acc[w] >> 8) & 0x00FF00FFu;
            const uint32_t hit = ((sig_e[w] - e) & msk_e[w]) | ((sig_o[w] - o) & msk_o[w]);
            if (hit) {
#pragma unroll
              for (int f = 0; f < 4; ++f) {
                // rare path: thresholds from LDS, not held in registers
                const uint32_t S = (acc[w] >> (8 * f)) & 0xFFu;
                const int g = PairSlot<LWB, WPR>::pair(w, f);
                if (pb[g] >= 0 && S <= psig[g]) emit(g, S);
              }
            }
          }
        } else {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int w = PairSlot<LWB, WPR>::word(g), f = PairSlot<LWB, WPR>::field(g);
            uint32_t S;
            if constexpr (FP) S = fkey(accf[w]);
            else S = LWB == 32 ? acc[w] : ((acc[w] >> (f * LWB)) & MASK);
            if (PHASE == 1) {
              lmin[g] = S < lmin[g] ? S : lmin[g];
            } else if (live[g] && S <= sig[g]) {
              emit(g, S);
            }
          }
        }
      }
      }  // vectors of the step
    }
    if (PHASE == 1 && a.kmax <= 64) {
      // the k-th smallest of a wave's per-lane minima bounds the pair's k-th
      // smallest (each minimum is a distinct vector): the wave's k smallest
      // minima go to the query's bound buffer, and the bound is taken over
      // all of them.  The k-th smallest minimum x is found bit by bit (the
      // largest x with fewer than k minima below it; counts are ballot bit
      // counts, no cross-lane shuffles); the minima below x and the
      // lowest-lane ones equal to x make up the k.
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g >= np_u) break;
        const uint32_t v = lmin[g];
        const int q = pq[g];
        const int kk = a.kq ? a.kq[q] : a.kconst;
        uint32_t x = 0;
        for (int bit = 31; bit >= 0; --bit) {
          const uint32_t t = x | (1u << bit);
          if (__popcll(__ballot(v < t)) < kk) x = t;
        }
        const uint64_t below = __ballot(v < x), eqm = __ballot(v == x);
        const int need = kk - __popcll(below);
        const uint64_t lower_lanes = (1ull << lane) - 1;
        // (lanes that scanned no vector hold the largest key: never sent)
        const bool e = (v < x || (v == x && __popcll(eqm & lower_lanes) < need)) && v != 0xFFFFFFFFu;
        // the candidate buffer serves as the bound buffer (emptied again
        // before phase 2); entries beyond its capacity are dropped, which
        // only loosens the bound
        const uint64_t bal = __ballot(e);
        uint32_t base = 0;
        if (lane == 0 && bal) base = atomicAdd(&a.ccount[q], (uint32_t)__popcll(bal));
        base = (uint32_t)__shfl((int)base, 0);
        const uint32_t pos = base + (uint32_t)__popcll(bal & lower_lanes);
        if (e && pos < a.capq) {
          uint64_t key;
          if constexpr (FP) key = (uint64_t)v;
          else key = ikey(pbase[g] + ((int64_t)v << ps[g]));
          a.ckey[(size_t)q * a.capq + pos] = key;
        }
      }
    } else if (PHASE == 1) {
      // k > 64: the k-th smallest of the workgroup's per-thread minima
      // (bitonic sort over a power-of-two row, padded with the largest key)
      constexpr int TP = kThreadsP2;
      __syncthreads();  // the LUT space is reused below
      uint32_t* lm = reinterpret_cast<uint32_t*>(lds + L.lmin);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        lm[g * TP + tid] = lmin[g];
        if (tid + kThreads < TP) lm[g * TP + kThreads + tid] = 0xFFFFFFFFu;
      }
      __syncthreads();
      for (int size = 2; size <= TP; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          for (int i = tid; i < G * (TP / 2); i += kThreads) {
            const int g = i / (TP / 2), ii = i % (TP / 2);
            const int pos = 2 * ii - (ii & (stride - 1));
            const bool asc = (pos & size) == 0;
            uint32_t* arr = lm + g * TP;
            const uint32_t x0 = arr[pos], x1 = arr[pos + stride];
            if ((x0 > x1) == asc) { arr[pos] = x1; arr[pos + stride] = x0; }
          }
          __syncthreads();
        }
      // the k smallest of each pair's minima to its query's bound buffer
      for (int i = tid; i < np_u * TP; i += kThreads) {
        const int g = i / TP, r = i % TP;
        const int q = pq[g];
        const int kk = a.kq ? a.kq[q] : a.kconst;
        const uint32_t val = lm[g * TP + r];
        if (r < kk && val != 0xFFFFFFFFu) {
          const uint32_t pos = atomicAdd(&a.ccount[q], 1u);
          if (pos < a.capq) {
            uint64_t key;
            if constexpr (FP) key = (uint64_t)val;
            else key = ikey(pbase[g] + ((int64_t)val << ps[g]));
            a.ckey[(size_t)q * a.capq + pos] = key;
          }
        }
      }
    }
}

// persistent scan of one lane class: workgroups claim units of their class
// from a device counter; the next unit is claimed while the current one is
// processed (index at the start, descriptor before the scan, published at
// the end)
template <int LWB, int MT, int PHASE, int DT, int NR>
__global__ __launch_bounds__(kThreads, 2) void k_scan(ScanArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int WPR = variant_wpr(MT, NR);
  constexpr bool FP = LWB == 0;
  constexpr int G = WPR * Lane<LWB>::W;
  constexpr bool CRES = FP && MT != 0 && MT <= 16;
  const int M = MT ? MT : a.M;
  const ScanLds L = scan_lds_layout(G, WPR, M, a.d, FP, PHASE);
  if (__builtin_amdgcn_groupstaticsize() != 0) {  // the LUT must start at LDS address 0
    if (threadIdx.x == 0) atomicOr(&a.flags[0], 16);
    return;
  }
  if (PHASE == 3 && *a.any_retry == 0) return;  // re-run of phase 2 with nothing to do
  int& s_u = *reinterpret_cast<int*>(lds + L.ctl);
  int4& s_unit = *reinterpret_cast<int4*>(lds + L.ctl + 16);
  const int tid = threadIdx.x;
  const int64_t ub = a.unitoff[(size_t)a.cls * a.nlist];
  const int64_t ue = a.unitoff[(size_t)(a.cls + 1) * a.nlist];
  const int own_j = tid % kKsub, own_m0 = tid / kKsub;
  const bool owner = tid < kMPar * kKsub;
  Owned<WPR, CRES ? MT : 0> own;
  if constexpr (CRES) {
#pragma unroll
    for (int i = 0; i < MT / kMPar; ++i)
#pragma unroll
      for (int t = 0; t < kMaxDsub; ++t)
        own.c[i][t] = owner && t < a.dsub
                          ? a.codebook[((size_t)(kMPar * i + own_m0) * kKsub + own_j) * a.dsub + t] : 0.f;
  }
  UnitQueue uq(a.counter, ue - ub, a.steal);
  if (tid == 0) {
    const int64_t uu = uq.next();
    s_u = (int)uu;
    if (ub + uu < ue) s_unit = a.units[ub + uu];
  }
  if (tid == 0)
    for (int i = 0; i < 3; ++i) reinterpret_cast<uint64_t*>(lds + L.ctl + 32)[i] = 0;
  __syncthreads();
  for (;;) {
    if (ub + s_u >= ue) break;
    int next_u = 0;
    int4 next_unit = make_int4(0, 0, 0, 0);
    if (tid == 0) next_u = (int)uq.next();
    scan_unit<LWB, MT, PHASE, DT, NR>(a, lds, L, own, s_unit, [&] {
      if (tid == 0 && ub + next_u < ue) next_unit = a.units[ub + next_u];
    });
    __syncthreads();
    if (tid == 0) {
      s_u = next_u;
      s_unit = next_unit;
    }
    __syncthreads();
  }
  if (PHASE == 2 && tid == 0 && a.work)
    for (int i = 0; i < 3; ++i)
      atomicAdd((unsigned long long*)&a.work[i],
                (unsigned long long)reinterpret_cast<const uint64_t*>(lds + L.ctl + 32)[i]);
}

// all three lane classes of an integer policy in one persistent launch, in
// the order 32-bit, 16-bit, 8-bit units (each largest list first): the few
// wide units start early and the many 8-bit units fill the tail.  The LDS
// tile of the 8-bit class (the most pairs per unit) serves every class.
template <int MT, int PHASE, int DT, int NR>
__global__ __launch_bounds__(kThreads, 2) void k_scan_mix(ScanArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int WPR = variant_wpr(MT, NR);
  const int M = MT ? MT : a.M;
  const ScanLds L = scan_lds_layout(WPR * Lane<8>::W, WPR, M, a.d, false, PHASE);
  if (__builtin_amdgcn_groupstaticsize() != 0) {  // the LUT must start at LDS address 0
    if (threadIdx.x == 0) atomicOr(&a.flags[0], 16);
    return;
  }
  if (PHASE == 3 && *a.any_retry == 0) return;  // re-run of phase 2 with nothing to do
  int& s_u = *reinterpret_cast<int*>(lds + L.ctl);
  int& s_cls = *reinterpret_cast<int*>(lds + L.ctl + 4);
  int4& s_unit = *reinterpret_cast<int4*>(lds + L.ctl + 16);
  const int tid = threadIdx.x;
  const int64_t* uo = a.unitoff;
  const int64_t n2 = uo[3 * (size_t)a.nlist] - uo[2 * (size_t)a.nlist];
  const int64_t n1 = uo[2 * (size_t)a.nlist] - uo[a.nlist];
  const int64_t total = uo[3 * (size_t)a.nlist] - uo[0];
  // unit number in launch order -> (class, row of the class-major unit table)
  auto locate = [&](int64_t u, int& cls) -> int64_t {
    if (u < n2) { cls = 2; return uo[2 * (size_t)a.nlist] + u; }
    if (u < n2 + n1) { cls = 1; return uo[a.nlist] + (u - n2); }
    cls = 0;
    return uo[0] + (u - n2 - n1);
  };
  Owned<WPR, 0> own;
  UnitQueue uq(a.counter, total, a.steal);
  if (tid == 0) {
    const int uu = (int)uq.next();
    s_u = uu;
    if (uu < total) {
      int c;
      s_unit = a.units[locate(uu, c)];
      s_cls = c;
    }
  }
  if (tid == 0)
    for (int i = 0; i < 3; ++i) reinterpret_cast<uint64_t*>(lds + L.ctl + 32)[i] = 0;
  __syncthreads();
  for (;;) {
    if (s_u >= total) break;
    int next_u = 0, next_cls = 0;
    int4 next_unit = make_int4(0, 0, 0, 0);
    if (tid == 0) next_u = (int)uq.next();
    auto fetch = [&] {
      if (tid == 0 && next_u < total) next_unit = a.units[locate(next_u, next_cls)];
    };
    const int cls = s_cls;
    if (cls == 0) scan_unit<8, MT, PHASE, DT, NR>(a, lds, L, own, s_unit, fetch);
    else if (cls == 1) scan_unit<16, MT, PHASE, DT, NR>(a, lds, L, own, s_unit, fetch);
    else scan_unit<32, MT, PHASE, DT, NR>(a, lds, L, own, s_unit, fetch);
    __syncthreads();
    if (tid == 0) {
      s_u = next_u;
      s_unit = next_unit;
      s_cls = next_cls;
    }
    __syncthreads();
  }
  if (PHASE == 2 && tid == 0 && a.work)
    for (int i = 0; i < 3; ++i)
      atomicAdd((unsigned long long*)&a.work[i],
                (unsigned long long)reinterpret_cast<const uint64_t*>(lds + L.ctl + 32)[i]);
}

// ------------------------------------------------------------------ bound
// tau[q] = the k-th smallest key of the query's phase-1 bound buffer (every
// entry is the estimate of a distinct vector, so it bounds the query's k-th
// smallest estimate from above), or no bound with fewer than k entries; the
// buffer is emptied for phase 2.  Queries with at most 64 entries: one wave
// each (register bitonic sort); the rest: k_tau, a workgroup each.
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
  int* s_n = reinterpret_cast<int*>(lds + capq * 8);
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
      int np2 = 1;
      while (np2 < n) np2 <<= 1;
      for (int i = threadIdx.x; i < np2; i += blockDim.x) keys[i] = i < n ? ckey[(size_t)qq * capq + i] : ~0ull;
      __syncthreads();
      block_bitonic_u64(keys, np2);
      const int kk = kq ? kq[qq] : kconst;
      if (threadIdx.x == 0) {
        tau[qq] = n >= kk ? keys[kk - 1] : ~0ull;
        ccount[qq] = 0;
      }
      __syncthreads();  // the LDS is reused by the next query
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

// queries with more than 64 candidates: a workgroup per query (strided over
// the queries), bitonic sort in LDS
__global__ __launch_bounds__(256) void k_merge(MergeArgs a, int nq) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
  int64_t* vals = reinterpret_cast<int64_t*>(lds + a.capq * 8);
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint32_t cnt = a.ccount[q];
    if (cnt > a.capq && threadIdx.x == 0) atomicOr(&a.flags[0], 2);
    const int n = (int)(cnt < a.capq ? cnt : a.capq);
    if (n <= 64) continue;  // uniform over the workgroup
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
                           u32x4* __restrict__ bsw, u32x4* __restrict__ bsw16) {
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
  uint32_t h[4] = {0, 0, 0, 0};
  if ((kg & 1) == 0) {
    for (int t = 0; t < 8; ++t) v[t] = (float)ci[t];
    for (int t = 0; t < 4; ++t) h[t] = f16_bits(v[2 * t]) | (f16_bits(v[2 * t + 1]) << 16);
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
  hipLaunchKernelGGL(k_prep_bsw, dim3((total + 255) / 256), dim3(256), 0, st, dv.codebook, ix->M, ix->dsub,
                     ix->grid_e, ix->grid_kind, reinterpret_cast<u32x4*>(dv.bsw),
                     reinterpret_cast<u32x4*>(dv.bsw16));
  return hipGetLastError();
}

// LC matrix dtype of an AMP_LUT_* value (0 selects BF16; the FP8 value is
// rejected before a search launches)
static int dt_of(int lut_dtype) {
  return lut_dtype == AMP_LUT_F16 ? DT_F16 : DT_BF16;
}

// subspace count of the scan variant that runs a lane class (0: generic):
// registers-resident variants exist for M = 8, 16, 24 with the BF16 LUT build
// (the FP32 LUT has no LC dtype)
// (wpr: the words per row the queue packed for; a batch too sparse to fill
// wide rows runs the generic one-word variant, see scan_wpr)
static int scan_mt(int lwb, int M, int dt) {
  if (lwb != 0 && dt != DT_BF16) return 0;
  return (M == 8 || M == 16 || M == 24) ? M : 0;
}
// one-word rows on a specialised variant
static int scan_nr(int mt, int wpr) { return (wpr == 1 && kernel_wpr(mt) != 1) ? 1 : 0; }

static size_t scan_lds_bytes(int lw_bits, int phase, int M, int d, int wpr) {
  const bool fp = lw_bits == 0;
  const int G = fp ? wpr : wpr * (32 / lw_bits);
  return (size_t)scan_lds_layout(G, wpr, M, d, fp, phase).total;
}

int scan_wpr(int M, bool fp32, int lut_dtype, bool narrow) {
  return narrow ? 1 : kernel_wpr(scan_mt(fp32 ? 0 : 8, M, dt_of(lut_dtype)));
}

typedef void (*ScanFn)(ScanArgs);
template <int LWB, int MT, int PH, int DT, int NR>
static ScanFn scan_fn() { return k_scan<LWB, MT, PH, DT, NR>; }

// kernels specialised for the subspace counts 8, 16 and 24 (codes and, for
// the FP32 LUT, codewords kept in registers) with the BF16 LUT build, with
// wide or one-word rows; any other M, and the FP16 LUT build, run the
// generic variant
static ScanFn pick_scan(int lwb, int M, int ph, int dt, int wpr) {
  const int mt = scan_mt(lwb, M, dt), nr = scan_nr(mt, wpr);
#define AMP_PH(L, MT, DTV, NRV)                                                            \
  return ph == 1 ? scan_fn<L, MT, 1, DTV, NRV>()                                           \
                 : (ph == 2 ? scan_fn<L, MT, 2, DTV, NRV>() : scan_fn<L, MT, 3, DTV, NRV>());
#define AMP_PICK_M(L, MT) \
  if (mt == MT) {         \
    if (nr) { AMP_PH(L, MT, DT_BF16, 1) } \
    AMP_PH(L, MT, DT_BF16, 0)             \
  }
#define AMP_PICK(L)                                  \
  if (lwb == L) {                                    \
    if (L != 0 && dt == DT_F16) { AMP_PH(L, 0, DT_F16, 0) } \
    AMP_PICK_M(L, 8)                                 \
    AMP_PICK_M(L, 16)                                \
    AMP_PICK_M(L, 24)                                \
    AMP_PH(L, 0, DT_BF16, 0)                         \
  }
  AMP_PICK(0)
  AMP_PICK(8)
  AMP_PICK(16)
  AMP_PICK(32)
#undef AMP_PICK
#undef AMP_PICK_M
#undef AMP_PH
  return nullptr;
}

template <int MT, int PH, int DT, int NR>
static ScanFn mix_fn() { return k_scan_mix<MT, PH, DT, NR>; }

// the mixed-class variant of the same specialisation as pick_scan's
static ScanFn pick_mix(int M, int ph, int dt, int wpr) {
  const int mt = scan_mt(8, M, dt), nr = scan_nr(mt, wpr);
#define AMP_PH(MT, DTV, NRV) \
  return ph == 1 ? mix_fn<MT, 1, DTV, NRV>() : (ph == 2 ? mix_fn<MT, 2, DTV, NRV>() : mix_fn<MT, 3, DTV, NRV>());
  if (dt == DT_F16) { AMP_PH(0, DT_F16, 0) }
#define AMP_MIX_M(MT)          \
  if (mt == MT) {              \
    if (nr) { AMP_PH(MT, DT_BF16, 1) } \
    AMP_PH(MT, DT_BF16, 0)     \
  }
  AMP_MIX_M(8)
  AMP_MIX_M(16)
  AMP_MIX_M(24)
#undef AMP_MIX_M
  AMP_PH(0, DT_BF16, 0)
#undef AMP_PH
}

static int g_num_cu = 0;

// lwb < 0: every integer lane class in one launch (k_scan_mix)
static hipError_t launch_scan(int lwb, int ph, int dt, int wpr, const ScanArgs& sa, hipStream_t st) {
  // phase 3 (the re-run) usually has nothing to do: one workgroup per CU
  const bool mix = lwb < 0;
  ScanFn fn = mix ? pick_mix(sa.M, ph, dt, wpr) : pick_scan(lwb, sa.M, ph, dt, wpr);
  // the queue packed units for `wpr` words per row: the variant must agree
  const int mt = scan_mt(mix ? 8 : lwb, sa.M, dt);
  if (!fn || variant_wpr(mt, scan_nr(mt, wpr)) != wpr) return hipErrorInvalidValue;
  const size_t lds = scan_lds_bytes(mix ? 8 : lwb, ph, sa.M, sa.d, wpr);
  hipError_t e = hipFuncSetAttribute(kaddr(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kaddr(fn), kThreads, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  if (!g_num_cu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  hipLaunchKernelGGL(fn, dim3(g_num_cu * (ph == 3 ? 1 : per_cu)), dim3(kThreads), lds, st, sa);
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
                         const ModelArgs& ma, int64_t* out_ids, float* out_dist, int64_t* out_qdist,
                         float* out_coarse, hipStream_t st, hipEvent_t* ev) {
  const DeviceIndex& dv = ix->dev;
  const bool fp32 = sd.policy == AMP_POLICY_FP32;
  const int ncls = fp32 ? 1 : kNCls;
  const int NB = ncls * sd.nlist;
  const size_t npairs = (size_t)sd.nq * sd.npmax;
  auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], st); };
  mark(0);
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
  if (sd.metric == AMP_L1) {
    hipLaunchKernelGGL(k_coarse_l1, dim3((sd.nlist + CL_T - 1) / CL_T, (sd.nq + CL_T - 1) / CL_T), dim3(256), 0,
                       st, queries, dv.centroids, coarse, sd.nq, sd.nlist, sd.d);
  } else {
    hipLaunchKernelGGL(k_sqnorm, dim3((sd.nq + 3) / 4), dim3(256), 0, st, queries, sd.nq, sd.d, ws.qnorm);
    hipLaunchKernelGGL(k_coarse, dim3((sd.nlist + CL_T - 1) / CL_T, (sd.nq + CL_T - 1) / CL_T), dim3(256), 0, st,
                       queries, dv.centroids, ws.qnorm, dv.cnorm, coarse, sd.nq, sd.nlist, sd.d, sd.metric);
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
  // resets, one launch
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
    ra.nq = (size_t)sd.nq;
    hipLaunchKernelGGL(k_reset, dim3(256), dim3(256), 0, st, ra);
  }
  // PPM
  PairArgs pa;
  pa.Q = queries;
  pa.C = dv.centroids;
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
  qa.wpr = sd.wpr;
  qa.chunk[0] = sd.chunk1;
  qa.chunk[1] = sd.chunk;
  qa.max_units = sd.max_units;
  const int qb = (int)((npairs + 255) / 256);
  hipLaunchKernelGGL(k_qhist, dim3(qb), dim3(256), 0, st, qa);
  hipLaunchKernelGGL(k_qtot, dim3((2 * NB + 255) / 256), dim3(256), 0, st, qa, fp32 ? 1 : 0);
  hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, st, qa, fp32 ? 1 : 0);
  hipLaunchKernelGGL(k_qscatter, dim3(qb), dim3(256), 0, st, qa);
  hipLaunchKernelGGL(k_qunits, dim3(512), dim3(256), 0, st, qa, fp32 ? 1 : 0);
  mark(4);
  // LC + DC, phase 1 then phase 2
  ScanArgs sa;
  sa.Q = queries;
  sa.C = dv.centroids;
  sa.codebook = dv.codebook;
  sa.bsw = reinterpret_cast<const u32x4*>(dv.bsw);
  sa.bsw16 = reinterpret_cast<const u32x4*>(dv.bsw16);
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
  sa.kconst = sd.kconst;
  sa.kmax = sd.kmax;
  sa.chunk = sd.chunk;  // per phase below
  sa.capq = sd.capq;
  sa.retry = nullptr;
  sa.tau_id = nullptr;
  sa.any_retry = nullptr;
  sa.work = nullptr;
  sa.steal = sd.queue;
  hipError_t err = hipSuccess;
  // the lane classes run one after another on the caller's stream, each a
  // persistent kernel over its own unit range.  (Running them concurrently
  // on separate streams was measured slower on the mid-size workload: scan
  // phase 2 took 1.86 ms against 1.50 ms serially.)
  const int dt = dt_of(sd.lut_dtype);
  for (int ph = 1; ph <= 2; ++ph) {
    sa.sorted = ws.sorted + (ph == 2 ? npairs : 0);
    sa.unitoff = ws.unitoff + (ph == 2 ? (NB + 1) : 0);
    sa.units = ws.units + (ph == 2 ? sd.max_units : 0);
    sa.chunk = ph == 2 ? sd.chunk : sd.chunk1;
    int sa_lwb;
    if (fp32 || sd.policy == AMP_POLICY_FIXED) {
      // one lane class holds every pair: its own kernel
      const int c = fp32 ? 0 : lane_class(sd.M, sd.fixed_bits);
      sa.cls = c;
      sa.counter = ws.counters + ((ph - 1) * (kNCls + 1) + c) * kQueueSlot;
      sa_lwb = fp32 ? 0 : lane_bits(c);
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
      const size_t tlds = sd.capq * 8 + 4 * (1 + 256);  // sort row + list of the queries to sort
      err = hipFuncSetAttribute(kaddr(k_tau), hipFuncAttributeMaxDynamicSharedMemorySize, (int)tlds);
      if (err != hipSuccess) return err;
      hipLaunchKernelGGL(k_tau, dim3(sd.nq < 512 ? sd.nq : 512), dim3(256), tlds, st, ws.ccount, ws.ckey, ws.tau,
                         ws.kq, sd.kconst, sd.nq, sd.capq);
    }
    mark(4 + ph);
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
      for (int rr = 0; rr < 2; ++rr) {
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
  const size_t mlds = sd.capq * 16;
  err = hipFuncSetAttribute(kaddr(k_merge), hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_merge_wave, dim3((sd.nq + 3) / 4), dim3(256), 0, st, ma2, sd.nq);
  hipLaunchKernelGGL(k_merge, dim3(sd.nq < 512 ? sd.nq : 512), dim3(256), mlds, st, ma2, sd.nq);
  mark(7);
  return hipGetLastError();
}

}  // namespace amp
