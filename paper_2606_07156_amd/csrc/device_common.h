// Device helpers shared by the kernel translation units of the search
// library (kernels.hip and the scan translation units).
#pragma once
#include "amp_internal.h"

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

// quantiser shift of a pair of width b: the smallest s with
// (R + n hf(s)) >> s <= n (2^b - 1), hf(s) = 2^(s-1) (0 for s = 0).  One
// width per pair: R the largest subspace range, n = 1; per-(pair, subspace)
// widths: R the sum of the ranges, n = M (the pair's lane budget)
__device__ __forceinline__ int quant_shift(int64_t R, int n, int b) {
  const int64_t top = (int64_t)n * ((1ll << b) - 1);
  int sh = 0;
  while (((R + (sh ? (int64_t)n << (sh - 1) : 0)) >> sh) > top) ++sh;
  return sh;
}

// byte permute: byte i of the result is byte sel_i of the 8-byte value
// (hi : lo), sel_i in 0..7 (0..3: bytes of lo, 4..7: bytes of hi)
__device__ __forceinline__ uint32_t byte_perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// an inner-product query table of width index wi (width 4 (wi + 1)) is kept
// as bytes for width 4 with one width per pair (entries at most 15; the
// pairs of the 4-bit lane class are exactly these); per-subspace widths bound
// only the sum of a row, so their tables stay uint16
__host__ __device__ __forceinline__ bool ip_bytes(int gran, int wi, int M) { return gran == 0 && wi == 0 && M <= 2184; }

__device__ __forceinline__ uint32_t bf16_bits(float v) {  // exact inputs only
  return __float_as_uint(v) >> 16;
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

// LC matrix dtypes of the integer LUT build.  BF16 and FP16 sums of grid
// products are exact; the FP8 (e4m3) build puts the dimension products on
// the FP8 MFMA, whose sums of e4m3-grid products are not always exact: its
// entries are the rounded FP32 results.
enum { DT_BF16 = 1, DT_F16 = 2, DT_F8 = 3 };

// four floats as OCP e4m3 bytes (the hardware conversion; exact for the
// e4m3-representable integers of the e4m3 operand grid)
__device__ __forceinline__ uint32_t f8_bits4(float v0, float v1, float v2, float v3) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(v0, v1, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(v2, v3, w, true);
  return (uint32_t)w;
}

__device__ __forceinline__ uint32_t f16_bits(float v) {  // exact inputs only
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
}
}  // namespace amp
