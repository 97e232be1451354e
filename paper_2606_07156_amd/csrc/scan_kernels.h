// Scan kernels of the search (LC, quantisation, DC scan, unit top-k):
// templates instantiated per phase in scan_ph1.hip, scan_ph2.hip and
// scan_ph3.hip (three translation units that compile side by side).
#pragma once
#include "device_common.h"

namespace amp {

// ------------------------------------------------------------------ scan
struct ScanArgs {
  const float* Q;
  const float* C;
  const float* codebook;   // FP32 policy
  const u32x4* bsw;        // integer policy MFMA B fragments (BF16, with aug slots)
  const u32x4* bsw16;      // FP16 dims fragments
  const u32x2* bsw8;       // FP8 (e4m3) dims fragments
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
  // inner product: the query's table built once per query (integer: exact T
  // with its row minima and span; FP32 policy: FP32 dot products), and the
  // pairs' exact bases
  const int32_t* iptab;     // [nq][M][256] (FP32 policy: the FP32 dot products)
  const uint16_t* iptq;     // [nq][4][M][256] quantised tables per width (bytes where ip_bytes)
  const int32_t* ipsh;      // [nq][4] their shifts
  const int64_t* pbase_g;   // [nq][npmax]
  int32_t* tab_out;         // LUT pass 1 that also stores T (per-query table build, LUT export)
  uint16_t* ex_q;           // LUT export: quantised entries [pair][M][256]
  int nq, d, M, dsub, nlist, npmax, grid_e, grid_kind, metric, kconst, kmax, cls;
  int steal;                // unit queue: 0 one counter, 1 per-XCD ranges with stealing
  int gran;                 // quantiser granularity: 0 one width per pair, 1 per-(pair, subspace) widths
  int noskip;               // 1: no pair is skipped whole by its base (measurement of the full scan's traffic)
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
// the 4-bit class (eight pairs per word) packs half the words per row of
// the variant (at least one): as many pairs per unit as the 8-bit class
// from two words per row on, so that its tile (and the registers that hold
// per-pair thresholds) does not grow where the LUT is small
__host__ __device__ constexpr int nib_wpr(int wpr) { return wpr > 1 ? wpr / 2 : 1; }
// words per row and pairs per unit of a lane class (lwb 0: FP32 LUT; -1: the
// mixed-class kernel, whose tile takes the most pairs of any class)
__host__ __device__ constexpr int class_wpr(int lwb, int wpr) { return lwb == 4 ? nib_wpr(wpr) : wpr; }
__host__ __device__ constexpr int unit_pairs(int lwb, int wpr) {
  return lwb < 0 ? (nib_wpr(wpr) * 8 > wpr * 4 ? nib_wpr(wpr) * 8 : wpr * 4)
                 : (lwb == 0 ? wpr : class_wpr(lwb, wpr) * (32 / lwb));
}

// row stride (int16 elements) of the integer residuals in LDS: each row is
// padded by 32 bytes, so the eight rows that the LC A-operand build reads at
// once (d a multiple of 64 puts them all in one bank otherwise) fall in
// distinct banks, as do the two subspaces of an m-pair
__host__ __device__ constexpr int ri_stride(int d) { return d + 16; }

// LDS carve-up of one scan workgroup (all offsets in bytes, 16-aligned)
struct ScanLds {
  int lut, ri, rr, lo, hi, pq, pb, ps, pbase, psig, pid, ctl, total;
};
__host__ __device__ inline ScanLds scan_lds_layout(int G, int wpr, int M, int d, bool fp32, int phase, int nt) {
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
  L.pid = take(G * 4);
  // unit-claim control words: kept in the dynamic LDS too, so that the LUT
  // starts at LDS address 0 and row addresses fold into instruction offsets
  L.ctl = take(64);  // unit index, class, re-run vote, live vote, unit descriptor, 4 work counters
  L.total = o;
  return L;
}

template <int LWB>  // lane bits 4/8/16/32, 0 = FP32 LUT
struct Lane {
  static constexpr int W = LWB ? 32 / LWB : 1;
  static constexpr uint32_t MASK = LWB == 32 || LWB == 0 ? 0xFFFFFFFFu : ((1u << LWB) - 1);
};

// where pair g of a work unit sits in a LUT row: word and field.  The 8-bit
// class with four words per row interleaves the pairs (word 2 h + t holds
// pairs 8 t + 4 h + 0..3) so that a lane of the LUT build writes its two
// words with one 8-byte store.  The 4-bit class keeps pairs 8 w + 0..3 in
// the low nibbles of word w's bytes and pairs 8 w + 4..7 in the high ones
// (field 2 i: pair 8 w + i, field 2 i + 1: pair 8 w + 4 + i), so that one
// mask and one shift split a word into two words of 8-bit lanes, each in
// pair order.  Every other layout is word g / W, field g % W.
template <int LWB, int WPR>
struct PairSlot {
  static constexpr bool IL = LWB == 8 && WPR == 4;
  static constexpr bool NB = LWB == 4;
  static constexpr int W = Lane<LWB>::W;
  __host__ __device__ static constexpr int word(int g) { return IL ? (((g >> 2) & 1) << 1) | (g >> 3) : g / W; }
  __host__ __device__ static constexpr int field(int g) {
    return IL ? (g & 3) : (NB ? (((g & 3) << 1) | ((g >> 2) & 1)) : g % W);
  }
  __host__ __device__ static constexpr int pair(int w, int f) {
    return IL ? ((w & 1) << 3) | ((w >> 1) << 2) | f : (NB ? w * 8 + ((f & 1) << 2) + (f >> 1) : w * W + f);
  }
};

// where the scan holds pair g's sum (phases 2, 3 test four or eight sums at
// once): the test word (8-bit class: fields 0, 2 / 1, 3 of a LUT word's
// lanes; 4-bit class: the four words of widened sums, pairs 0, 2 / 1, 3 of
// the low nibbles, then 4, 6 / 5, 7 of the high ones) and its 16-bit half
template <int LWB, int WPR>
__host__ __device__ constexpr int test_word(int g) {
  return LWB == 4 ? ((((g & 7) >> 2) << 1) | (g & 1)) : (PairSlot<LWB, WPR>::field(g) & 1);
}
template <int LWB, int WPR>
__host__ __device__ constexpr int test_half(int g) {
  return LWB == 4 ? ((g & 3) >> 1) : (PairSlot<LWB, WPR>::field(g) >> 1);
}

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

// A operand of one 8-pair tile gt of an m-pair: rows (subspace slot ms,
// pair g) = ms*8 + g; K holds [dims m0 | aug m0 | dims m1 | aug m1], 8 slots
// each (see lut_mpair).  Pairs at or beyond np_u get zero rows.
template <int DT, int PASS, bool IP>
__device__ __forceinline__ void mpair_a_tile(const ScanArgs& a, const char* lds, const ScanLds& L, int M, int np_u,
                                             int mp, int gt, bf16x8& A, u32x4& Ad) {
  constexpr int pass = PASS;
  constexpr bool ip = IP;
  const int lane = threadIdx.x & 63;
  const int16_t* ri = reinterpret_cast<const int16_t*>(lds + L.ri);
  const int32_t* rr = reinterpret_cast<const int32_t*>(lds + L.rr);
  const int32_t* lo = reinterpret_cast<const int32_t*>(lds + L.lo);
  const int32_t* ps = reinterpret_cast<const int32_t*>(lds + L.ps);
  const int row = lane & 15, kg = lane >> 4;
  const int ms_row = row >> 3;
  const int dsub = a.dsub;
  const int rs = ri_stride(a.d);
  const int g = gt * 8 + (row & 7);
  const int m = 2 * mp + ms_row;
  uint32_t pk[4] = {0, 0, 0, 0}, pd[4] = {0, 0, 0, 0};
  constexpr bool Q2 = PASS == 2 || PASS == 5;  // the quantising passes (5: the LUT export)
  if (g < np_u && (kg >> 1) == ms_row) {
    const int s = !Q2 ? 0 : ps[g];
    const float sc = DT == DT_BF16 ? ldexpf(1.f, -s) : 1.f;
    if ((kg & 1) == 0) {
      // (FP8: -ri, exact in e4m3; the L2 factor 2 is applied to the FP8
      // MFMA's result on the VALU)
      const int coef = (ip || DT == DT_F8) ? -1 : -2;
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
      } else if constexpr (DT == DT_F16) {
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = t < dsub ? (float)(coef * rv[t]) : 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) pd[t] = f16_bits(v[2 * t]) | (f16_bits(v[2 * t + 1]) << 16);
      } else {
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = t < dsub ? (float)(coef * rv[t]) : 0.f;
        pd[0] = f8_bits4(v[0], v[1], v[2], v[3]);
        pd[1] = f8_bits4(v[4], v[5], v[6], v[7]);
      }
    } else {
      int32_t X = ip ? 0 : rr[g * M + m];
      // lo holds off = hf(s) - min after pass 1 (folded in, except for the
      // FP8 build: its entries are offset and shifted after rounding)
      if (Q2 && DT != DT_F8) X += lo[g * M + m];
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
  A = __builtin_bit_cast(bf16x8, u);
  Ad = (u32x4){pd[0], pd[1], pd[2], pd[3]};
}

// one 16x16 tile of T (+ the aug terms): BF16 MFMA of everything (BF16
// build) or of the aug terms, then the dims on the FP16 MFMA or, FP8 build,
// on the FP8 MFMA (-ri.cbi, doubled for L2)
template <int DT, bool IP>
__device__ __forceinline__ f4 mpair_mfma(const bf16x8& A, const u32x4& Ad, const u32x4& B, const u32x4& Bd) {
  f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, B), (f4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  if constexpr (DT == DT_F16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, Ad), __builtin_bit_cast(f16x8, Bd), acc,
                                                 0, 0, 0);
  } else if constexpr (DT == DT_F8) {
    const long a8 = (long)(((uint64_t)Ad[1] << 32) | Ad[0]);
    const long b8 = (long)(((uint64_t)Bd[1] << 32) | Bd[0]);
    // the dot products into an accumulator of their own, added on the VALU
    // (integers below 2^24: exact), so that this MFMA never takes the BF16
    // MFMA's result as its C operand
    const f4 p = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a8, b8, (f4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += (IP ? 1.f : 2.f) * p[i];
  }
  return acc;
}

// Row minima of an m-pair's exact integer LUT for np_u pairs (L2: min over
// the 256 codewords of T, written to L.lo), one 8-pair tile at a time, so
// that only one tile's accumulators are live: the B fragments (kept in
// registers) serve any number of tiles.
template <int DT>
__device__ __forceinline__ void lut_row_minima(const ScanArgs& a, char* lds, const ScanLds& L, int M, int np_u,
                                               int mp, const u32x4 (&B)[16], const u32x4 (&Bd)[16]) {
  const int lane = threadIdx.x & 63, kg = lane >> 4;
  int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
  const int m_out = 2 * mp + (kg >> 1);
  const int ntiles = (np_u + 7) >> 3;
#pragma unroll 1
  for (int gt = 0; gt < ntiles; ++gt) {
    bf16x8 A;
    u32x4 Ad;
    mpair_a_tile<DT, 1, false>(a, lds, L, M, np_u, mp, gt, A, Ad);
    int mn[4] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
#pragma unroll
    for (int jt = 0; jt < 16; ++jt) {
      const f4 acc = mpair_mfma<DT, false>(A, Ad, B[jt], Bd[jt]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // exact non-negative values: bit patterns order as integers (FP8
        // build: the rounded value)
        const int t = DT == DT_F8 ? (int)rintf(acc[i]) : __float_as_int(acc[i]);
        mn[i] = t < mn[i] ? t : mn[i];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = row16_reduce<false>(mn[i]);
      const int v = DT == DT_F8 ? r : (int)__int_as_float(r);
      const int g = gt * 8 + 4 * (kg & 1) + i;
      if ((lane & 15) == 15 && g < np_u) lo[g * M + m_out] = v;
    }
  }
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
  constexpr bool INTV = IP || DT == DT_F8;  // entries held as integers (else L2 float bit patterns)
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
  for (int gt = 0; gt < NGT; ++gt) mpair_a_tile<DT, PASS, IP>(a, lds, L, M, np_u, mp, gt, A[gt], Ad[gt]);
  // D rows of this lane: (ms = kg>>1, g = gt*8 + 4*(kg&1) + i), column j
  const int m_out = 2 * mp + (kg >> 1);
  float rsc[NGT][4];  // 2^-s of each row (used after a non-BF16 build)
#pragma unroll
  for (int gt = 0; gt < NGT; ++gt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int g = gt * 8 + 4 * (kg & 1) + i;
      rsc[gt][i] = (DT == DT_BF16 || !(PASS == 2 || PASS == 5) || g >= np_u) ? 1.f : ldexpf(1.f, -ps[g]);
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
      const f4 acc = mpair_mfma<DT, IP>(A[gt], Ad[gt], B[jt], Bdj);
      const int g0 = gt * 8 + 4 * (kg & 1);
      if constexpr (PASS == 1 || PASS == 4) {
        // exact integers: for L2 (T >= 0) the float bit patterns order as
        // integers; inner product values may be negative and are converted;
        // the FP8 build's entries are its rounded FP32 results
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t = INTV ? (DT == DT_F8 ? (int)rintf(acc[i]) : (int)acc[i]) : __float_as_int(acc[i]);
          mn[gt][i] = t < mn[gt][i] ? t : mn[gt][i];
          mx[gt][i] = t > mx[gt][i] ? t : mx[gt][i];
          if constexpr (PASS == 4) {
            // the per-query table build (and the LUT export) also keep the
            // entries; row g's destination index is in L.pq
            const int g = g0 + i;
            const int q = g < np_u ? reinterpret_cast<const int32_t*>(lds + L.pq)[g] : -1;
            if (q >= 0) a.tab_out[((size_t)q * M + m_out) * kKsub + j] = INTV ? t : (int)acc[i];
          }
        }
      } else if (g0 < G) {
        uint32_t qv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if constexpr (DT == DT_F8) {
            // offset and shift after rounding, clamped to the width (the
            // entries are the same rounded values as in pass 1)
            const int g = g0 + i;
            const int bw = reinterpret_cast<const int32_t*>(lds + L.pb)[g];
            const int top = bw > 0 ? (1 << bw) - 1 : 0;
            const int sh = g < np_u ? ps[g] : 0;
            int v = g < np_u ? ((int)rintf(acc[i]) + lo[g * M + m_out]) >> sh : 0;
            v = v < 0 ? 0 : (v > top ? top : v);
            qv[i] = (uint32_t)v;
          } else {
            const float vv = DT == DT_BF16 ? acc[i] : acc[i] * rsc[gt][i];  // power-of-two scale: exact
            qv[i] = (uint32_t)vv;  // exact and >= 0: truncation = floor
          }
        }
        if constexpr (PASS == 5) {
          // LUT export: the quantised entries to global memory, row g's
          // destination index in L.pq
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int g = g0 + i;
            const int q = g < np_u ? reinterpret_cast<const int32_t*>(lds + L.pq)[g] : -1;
            if (q >= 0) a.ex_q[((size_t)q * M + m_out) * kKsub + j] = (uint16_t)qv[i];
          }
          continue;
        }
        uint32_t* dst = lut + (size_t)(m_out * kKsub + j) * WPR;
        if constexpr (LWB == 4) {
          // pairs g0 .. g0 + 3 of word gt: low nibbles of its bytes (kg
          // even, g0 = 8 gt) or high nibbles (kg odd); the two halves meet
          // across lanes 16 apart and the even lane stores the row's words
          const uint32_t h = (qv[0] | (qv[1] << 8) | (qv[2] << 16) | (qv[3] << 24)) << (4 * (kg & 1));
          wv8[gt] = h | (uint32_t)__shfl_xor((int)h, 16);
          if (gt == NGT - 1 && (kg & 1) == 0) {
            if constexpr (WPR == 4) *reinterpret_cast<u32x4*>(dst) = (u32x4){wv8[0], wv8[1], wv8[2], wv8[3]};
            else if constexpr (WPR == 2) *reinterpret_cast<u32x2*>(dst) = (u32x2){wv8[0], wv8[1]};
            else dst[0] = wv8[0];
          }
        } else if constexpr (PairSlot<LWB, WPR>::IL) {
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
  if constexpr (PASS == 1 || PASS == 4) {
#pragma unroll
    for (int gt = 0; gt < NGT; ++gt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int a0 = row16_reduce<false>(mn[gt][i]), b0 = row16_reduce<true>(mx[gt][i]);
        if (!INTV) {
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

// FP32 LUT entries are built by thread (m, j) = (MPAR i + tid / 256, tid % 256),
// MPAR = threads / 256 subspaces side by side; the variants specialised for
// a subspace count (256 threads) keep the codewords of their entries in
// registers
constexpr int kMPar = kThreads / kKsub;
template <int WPR, int MT>
struct Owned {
  // codewords of the FP32 LUT entries a thread owns
  static constexpr int NM = MT ? MT / kMPar : 1;
  float c[NM][kMaxDsub];
};

// One work unit (G pairs of one list, lane class LWB; 0 = FP32 LUT): RC, LC,
// quantisation, DC scan, and the phase's bound or candidate forwarding.
// L may be the layout of a larger tile (the mixed-class kernel).
template <int LWB, int MT, int PHASE, int DT, int NR, int NT, typename Own, typename Fetch>
__device__ __forceinline__ void scan_unit(const ScanArgs& a, char* lds, const ScanLds& L, const Own& own,
                                          const int4 unit, Fetch&& fetch_next) {
  constexpr int WPR = class_wpr(LWB, variant_wpr(MT, NR));
  constexpr bool FP = LWB == 0;
  constexpr int W = Lane<LWB>::W;
  constexpr int G = WPR * W;
  constexpr uint32_t MASK = Lane<LWB>::MASK;
  constexpr bool CRES = FP && MT != 0 && MT <= 16;  // FP32 codewords stay in registers
  constexpr int MPAR = NT / kKsub;  // FP32 LUT: subspaces built side by side
  static_assert(!CRES || NT == kThreads, "FP32 codewords in registers: 256-thread workgroups");
  static_assert(NT % 64 == 0 && (NT & (NT - 1)) == 0, "NT: a power of two number of waves");
  const int M = MT ? MT : a.M;
  // 4-bit entries (width 4, one width per pair): a word's low and high
  // nibbles are added into the 8-bit lanes of two words, whose sums of
  // kWideChunk subspaces are widened into 16-bit lanes (at most 2^15 - 1,
  // guard bit 15) between chunks
  constexpr bool NIB = LWB == 4;
  const uint32_t SMASK = NIB ? 0x7FFFu : MASK;
  int32_t* pq = reinterpret_cast<int32_t*>(lds + L.pq);
  int32_t* pb = reinterpret_cast<int32_t*>(lds + L.pb);
  int32_t* ps = reinterpret_cast<int32_t*>(lds + L.ps);
  int64_t* pbase = reinterpret_cast<int64_t*>(lds + L.pbase);
  uint32_t* psig = reinterpret_cast<uint32_t*>(lds + L.psig);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int own_j = tid % kKsub, own_m0 = tid / kKsub;
  const bool owner = tid < MPAR * kKsub;
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
    int32_t* ppid = reinterpret_cast<int32_t*>(lds + L.pid);
    if (tid < G) {
      if (tid < np_u) {
        const int pid = a.sorted[unit.y + tid];
        ppid[tid] = pid;
        pq[tid] = pid / a.npmax;
        pb[tid] = a.pbits[pid];
      } else {
        ppid[tid] = -1;
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
    if (FP || !ip) {
      const int d4 = a.d >> 2;
      const int gstep = NT / d4, tstep = NT - gstep * d4;
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
          if (PHASE >= 2 && !a.noskip && fkey(reinterpret_cast<const float*>(lds + L.pbase)[g]) > sig) live = false;
        } else {
          const int64_t t = ikey_val(tk);
          if (t < pbase[g]) {
            // (noskip: the pair is scanned all the same; only a vector at
            // its base could pass, a candidate beyond the bound that the
            // merge ranks below the top k)
            live = a.noskip != 0;
          } else {
            const int64_t dd = (t - pbase[g]) >> ps[g];
            sig = dd > (int64_t)SMASK ? SMASK : (uint32_t)dd;
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
      for (int e = tid; e < np_u * M; e += NT) {
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
              if constexpr (MM == 1) {
                // the query's FP32 dot products, built once per query (the
                // same FMA chain)
                dot = __int_as_float(a.iptab[((size_t)pq[g] * M + m) * kKsub + own_j]);
              } else {
#pragma unroll
                for (int t = 0; t < kMaxDsub; ++t)
                  if (t < a.dsub) dot = fmaf(r[t], c[t], dot);
              }
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
            for (int i = 0; i < MT / MPAR; ++i) entry(mtag, MPAR * i + own_m0, own.c[i]);
          }
        } else if (owner) {
          for (int m = own_m0; m < M; m += MPAR) {
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
    } else if (ip) {
      // inner product: the LUT is the query's, quantised once per (query,
      // width) with the query's shift; the pair's base is its exact base.
      // The unit copies its pairs' tables into the packed rows.
      if (tid == 0) *reinterpret_cast<int*>(lds + L.ctl + 12) = 0;  // live-pair count of the unit
      __syncthreads();
      int32_t* pw = reinterpret_cast<int32_t*>(lds + L.lo);  // [G]: table index (query, width) of each pair
      if (tid < G) {
        if (tid < np_u) {
          const int wi = (pb[tid] >> 2) - 1;
          pw[tid] = pq[tid] * 4 + wi;
          ps[tid] = a.ipsh[pq[tid] * 4 + wi];
          pbase[tid] = a.pbase_g[ppid[tid]];
        }
        if (PHASE >= 2 && pair_threshold(tid)) atomicAdd(reinterpret_cast<int*>(lds + L.ctl + 12), 1);
      }
      __syncthreads();
      if constexpr (PHASE >= 2) {
        const int nlive = *reinterpret_cast<int*>(lds + L.ctl + 12);
        if (PHASE == 2 && tid == 0 && a.work) {
          uint64_t* wc = reinterpret_cast<uint64_t*>(lds + L.ctl + 32);
          wc[0] += (uint64_t)(nlive * (v1 - v0) * M);
          wc[1] += (uint64_t)nlive;
          wc[2] += (uint64_t)(np_u - nlive);
          // what the unit reads: its chunk's codes once and the live pairs'
          // quantised tables (bytes for the 4-bit class, else uint16)
          if (nlive) wc[3] += (uint64_t)((v1 - v0) * M) + (uint64_t)nlive * M * kKsub * (LWB == 4 ? 1 : 2);
        }
        if (!nlive) {
          fetch_next();
          return;
        }
      }
      uint32_t* lut = reinterpret_cast<uint32_t*>(lds + L.lut);
      const size_t tsz = (size_t)M * kKsub;
      // one 16-byte load per pair and step (16 byte entries or 8 uint16
      // ones); the loads of U steps are issued before any is consumed
      constexpr int U = G >= 16 ? 1 : (G >= 8 ? 2 : 4);
      auto copy = [&](auto by_tag) {
        constexpr bool BY = decltype(by_tag)::value;
        constexpr int EPS = BY ? 16 : 8;  // entries per step
        const int ns = M * kKsub / EPS;
        for (int eb = tid; eb < ns; eb += U * NT) {
          u32x4 xs[U][G];
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const int es = eb + u * NT;
              xs[u][g] = (u32x4){0u, 0u, 0u, 0u};  // absent and dead pairs: zero fields
              if (g < np_u && pb[g] >= 0 && es < ns)
                xs[u][g] = *reinterpret_cast<const u32x4*>(
                    reinterpret_cast<const uint8_t*>(a.iptq + (size_t)pw[g] * tsz) + (size_t)es * 16);
            }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int es = eb + u * NT;
            if (es >= ns) continue;
            uint32_t wds[EPS][WPR];
            if constexpr (BY && LWB == 4) {
              // byte entries (at most 15) of the word's eight pairs: for each
              // four entries, pairs 8 w + 0..3 and 8 w + 4..7 are two 4 x 4
              // byte transposes (eight byte permutes each), the second moved
              // into the high nibbles
#pragma unroll
              for (int w = 0; w < WPR; ++w)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  uint32_t t4[2][4];
#pragma unroll
                  for (int h = 0; h < 2; ++h) {
                    const uint32_t pa = xs[u][8 * w + 4 * h + 0][j], pb2 = xs[u][8 * w + 4 * h + 1][j];
                    const uint32_t pc = xs[u][8 * w + 4 * h + 2][j], pd = xs[u][8 * w + 4 * h + 3][j];
                    const uint32_t ab0 = byte_perm(pb2, pa, 0x05010400u), ab1 = byte_perm(pb2, pa, 0x07030602u);
                    const uint32_t cd0 = byte_perm(pd, pc, 0x05010400u), cd1 = byte_perm(pd, pc, 0x07030602u);
                    t4[h][0] = byte_perm(cd0, ab0, 0x05040100u);
                    t4[h][1] = byte_perm(cd0, ab0, 0x07060302u);
                    t4[h][2] = byte_perm(cd1, ab1, 0x05040100u);
                    t4[h][3] = byte_perm(cd1, ab1, 0x07060302u);
                  }
#pragma unroll
                  for (int i = 0; i < 4; ++i) wds[4 * j + i][w] = t4[0][i] | (t4[1][i] << 4);
                }
            } else if constexpr (!BY && LWB == 16) {
              // uint16 entries of two pairs: one byte permute per word
#pragma unroll
              for (int w = 0; w < WPR; ++w)
#pragma unroll
                for (int k = 0; k < EPS; ++k)
                  wds[k][w] = byte_perm(xs[u][PairSlot<LWB, WPR>::pair(w, 1)][k >> 1],
                                        xs[u][PairSlot<LWB, WPR>::pair(w, 0)][k >> 1],
                                        (k & 1) ? 0x07060302u : 0x05040100u);
            } else {
#pragma unroll
              for (int k = 0; k < EPS; ++k)
#pragma unroll
                for (int w = 0; w < WPR; ++w) {
                  uint32_t wd = 0;
#pragma unroll
                  for (int f = 0; f < W; ++f) {
                    const u32x4 x = xs[u][PairSlot<LWB, WPR>::pair(w, f)];
                    const uint32_t qv =
                        BY ? (x[k >> 2] >> (8 * (k & 3))) & 0xFFu : (x[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
                    wd |= LWB == 32 ? qv : (qv << (f * LWB));
                  }
                  wds[k][w] = wd;
                }
            }
#pragma unroll
            for (int k = 0; k < EPS; ++k) {
              uint32_t* dst = lut + ((size_t)es * EPS + k) * WPR;
#pragma unroll
              for (int w = 0; w < WPR; ++w) dst[w] = wds[k][w];
            }
          }
        }
      };
      // the 4-bit lane class holds width-4 pairs of one width per pair only,
      // whose tables are bytes (ip_bytes); every other table is uint16
      if constexpr (LWB == 4) copy(std::true_type{});
      else copy(std::false_type{});
      __syncthreads();
    } else {
      int32_t* rr = reinterpret_cast<int32_t*>(lds + L.rr);
      const int16_t* ri = reinterpret_cast<const int16_t*>(lds + L.ri);
      const bool vec8 = a.dsub == 8 && (a.d & 7) == 0;  // 16-byte aligned subspace rows
      for (int e = tid; e < np_u * M; e += NT) {
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
            sacc += v * v;
          }
        }
        rr[e] = sacc;
      }
      __syncthreads();
      // the 16 B fragments of an m-pair are issued together, then consumed
      auto build = [&](auto pass_tag, auto ip_tag) {
        constexpr int PASS = decltype(pass_tag)::value;
        constexpr bool IPM = decltype(ip_tag)::value;
        for (int mp = wave; mp < M / 2; mp += NT / 64) {
          u32x4 Bt[16], Bd[16];
#pragma unroll
          for (int jt = 0; jt < 16; ++jt) {
            const size_t fi = ((size_t)mp * 16 + jt) * 64 + lane;
            Bt[jt] = a.bsw[fi];
            if constexpr (DT == DT_F16) {
              Bd[jt] = a.bsw16[fi];
            } else if constexpr (DT == DT_F8) {
              const u32x2 b8 = a.bsw8[fi];
              Bd[jt] = (u32x4){b8[0], b8[1], 0u, 0u};
            } else {
              Bd[jt] = (u32x4){0u, 0u, 0u, 0u};
            }
          }
          lut_mpair<LWB, WPR, DT, PASS, IPM>(a, lds, L, M, np_u, mp, Bt, Bd);
        }
      };
      using P1 = std::integral_constant<int, 1>;
      using P2 = std::integral_constant<int, 2>;
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
          for (int e = tid; e < np_u * M; e += NT) {
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
          for (int e = tid; e < M * kKsub; e += NT) {
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
        int64_t bsum = 0, rsum = 0;
        if (g < np_u)
          for (int m = r; m < M; m += 16) {
            const int32_t l = lo[g * M + m], h = hi[g * M + m];
            span = h - l > span ? h - l : span;
            rsum += h - l;
            bsum += l - (ip ? rrp[g * M + m] : 0);
          }
        span = row16_reduce<true>(span);
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          bsum += __shfl_xor(bsum, off, 16);
          rsum += __shfl_xor(rsum, off, 16);
        }
        if (r == 15 && g < G) {
          if (g < np_u) {
            const int sh = a.gran ? quant_shift(rsum, M, pb[g]) : quant_shift(span, 1, pb[g]);
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
          // what the unit reads: the pairs' query rows and the centroid (its
          // residuals), and, if a pair is live, its chunk's codes once
          wc[3] += (uint64_t)(np_u + 1) * a.d * 4 + (nlive ? (uint64_t)((v1 - v0) * M) : 0ull);
        }
        if (!nlive) {
          fetch_next();
          return;
        }
      }
      {
        // lo -> the offset hf(s) - lo that pass 2 adds before the shift
        int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
        for (int e = tid; e < np_u * M; e += NT) {
          const int g = e / M, sh = ps[g];
          lo[e] = (sh ? (1 << (sh - 1)) : 0) - lo[e];
        }
      }
      __syncthreads();
      if (l1) build_l1(2);
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
        for (int m0 = 0; m0 < M; m0 += NT / 16) {
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
          // what the unit reads: its LUT sources (inner product: the pairs'
          // FP32 dot-product tables; L2 / L1: the query rows, the centroid
          // and the codebook) and, if a pair is live, its chunk's codes once
          wc[3] += (ip ? (uint64_t)np_u * M * kKsub * 4
                       : (uint64_t)(np_u + 1) * a.d * 4 + (uint64_t)M * kKsub * a.dsub * 4) +
                   (nlive ? (uint64_t)((v1 - v0) * M) : 0ull);
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
    // packed thresholds (phases 2, 3) of the 4- and 8-bit lane classes: the
    // sums of a LUT word's pairs sit in the 16-bit halves of NTW test words
    // (8-bit: fields 0, 2 and 1, 3 with guard bit 8; 4-bit: the widened
    // sums, guard bit 15); a sum passes iff (sigma | guard) - sum keeps the
    // guard bit, and dead pairs have no guard bit in the mask (never hit)
    constexpr int NTW = NIB ? 4 : 2;
    uint32_t sigw[WPR][NTW], mskw[WPR][NTW];
    if constexpr (PHASE >= 2 && (LWB == 8 || NIB)) {
      const uint32_t top = NIB ? 0x7FFFu : 255u, guard = NIB ? 0x8000u : 0x100u;
#pragma unroll
      for (int w = 0; w < WPR; ++w)
#pragma unroll
        for (int t = 0; t < NTW; ++t) sigw[w][t] = mskw[w][t] = 0;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int w = PairSlot<LWB, WPR>::word(g), t = test_word<LWB, WPR>(g), h = test_half<LWB, WPR>(g);
        const uint32_t sg = live[g] ? (sig[g] > top ? top : sig[g]) : top;
        sigw[w][t] |= (sg | guard) << (16 * h);
        mskw[w][t] |= (live[g] ? guard : 0u) << (16 * h);
      }
    }
    lds_u32* lut = reinterpret_cast<lds_u32*>((uintptr_t)L.lut);  // LDS address (see lds_u32)
    // code dwords per vector held in registers: MT / 4 for a specialised
    // variant; the generic integer BF16 one holds up to kRegMQ (M <= 4
    // kRegMQ) with its loops unrolled to that bound and branches on M.
    // Longer rows, the FP16 / FP8 builds (whose B fragments leave no
    // registers for it) and the FP32 LUT (one dependent chain of FP32 adds
    // per vector: measured slower with the codes in registers) read the
    // codes from memory as they are scanned.
    constexpr bool RG = MT == 0 && DT == DT_BF16 && !FP;
    constexpr int MQ = MT ? MT / 4 : (RG ? kRegMQ : 1);
    const bool regc = MT != 0 || (RG && M <= 4 * kRegMQ);
    // vectors per thread and step: one-word rows (a few pairs per list, the
    // streaming case) make a vector cheap to scan, so four are kept in flight
    // to cover HBM latency; wide rows are compute-bound at one
    constexpr int PV = (NR && MT != 0) ? 4 : 1;
    uint32_t cw_next[PV][MQ];
    auto load_codes = [&](int64_t v, uint32_t* cw) {
      const uint32_t* cp = reinterpret_cast<const uint32_t*>(a.codes + (size_t)(L0 + v) * M);
#pragma unroll
      for (int i = 0; i < MQ; ++i)
        if (MT != 0 || 4 * i < M) cw[i] = cp[i];
    };
    if (regc) {
#pragma unroll
      for (int pv = 0; pv < PV; ++pv) {
        const int64_t v = v0 + tid + pv * NT;
        if (v < v1) load_codes(v, cw_next[pv]);
      }
    }
    fetch_next();  // the next unit's descriptor, read while this one scans
    for (int64_t vb = v0; vb < v1; vb += NT * PV) {
      uint32_t cwg[PV][MQ];
#pragma unroll
      for (int pv = 0; pv < PV; ++pv)
#pragma unroll
        for (int i = 0; i < MQ; ++i) cwg[pv][i] = cw_next[pv][i];
      if (regc) {
#pragma unroll
        for (int pv = 0; pv < PV; ++pv) {
          const int64_t vn = vb + tid + (PV + pv) * NT;
          if (vn < v1) load_codes(vn, cw_next[pv]);
        }
      }
#pragma unroll
      for (int pv = 0; pv < PV; ++pv) {
      const int64_t v = vb + tid + pv * NT;
      if (v < v1) {
        // acc: the lanes of each LUT word (4-bit class: the low nibbles, with
        // the high ones in accb), wz: the 4-bit class's widened sums
        uint32_t acc[WPR], accb[WPR], wz[WPR][4];
        float accf[WPR];
#pragma unroll
        for (int w = 0; w < WPR; ++w) {
          acc[w] = 0;
          accb[w] = 0;
          accf[w] = 0.f;
#pragma unroll
          for (int t = 0; t < 4; ++t) wz[w][t] = 0;
        }
        // 4 ND subspaces from ND code dwords: the ND * 4 row reads are issued
        // before any is added (a scheduling barrier keeps the adds behind
        // them: left alone, the compiler waited after every second read of
        // the long variants), then added in subspace order; the 8-bit sums
        // are widened at every kWideChunk-th subspace (chunks never straddle
        // one)
        auto stepn = [&](auto nd_tag, const uint32_t* c, int m0) {
          constexpr int ND = decltype(nd_tag)::value;
          uint32_t x[4 * ND][WPR];
#pragma unroll
          for (int k = 0; k < 4 * ND; ++k) {
            const int rowi = ((m0 + k) * kKsub + ((c[k >> 2] >> (8 * (k & 3))) & 255u)) * WPR;
            lut_row_load<WPR>(lut, rowi, x[k]);
          }
          // (the short straight-line variants, M <= 24, are left to the
          // scheduler: the barrier made the M = 24 scan 30 % slower)
          if constexpr (MT == 0 || MT > 24) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int k = 0; k < 4 * ND; ++k)
#pragma unroll
            for (int w = 0; w < WPR; ++w) {
              if constexpr (FP) {
                accf[w] += __uint_as_float(x[k][w]);
              } else if constexpr (NIB) {
                acc[w] += x[k][w] & 0x0F0F0F0Fu;
                accb[w] += (x[k][w] >> 4) & 0x0F0F0F0Fu;
              } else {
                acc[w] += x[k][w];
              }
            }
          if constexpr (NIB) {
            if (((m0 + 4 * ND) % kWideChunk) == 0 || m0 + 4 * ND >= M) {
              // widen the chunk's 8-bit sums: bytes 0, 2 and 1, 3 of the
              // low- and high-nibble words into the 16-bit halves of four
#pragma unroll
              for (int w = 0; w < WPR; ++w) {
                wz[w][0] += acc[w] & 0x00FF00FFu;
                wz[w][1] += (acc[w] >> 8) & 0x00FF00FFu;
                wz[w][2] += accb[w] & 0x00FF00FFu;
                wz[w][3] += (accb[w] >> 8) & 0x00FF00FFu;
                acc[w] = 0;
                accb[w] = 0;
              }
            }
          }
        };
        using One = std::integral_constant<int, 1>;
        using Two = std::integral_constant<int, 2>;
        static_assert(kWideChunk % 8 == 0, "two-dword chunks must not straddle a widening point");
        if (regc) {
#pragma unroll
          for (int i = 0; i < MQ; i += 2) {
            if (i + 1 < MQ && (MT != 0 || 4 * i + 8 <= M)) stepn(Two{}, &cwg[pv][i], 4 * i);
            else if (MT != 0 || 4 * i < M) stepn(One{}, &cwg[pv][i], 4 * i);
          }
        } else {
          const uint32_t* cpg = reinterpret_cast<const uint32_t*>(a.codes + (size_t)(L0 + v) * M);
          for (int m4 = 0; m4 < M; m4 += 4) {
            const uint32_t c4 = cpg[m4 >> 2];
            stepn(One{}, &c4, m4);
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
        // the test word t of LUT word w (8-bit: fields 0, 2 / 1, 3; 4-bit:
        // the widened sums)
        auto tword = [&](int w, int t) -> uint32_t {
          if constexpr (NIB) return wz[w][t];
          else return t ? (acc[w] >> 8) & 0x00FF00FFu : acc[w] & 0x00FF00FFu;
        };
        if constexpr (PHASE >= 2 && (LWB == 8 || NIB)) {
          // every sum of a LUT word tested against its threshold at once, in
          // the 16-bit halves of its test words
#pragma unroll
          for (int w = 0; w < WPR; ++w) {
            uint32_t hit = 0;
#pragma unroll
            for (int t = 0; t < NTW; ++t) hit |= (sigw[w][t] - tword(w, t)) & mskw[w][t];
            if (hit) {
#pragma unroll
              for (int f = 0; f < W; ++f) {
                // rare path: thresholds from LDS, not held in registers
                const int g = PairSlot<LWB, WPR>::pair(w, f);
                const uint32_t S = (tword(w, test_word<LWB, WPR>(g)) >> (16 * test_half<LWB, WPR>(g))) & 0xFFFFu;
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
            else if constexpr (NIB) S = (wz[w][test_word<LWB, WPR>(g)] >> (16 * test_half<LWB, WPR>(g))) & 0xFFFFu;
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
    if (PHASE == 1) {
      // the k-th smallest of a wave's per-lane minima bounds the pair's k-th
      // smallest (each minimum is a distinct vector): the wave's min(k, 64)
      // smallest minima go to the query's bound buffer, and the bound is
      // taken over all of them (for k > 64 every lane's minimum goes: the k
      // smallest entries of the buffer are then the pair's k smallest
      // minima, as a workgroup-wide selection would give).  The kw-th
      // smallest minimum x is found bit by bit (the largest x with fewer
      // than kw minima below it; counts are ballot bit counts, no
      // cross-lane shuffles); the minima below x and the lowest-lane ones
      // equal to x make up the kw.
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g >= np_u) break;
        const uint32_t v = lmin[g];
        const int q = pq[g];
        const int kq = a.kq ? a.kq[q] : a.kconst;
        const int kk = kq < 64 ? kq : 64;
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
    }
}

// workgroups per CU the register allocation of a scan variant must allow:
// one of 512 threads; three of 256 for M = 24 (its 48 KB LUT leaves LDS for
// three), else two
__host__ __device__ constexpr int scan_min_blocks(int MT, int NT) { return NT == 512 ? 1 : (MT == 24 ? 3 : 2); }

// persistent scan of one lane class: workgroups claim units of their class
// from a device counter; the next unit is claimed while the current one is
// processed (index at the start, descriptor before the scan, published at
// the end)
template <int LWB, int MT, int PHASE, int DT, int NR, int NT>
__global__ __launch_bounds__(NT, scan_min_blocks(MT, NT))
    __attribute__((amdgpu_waves_per_eu(NT / 64 * scan_min_blocks(MT, NT) / 4, NT == 512 ? 2 : 8))) void k_scan(ScanArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int WPR = class_wpr(LWB, variant_wpr(MT, NR));
  constexpr bool FP = LWB == 0;
  constexpr int G = WPR * Lane<LWB>::W;
  constexpr bool CRES = FP && MT != 0 && MT <= 16;
  constexpr int MPAR = NT / kKsub;
  static_assert(!CRES || NT == kThreads, "FP32 codewords in registers: 256-thread workgroups");
  const int M = MT ? MT : a.M;
  const ScanLds L = scan_lds_layout(G, WPR, M, a.d, FP, PHASE, NT);
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
  const bool owner = tid < MPAR * kKsub;
  Owned<WPR, CRES ? MT : 0> own;
  if constexpr (CRES) {
#pragma unroll
    for (int i = 0; i < MT / MPAR; ++i)
#pragma unroll
      for (int t = 0; t < kMaxDsub; ++t)
        own.c[i][t] = owner && t < a.dsub
                          ? a.codebook[((size_t)(MPAR * i + own_m0) * kKsub + own_j) * a.dsub + t] : 0.f;
  }
  UnitQueue uq(a.counter, ue - ub, a.steal);
  if (tid == 0) {
    const int64_t uu = uq.next();
    s_u = (int)uu;
    if (ub + uu < ue) s_unit = a.units[ub + uu];
  }
  if (tid == 0)
    for (int i = 0; i < 4; ++i) reinterpret_cast<uint64_t*>(lds + L.ctl + 32)[i] = 0;
  __syncthreads();
  for (;;) {
    if (ub + s_u >= ue) break;
    int next_u = 0;
    int4 next_unit = make_int4(0, 0, 0, 0);
    if (tid == 0) next_u = (int)uq.next();
    scan_unit<LWB, MT, PHASE, DT, NR, NT>(a, lds, L, own, s_unit, [&] {
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
    for (int i = 0; i < 4; ++i)
      atomicAdd((unsigned long long*)&a.work[i],
                (unsigned long long)reinterpret_cast<const uint64_t*>(lds + L.ctl + 32)[i]);
}

// all three lane classes of an integer policy in one persistent launch, in
// the order 32-bit, 16-bit, then 4-bit (one width per pair) or 8-bit units
// (each largest list first): the few wide units start early and the many
// narrow units fill the tail.  The LDS tile of the 4-bit class (the most
// pairs per unit) serves every class.
template <int MT, int PHASE, int DT, int NR, int NT>
__global__ __launch_bounds__(NT, scan_min_blocks(MT, NT))
    __attribute__((amdgpu_waves_per_eu(NT / 64 * scan_min_blocks(MT, NT) / 4, NT == 512 ? 2 : 8))) void k_scan_mix(ScanArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int WPR = variant_wpr(MT, NR);
  const int M = MT ? MT : a.M;
  const ScanLds L = scan_lds_layout(unit_pairs(-1, WPR), WPR, M, a.d, false, PHASE, NT);
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
    for (int i = 0; i < 4; ++i) reinterpret_cast<uint64_t*>(lds + L.ctl + 32)[i] = 0;
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
    if (cls == 0 && !a.gran) scan_unit<4, MT, PHASE, DT, NR, NT>(a, lds, L, own, s_unit, fetch);
    else if (cls == 0) scan_unit<8, MT, PHASE, DT, NR, NT>(a, lds, L, own, s_unit, fetch);
    else if (cls == 1) scan_unit<16, MT, PHASE, DT, NR, NT>(a, lds, L, own, s_unit, fetch);
    else scan_unit<32, MT, PHASE, DT, NR, NT>(a, lds, L, own, s_unit, fetch);
    __syncthreads();
    if (tid == 0) {
      s_u = next_u;
      s_unit = next_unit;
      s_cls = next_cls;
    }
    __syncthreads();
  }
  if (PHASE == 2 && tid == 0 && a.work)
    for (int i = 0; i < 4; ++i)
      atomicAdd((unsigned long long*)&a.work[i],
                (unsigned long long)reinterpret_cast<const uint64_t*>(lds + L.ctl + 32)[i]);
}

// LC matrix dtype of an AMP_LUT_* value (0 selects BF16; the FP8 value is
// rejected before a search launches)
inline int dt_of(int lut_dtype) {
  return lut_dtype == AMP_LUT_F16 ? DT_F16 : (lut_dtype == AMP_LUT_F8E4M3 ? DT_F8 : DT_BF16);
}


// subspace count of the scan variant that runs a lane class (0: generic):
// variants with straight-line code for their subspace count (codes in
// registers) exist for M = 8, 16, 24, 32, 64 (256-thread workgroups) and
// M = 96, 120, 128 (512-thread workgroups: one workgroup fills a CU's LDS),
// for the integer lane classes with the BF16 LUT build and for the FP32 LUT
// (which has no LC dtype)
// (wpr: the words per row the queue packed for; a batch too sparse to fill
// wide rows runs the generic one-word variant, see scan_wpr)
inline bool scan_mt_wide(int M) { return M == 96 || M == 120 || M == 128; }
inline int scan_mt(int lwb, int M, int dt) {
  if (lwb != 0 && dt != DT_BF16) return 0;
  if (M == 8 || M == 16 || M == 24) return M;
  if (M == 32 || M == 64 || scan_mt_wide(M)) return M;
  return 0;
}
// one-word rows on a specialised variant
inline int scan_nr(int mt, int wpr) { return (wpr == 1 && kernel_wpr(mt) != 1) ? 1 : 0; }


typedef void (*ScanFn)(ScanArgs);
// the kernel of a lane class (lwb 0 = FP32 LUT, 8/16/32) or, with lwb < 0,
// the mixed-class kernel, for one phase; nullptr if none fits
ScanFn pick_scan_ph1(int lwb, int M, int dt, int wpr, int nt);
ScanFn pick_scan_ph2(int lwb, int M, int dt, int wpr, int nt);
ScanFn pick_scan_ph3(int lwb, int M, int dt, int wpr, int nt);

}  // namespace amp

namespace amp {

// ------------------------------------------------------------------ exact pair bases
// The base of a (query, probed list) pair, sum over the subspaces of the
// minimum of the exact integer LUT row (inner product: minus qi.ci), bounds
// every integer distance estimate of its list from below.  A pair whose base
// exceeds its query's phase-1 bound cannot reach the top-k: it is left out of
// the full scan's work queue (the same test the scan applies after LUT pass
// 1, made before any unit is formed).  L2 and L1: the LUT minima of every
// pair (LUT pass 1 on MFMA, or on the VALU for L1); inner product: the table
// is the query's, built once per query with its minima, and each pair adds
// its own -qi.ci.
struct BaseArgs {
  const float* Q;
  const float* C;
  const u32x4* bsw;
  const u32x4* bsw16;
  const u32x2* bsw8;
  const int16_t* cbi16;
  const int16_t* ci16;     // [nlist][d] grid centroids
  const int32_t* probes;
  int64_t* pbase;          // [nq][npmax]
  // inner product
  int16_t* qi16;           // [nq][d] queries on the grid
  int32_t* iptab;          // [nq][M][256]
  int32_t* iplo;           // [nq][M]
  int32_t* ipspan;         // [nq]
  int64_t* iplsum;         // [nq]
  uint16_t* iptq;          // [nq][4][M][256] (bytes where ip_bytes)
  int32_t* ipsh;           // [nq][4]
  int32_t* ipmask;         // [nq]
  const uint8_t* pbits;    // [nq][npmax]
  const float* codebook;   // FP32 policy table
  int nq, d, M, dsub, npmax, grid_e, grid_kind, metric;
  int G;                   // pairs per workgroup of k_base
  int gran;                // quantiser granularity (as ScanArgs)
};

__host__ __device__ inline ScanLds base_lds_layout(int G, int M, int d) {
  ScanLds L{};
  int o = 0;
  auto take = [&](int bytes) { int r = o; o += (bytes + 15) & ~15; return r; };
  L.lut = 0;  // (no LUT: pass 1 only)
  L.ri = take(G * ri_stride(d) * 2);
  L.rr = take(G * M * 4);
  L.lo = take(G * M * 4);
  L.hi = take(G * M * 4);
  L.ps = take(G * 4);
  L.pq = take(G * 4);
  L.pb = take(G * 4);
  L.ctl = take(64);
  L.total = o;
  return L;
}

// the B fragments of one m-pair, issued together (as in the scan)
template <int DT>
__device__ __forceinline__ void base_frags(const BaseArgs& b, int mp, int lane, u32x4 (&Bt)[16], u32x4 (&Bd)[16]) {
#pragma unroll
  for (int jt = 0; jt < 16; ++jt) {
    const size_t fi = ((size_t)mp * 16 + jt) * 64 + lane;
    Bt[jt] = b.bsw[fi];
    if constexpr (DT == DT_F16) {
      Bd[jt] = b.bsw16[fi];
    } else if constexpr (DT == DT_F8) {
      const u32x2 b8 = b.bsw8[fi];
      Bd[jt] = (u32x4){b8[0], b8[1], 0u, 0u};
    } else {
      Bd[jt] = (u32x4){0u, 0u, 0u, 0u};
    }
  }
}

// L2 / L1: b.G consecutive pair slots per workgroup (any queries, any
// lists; empty slots have zero rows and write nothing).  Every m-pair's B
// fragments, loaded once per workgroup and wave, serve all G pairs.
template <int DT>
__global__ __launch_bounds__(kThreads) void k_base(BaseArgs b) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int G = b.G;
  const ScanLds L = base_lds_layout(G, b.M, b.d);
  ScanArgs a{};
  a.d = b.d;
  a.dsub = b.dsub;
  a.M = b.M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = b.M;
  const size_t n = (size_t)b.nq * b.npmax;
  const size_t i0 = (size_t)blockIdx.x * G;
  int* sp = reinterpret_cast<int*>(lds + L.ps);
  for (int g = tid; g < G; g += kThreads) sp[g] = i0 + g < n ? b.probes[i0 + g] : -1;
  __syncthreads();
  // RC onto the grid (the scan's arithmetic: FP32 subtraction, then the grid)
  const int d4 = b.d >> 2, rs4 = ri_stride(b.d) >> 2;
  for (int e = tid; e < G * d4; e += kThreads) {
    const int g = e / d4, t4 = e - g * d4;
    const int p = sp[g];
    u32x2 v = {0u, 0u};
    if (p >= 0) {
      const size_t q = (i0 + g) / b.npmax;
      const float4 qv = reinterpret_cast<const float4*>(b.Q + q * b.d)[t4];
      const float4 cv = reinterpret_cast<const float4*>(b.C + (size_t)p * b.d)[t4];
      const float rx = qv.x - cv.x, ry = qv.y - cv.y, rz = qv.z - cv.z, rw = qv.w - cv.w;
      const uint32_t v0 = (uint32_t)grid_val(rx, b.grid_e, b.grid_kind) & 0xFFFFu;
      const uint32_t v1 = (uint32_t)grid_val(ry, b.grid_e, b.grid_kind) & 0xFFFFu;
      const uint32_t v2 = (uint32_t)grid_val(rz, b.grid_e, b.grid_kind) & 0xFFFFu;
      const uint32_t v3 = (uint32_t)grid_val(rw, b.grid_e, b.grid_kind) & 0xFFFFu;
      v = (u32x2){v0 | (v1 << 16), v2 | (v3 << 16)};
    }
    reinterpret_cast<u32x2*>(lds + L.ri)[g * rs4 + t4] = v;
  }
  __syncthreads();
  const int16_t* ri = reinterpret_cast<const int16_t*>(lds + L.ri);
  int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
  if (b.metric == AMP_L1) {
    // a thread per (pair, subspace) row: minimum over the codewords on the VALU
    for (int e = tid; e < G * M; e += kThreads) {
      const int g = e / M, m = e % M;
      int rv[kMaxDsub];
#pragma unroll
      for (int t = 0; t < kMaxDsub; ++t) rv[t] = t < b.dsub ? (int)ri[g * ri_stride(b.d) + m * b.dsub + t] : 0;
      int mn = 0x7FFFFFFF;
      const int16_t* cb = b.cbi16 + (size_t)m * kKsub * 8;
      for (int j = 0; j < kKsub; ++j) {
        int v = 0;
#pragma unroll
        for (int t = 0; t < kMaxDsub; ++t) v += abs(rv[t] - (int)cb[j * 8 + t]);
        mn = v < mn ? v : mn;
      }
      lo[e] = mn;
    }
  } else {
    int32_t* rr = reinterpret_cast<int32_t*>(lds + L.rr);
    for (int e = tid; e < G * M; e += kThreads) {
      const int g = e / M, m = e % M;
      int32_t sacc = 0;
      for (int t = 0; t < b.dsub; ++t) {
        const int v = ri[g * ri_stride(b.d) + m * b.dsub + t];
        sacc += v * v;
      }
      rr[e] = sacc;
    }
    __syncthreads();
    for (int mp = wave; mp < M / 2; mp += kThreads / 64) {
      u32x4 Bt[16], Bd[16];
      base_frags<DT>(b, mp, lane, Bt, Bd);
      lut_row_minima<DT>(a, lds, L, M, G, mp, Bt, Bd);
    }
  }
  __syncthreads();
  for (int g = tid; g < G; g += kThreads)
    if (sp[g] >= 0) {
      int64_t sum = 0;
      for (int m = 0; m < M; ++m) sum += lo[g * M + m];
      b.pbase[i0 + g] = sum;
    }
}

// LUT export (test hook, L2): for kBaseExport consecutive pair slots, the
// LUT exactly as the scan builds it (pass 1, shift and base, pass 2) with the
// quantised entries, shift and base (and, optionally, the entries before
// quantisation) written to global memory
constexpr int kBaseExport = 16;
template <int DT>
__global__ __launch_bounds__(kThreads) void k_export(BaseArgs b, uint16_t* exq, int32_t* exs, int64_t* exb,
                                                     int32_t* ext) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int G = kBaseExport;
  const ScanLds L = base_lds_layout(G, b.M, b.d);
  ScanArgs a{};
  a.d = b.d;
  a.dsub = b.dsub;
  a.M = b.M;
  a.tab_out = ext;
  a.ex_q = exq;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = b.M;
  const size_t n = (size_t)b.nq * b.npmax;
  const size_t i0 = (size_t)blockIdx.x * G;
  int32_t* sp = reinterpret_cast<int32_t*>(lds + L.ps);
  int32_t* pq = reinterpret_cast<int32_t*>(lds + L.pq);
  int32_t* pb = reinterpret_cast<int32_t*>(lds + L.pb);
  int32_t* lo = reinterpret_cast<int32_t*>(lds + L.lo);
  const int32_t* hi = reinterpret_cast<const int32_t*>(lds + L.hi);
  __shared__ int s_probe[G];
  if (tid < G) {
    const bool ok = i0 + tid < n && b.probes[i0 + tid] >= 0;
    s_probe[tid] = ok ? b.probes[i0 + tid] : -1;
    pq[tid] = ok ? (int)(i0 + tid) : -1;  // destination row
    pb[tid] = ok ? b.pbits[i0 + tid] : 16;
  }
  __syncthreads();
  const int d4 = b.d >> 2, rs4 = ri_stride(b.d) >> 2;
  for (int e = tid; e < G * d4; e += kThreads) {
    const int g = e / d4, t4 = e - g * d4;
    const int p = s_probe[g];
    u32x2 v = {0u, 0u};
    if (p >= 0) {
      const size_t q = (i0 + g) / b.npmax;
      const float4 qv = reinterpret_cast<const float4*>(b.Q + q * b.d)[t4];
      const float4 cv = reinterpret_cast<const float4*>(b.C + (size_t)p * b.d)[t4];
      const uint32_t v0 = (uint32_t)grid_val(qv.x - cv.x, b.grid_e, b.grid_kind) & 0xFFFFu;
      const uint32_t v1 = (uint32_t)grid_val(qv.y - cv.y, b.grid_e, b.grid_kind) & 0xFFFFu;
      const uint32_t v2 = (uint32_t)grid_val(qv.z - cv.z, b.grid_e, b.grid_kind) & 0xFFFFu;
      const uint32_t v3 = (uint32_t)grid_val(qv.w - cv.w, b.grid_e, b.grid_kind) & 0xFFFFu;
      v = (u32x2){v0 | (v1 << 16), v2 | (v3 << 16)};
    }
    reinterpret_cast<u32x2*>(lds + L.ri)[g * rs4 + t4] = v;
  }
  __syncthreads();
  {
    const int16_t* ri = reinterpret_cast<const int16_t*>(lds + L.ri);
    int32_t* rr = reinterpret_cast<int32_t*>(lds + L.rr);
    for (int e = tid; e < G * M; e += kThreads) {
      const int g = e / M, m = e % M;
      int32_t sacc = 0;
      for (int t = 0; t < b.dsub; ++t) {
        const int v = ri[g * ri_stride(b.d) + m * b.dsub + t];
        sacc += v * v;
      }
      rr[e] = sacc;
    }
  }
  __syncthreads();
  for (int mp = wave; mp < M / 2; mp += kThreads / 64) {
    u32x4 Bt[16], Bd[16];
    base_frags<DT>(b, mp, lane, Bt, Bd);
    if (ext) lut_mpair<32, G, DT, 4, false>(a, lds, L, M, G, mp, Bt, Bd);
    else lut_mpair<32, G, DT, 1, false>(a, lds, L, M, G, mp, Bt, Bd);
  }
  __syncthreads();
  int32_t* ps = sp;  // (the probe ids are in s_probe now)
  if (tid < G) {
    int32_t span = 0;
    int64_t bsum = 0, rsum = 0;
    for (int m = 0; m < M; ++m) {
      span = hi[tid * M + m] - lo[tid * M + m] > span ? hi[tid * M + m] - lo[tid * M + m] : span;
      rsum += hi[tid * M + m] - lo[tid * M + m];
      bsum += lo[tid * M + m];
    }
    const int sh = b.gran ? quant_shift(rsum, M, pb[tid]) : quant_shift(span, 1, pb[tid]);
    ps[tid] = sh;
    if (pq[tid] >= 0) {
      exs[pq[tid]] = sh;
      exb[pq[tid]] = bsum;
    }
  }
  __syncthreads();
  for (int e = tid; e < G * M; e += kThreads) {
    const int g = e / M, sh = ps[g];
    lo[e] = (sh ? (1 << (sh - 1)) : 0) - lo[e];
  }
  __syncthreads();
  for (int mp = wave; mp < M / 2; mp += kThreads / 64) {
    u32x4 Bt[16], Bd[16];
    base_frags<DT>(b, mp, lane, Bt, Bd);
    lut_mpair<32, G, DT, 5, false>(a, lds, L, M, G, mp, Bt, Bd);
  }
}

constexpr int kTabQ = 8;  // queries per workgroup of the table build (one 8-row MFMA tile)

// inner product, integer policies: each query's exact table T[m][j] =
// -qi_m . cbi_mj (LUT pass 1 on MFMA, the entries kept), its row minima, the
// largest row span and the sum of the minima; the pair bases, which held
// qi.ci, become the sum of the minima - qi.ci
template <int DT>
__global__ __launch_bounds__(kThreads) void k_iptab(BaseArgs b) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const ScanLds L = base_lds_layout(kTabQ, b.M, b.d);
  ScanArgs a{};
  a.d = b.d;
  a.dsub = b.dsub;
  a.M = b.M;
  a.tab_out = b.iptab;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = b.M;
  const int q0 = blockIdx.x * kTabQ;
  const int nqb = b.nq - q0 < kTabQ ? b.nq - q0 : kTabQ;
  int32_t* pq = reinterpret_cast<int32_t*>(lds + L.pq);
  if (tid < kTabQ) pq[tid] = q0 + tid;
  const int d4 = b.d >> 2, rs4 = ri_stride(b.d) >> 2;
  for (int e = tid; e < kTabQ * d4; e += kThreads) {
    const int g = e / d4, t4 = e - g * d4;
    u32x2 v = {0u, 0u};
    if (g < nqb) v = reinterpret_cast<const u32x2*>(b.qi16 + (size_t)(q0 + g) * b.d)[t4];
    reinterpret_cast<u32x2*>(lds + L.ri)[g * rs4 + t4] = v;
  }
  __syncthreads();
  for (int mp = wave; mp < M / 2; mp += kThreads / 64) {
    u32x4 Bt[16], Bd[16];
    base_frags<DT>(b, mp, lane, Bt, Bd);
    lut_mpair<32, kTabQ, DT, 4, true>(a, lds, L, M, nqb, mp, Bt, Bd);
  }
  __syncthreads();
  const int32_t* lo = reinterpret_cast<const int32_t*>(lds + L.lo);
  const int32_t* hi = reinterpret_cast<const int32_t*>(lds + L.hi);
  for (int e = tid; e < nqb * M; e += kThreads) b.iplo[(size_t)q0 * M + e] = lo[e];
  // per query (a wave each): span and sum of minima
  // (per-subspace granularity: the sum of the row spans instead of the
  // largest)
  for (int g = wave; g < nqb; g += kThreads / 64) {
    int32_t span = 0;
    int64_t sum = 0, rsum = 0;
    for (int m = lane; m < M; m += 64) {
      span = hi[g * M + m] - lo[g * M + m] > span ? hi[g * M + m] - lo[g * M + m] : span;
      rsum += hi[g * M + m] - lo[g * M + m];
      sum += lo[g * M + m];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int32_t o = __shfl_xor(span, off);
      span = o > span ? o : span;
      sum += __shfl_xor(sum, off);
      rsum += __shfl_xor(rsum, off);
    }
    if (lane == 0) {
      b.ipspan[q0 + g] = b.gran ? rsum : span;
      b.iplsum[q0 + g] = sum;
      reinterpret_cast<int64_t*>(lds + L.rr)[g] = sum;  // (rr is not used by the inner-product build)
    }
  }
  __syncthreads();
  // the pair bases: sum of the query's row minima - qi.ci (pbase held qi.ci)
  const int64_t* psum = reinterpret_cast<const int64_t*>(lds + L.rr);
  for (int e = tid; e < nqb * b.npmax; e += kThreads) {
    const size_t i = (size_t)q0 * b.npmax + e;
    if (b.probes[i] >= 0) b.pbase[i] = psum[e / b.npmax] - b.pbase[i];
  }
}

}  // namespace amp
