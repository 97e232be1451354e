// Internal declarations shared by the host side (capi.cpp) and the kernels
// (kernels.hip) of the adaptive-precision IVF-PQ search library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/amp.h"

namespace amp {

// -------------------------------------------------------------- constants
constexpr int kKsub = AMP_KSUB;
// threads per workgroup of the scan: 256, two workgroups per CU (384 and 512
// were measured slower on the mid workload: registers spill at three or four
// waves per SIMD, and the per-wave phase-1 bound loosens as waves cover less
// of a list)
constexpr int kThreads = 256;
constexpr int kThreadsP2 = 256;        // the next power of two (phase-1 sort rows)
static_assert(kThreadsP2 >= kThreads && (kThreadsP2 & (kThreadsP2 - 1)) == 0, "kThreadsP2");
constexpr int kMaxDsub = 8;            // one MFMA lane group holds a subspace
constexpr int kTableN = 1024;          // predictor kernel table entries
constexpr int kNCls = 3;               // LUT lane-width classes: 8, 16, 32 bit
constexpr int kQSub = 16;              // queue sub-counters per (class, list) bucket
constexpr int kXcd = 8;                // XCDs of the device (ranges of a stealing unit queue)
constexpr int kCtrStride = 32;         // unit counters one 128-byte line apart
constexpr int kQueueSlot = kXcd * kCtrStride;  // u32 words per scan unit queue

// subspaces whose 4-bit entries (at most 15) an 8-bit lane adds before its
// sums are widened into 16-bit lanes
constexpr int kWideChunk = 16;
// code dwords per vector that the generic scan variant keeps in registers
// (M up to 4 kRegMQ subspaces); longer code rows are read as they are scanned
constexpr int kRegMQ = 32;
// lane-width class of a b-bit LUT for M subspaces: the sum of M entries of at
// most 2^b - 1 must fit in the lane; 4-bit widths with one width per pair
// (entries at most 15) are class 0 for any M, their 4-bit entries summed in
// 8-bit lanes that are widened every kWideChunk subspaces (up to M = 2184:
// sums below 2^15)
inline int lane_class(int M, int b, int gran = 0) {
  if (b == 4 && gran == 0 && M <= 2184) return 0;
  uint64_t top = (uint64_t)M * ((1ull << b) - 1);
  if (top <= 0xFFull) return 0;
  if (top <= 0xFFFFull) return 1;
  return 2;
}
// lane bits of a class: class 0 holds 4-bit entries with one width per pair
// (width-4 pairs only), 8-bit ones with per-subspace widths
inline int lane_bits(int cls, int gran) { return cls == 0 && gran == 0 ? 4 : 8 << cls; }

// -------------------------------------------------------------- device data
struct DeviceModel {
  int32_t n_sv = 0;
  int32_t* sv = nullptr;       // [n_sv][5]
  int32_t* beta = nullptr;     // [n_sv]
  int32_t* table = nullptr;    // [1024]
};

struct DeviceIndex {
  int device = -1;
  float* centroids = nullptr;  // [nlist][d]
  float* cnorm = nullptr;      // [nlist] squared norms (FP32, sequential order)
  float* codebook = nullptr;   // [M][256][dsub]
  uint4* bsw = nullptr;        // [M/2][16][64] MFMA B fragments (8 bf16 each)
  uint4* bsw16 = nullptr;      // [M/2][16][64] FP16 dims fragments
  uint2* bsw8 = nullptr;       // [M/2][16][64] FP8 (e4m3) dims fragments
  int16_t* cbi16 = nullptr;    // [M][256][8] grid codebook (L1 LUT build)
  int16_t* ci16 = nullptr;     // [nlist][d] grid centroids (inner product: qi.ci, d')
  int32_t* lorder = nullptr;   // [nlist] lists by decreasing size (ties: id)
  int32_t* lpos = nullptr;     // [nlist] position of each list in lorder
  uint8_t* codes = nullptr;    // [N][M]
  int64_t* ids = nullptr;      // [N]
  int64_t* offsets = nullptr;  // [nlist+1]
  int32_t* radq = nullptr;     // [nlist]
  DeviceModel model;
  // reduced-precision cluster locating (sub-space map, CL predictor)
  int8_t* clc = nullptr;       // [nlist][S][Kp] centroid codes, each slice zero-padded to Kp bytes
  uint16_t* clasg = nullptr;   // [nlist][S] sub-space of every centroid slice
  int8_t* clz = nullptr;       // [S][P][Kp] sub-space centres (codes), zero-padded
  int32_t* clr = nullptr;      // [S][P] radius
  int32_t* cln = nullptr;      // [S][P] count
  DeviceModel clmodel;
  uint32_t* cltab = nullptr;   // [S][P][P][32] exact CL predictor decisions by the 10-bit d' feature, or null
};

// what a captured search graph depends on
struct GraphKey {
  const void* q;
  const void *ids, *dist, *qdist, *probes, *bits, *coarse, *status;
  const void *kptr, *npptr;  // device per-query sizes (AMP_SEARCH_DEVICE_SIZES) or null
  void* stream;
  int64_t nq;
  int32_t k, nprobe, kind, fixed_bits;
  uint32_t allowed;
  int64_t margin;
  int32_t lut_dtype;
  uint64_t ws_gen, model_gen;
  int64_t chunk, chunk1;
  size_t capq;
  int32_t wpr;
  int32_t q_dtype;
  int32_t queue;
  int32_t cl_policy, cl_bits;
  const void *cl_dist, *cl_bits_out;
  int32_t gran;
  bool operator==(const GraphKey& o) const {
    return q == o.q && ids == o.ids && dist == o.dist && qdist == o.qdist && probes == o.probes &&
           bits == o.bits && coarse == o.coarse && status == o.status && kptr == o.kptr && npptr == o.npptr &&
           stream == o.stream && nq == o.nq && k == o.k &&
           nprobe == o.nprobe && kind == o.kind && fixed_bits == o.fixed_bits && allowed == o.allowed &&
           margin == o.margin && lut_dtype == o.lut_dtype && ws_gen == o.ws_gen && model_gen == o.model_gen &&
           chunk == o.chunk && chunk1 == o.chunk1 && capq == o.capq && wpr == o.wpr &&
           q_dtype == o.q_dtype && queue == o.queue && cl_policy == o.cl_policy && cl_bits == o.cl_bits &&
           cl_dist == o.cl_dist && cl_bits_out == o.cl_bits_out && gran == o.gran;
  }
};
struct GraphSlot {
  GraphKey key;
  hipGraphExec_t exec;
  uint64_t last_use;
};
constexpr size_t kMaxGraphs = 32;  // captured searches kept per scratch space (least recently used go)

// Scratch of one search: the index's own (grown on demand), a serving slot's
// (reserved at server creation), or carved out of the library's fixed
// scratch array (allocation-free entry point: never grown or freed).
struct Workspace {
  std::vector<void*> blocks;   // device allocations (empty for a fixed workspace)
  bool fixed = false;          // carved out of the fixed scratch array
  size_t cap_nq = 0, cap_np = 0, cap_k = 0;
  uint64_t generation = 0;     // bumped whenever the buffers move
  hipEvent_t ev_done = nullptr;  // end of the last search on this scratch (null: not tracked)
  std::vector<GraphSlot> graphs;  // captured searches on this scratch (least recently used go)
  // per query
  float* queries = nullptr;    // [nq][d] (host-mode staging, converted BF16 queries)
  uint16_t* qraw = nullptr;    // [nq][d] BF16 queries staged from the host
  int32_t* hstage = nullptr;   // pinned host [2][nq]: per-query k and nprobe on their way up
  hipEvent_t ev_stage = nullptr;  // the last upload from hstage has run
  int32_t* kq = nullptr;       // [nq]
  int32_t* npq = nullptr;      // [nq]
  float* qnorm = nullptr;      // [nq]
  float* coarse = nullptr;     // [nq][nlist]
  int32_t* probes = nullptr;   // [nq][npmax]
  uint8_t* pbits = nullptr;    // [nq][npmax]
  uint8_t* xbits = nullptr;    // [nq][npmax] explicit widths (uploaded)
  uint64_t* tau = nullptr;     // [nq] pruning threshold key
  int64_t* pbase = nullptr;    // [nq][npmax] exact base of each pair (integer policies)
  // inner product: the LUT is the query's (every probed list shares it), so
  // it is built once per query
  int16_t* qi16 = nullptr;     // [nq][d] queries on the operand grid
  int32_t* iptab = nullptr;    // [nq][M][256] exact integer table (FP32 policy: FP32 dot products)
  int32_t* iplo = nullptr;     // [nq][M] row minima of the integer table
  int32_t* ipspan = nullptr;   // [nq] largest row span (max - min); per-subspace widths: sum of the spans
  int64_t* iplsum = nullptr;   // [nq] sum of the row minima
  uint16_t* iptq = nullptr;    // [nq][4][M][256] quantised tables, one per width the query uses
  int32_t* ipsh = nullptr;     // [nq][4] their shifts
  int32_t* ipmask = nullptr;   // [nq] widths the query's pairs use (bit b/4 - 1)
  uint8_t* retry = nullptr;    // [nq] query takes part in the phase-2 re-run
  int64_t* tau_id = nullptr;   // [nq] id part of the re-run's bound
  // integer cluster locating (laid out when the index has a sub-space map)
  int8_t* clq = nullptr;       // [nq][S][Kp] query codes
  int32_t* clqn = nullptr;     // [nq][S][2] |vq_s|^2 at the two widths of the search
  uint32_t* clmask = nullptr;  // [nq][S][PW] sub-spaces at the low width (one bit each)
  int32_t* clcn = nullptr;     // [nlist][S][2] |vc_s|^2 at the two widths
  size_t cap_cl = 0;           // cl_layout_key of the index the buffers were laid out for
  uint32_t* ccount = nullptr;  // [nq] candidate count
  uint64_t* ckey = nullptr;    // [nq][capq]
  int64_t* cid = nullptr;      // [nq][capq]
  // queue (buckets are class-major: b = cls * nlist + list)
  int32_t* cnt = nullptr;      // [2][kQSub][NB] pairs per bucket and sub-counter
  int32_t* rank = nullptr;     // [2][nq*npmax] rank of a pair inside its bucket
  int4* units = nullptr;       // [2][max_units] work units
  int64_t cap_units = 0;
  int64_t* pairoff = nullptr;  // [2][NB+1]
  int64_t* unitoff = nullptr;  // [2][NB+1]
  int32_t* sorted = nullptr;   // [2][nq*npmax]
  uint32_t* counters = nullptr;// [2][kNCls+1][kQueueSlot] unit counters
  int32_t* flags = nullptr;    // [4]: error bits, phase-2 re-run requested (two rounds), -
  int32_t* status = nullptr;   // [1] device-side status word of the last search
  uint64_t* work = nullptr;    // [4]: phase-2 code bytes scanned, live pairs, dead pairs, -
  // outputs staged for host mode
  int64_t* o_ids = nullptr;
  float* o_dist = nullptr;
  int64_t* o_qdist = nullptr;
  size_t capq = 0;
};

}  // namespace amp

struct amp_index {
  // host copies
  int32_t d = 0, M = 0, dsub = 0, nlist = 0, metric = 0, grid_kind = 0, grid_e = 0;
  int64_t n = 0, max_list = 0;
  std::vector<float> centroids, codebook;
  std::vector<int64_t> offsets, ids;
  std::vector<uint8_t> codes;
  std::vector<int32_t> radq, sizes;
  // predictor (host copy)
  bool has_model = false;
  int32_t n_sv = 0;
  std::vector<int32_t> sv, beta, table;
  int64_t beta0 = 0, feat_lo[5] = {}, feat_mul[5] = {}, theta[3] = {};
  uint64_t g_mul = 0;
  // sub-space map of reduced-precision cluster locating (host copy)
  bool has_clmap = false;
  int32_t cl_S = 0, cl_P = 0, cl_w = 0, cl_ec = 0;
  float cl_o = 0.f;
  std::vector<int8_t> cl_codes;                   // [nlist][d]
  std::vector<int32_t> cl_assign, cl_centre, cl_radius, cl_count;
  // CL predictor (host copy)
  bool has_cl_model = false;
  int32_t cl_n_sv = 0;
  std::vector<int32_t> cl_sv, cl_beta, cl_table;
  int64_t cl_beta0 = 0, cl_feat_lo[5] = {}, cl_feat_mul[5] = {}, cl_theta[3] = {};
  uint64_t cl_g_mul = 0;
  bool dev_cl_stale = true;    // the device copy of the map / CL predictor is out of date
  // device side
  amp::DeviceIndex dev;
  bool dev_model_stale = true;
  amp::Workspace ws;
  uint64_t model_generation = 0, graph_clock = 0;
  // search schedules chosen by the autotuner, by (policy kind, batch bucket);
  // while tuning, tune_force replaces the lookup
  std::vector<amp_tune_entry> tune;
  bool tune_forcing = false;
  amp_tune_entry tune_force{};
  std::mutex mu;
};

namespace amp {

// -------------------------------------------------------------- errors
amp_status set_error(amp_status s, const char* fmt, ...);
// a host entry point's body with a failed host allocation (std::bad_alloc,
// also from worker threads that rethrow it) turned into AMP_ENOMEM: no C++
// exception crosses the C ABI
template <class F>
amp_status host_guard(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return set_error(AMP_ENOMEM, "host allocation failed");
  }
}
#define AMP_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::amp::set_error(AMP_EDEVICE, "%s failed: %s", #call,          \
                              hipGetErrorString(e_));                        \
  } while (0)

// -------------------------------------------------------------- launches
struct SearchDims {
  int nq, d, M, dsub, nlist, npmax, kmax, metric, grid_kind, grid_e;
  int kconst, npconst;   // used when the per-query arrays are null
  int wpr;               // LUT words per row
  int64_t chunk;         // list chunk length of one work unit (phase 2)
  int64_t chunk1;        // the same for the phase-1 bound (latency-bound: shorter)
  int64_t max_units;     // capacity of each phase's unit table
  size_t capq;
  const uint16_t* q_bf16;  // BF16 query rows to widen into q_conv first (null: FP32 queries)
  float* q_conv;
  bool want_work;        // count the phase-2 work (code bytes scanned, live / skipped pairs)
  int policy;            // AMP_POLICY_*
  int lut_dtype;         // AMP_LUT_* (0 = BF16)
  int gran;              // quantiser granularity: 0 one width per pair, 1 per-(pair, subspace) widths
  int noskip;            // 1: no pair skipped by its base (AMP_PAIR_SKIP=0; measurement of the full scan)
  int queue;             // scan unit queue: 0 one counter, 1 per-XCD ranges with stealing
  int fixed_bits;
  uint32_t allowed_mask;
  int64_t margin;
  const int32_t* k_dev;  // device per-query k / nprobe to check and copy into the
  const int32_t* np_dev; // workspace first (AMP_SEARCH_DEVICE_SIZES), or null
  int32_t* out_status;   // status word written at the end of the search, or null
  int reruns;            // phase-2 re-runs of overflowed queries (2; fewer only to test overflow reporting)
  const amp_lut_export* lut_export;  // test hook: every pair's LUT after the search, or null
  // cluster locating
  int cl_policy;         // AMP_CL_*
  int cl_lo, cl_hi;      // operand widths of the two classes (fixed: both the fixed width)
  int cl_S, cl_P, cl_w, cl_kp, cl_pw, cl_ec;
  float cl_o;
  const uint32_t* cl_tab;  // exact decision table of the CL predictor, or null (direct evaluation)
  int32_t* out_cl_dist;  // [nq][nlist] or null
  uint8_t* out_cl_bits;  // [nq][S][P] or null
};

struct ModelArgs {
  int32_t n_sv;
  const int32_t* sv;
  const int32_t* beta;
  const int32_t* table;
  int64_t beta0;
  int64_t feat_lo[5];
  int64_t feat_mul[5];
  uint64_t g_mul;
  int64_t theta[3];
};

// CL operand codes (host; the definition the search kernels follow)
void cl_params_host(const std::vector<float>& C, int metric, float* o, int* ec);
int8_t cl_code_host(float x, float o, int ec);

// padded bytes of one slice of CL codes (one MFMA K: 32 or 64)
inline int cl_kpad(int w) { return w <= 32 ? 32 : 64; }
// shape of a workspace's CL buffers (0: none): slices, padded slice bytes,
// mask words per (query, slice)
inline size_t cl_layout_key(const amp_index* ix) {
  if (!ix->has_clmap) return 0;
  return (size_t)ix->cl_S | ((size_t)cl_kpad(ix->cl_w) << 12) | ((size_t)((ix->cl_P + 31) / 32) << 20);
}

hipError_t launch_prep_index(const amp_index* ix, hipStream_t st);
hipError_t launch_search(const amp_index* ix, const Workspace& ws, const float* queries,
                         const SearchDims& sd, const ModelArgs& ma, const ModelArgs& clma, int64_t* out_ids,
                         float* out_dist, int64_t* out_qdist, float* out_coarse,
                         hipStream_t st, hipEvent_t* ev /* [AMP_N_STAGES+1] or null */);
// cluster locating on 8-bit codes (integer policies): order keys of the
// coarse distances into keys [nq][nlist]
hipError_t launch_cl(const amp_index* ix, const Workspace& ws, const float* queries, const SearchDims& sd,
                     const ModelArgs& clma, float* keys, hipStream_t st);
// the CL predictor's exact decision table [S][P][P][32] (bit d' feature value)
hipError_t launch_cltab(const amp_index* ix, const ModelArgs& clma, uint32_t* tab, hipStream_t st);
// the table is built when it takes at most this many bytes
constexpr size_t kClTabMaxBytes = 512ull << 20;
// index build: nearest centroid of n rows (dd floats, leading dimension ld)
// among k centroids [k][dd], with its squared distance (out_d may be null);
// xn [n] and cn [k] are scratch for the squared norms
hipError_t launch_assign(const float* X, int64_t n, int dd, int ld, const float* C, int k, float* xn, float* cn,
                         int32_t* out_a, float* out_d, hipStream_t st);
// out [n][d] = X [n][d] - C[a[i]]
hipError_t launch_residual(const float* X, const int32_t* a, const float* C, int64_t n, int d, float* out,
                           hipStream_t st);

// grow a search workspace (the index's own when w is null) to hold any search
// of at most nq queries, npmax probes and k <= kmax (a caller that must not
// stall on a reallocation while searches are in flight reserves up front);
// takes the index lock
amp_status reserve_workspace(amp_index* ix, int64_t nq, int npmax, int kmax, Workspace* w = nullptr);
// free a workspace's buffers, events and graphs (not a fixed one's buffers)
void release_workspace(Workspace& w);
// one search on a given workspace: the index's own, a serving slot's (sized
// beforehand by reserve_workspace), or a fixed one (never grown: a search that
// does not fit is rejected)
amp_status search_on(amp_index* ix, Workspace& w, const void* queries, int64_t nq, const int32_t* k,
                     const int32_t* nprobe, int32_t per_query, const amp_precision_policy* pol,
                     const amp_search_opts* opts, int64_t* out_ids, float* out_dist);
// lay the buffers of a workspace out in [base, base + bytes) (device memory)
// for searches of at most nq queries, npmax probes and k <= kmax, candidate
// capacity capq and `units` work units per phase; returns false (nothing
// set) if they do not fit.  Host-mode staging is left out.
bool carve_workspace(const amp_index* ix, Workspace& w, char* base, size_t bytes, int64_t nq, int npmax, int kmax,
                     size_t capq, int64_t units);
// candidate capacity of a search of at most kmax results (a power of two)
size_t plan_capq(int kmax);
// work units per phase of a search that keeps every list whole
inline int64_t whole_list_units(int64_t nq, int npmax) { return nq * npmax; }

// LUT words per row of the scan variants a search runs (the queue packs its
// work units to match)
int scan_wpr(int M, bool fp32, int lut_dtype, bool narrow);

}  // namespace amp
