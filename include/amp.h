/*
 * amp.h - C ABI of the MI355X cluster-adaptive IVF-PQ search library.
 *
 * The library answers top-k nearest-neighbour queries over a cluster-based
 * product-quantised (IVF-PQ) index (paper Sec. 2.1): cluster locating (CL),
 * residual calculation (RC), look-up-table construction (LC), distance
 * calculation (DC) and top-k selection (TS), with the precision of each probed
 * cluster's LUT chosen per (query, cluster) by a support-vector regressor over
 * size, radius and query-distance features (Sec. 3.3-3.4, Sec. 4.1 PPM).
 * Every stage of a search runs in HIP kernels on one gfx950 GPU.
 *
 * Conventions
 *  - Status: every call returns AMP_OK (0) or a negative amp_status.  On error
 *    the outputs are unspecified and the index is unchanged; nothing aborts.
 *    amp_last_error() returns a thread-local message for the last failure.
 *  - Ownership: handles (amp_index) are owned by the library and released
 *    with amp_index_free().  Every buffer passed in is owned by the caller and
 *    only read (inputs) or written (outputs) during the call (host mode) or
 *    until the stream reaches the end of the call (device mode).
 *  - Memory: amp_search_opts.mem says whether queries and outputs are host or
 *    device pointers.  Host mode is synchronous.  Device mode enqueues all
 *    work on amp_search_opts.stream (a hipStream_t, NULL = default stream)
 *    and returns without waiting.
 *  - Results are ordered ascending by (distance, id).  Fewer than k
 *    candidates: the tail is padded with id -1, distance +inf, integer
 *    distance INT64_MAX.
 *  - An index is immutable once built; searches may run concurrently on
 *    different streams (they serialise on the index's scratch space).
 */
#ifndef AMP_H
#define AMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t amp_status;
enum {
  AMP_OK = 0,
  AMP_EINVAL = -1,       /* bad argument (null pointer, size out of range)    */
  AMP_ENOMEM = -2,       /* host or device allocation failed                  */
  AMP_EDEVICE = -3,      /* HIP runtime error or no usable gfx950 device      */
  AMP_EIO = -4,          /* file could not be opened / read / written         */
  AMP_EFORMAT = -5,      /* index file corrupt, truncated or wrong version     */
  AMP_EBUSY = -6,
  AMP_ECANCELED = -7,
  AMP_EUNSUPPORTED = -8, /* valid request the library does not implement      */
  AMP_EOVERFLOW = -9     /* a query's candidate buffer overflowed             */
};

enum { AMP_L2 = 0, AMP_IP = 1, AMP_L1 = 2 };    /* metric: squared L2, inner     *
                                                  * product, L1 (sum of absolute *
                                                  * differences)                 */
enum { AMP_GRID_U9 = 0, AMP_GRID_E4M3 = 1 };     /* LC operand grid             */
enum { AMP_MEM_HOST = 0, AMP_MEM_DEVICE = 1 };
enum {                                           /* precision policy kind       */
  AMP_POLICY_FP32 = 0,      /* full-precision FP32 LUT and FP32 sums           */
  AMP_POLICY_FIXED = 1,     /* every probed cluster at fixed_bits              */
  AMP_POLICY_ADAPTIVE = 2,  /* regressor picks the width per probed cluster    */
  AMP_POLICY_EXPLICIT = 3   /* caller gives the width per (query, probe rank)  */
};
enum { AMP_LUT_BF16 = 1, AMP_LUT_F16 = 2, AMP_LUT_F8E4M3 = 3 }; /* LC matrix dtype */
enum { AMP_F32 = 0, AMP_BF16 = 1 };  /* element type of query and base rows */

#define AMP_KSUB 256        /* codewords per subspace                          */
#define AMP_MAX_K 1024
#define AMP_MAX_NPROBE 256
#define AMP_MAX_NLIST 8192
#define AMP_N_FEAT 5

typedef struct amp_index amp_index;

/*
 * Arrays of an IVF-PQ index (Sec. 2.1).  All host pointers, read during
 * amp_index_from_arrays and copied.  N = list_offsets[nlist].
 *   centroids    [nlist][d] float   coarse centroids
 *   codebook     [M][256][d/M] float  residual PQ codebook shared by all lists
 *   list_offsets [nlist+1] int64    list p holds positions [off[p], off[p+1])
 *   ids          [N] int64          id of each position; strictly increasing
 *                                   inside each list (ties in the search are
 *                                   broken by id)
 *   codes        [N][M] uint8       PQ codes by position
 *   radq         [nlist] int32      list radius max ||x - c|| in grid units
 * grid_e: the LC operand grid step is h = 2^grid_e; grid_kind selects the
 * 9-bit integer grid (|v| <= 255) or the e4m3-representable integers.
 * Constraints: d % M == 0, d/M <= 8, M even, M % 4 == 0, nlist <= 8192.
 */
typedef struct amp_index_arrays {
  int32_t d, M, nlist, metric, grid_kind, grid_e;
  const float* centroids;
  const float* codebook;
  const int64_t* list_offsets;
  const int64_t* ids;
  const uint8_t* codes;
  const int32_t* radq;
} amp_index_arrays;

/*
 * Fixed-point RBF support-vector regressor of the precision predictor
 * (Sec. 3.4: Gaussian kernel read from a table at run time).  For pair
 * (q, p) with features x = {d', r1, r2, n1, n2} (Sec. 3.3):
 *   L_f = 256*k + ((y << 8) >> k) - 256,  y = x_f + 1, k = leading-bit index
 *   u_f = clamp(((L_f - feat_lo[f]) * feat_mul[f]) >> 16, 0, 1023)
 *   y   = beta0 + sum_i beta[i] * table[min(1023, (g_mul * |u - sv_i|^2) >> 32)]
 *   bits = smallest allowed b in {4,8,12} with y + margin <= theta[b/4-1],
 *          else the largest allowed width.
 * sv [n_sv][5] int32 in [0, 1023] (the feature range), beta [n_sv] int32
 * (Q20), table [1024] int32 (Q20), beta0 and theta in Q40.  n_sv <= 4096,
 * g_mul < 2^32 (else AMP_EINVAL).  Host pointers, copied.
 */
typedef struct amp_predictor_model {
  int32_t n_sv;
  const int32_t* sv;
  const int32_t* beta;
  const int32_t* table;
  int64_t beta0;
  int64_t feat_lo[AMP_N_FEAT];
  int64_t feat_mul[AMP_N_FEAT];
  uint64_t g_mul;
  int64_t theta[3];
} amp_predictor_model;

/*
 * Precision policy of a search.
 *   kind              AMP_POLICY_*
 *   fixed_bits        width for AMP_POLICY_FIXED: 4, 8, 12 or 16
 *   allowed_bits_mask bit b set => width b allowed (ADAPTIVE); 0 = all four
 *   lut_dtype         AMP_LUT_* matrix dtype of the integer LUT build
 *                     (0 = BF16).  BF16 and FP16 give the exact integer LUT
 *                     (the result does not depend on the choice).
 *                     AMP_LUT_F8E4M3 (indexes on the e4m3 operand grid, L2
 *                     or inner product; else AMP_EINVAL): the dimension
 *                     products on the FP8 MFMA, whose FP32 sums of e4m3-grid
 *                     products are not always exact; the entries are those
 *                     sums rounded to integers (quantised entries clamped
 *                     to the width), so results may differ from the exact
 *                     LUT's
 *   margin_q40        added to the regressor score before thresholding
 *   explicit_bits     host [nq][npmax] uint8 widths by probe rank (EXPLICIT)
 *   granularity       of the LUT quantiser (Sec. 5.3 finer LC precision;
 *                     integer policies): with lo_m the minimum and R_m the
 *                     range of subspace m's entries, hf(s) = 2^(s-1) (0 for
 *                     s = 0), entries Q = (T - lo_m + hf(s)) >> s and the
 *                     estimate sum_m lo_m + (sum_m Q) << s:
 *                     AMP_GRAN_PAIR (0): one width for every subspace of the
 *                       pair, s the smallest with
 *                       (max_m R_m + hf(s)) >> s <= 2^b - 1;
 *                     AMP_GRAN_SUBSPACE (1): a width per (pair, subspace):
 *                       the pair's lane budget M (2^b - 1) is shared by its
 *                       subspaces in proportion to their ranges, s the
 *                       smallest with (sum_m R_m + M hf(s)) >> s <= M (2^b - 1)
 *                       (subspace m's entries then take about
 *                       log2((R_m + hf(s)) >> s) bits; one shift for all
 *                       subspaces, since the packed sums add entries in
 *                       common units).  The predictor should be trained
 *                       with the same granularity (amp_train_params).
 */
enum { AMP_GRAN_PAIR = 0, AMP_GRAN_SUBSPACE = 1 };
typedef struct amp_precision_policy {
  int32_t kind;
  int32_t fixed_bits;
  uint32_t allowed_bits_mask;
  int32_t lut_dtype;
  int64_t margin_q40;
  const uint8_t* explicit_bits;
  int32_t granularity;
} amp_precision_policy;

/*
 * Options of a search.  Optional outputs (NULL = not wanted) live in the
 * same memory space as the main outputs (opts.mem):
 *   out_qdist  [nq][kmax] int64  integer distance estimates (-1 under FP32)
 *   out_probes [nq][npmax] int32 probed lists by rank (-1 padded)
 *   out_bits   [nq][npmax] uint8 LUT width of each probed list (32 = FP32)
 *   out_coarse [nq][nlist] float coarse (CL) distances
 * stage_ms (host, [AMP_N_STAGES] float, optional): per-stage GPU time of this
 * call from events on the stream (stages listed with AMP_N_STAGES); forces a
 * synchronisation at the end.
 * q_dtype: AMP_F32 (0) or AMP_BF16 query rows (bfloat16 bit patterns,
 * uint16); BF16 rows are widened to FP32 on the device (exact) as the first
 * step of the search, so a BF16 query searches exactly as the FP32 query of
 * the same value.
 * Per-query k / nprobe host arrays are staged through pinned memory: the
 * call does not wait for earlier searches on the stream, and the caller may
 * reuse the arrays when it returns.
 * work (host, [4] int64, optional): work of the full scan (phase 2): code
 * bytes scanned summed over the live (query, list) pairs, live pairs, pairs
 * skipped whole because their LUT base exceeds the query's bound, and the
 * bytes its work units read (each unit's list chunk once, however many
 * pairs it serves, plus its LUT sources: inner product the live pairs'
 * quantised tables, L2 / L1 the query rows and the centroid); forces a
 * synchronisation at the end (not with AMP_SEARCH_GRAPH).
 * out_status (optional, int32, same memory space as the outputs; device mode
 * also accepts pinned host memory): the status of the search as the device
 * saw it, written when the stream reaches the end of the call: AMP_OK,
 * AMP_EOVERFLOW (a query's candidates still overflowed its buffer after the
 * re-runs, or the work-unit table overflowed: results may miss candidates),
 * AMP_EINVAL (an AMP_SEARCH_DEVICE_SIZES entry was out of range: it was
 * clamped into range) or AMP_EDEVICE (internal error).  In host mode the
 * return value carries the same status.
 * kmax, npmax: with AMP_SEARCH_DEVICE_SIZES, the bounds of the device k and
 * nprobe entries (they size the outputs: [nq][kmax], [nq][npmax]).
 * lut_export (test hook, optional, device mode, integer policies, L2 or
 * inner product, not with AMP_SEARCH_GRAPH): the quantised LUT of every
 * (query, probe rank) pair as the search builds it, for the replay check of
 * the integer stages:
 *   q     [nq][npmax][M][256] uint16  entries Q (after the shift)
 *   shift [nq][npmax] int32           shift s of the pair
 *   base  [nq][npmax] int64           base (sum of the subspace minima; inner
 *                                     product: with the -qi.ci term)
 *   t     [nq][npmax][M][256] int32   optional (NULL: not wanted): the
 *                                     entries before quantisation (T; the FP8
 *                                     build's rounded FP32 results)
 * Rows of probe ranks at or beyond a query's nprobe are left unwritten.  The
 * export is an extra LUT build after the search with the same kernels'
 * arithmetic (inner product: a copy of the query's tables); the search itself
 * is unchanged.
 */
#define AMP_N_STAGES 9  /* stage_ms: CL, top-nprobe, predictor, pair bases, queue,
                           phase-1 scan (+ bound, + the full scan's queue),
                           phase-2 scan, re-runs + merge, total */
#define AMP_SEARCH_GRAPH 1u  /* flags: capture the search as a HIP graph once
                                and replay it while queries/outputs pointers,
                                sizes, policy and stream are unchanged (device
                                mode, a created stream, constant k and nprobe
                                or AMP_SEARCH_DEVICE_SIZES, no stage_ms, not
                                EXPLICIT).  Replays read the current contents
                                of the query buffer (and of the device k /
                                nprobe arrays). */
#define AMP_SEARCH_DEVICE_SIZES 2u  /* flags: k and nprobe point to device
                                arrays of nq int32 (per_query must be 1,
                                device mode); opts.kmax / opts.npmax bound
                                them.  Entries outside [1, kmax] / [1, npmax]
                                are clamped and reported through out_status
                                (AMP_EINVAL).  The search reads the arrays
                                on the stream, so a captured graph may be
                                replayed with new per-query sizes. */
typedef struct amp_lut_export {
  uint16_t* q;
  int32_t* shift;
  int64_t* base;
  int32_t* t;
} amp_lut_export;

/*
 * Cluster locating (CL) policy of a search (amp_search_opts.cl_policy):
 *   AMP_CL_FP32      FP32 coarse distances of the FP32 centroids (default)
 *   AMP_CL_FIXED     integer coarse distances of 8-bit codes, every partial
 *                    distance at cl_bits (1..8) operand bits
 *   AMP_CL_ADAPTIVE  the same with a width per (query, dimension slice,
 *                    sub-space) from the CL predictor: cl_bits (1..7, 0 = 4)
 *                    or 8 bits
 * The integer policies need the index's sub-space map (amp_index_build_cl_map;
 * ADAPTIVE also a CL predictor), else AMP_EINVAL; not with out_coarse.  See
 * amp_cl_map for the arithmetic.
 * Optional outputs (same memory space as the other outputs):
 *   out_cl_dist [nq][nlist] int32  the integer coarse distances D_i
 *   out_cl_bits [nq][S][P] uint8   the width of every (slice, sub-space)
 *                                  (ADAPTIVE)
 */
enum { AMP_CL_FP32 = 0, AMP_CL_FIXED = 1, AMP_CL_ADAPTIVE = 2 };

typedef struct amp_search_opts {
  int32_t mem;
  void* stream;
  int64_t* out_qdist;
  int32_t* out_probes;
  uint8_t* out_bits;
  float* out_coarse;
  float* stage_ms;
  uint32_t flags;
  int32_t q_dtype;
  int64_t* work;
  int32_t* out_status;
  int32_t kmax, npmax;
  const amp_lut_export* lut_export;
  int32_t cl_policy, cl_bits;
  int32_t* out_cl_dist;
  uint8_t* out_cl_bits;
} amp_search_opts;

/* Build an index handle from arrays (copied).  Validates every constraint
 * listed with amp_index_arrays, including id order inside lists. */
amp_status amp_index_from_arrays(const amp_index_arrays* arrays, amp_index** out);

/*
 * Build an IVF-PQ index (Sec. 2.1) from n host vectors base [n][d] (FP32, or
 * BF16 bit patterns with base_dtype = AMP_BF16, widened exactly) on the
 * current HIP device: k-means coarse quantiser of nlist centroids,
 * residual product quantiser of M subspaces with one 256-word codebook per
 * subspace shared by all lists, PQ codes by nearest codeword, lists stored
 * contiguously with ids increasing inside a list, per-list radius (Sec. 3.3
 * feature) in grid units, and the LC operand grid step h = 2^grid_e.
 *   ids            host [n] int64, or NULL for 0..n-1
 *   nlist, M       as in amp_index_arrays (d % M == 0, d/M <= 8, M % 4 == 0,
 *                  1 <= nlist <= min(n, 8192))
 *   kmeans_iters   Lloyd iterations of every k-means (0..1000)
 *   seed           seeds the training samples and initial centroids
 *   metric         AMP_L2, AMP_IP or AMP_L1 (the coarse quantiser and the
 *                  codebooks are trained under L2 for every metric)
 *   grid_kind      AMP_GRID_U9 or AMP_GRID_E4M3
 *   integer_data   non-zero: the vectors hold integers; centroids and
 *                  codewords are rounded to integers after training, every
 *                  vector is assigned to the rounded centroids and h = 1
 * k-means trains on at most 256 points per centroid (a seeded sample), starts
 * from the first distinct points of a seeded order, breaks ties to the lower
 * centroid index and reseeds an empty cluster with the training point
 * farthest from its centroid.  Otherwise h is the smallest power of two with
 * every codeword and residual magnitude (inner product: also every centroid
 * and vector magnitude) within the grid's largest value (255 for U9, 448 for
 * E4M3).  Distances and assignments run on the device in FP32; means, radius
 * and layout on the host (FP64 sums).  The result is an index as from
 * amp_index_from_arrays, without a predictor.  AMP_EINVAL for bad arguments,
 * AMP_EUNSUPPORTED beyond the limits, AMP_EDEVICE on a HIP failure; *out is
 * NULL on failure.
 */
typedef struct amp_build_params {
  int32_t nlist, M, kmeans_iters, metric, grid_kind, integer_data, base_dtype;
  uint64_t seed;
} amp_build_params;

amp_status amp_index_build(const void* base, int64_t n, int32_t d, const int64_t* ids,
                           const amp_build_params* params, amp_index** out);

/* Borrow the arrays of an index (pointers into the handle, valid until it is
 * freed or modified); the same layout amp_index_from_arrays takes. */
amp_status amp_index_get_arrays(const amp_index* index, amp_index_arrays* out);

/* Attach (or replace) the precision predictor of an index (copied). */
amp_status amp_index_set_predictor(amp_index* index, const amp_predictor_model* model);

/*
 * Offline fit of the precision predictor (Sec. 3.3-3.4) on training queries
 * (host [nq][d] float).  For every (query, probed list) pair of a search at
 * (k, nprobe) the trainer computes the features {d', r1, r2, n1, n2} and a
 * label: the smallest allowed width whose worst-case LUT quantisation error
 * M * 2^(s-1) (s from the quantiser of params->granularity) stays below the
 * list's margin between the query's k neighbours
 * and its non-neighbours (exact integer ADC distances on the operand grid,
 * Sec. 3.3 label definition).  It keeps n_samples pairs stratified by label,
 * fits an epsilon-SVR with the Gaussian kernel exp(-gamma |du|^2) on the
 * 10-bit feature grid by SMO (at most max_iter pair updates, tolerance tol),
 * exports it to fixed point and attaches it to the index.  Host computation
 * only; the search kernels evaluate the model.
 */
typedef struct amp_train_params {
  int32_t n_samples;          /* paper: 1280 */
  int32_t max_iter;           /* 0 = 100000 */
  double gamma, C, epsilon, tol;
  uint32_t allowed_bits_mask; /* 0 = {4, 8, 12, 16} */
  uint64_t seed;
  int32_t granularity;        /* AMP_GRAN_*: the quantiser whose error the labels bound */
} amp_train_params;

typedef struct amp_train_report {
  int64_t n_pairs;            /* labelled pairs */
  int64_t label_hist[4];      /* pairs labelled 4, 8, 12, 16 bits */
  int32_t n_samples, n_sv, smo_iterations;
  double train_rmse;          /* of the real-valued regressor on the sample */
} amp_train_report;

amp_status amp_index_train_predictor(amp_index* index, const float* train_queries, int64_t nq,
                                     int32_t k, int32_t nprobe, const amp_train_params* params,
                                     amp_train_report* report /* optional */);

/* The solver amp_index_train_predictor uses, exposed for testing: fit
 * f(x) = sum_i coef[i] K(x_i, x) + bias to targets y [l] for a host kernel
 * matrix K [l][l] (row-major, symmetric positive semi-definite) by the
 * epsilon-insensitive SVR dual with box C, tolerance tol, at most max_iter
 * pair updates.  coef [l] and bias are written; iterations may be NULL. */
amp_status amp_svr_fit(const double* K, const double* y, int32_t l, double C, double eps, double tol,
                       int32_t max_iter, double* coef, double* bias, int32_t* iterations);

/* Copy the index's predictor into caller buffers: sv [capacity][5], beta
 * [capacity], table [1024] (host).  out->n_sv is always set; if capacity is
 * below it nothing else is written and AMP_EINVAL is returned, so a first
 * call with capacity 0 sizes the buffers.  AMP_EINVAL if no predictor. */
amp_status amp_index_get_predictor(const amp_index* index, amp_predictor_model* out, int32_t* sv,
                                   int32_t* beta, int32_t* table, int32_t capacity);

/*
 * Autotuner of the search schedule.  A search's schedule (not its result:
 * results are the same under every choice) has five knobs: the list chunk of
 * a phase-2 work unit and of a phase-1 (bound) unit, the LUT row width (one
 * 32-bit word per row, or the widest packing of the lane class), the LC
 * matrix dtype (BF16 or FP16) for policies that leave it open, and the work
 * queue of the scan kernels (one counter over the cost-sorted units, or one
 * range per XCD with stealing from the neighbouring ranges).  By default
 * they follow fixed rules of the batch shape.  amp_index_autotune times
 * candidate schedules on the current device for a representative batch
 * (queries: host [nq][d], q_dtype rows; k / nprobe as in amp_search; one
 * coordinate at a time, `repeats` timed searches per trial, 0 = 5) and
 * records the fastest in the index's table under (policy kind, batch-size
 * bucket ceil(log2 nq)); later searches of that policy kind and bucket use
 * it.  Environment overrides (AMP_CHUNK, AMP_CHUNK1, AMP_NARROW) still take
 * precedence.  Not to be called while other searches run on the index.
 *   chunk, chunk1  list chunk of a phase-2 / phase-1 unit (0 = automatic)
 *   narrow         1 one-word LUT rows, 0 widest rows, -1 automatic
 *   lut_dtype      AMP_LUT_BF16 / AMP_LUT_F16 (0 = automatic)
 *   queue          0 one counter over the cost-sorted unit order; 1 the
 *                  order cut into eight contiguous ranges, one per XCD (the
 *                  units of a list stay on one XCD's L2), a workgroup taking
 *                  from its own XCD's range, then from the next ranges in
 *                  ring order once its own is used up (work stealing)
 *   ms, ms_default median time of the tuned and of the automatic schedule
 *   trials         schedules timed
 */
typedef struct amp_tune_entry {
  int32_t policy_kind, nq_log2;
  int64_t chunk, chunk1;
  int32_t narrow, lut_dtype, queue;
  float ms, ms_default;
  int32_t trials;
} amp_tune_entry;

amp_status amp_index_autotune(amp_index* index, const void* queries, int64_t nq, const int32_t* k,
                              const int32_t* nprobe, int32_t per_query, const amp_precision_policy* policy,
                              int32_t q_dtype, int32_t repeats, amp_tune_entry* out /* optional */);
/* Read the tuning table (count always set; entries NULL: size query;
 * capacity below count: nothing copied, AMP_EINVAL) or replace it (count 0
 * clears; entries are validated: chunks 0 or >= 256, narrow -1..1,
 * queue 0..1). */
amp_status amp_index_get_tuning(const amp_index* index, amp_tune_entry* entries, int32_t capacity, int32_t* count);
amp_status amp_index_set_tuning(amp_index* index, const amp_tune_entry* entries, int32_t count);

/*
 * Vector space division for cluster locating with adaptive operand precision
 * (Sec. 3.1: dimension slices, then clusters of each slice; Sec. 3.3
 * sub-space features; Sec. 4.1 the distance module's CL pass summing
 * partial distances over slices; Sec. 4.2 MSB-first operand bits).
 *
 * Codes: every centroid and query value x becomes the 8-bit signed code
 * v = clamp(round_half_even((x - o) * 2^-ec), -128, 127), x - o rounded once
 * to FP32; o is the FP32 midpoint of the centroids' value range (inner
 * product: 0) and ec the smallest exponent with every centroid value within
 * 127 * 2^ec of o.  A b-bit operand keeps the top b bits of the code (floor
 * to a multiple of 2^(8-b)).
 * Slices: S equal runs of w = d / S consecutive dimensions.  In each slice
 * the nlist centroid codes are clustered into P sub-spaces (k-means, FP64,
 * `iters` Lloyd steps from P distinct seeded starting points, empty clusters
 * reseeded from the farthest point); the centres are then rounded to
 * integers (half away from zero) and every centroid slice is assigned to its
 * nearest rounded centre (ties: lower index).  radius = ceil of the largest
 * member distance, count = members.
 * Distances: for query q, slice s of centroid i is computed at the width b of
 * its sub-space assign[i][s]; D_i = sum_s sum_t (vq_t^(b) - vc_it^(b))^2
 * (L2) or -sum_s sum_t vq_t^(b) vc_it^(b) (inner product), exact integers;
 * the probes are the nprobe smallest (D_i, i).
 * Predictor: for slice s and sub-space u the features {d', r1, r2, n1, n2}:
 * d' = |vq_s - centre_su|^2, r1 / n1 of C1 (the sub-space with the smallest
 * d', ties: lower index), r2 / n2 of u; the model is evaluated as
 * amp_predictor_model describes, and the width is the low width if
 * y <= theta[0], else 8 bits.
 *
 * amp_index_build_cl_map: host computation on the index's centroids.
 * Requires d % S == 0, d / S <= 64, 1 <= P <= min(nlist, 1024), metric L2 or
 * inner product (else AMP_EINVAL / AMP_EUNSUPPORTED).  Replaces any earlier
 * map and drops the CL predictor.
 * amp_index_get_cl_map: borrow the map (pointers into the handle, valid
 * until it is freed or the map rebuilt); AMP_EINVAL if there is none.
 *   assign [nlist][S], centre [S][P][w], radius [S][P], count [S][P] int32.
 */
typedef struct amp_cl_map {
  int32_t S, P, w;
  float o;
  int32_t ec;
  const int32_t* assign;
  const int32_t* centre;
  const int32_t* radius;
  const int32_t* count;
} amp_cl_map;

amp_status amp_index_build_cl_map(amp_index* index, int32_t S, int32_t P, int32_t iters, uint64_t seed);
amp_status amp_index_get_cl_map(const amp_index* index, amp_cl_map* out);

/* The CL predictor (same fixed-point form as amp_predictor_model; only
 * theta[0] is used): set (copied; needs a sub-space map, AMP_EINVAL
 * otherwise), get (as amp_index_get_predictor). */
amp_status amp_index_set_cl_predictor(amp_index* index, const amp_predictor_model* model);
amp_status amp_index_get_cl_predictor(const amp_index* index, amp_predictor_model* out, int32_t* sv,
                                      int32_t* beta, int32_t* table, int32_t capacity);

/*
 * Offline fit of the CL predictor (Sec. 3.3-3.4; the paper's CL setting is
 * gamma = 0.1, C = 10) on training queries (host [nq][d] float).  For each
 * query the trainer takes the full-width (8-bit) integer distances D_i and
 * the margin of every centroid against the nprobe boundary (a probed
 * centroid: D of the (nprobe+1)-th minus D_i; another: D_i minus D of the
 * nprobe-th); for slice s and sub-space u the label is the low width
 * low_bits if twice the largest change of a member's D_i caused by computing
 * its slice s at low_bits stays below the smallest member margin, else 8.
 * Empty sub-spaces give no sample.  n_samples pairs stratified by label, an
 * epsilon-SVR (gamma, C, epsilon, tol, max_iter as in amp_train_params;
 * allowed_bits_mask is ignored) fitted by SMO, exported to fixed point with
 * theta[0] halfway between the two labels, attached to the index.
 * report->label_hist[0] counts low labels, [1] full-width ones.
 */
amp_status amp_index_train_cl_predictor(amp_index* index, const float* train_queries, int64_t nq,
                                        int32_t nprobe, int32_t low_bits, const amp_train_params* params,
                                        amp_train_report* report /* optional */);

/* Copy the index to device `device` (hipGetDevice numbering) and derive the
 * device-side tables (centroid norms, grid codebook).  Called implicitly by
 * the first search on the current device. */
amp_status amp_index_to_device(amp_index* index, int32_t device);

/* Versioned binary file with a checksum per section. */
amp_status amp_index_save(const amp_index* index, const char* path);
amp_status amp_index_load(const char* path, amp_index** out);

/* Basic properties: d, M, nlist, N (any pointer may be NULL). */
amp_status amp_index_info(const amp_index* index, int32_t* d, int32_t* M,
                          int32_t* nlist, int64_t* n);

/*
 * Search nq queries ([nq][d] float, or BF16 with opts.q_dtype, row-major).  k and nprobe are host
 * arrays of nq entries when per_query != 0, else single values; kmax and
 * npmax are their maxima.  Outputs: out_ids [nq][kmax] int64 and out_dist
 * [nq][kmax] float (h^2 * integer estimate for integer policies, h * it under
 * L1, FP32 sum for the FP32 policy).  Requires 1 <= k <= AMP_MAX_K, 1 <= nprobe <=
 * min(nlist, AMP_MAX_NPROBE); AMP_POLICY_ADAPTIVE requires a predictor.
 * In device mode an FP32 query buffer must be 16-byte aligned (rows are read
 * as float4; d is a multiple of 4), a BF16 one 2-byte aligned, else
 * AMP_EINVAL.
 */
amp_status amp_search(amp_index* index, const void* queries, int64_t nq,
                      const int32_t* k, const int32_t* nprobe, int32_t per_query,
                      const amp_precision_policy* policy, const amp_search_opts* opts,
                      int64_t* out_ids, float* out_dist);

/*
 * amp_search without allocation, for callers that cannot allocate device or
 * host memory during a search: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same arguments, results and
 * errors as amp_search, with these differences:
 *  - the search's scratch is a fixed array of device memory, 64 MiB per
 *    device, that the library holds from its first use on a device until the
 *    process ends; a search that does not fit it (roughly: nq * nlist * 4 +
 *    nq * npmax * 40 + nq * capq * 16 bytes, capq the candidate capacity, at
 *    least k rounded up to a power of two) is rejected with AMP_EINVAL;
 *  - every call on a device shares that device's array: calls that overlap on
 *    one device (different streams, threads) race and give wrong results;
 *    successive calls on one stream are safe;
 *  - device mode only; per-query sizes only as device arrays
 *    (AMP_SEARCH_DEVICE_SIZES); no EXPLICIT policy, AMP_SEARCH_GRAPH,
 *    stage_ms or work;
 *  - the index must be resident on the current device with its predictor
 *    (amp_index_to_device after the last amp_index_set_predictor), else
 *    AMP_EINVAL;
 *  - long lists are not split into several work units (a batch of few
 *    queries over very long lists runs slower than with amp_search);
 *  - overflows are reported through opts.out_status only (the return value
 *    covers the enqueue).
 */
amp_status amp_search_noalloc(amp_index* index, const void* queries, int64_t nq,
                              const int32_t* k, const int32_t* nprobe, int32_t per_query,
                              const amp_precision_policy* policy, const amp_search_opts* opts,
                              int64_t* out_ids, float* out_dist);

/*
 * Serving loop: single-query requests, continuously batched onto the search
 * path of the device current at creation (the paper's problem statement,
 * Sec. 1 / Sec. 2.1, served one query at a time).
 *
 * Requests are copied at submission into a pool of max_pending pinned query
 * slots: that pool is the admission bound (memory-based admission), a full
 * pool rejects with AMP_EBUSY.  A worker thread gathers queued requests of
 * one precision policy (the oldest request's) into batches of at most
 * max_batch queries and runs each as one device-mode search with per-query k
 * and nprobe.  Two batches may be in flight, each on an execution slot of its
 * own (a stream of default priority, search scratch, staging), so that their
 * searches overlap on the device.  A batch is padded to a size bucket (powers
 * of two up to 128, then multiples of 128) and its search replays a HIP graph
 * captured once per (slot, bucket, policy), the per-query k and nprobe
 * uploaded to the device with the queries.  An idle device waits up to
 * batch_window_us after the oldest request's arrival for a batch to fill (0:
 * launch at once).  Results are the same as amp_search of that query alone; a
 * batch whose search reports an error on the device (AMP_EOVERFLOW: a
 * query's candidate buffer overflowed) completes its requests with that
 * status.
 *   max_batch    1..65536 (0 = 1024)       max_pending 1..2^22 (0 = 4*max_batch)
 *   max_k        1..1024 (0 = 100)         max_nprobe  1..min(nlist, 256) (0 = that)
 *   q_dtype      AMP_F32 or AMP_BF16 query rows
 *   policy       default of requests that name none (not EXPLICIT)
 * Pinned host memory, with B the largest bucket (max_batch rounded up to its
 * bucket): max_pending * d * sizeof(row element) + 2 * B * (d * sizeof(row
 * element) + 8 + max_k * 20) bytes; device memory the same staging plus two
 * search workspaces reserved at creation for B queries, max_nprobe probes and
 * max_k results.  The index must outlive the server; other searches on it
 * are allowed (they use the index's own scratch space).
 */
typedef struct amp_server amp_server;

typedef struct amp_server_config {
  int32_t max_batch, max_pending, max_k, max_nprobe, batch_window_us, q_dtype;
  amp_precision_policy policy;
} amp_server_config;

/*
 * One request.  query: host row of d elements (q_dtype), copied during the
 * call.  out_ids [k] int64, out_dist [k] float and out_qdist [k] int64
 * (optional) are host buffers the caller keeps valid until completion; they
 * are written before done(user, AMP_OK) runs.  done (optional) runs on the
 * server's worker thread with no server lock held, once per admitted request
 * with AMP_OK, AMP_ECANCELED (outputs untouched) or the error of its batch; it
 * may submit or cancel, but must not flush or destroy the server.  policy:
 * NULL = the server's default.  arrival_ns: CLOCK_MONOTONIC time the request
 * arrived (latency is measured from it; 0 = the time of submission).
 */
typedef struct amp_request {
  const void* query;
  int32_t k, nprobe;
  int64_t* out_ids;
  float* out_dist;
  int64_t* out_qdist;
  void (*done)(void* user, amp_status status);
  void* user;
  const amp_precision_policy* policy;
  int64_t arrival_ns;
} amp_request;

/* Counters since creation or the last reset; latency percentiles over the
 * requests completed with AMP_OK in that window (arrival to results written). */
typedef struct amp_server_report {
  int64_t submitted, rejected, completed, cancelled, failed, batches, pending, in_flight;
  double elapsed_s, qps, mean_batch, p50_ms, p99_ms, max_ms;
} amp_server_report;

/* Start a server on the current device (moves the index there and reserves
 * its search scratch).  AMP_EINVAL for a bad configuration or policy. */
amp_status amp_server_create(amp_index* index, const amp_server_config* config, amp_server** out);
/* Admit a request (AMP_EBUSY when the pool is full or the server is
 * stopping; AMP_EINVAL for k, nprobe or policy out of range, nothing queued).
 * *ticket (optional) identifies it for amp_server_cancel. */
amp_status amp_server_submit(amp_server* server, const amp_request* request, uint64_t* ticket);
/* Cancel a queued request (its done runs at once with AMP_ECANCELED) or an
 * in-flight one (its results are dropped; done runs at completion with
 * AMP_ECANCELED).  AMP_EINVAL if the ticket is neither queued nor in flight. */
amp_status amp_server_cancel(amp_server* server, uint64_t ticket);
/* Block until every admitted request has completed (not from a callback). */
amp_status amp_server_flush(amp_server* server);
/* Read the counters; reset != 0 starts a new window. */
amp_status amp_server_stats(amp_server* server, amp_server_report* out, int32_t reset);
/* Stop admission, finish every admitted request, join the worker, free. */
void amp_server_destroy(amp_server* server);

void amp_index_free(amp_index* index);
const char* amp_status_str(amp_status status);
const char* amp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMP_H */
