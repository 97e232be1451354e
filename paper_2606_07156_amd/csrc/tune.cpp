// Autotuner of the search schedule: list chunk of the phase-2 and phase-1
// work units, LUT row width and LC matrix dtype, timed on the device for a
// representative batch and kept per (policy kind, batch-size bucket).
//
// The knobs change how work is cut and packed, never what is computed, so a
// tuned search returns the same results as the automatic schedule.
#include <algorithm>
#include <cstring>
#include <vector>

#include "amp_internal.h"

using namespace amp;

namespace {

int bucket_of(int64_t nq) {
  int lg = 0;
  while ((1ll << lg) < nq) ++lg;
  return lg;
}

struct Trial {
  amp_index* ix;
  const void* dq;
  int64_t nq;
  const int32_t *k, *np;
  int32_t per_query;
  amp_precision_policy pol;
  amp_search_opts opts;
  int64_t* dids;
  float* ddist;
  hipEvent_t e0, e1;
  int repeats;

  // median over `repeats` timed searches (after one untimed) of a schedule
  amp_status time(const amp_tune_entry& cfg, float* ms) {
    ix->tune_force = cfg;
    ix->tune_forcing = true;
    std::vector<float> t;
    amp_status s = amp_search(ix, dq, nq, k, np, per_query, &pol, &opts, dids, ddist);
    hipStream_t st = static_cast<hipStream_t>(opts.stream);
    for (int r = 0; r < repeats && s == AMP_OK; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) s = set_error(AMP_EDEVICE, "event record failed");
      if (s == AMP_OK) s = amp_search(ix, dq, nq, k, np, per_query, &pol, &opts, dids, ddist);
      if (s == AMP_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        s = set_error(AMP_EDEVICE, "event wait failed");
      float x = 0.f;
      if (s == AMP_OK) hipEventElapsedTime(&x, e0, e1);
      t.push_back(x);
    }
    ix->tune_forcing = false;
    if (s != AMP_OK) return s;
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    *ms = t[t.size() / 2];
    return AMP_OK;
  }
};

amp_status check_entry(const amp_tune_entry& e) {
  if (e.policy_kind < AMP_POLICY_FP32 || e.policy_kind > AMP_POLICY_EXPLICIT)
    return set_error(AMP_EINVAL, "tuning entry: bad policy kind %d", e.policy_kind);
  if (e.nq_log2 < 0 || e.nq_log2 > 24) return set_error(AMP_EINVAL, "tuning entry: nq_log2 %d", e.nq_log2);
  if (e.chunk < 0 || e.chunk1 < 0 || (e.chunk > 0 && e.chunk < 256) || (e.chunk1 > 0 && e.chunk1 < 256))
    return set_error(AMP_EINVAL, "tuning entry: chunks must be 0 or at least 256");
  if (e.narrow < -1 || e.narrow > 1) return set_error(AMP_EINVAL, "tuning entry: narrow %d", e.narrow);
  if (e.lut_dtype != 0 && e.lut_dtype != AMP_LUT_BF16 && e.lut_dtype != AMP_LUT_F16)
    return set_error(AMP_EINVAL, "tuning entry: LUT dtype %d", e.lut_dtype);
  if (e.queue < 0 || e.queue > 1) return set_error(AMP_EINVAL, "tuning entry: queue %d", e.queue);
  return AMP_OK;
}

void put_entry(amp_index* ix, const amp_tune_entry& e) {
  for (amp_tune_entry& x : ix->tune)
    if (x.policy_kind == e.policy_kind && x.nq_log2 == e.nq_log2) {
      x = e;
      return;
    }
  ix->tune.push_back(e);
}

}  // namespace

static amp_status amp_index_autotune_body(amp_index* ix, const void* queries, int64_t nq, const int32_t* k,
                                         const int32_t* nprobe, int32_t per_query, const amp_precision_policy* pol,
                                         int32_t q_dtype, int32_t repeats, amp_tune_entry* out);
extern "C" amp_status amp_index_autotune(amp_index* ix, const void* queries, int64_t nq, const int32_t* k,
                                         const int32_t* nprobe, int32_t per_query, const amp_precision_policy* pol,
                                         int32_t q_dtype, int32_t repeats, amp_tune_entry* out) {
  return host_guard([&] { return amp_index_autotune_body(ix, queries, nq, k, nprobe, per_query, pol, q_dtype, repeats, out); });
}

static amp_status amp_index_autotune_body(amp_index* ix, const void* queries, int64_t nq, const int32_t* k,
                                         const int32_t* nprobe, int32_t per_query, const amp_precision_policy* pol,
                                         int32_t q_dtype, int32_t repeats, amp_tune_entry* out) {
  if (!ix || !queries || !k || !nprobe || !pol) return set_error(AMP_EINVAL, "null argument");
  if (nq <= 0 || nq > (1 << 24)) return set_error(AMP_EINVAL, "nq %lld out of range", (long long)nq);
  if (q_dtype != AMP_F32 && q_dtype != AMP_BF16) return set_error(AMP_EINVAL, "bad query dtype %d", q_dtype);
  if (pol->kind == AMP_POLICY_EXPLICIT) return set_error(AMP_EINVAL, "the explicit policy is a test hook, not tuned");
  if (repeats < 0 || repeats > 100) return set_error(AMP_EINVAL, "repeats %d outside [0, 100]", repeats);
  int kmax = 0;
  for (int64_t i = 0; i < (per_query ? nq : 1); ++i) kmax = std::max(kmax, k[i]);
  if (kmax < 1 || kmax > AMP_MAX_K) return set_error(AMP_EINVAL, "k outside [1, %d]", AMP_MAX_K);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(AMP_EDEVICE, "no HIP device");
  }
  const size_t esz = q_dtype == AMP_BF16 ? 2 : 4;
  void* dq = nullptr;
  int64_t* dids = nullptr;
  float* ddist = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  amp_status s = AMP_OK;
  if (hipMalloc(&dq, (size_t)nq * ix->d * esz) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&dids), (size_t)nq * kmax * 8) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&ddist), (size_t)nq * kmax * 4) != hipSuccess ||
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess ||
      hipMemcpy(dq, queries, (size_t)nq * ix->d * esz, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    s = set_error(AMP_ENOMEM, "autotune: device buffers");
  }
  amp_tune_entry best{};
  best.policy_kind = pol->kind;
  best.nq_log2 = bucket_of(nq);
  best.narrow = -1;
  int trials = 0;
  if (s == AMP_OK) {
    Trial tr{ix, dq, nq, k, nprobe, per_query, *pol, {}, dids, ddist, e0, e1, repeats ? repeats : 5};
    tr.opts.mem = AMP_MEM_DEVICE;
    tr.opts.stream = st;
    tr.opts.q_dtype = q_dtype;
    float t_best = 0.f;
    s = tr.time(best, &t_best);  // the automatic schedule
    ++trials;
    best.ms_default = t_best;
    auto try_cfg = [&](const amp_tune_entry& c) {
      float t = 0.f;
      if (s != AMP_OK) return;
      s = tr.time(c, &t);
      ++trials;
      if (s == AMP_OK && t < t_best) {
        t_best = t;
        best = c;
      }
    };
    // one coordinate at a time, keeping the best so far
    const int64_t whole = std::max<int64_t>(ix->max_list, 256);
    const bool fp32 = pol->kind == AMP_POLICY_FP32;
    {
      amp_tune_entry base = best;
      for (int nw = 0; nw <= 1; ++nw) {
        const int lut = pol->lut_dtype ? pol->lut_dtype : base.lut_dtype;
        // only distinct row widths are worth timing
        if (scan_wpr(ix->M, fp32, lut, nw == 1) == scan_wpr(ix->M, fp32, lut, nw == 0) && nw == 1) continue;
        amp_tune_entry c = base;
        c.narrow = nw;
        try_cfg(c);
      }
    }
    {
      amp_tune_entry base = best;
      const int64_t cands[] = {whole, 65536, 32768, 16384, 8192, 4096};
      for (int64_t c0 : cands) {
        if (c0 != whole && c0 >= whole) continue;
        amp_tune_entry c = base;
        c.chunk = c0;
        try_cfg(c);
      }
    }
    {
      amp_tune_entry base = best;
      const int64_t cands[] = {whole, 16384, 4096, 1024};
      for (int64_t c0 : cands) {
        if (c0 != whole && c0 >= whole) continue;
        amp_tune_entry c = base;
        c.chunk1 = c0;
        try_cfg(c);
      }
    }
    if (!fp32 && !pol->lut_dtype) {
      amp_tune_entry base = best;
      for (int dtp : {AMP_LUT_BF16, AMP_LUT_F16}) {
        amp_tune_entry c = base;
        c.lut_dtype = dtp;
        try_cfg(c);
      }
    }
    {
      amp_tune_entry c = best;  // work stealing between XCD ranges
      c.queue = 1;
      try_cfg(c);
    }
    best.ms = t_best;
    best.trials = trials;
  }
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (dq) (void)hipFree(dq);
  if (dids) (void)hipFree(dids);
  if (ddist) (void)hipFree(ddist);
  if (s != AMP_OK) return s;
  {
    std::lock_guard<std::mutex> lk(ix->mu);
    put_entry(ix, best);
  }
  if (out) *out = best;
  return AMP_OK;
}

extern "C" amp_status amp_index_get_tuning(const amp_index* ix, amp_tune_entry* entries, int32_t capacity,
                                           int32_t* count) {
  if (!ix || !count) return set_error(AMP_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(const_cast<amp_index*>(ix)->mu);
  *count = (int32_t)ix->tune.size();
  if (!entries) return AMP_OK;  // size query
  if (capacity < *count) return set_error(AMP_EINVAL, "capacity %d < %d entries", capacity, *count);
  std::copy(ix->tune.begin(), ix->tune.end(), entries);
  return AMP_OK;
}

static amp_status amp_index_set_tuning_body(amp_index* ix, const amp_tune_entry* entries, int32_t count);
extern "C" amp_status amp_index_set_tuning(amp_index* ix, const amp_tune_entry* entries, int32_t count) {
  return host_guard([&] { return amp_index_set_tuning_body(ix, entries, count); });
}

static amp_status amp_index_set_tuning_body(amp_index* ix, const amp_tune_entry* entries, int32_t count) {
  if (!ix || count < 0 || (count && !entries)) return set_error(AMP_EINVAL, "bad arguments");
  for (int32_t i = 0; i < count; ++i) {
    amp_status s = check_entry(entries[i]);
    if (s != AMP_OK) return s;
  }
  std::lock_guard<std::mutex> lk(ix->mu);
  ix->tune.clear();
  for (int32_t i = 0; i < count; ++i) put_entry(ix, entries[i]);
  return AMP_OK;
}
