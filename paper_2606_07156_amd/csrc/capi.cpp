// C ABI of the adaptive-precision IVF-PQ search: argument validation, index
// residency on the device, the index file format and the search driver.  All
// arithmetic of a search runs in the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <type_traits>

#include "amp_internal.h"

namespace amp {

static thread_local char g_err[512] = "";

amp_status set_error(amp_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

static size_t env_size(const char* name, size_t dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  long long x = atoll(v);
  return x > 0 ? (size_t)x : dflt;
}

template <typename T>
static amp_status dalloc(T** p, size_t n, std::vector<void*>* track = nullptr) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
  if (e != hipSuccess) {
    hipGetLastError();
    return set_error(AMP_ENOMEM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
  }
  if (track) track->push_back(*p);
  return AMP_OK;
}

static void free_device_index(DeviceIndex& d) {
  void* ptrs[] = {d.centroids, d.cnorm, d.codebook, d.bsw, d.bsw16, d.bsw8, d.cbi16, d.ci16, d.lorder, d.lpos, d.codes, d.ids,
                  d.offsets, d.radq, d.model.sv, d.model.beta, d.model.table, d.clc, d.clasg, d.clz, d.clr,
                  d.cln, d.clmodel.sv, d.clmodel.beta, d.clmodel.table, d.cltab};
  for (void* p : ptrs)
    if (p) hipFree(p);
  d = DeviceIndex();
}

static void free_workspace(Workspace& w) {
  for (GraphSlot& g : w.graphs) hipGraphExecDestroy(g.exec);
  for (void* p : w.blocks) hipFree(p);
  if (w.hstage) hipHostFree(w.hstage);
  if (w.ev_stage) hipEventDestroy(w.ev_stage);
  if (w.ev_done) hipEventDestroy(w.ev_done);
  const uint64_t gen = w.generation;
  w = Workspace();
  w.generation = gen + 1;
}

void release_workspace(Workspace& w) { free_workspace(w); }

}  // namespace amp

using namespace amp;

extern "C" {

const char* amp_status_str(amp_status s) {
  switch (s) {
    case AMP_OK: return "ok";
    case AMP_EINVAL: return "invalid argument";
    case AMP_ENOMEM: return "out of memory";
    case AMP_EDEVICE: return "device error";
    case AMP_EIO: return "i/o error";
    case AMP_EFORMAT: return "bad index file";
    case AMP_EBUSY: return "busy";
    case AMP_ECANCELED: return "canceled";
    case AMP_EUNSUPPORTED: return "unsupported";
    case AMP_EOVERFLOW: return "candidate buffer overflow";
    default: return "unknown status";
  }
}

const char* amp_last_error(void) { return g_err; }

amp_status amp_index_from_arrays(const amp_index_arrays* a, amp_index** out) {
  if (!a || !out) return set_error(AMP_EINVAL, "null argument");
  *out = nullptr;
  if (!a->centroids || !a->codebook || !a->list_offsets || !a->ids || !a->codes || !a->radq)
    return set_error(AMP_EINVAL, "null array in amp_index_arrays");
  if (a->d <= 0 || a->M <= 0 || a->nlist <= 0) return set_error(AMP_EINVAL, "d, M, nlist must be positive");
  if (a->d % a->M) return set_error(AMP_EINVAL, "d (%d) must be a multiple of M (%d)", a->d, a->M);
  if (a->d / a->M > kMaxDsub) return set_error(AMP_EUNSUPPORTED, "d/M = %d > %d", a->d / a->M, kMaxDsub);
  if (a->M % 4) return set_error(AMP_EUNSUPPORTED, "M (%d) must be a multiple of 4", a->M);
  if (a->nlist > AMP_MAX_NLIST) return set_error(AMP_EINVAL, "nlist %d > %d", a->nlist, AMP_MAX_NLIST);
  if (a->metric != AMP_L2 && a->metric != AMP_IP && a->metric != AMP_L1)
    return set_error(AMP_EINVAL, "bad metric %d", a->metric);
  if (a->grid_kind != AMP_GRID_U9 && a->grid_kind != AMP_GRID_E4M3)
    return set_error(AMP_EINVAL, "bad grid kind %d", a->grid_kind);
  if (a->grid_e < -60 || a->grid_e > 60) return set_error(AMP_EINVAL, "grid exponent out of range");
  if (a->list_offsets[0] != 0) return set_error(AMP_EINVAL, "list_offsets[0] must be 0");
  for (int p = 0; p < a->nlist; ++p)
    if (a->list_offsets[p + 1] < a->list_offsets[p]) return set_error(AMP_EINVAL, "list_offsets not monotone");
  const int64_t n = a->list_offsets[a->nlist];
  if (n >= (1ll << 31)) return set_error(AMP_EUNSUPPORTED, "more than 2^31 vectors");
  for (int p = 0; p < a->nlist; ++p)
    for (int64_t i = a->list_offsets[p] + 1; i < a->list_offsets[p + 1]; ++i)
      if (a->ids[i] <= a->ids[i - 1])
        return set_error(AMP_EINVAL, "ids not strictly increasing inside list %d", p);
  amp_index* ix = new (std::nothrow) amp_index();
  if (!ix) return set_error(AMP_ENOMEM, "host allocation failed");
  try {
    ix->d = a->d;
    ix->M = a->M;
    ix->dsub = a->d / a->M;
    ix->nlist = a->nlist;
    ix->metric = a->metric;
    ix->grid_kind = a->grid_kind;
    ix->grid_e = a->grid_e;
    ix->n = n;
    for (int p = 0; p < a->nlist; ++p)
      ix->max_list = std::max<int64_t>(ix->max_list, a->list_offsets[p + 1] - a->list_offsets[p]);
    ix->centroids.assign(a->centroids, a->centroids + (size_t)a->nlist * a->d);
    ix->codebook.assign(a->codebook, a->codebook + (size_t)a->M * kKsub * ix->dsub);
    ix->offsets.assign(a->list_offsets, a->list_offsets + a->nlist + 1);
    ix->ids.assign(a->ids, a->ids + n);
    ix->codes.assign(a->codes, a->codes + (size_t)n * a->M);
    ix->radq.assign(a->radq, a->radq + a->nlist);
  } catch (...) {
    delete ix;
    return set_error(AMP_ENOMEM, "host allocation failed");
  }
  *out = ix;
  return AMP_OK;
}

static amp_status set_predictor_impl(amp_index* ix, const amp_predictor_model* m);
amp_status amp_index_set_predictor(amp_index* ix, const amp_predictor_model* m) {
  return host_guard([&] { return set_predictor_impl(ix, m); });
}

static amp_status set_predictor_impl(amp_index* ix, const amp_predictor_model* m) {
  if (!ix || !m) return set_error(AMP_EINVAL, "null argument");
  if (m->n_sv < 0 || m->n_sv > 4096) return set_error(AMP_EINVAL, "n_sv %d outside [0, 4096]", m->n_sv);
  if ((m->n_sv && (!m->sv || !m->beta)) || !m->table) return set_error(AMP_EINVAL, "null model array");
  if (m->g_mul >= (1ull << 32)) return set_error(AMP_EINVAL, "g_mul must be below 2^32");
  for (int64_t i = 0; i < 5 * (int64_t)m->n_sv; ++i)
    if (m->sv[i] < 0 || m->sv[i] > 1023)
      return set_error(AMP_EINVAL, "support vector coordinate %d outside the feature range [0, 1023]", m->sv[i]);
  // the copies first (they may fail), then the index changes at once
  std::vector<int32_t> sv(m->sv, m->sv + 5 * (size_t)m->n_sv), beta(m->beta, m->beta + m->n_sv),
      table(m->table, m->table + kTableN);
  std::lock_guard<std::mutex> lk(ix->mu);
  ix->n_sv = m->n_sv;
  ix->sv.swap(sv);
  ix->beta.swap(beta);
  ix->table.swap(table);
  ix->beta0 = m->beta0;
  for (int f = 0; f < 5; ++f) {
    ix->feat_lo[f] = m->feat_lo[f];
    ix->feat_mul[f] = m->feat_mul[f];
  }
  for (int i = 0; i < 3; ++i) ix->theta[i] = m->theta[i];
  ix->g_mul = m->g_mul;
  ix->has_model = true;
  ix->dev_model_stale = true;
  ix->model_generation++;
  return AMP_OK;
}

amp_status amp_index_get_predictor(const amp_index* ix, amp_predictor_model* m, int32_t* sv, int32_t* beta,
                                   int32_t* table, int32_t capacity) {
  if (!ix || !m) return set_error(AMP_EINVAL, "null argument");
  if (!ix->has_model) return set_error(AMP_EINVAL, "index has no predictor");
  m->n_sv = ix->n_sv;
  if (capacity < ix->n_sv) return set_error(AMP_EINVAL, "capacity %d below n_sv %d", capacity, ix->n_sv);
  if ((ix->n_sv && (!sv || !beta)) || !table) return set_error(AMP_EINVAL, "null output buffer");
  std::copy(ix->sv.begin(), ix->sv.end(), sv);
  std::copy(ix->beta.begin(), ix->beta.end(), beta);
  std::copy(ix->table.begin(), ix->table.end(), table);
  m->sv = sv;
  m->beta = beta;
  m->table = table;
  m->beta0 = ix->beta0;
  for (int f = 0; f < 5; ++f) m->feat_lo[f] = ix->feat_lo[f], m->feat_mul[f] = ix->feat_mul[f];
  for (int i = 0; i < 3; ++i) m->theta[i] = ix->theta[i];
  m->g_mul = ix->g_mul;
  return AMP_OK;
}

static amp_status upload_model(amp_index* ix) {
  DeviceModel& dm = ix->dev.model;
  if (dm.sv) hipFree(dm.sv);
  if (dm.beta) hipFree(dm.beta);
  if (dm.table) hipFree(dm.table);
  dm = DeviceModel();
  amp_status s;
  if ((s = dalloc(&dm.sv, 5 * (size_t)std::max(1, ix->n_sv))) != AMP_OK) return s;
  if ((s = dalloc(&dm.beta, (size_t)std::max(1, ix->n_sv))) != AMP_OK) return s;
  if ((s = dalloc(&dm.table, (size_t)kTableN)) != AMP_OK) return s;
  if (ix->n_sv) {
    AMP_HIP(hipMemcpy(dm.sv, ix->sv.data(), ix->sv.size() * 4, hipMemcpyHostToDevice));
    AMP_HIP(hipMemcpy(dm.beta, ix->beta.data(), ix->beta.size() * 4, hipMemcpyHostToDevice));
  }
  AMP_HIP(hipMemcpy(dm.table, ix->table.data(), kTableN * 4, hipMemcpyHostToDevice));
  dm.n_sv = ix->n_sv;
  ix->dev_model_stale = false;
  return AMP_OK;
}

static ModelArgs cl_model_args(const amp_index* ix) {
  ModelArgs clma{};
  if (ix->has_cl_model) {
    clma.n_sv = ix->cl_n_sv;
    clma.sv = ix->dev.clmodel.sv;
    clma.beta = ix->dev.clmodel.beta;
    clma.table = ix->dev.clmodel.table;
    clma.beta0 = ix->cl_beta0;
    for (int f = 0; f < 5; ++f) clma.feat_lo[f] = ix->cl_feat_lo[f], clma.feat_mul[f] = ix->cl_feat_mul[f];
    clma.g_mul = ix->cl_g_mul;
    for (int i = 0; i < 3; ++i) clma.theta[i] = ix->cl_theta[i];
  }
  return clma;
}

// the sub-space map of integer cluster locating (codes padded per slice to
// one MFMA K) and the CL predictor, to the index's device
static amp_status upload_cl(amp_index* ix) {
  DeviceIndex& d = ix->dev;
  void* old[] = {d.clc, d.clasg, d.clz, d.clr, d.cln, d.clmodel.sv, d.clmodel.beta, d.clmodel.table, d.cltab};
  for (void* p : old)
    if (p) hipFree(p);
  d.cltab = nullptr;
  d.clc = nullptr;
  d.clasg = nullptr;
  d.clz = nullptr;
  d.clr = d.cln = nullptr;
  d.clmodel = DeviceModel();
  if (!ix->has_clmap) {
    ix->dev_cl_stale = false;
    return AMP_OK;
  }
  const size_t nl = ix->nlist, S = ix->cl_S, P = ix->cl_P, w = ix->cl_w, kp = cl_kpad(ix->cl_w), dd = ix->d;
  std::vector<int8_t> codes(nl * S * kp, 0), cent(S * P * kp, 0);
  std::vector<uint16_t> asg(nl * S);
  for (size_t i = 0; i < nl; ++i)
    for (size_t s = 0; s < S; ++s) {
      for (size_t t = 0; t < w; ++t) codes[(i * S + s) * kp + t] = ix->cl_codes[i * dd + s * w + t];
      asg[i * S + s] = (uint16_t)ix->cl_assign[i * S + s];
    }
  for (size_t s = 0; s < S; ++s)
    for (size_t u = 0; u < P; ++u)
      for (size_t t = 0; t < w; ++t) cent[(s * P + u) * kp + t] = (int8_t)ix->cl_centre[(s * P + u) * w + t];
  amp_status st;
  if ((st = dalloc(&d.clc, codes.size())) || (st = dalloc(&d.clasg, asg.size())) ||
      (st = dalloc(&d.clz, cent.size())) || (st = dalloc(&d.clr, S * P)) || (st = dalloc(&d.cln, S * P)))
    return st;
  AMP_HIP(hipMemcpy(d.clc, codes.data(), codes.size(), hipMemcpyHostToDevice));
  AMP_HIP(hipMemcpy(d.clasg, asg.data(), asg.size() * 2, hipMemcpyHostToDevice));
  AMP_HIP(hipMemcpy(d.clz, cent.data(), cent.size(), hipMemcpyHostToDevice));
  AMP_HIP(hipMemcpy(d.clr, ix->cl_radius.data(), S * P * 4, hipMemcpyHostToDevice));
  AMP_HIP(hipMemcpy(d.cln, ix->cl_count.data(), S * P * 4, hipMemcpyHostToDevice));
  if (ix->has_cl_model) {
    DeviceModel& dm = d.clmodel;
    if ((st = dalloc(&dm.sv, 5 * (size_t)std::max(1, ix->cl_n_sv))) ||
        (st = dalloc(&dm.beta, (size_t)std::max(1, ix->cl_n_sv))) || (st = dalloc(&dm.table, (size_t)kTableN)))
      return st;
    if (ix->cl_n_sv) {
      AMP_HIP(hipMemcpy(dm.sv, ix->cl_sv.data(), ix->cl_sv.size() * 4, hipMemcpyHostToDevice));
      AMP_HIP(hipMemcpy(dm.beta, ix->cl_beta.data(), ix->cl_beta.size() * 4, hipMemcpyHostToDevice));
    }
    AMP_HIP(hipMemcpy(dm.table, ix->cl_table.data(), kTableN * 4, hipMemcpyHostToDevice));
    dm.n_sv = ix->cl_n_sv;
    // the exact decision table (searches then read one bit per sub-space
    // instead of evaluating the regressor), when it is not too large
    const size_t words = S * P * P * 32;
    if (words * 4 <= kClTabMaxBytes) {
      if ((st = dalloc(&d.cltab, words)) != AMP_OK) return st;
      const ModelArgs clma = cl_model_args(ix);
      AMP_HIP(launch_cltab(ix, clma, d.cltab, nullptr));
      AMP_HIP(hipDeviceSynchronize());
    }
  }
  ix->dev_cl_stale = false;
  return AMP_OK;
}

static amp_status to_device_locked(amp_index* ix, int device) {
  if (ix->dev.device == device && ix->dev.centroids) return AMP_OK;
  free_device_index(ix->dev);
  free_workspace(ix->ws);
  AMP_HIP(hipSetDevice(device));
  DeviceIndex& d = ix->dev;
  amp_status s;
  const size_t nl = ix->nlist, dd = ix->d, M = ix->M, n = ix->n;
  if ((s = dalloc(&d.centroids, nl * dd)) || (s = dalloc(&d.cnorm, nl)) ||
      (s = dalloc(&d.codebook, M * kKsub * ix->dsub)) || (s = dalloc(&d.bsw, (M / 2) * 16 * 64)) ||
      (s = dalloc(&d.bsw16, (M / 2) * 16 * 64)) || (s = dalloc(&d.bsw8, (M / 2) * 16 * 64)) || (s = dalloc(&d.cbi16, M * kKsub * 8)) || (s = dalloc(&d.ci16, nl * dd)) ||
      (s = dalloc(&d.lorder, nl)) || (s = dalloc(&d.lpos, nl)) ||
      (s = dalloc(&d.codes, std::max<size_t>(1, n * M))) || (s = dalloc(&d.ids, std::max<size_t>(1, n))) ||
      (s = dalloc(&d.offsets, nl + 1)) || (s = dalloc(&d.radq, nl))) {
    free_device_index(d);
    return s;
  }
  AMP_HIP(hipMemcpy(d.centroids, ix->centroids.data(), nl * dd * 4, hipMemcpyHostToDevice));
  AMP_HIP(hipMemcpy(d.codebook, ix->codebook.data(), ix->codebook.size() * 4, hipMemcpyHostToDevice));
  if (n) {
    AMP_HIP(hipMemcpy(d.codes, ix->codes.data(), n * M, hipMemcpyHostToDevice));
    AMP_HIP(hipMemcpy(d.ids, ix->ids.data(), n * 8, hipMemcpyHostToDevice));
  }
  AMP_HIP(hipMemcpy(d.offsets, ix->offsets.data(), (nl + 1) * 8, hipMemcpyHostToDevice));
  AMP_HIP(hipMemcpy(d.radq, ix->radq.data(), nl * 4, hipMemcpyHostToDevice));
  {
    // work units are enumerated largest list first (longest-processing-time
    // order for the persistent scan); index metadata, computed once
    // (AMP_LIST_ORDER=natural keeps list-id order, for comparison)
    std::vector<int32_t> order(nl), pos(nl);
    for (size_t p = 0; p < nl; ++p) order[p] = (int32_t)p;
    const char* lo_env = getenv("AMP_LIST_ORDER");
    if (!lo_env || strcmp(lo_env, "natural") != 0)
      std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return ix->offsets[x + 1] - ix->offsets[x] > ix->offsets[y + 1] - ix->offsets[y];
      });
    for (size_t i = 0; i < nl; ++i) pos[order[i]] = (int32_t)i;
    AMP_HIP(hipMemcpy(d.lorder, order.data(), nl * 4, hipMemcpyHostToDevice));
    AMP_HIP(hipMemcpy(d.lpos, pos.data(), nl * 4, hipMemcpyHostToDevice));
  }
  AMP_HIP(launch_prep_index(ix, nullptr));
  AMP_HIP(hipDeviceSynchronize());
  d.device = device;
  ix->dev_model_stale = true;
  ix->dev_cl_stale = true;
  return AMP_OK;
}

static amp_status amp_index_to_device_body(amp_index* ix, int32_t device);
amp_status amp_index_to_device(amp_index* ix, int32_t device) {
  return host_guard([&] { return amp_index_to_device_body(ix, device); });
}

static amp_status amp_index_to_device_body(amp_index* ix, int32_t device) {
  if (!ix) return set_error(AMP_EINVAL, "null index");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    hipGetLastError();
    return set_error(AMP_EDEVICE, "no HIP device");
  }
  if (device < 0 || device >= count) return set_error(AMP_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(ix->mu);
  amp_status s = to_device_locked(ix, device);
  // the predictor goes up with the index (and again after a change), so that
  // searches that must not allocate find it resident
  if (s == AMP_OK && ix->has_model && ix->dev_model_stale) s = upload_model(ix);
  if (s == AMP_OK && ix->dev_cl_stale) s = upload_cl(ix);
  return s;
}

amp_status amp_index_info(const amp_index* ix, int32_t* d, int32_t* M, int32_t* nlist, int64_t* n) {
  if (!ix) return set_error(AMP_EINVAL, "null index");
  if (d) *d = ix->d;
  if (M) *M = ix->M;
  if (nlist) *nlist = ix->nlist;
  if (n) *n = ix->n;
  return AMP_OK;
}

void amp_index_free(amp_index* ix) {
  if (!ix) return;
  if (ix->dev.device >= 0) hipSetDevice(ix->dev.device);
  free_workspace(ix->ws);
  free_device_index(ix->dev);
  delete ix;
}

// ------------------------------------------------------------------ file format
// "AMPIDX\0\1" | u32 version | i32 d, M, nlist, metric, grid_kind, grid_e | i64 n
// | u32 has_model | sections: u32 tag, u64 bytes, u64 fnv1a-64, payload.
static const char kMagic[8] = {'A', 'M', 'P', 'I', 'D', 'X', 0, 1};
static const uint32_t kVersion = 1;

static uint64_t fnv1a(const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

static bool wr(FILE* f, const void* p, size_t n) { return fwrite(p, 1, n, f) == n; }
static bool wsec(FILE* f, uint32_t tag, const void* p, size_t n) {
  uint64_t bytes = n, h = fnv1a(p, n);
  return wr(f, &tag, 4) && wr(f, &bytes, 8) && wr(f, &h, 8) && (n == 0 || wr(f, p, n));
}

amp_status amp_index_save(const amp_index* ix, const char* path) {
  if (!ix || !path) return set_error(AMP_EINVAL, "null argument");
  FILE* f = fopen(path, "wb");
  if (!f) return set_error(AMP_EIO, "cannot open %s for writing", path);
  int32_t hdr[6] = {ix->d, ix->M, ix->nlist, ix->metric, ix->grid_kind, ix->grid_e};
  // flags: 1 LUT predictor, 2 sub-space map of integer CL, 4 CL predictor
  uint32_t hm = (ix->has_model ? 1u : 0u) | (ix->has_clmap ? 2u : 0u) | (ix->has_cl_model ? 4u : 0u);
  bool ok = wr(f, kMagic, 8) && wr(f, &kVersion, 4) && wr(f, hdr, sizeof hdr) && wr(f, &ix->n, 8) && wr(f, &hm, 4);
  ok = ok && wsec(f, 1, ix->centroids.data(), ix->centroids.size() * 4);
  ok = ok && wsec(f, 2, ix->codebook.data(), ix->codebook.size() * 4);
  ok = ok && wsec(f, 3, ix->offsets.data(), ix->offsets.size() * 8);
  ok = ok && wsec(f, 4, ix->ids.data(), ix->ids.size() * 8);
  ok = ok && wsec(f, 5, ix->codes.data(), ix->codes.size());
  ok = ok && wsec(f, 6, ix->radq.data(), ix->radq.size() * 4);
  if (hm & 1) {
    int64_t scal[15];
    scal[0] = ix->n_sv;
    scal[1] = ix->beta0;
    for (int i = 0; i < 5; ++i) scal[2 + i] = ix->feat_lo[i], scal[7 + i] = ix->feat_mul[i];
    scal[12] = ix->theta[0];
    scal[13] = ix->theta[1];
    scal[14] = ix->theta[2];
    ok = ok && wsec(f, 7, scal, sizeof scal) && wsec(f, 8, &ix->g_mul, 8);
    ok = ok && wsec(f, 9, ix->sv.data(), ix->sv.size() * 4) && wsec(f, 10, ix->beta.data(), ix->beta.size() * 4);
    ok = ok && wsec(f, 11, ix->table.data(), ix->table.size() * 4);
  }
  if (hm & 2) {
    int32_t cs[5] = {ix->cl_S, ix->cl_P, ix->cl_w, ix->cl_ec, 0};
    std::memcpy(&cs[4], &ix->cl_o, 4);
    ok = ok && wsec(f, 12, cs, sizeof cs) && wsec(f, 13, ix->cl_codes.data(), ix->cl_codes.size());
    ok = ok && wsec(f, 14, ix->cl_assign.data(), ix->cl_assign.size() * 4) &&
         wsec(f, 15, ix->cl_centre.data(), ix->cl_centre.size() * 4) &&
         wsec(f, 16, ix->cl_radius.data(), ix->cl_radius.size() * 4) &&
         wsec(f, 17, ix->cl_count.data(), ix->cl_count.size() * 4);
  }
  if (hm & 4) {
    int64_t scal[15];
    scal[0] = ix->cl_n_sv;
    scal[1] = ix->cl_beta0;
    for (int i = 0; i < 5; ++i) scal[2 + i] = ix->cl_feat_lo[i], scal[7 + i] = ix->cl_feat_mul[i];
    for (int i = 0; i < 3; ++i) scal[12 + i] = ix->cl_theta[i];
    ok = ok && wsec(f, 18, scal, sizeof scal) && wsec(f, 19, &ix->cl_g_mul, 8);
    ok = ok && wsec(f, 20, ix->cl_sv.data(), ix->cl_sv.size() * 4) &&
         wsec(f, 21, ix->cl_beta.data(), ix->cl_beta.size() * 4) &&
         wsec(f, 22, ix->cl_table.data(), ix->cl_table.size() * 4);
  }
  ok = (fclose(f) == 0) && ok;
  return ok ? AMP_OK : set_error(AMP_EIO, "write to %s failed", path);
}

static amp_status rsec(FILE* f, uint32_t tag, void* p, size_t n) {
  uint32_t t;
  uint64_t bytes, h;
  if (fread(&t, 4, 1, f) != 1 || fread(&bytes, 8, 1, f) != 1 || fread(&h, 8, 1, f) != 1)
    return set_error(AMP_EFORMAT, "truncated index file (section %u header)", tag);
  if (t != tag || bytes != n) return set_error(AMP_EFORMAT, "section %u: unexpected tag/size", tag);
  if (n && fread(p, 1, n, f) != n) return set_error(AMP_EFORMAT, "truncated index file (section %u)", tag);
  if (fnv1a(p, n) != h) return set_error(AMP_EFORMAT, "checksum mismatch in section %u", tag);
  return AMP_OK;
}

// reads an index file; the handle goes to *pix as soon as it exists (the
// caller frees it on failure and closes the file)
static amp_status index_read(FILE* f, const char* path, int64_t fsize, amp_index** pix);

amp_status amp_index_load(const char* path, amp_index** out) {
  if (!path || !out) return set_error(AMP_EINVAL, "null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return set_error(AMP_EIO, "cannot open %s", path);
  int64_t fsize = -1;
  if (fseek(f, 0, SEEK_END) == 0) fsize = (int64_t)ftell(f);
  rewind(f);
  amp_index* ix = nullptr;
  const amp_status s = host_guard([&] { return index_read(f, path, fsize, &ix); });
  fclose(f);
  if (s != AMP_OK) {
    if (ix) amp_index_free(ix);
    return s;
  }
  *out = ix;
  return AMP_OK;
}

static amp_status index_read(FILE* f, const char* path, int64_t fsize, amp_index** pix) {
  char mg[8];
  uint32_t ver = 0, hm = 0;
  int32_t hdr[6];
  int64_t n = 0;
  if (fread(mg, 1, 8, f) != 8 || memcmp(mg, kMagic, 8) != 0) {
    return set_error(AMP_EFORMAT, "%s is not an index file", path);
  }
  if (fread(&ver, 4, 1, f) != 1 || ver != kVersion) {
    return set_error(AMP_EFORMAT, "index file version %u, expected %u", ver, kVersion);
  }
  if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(&n, 8, 1, f) != 1 || fread(&hm, 4, 1, f) != 1) {
    return set_error(AMP_EFORMAT, "truncated header");
  }
  const int d = hdr[0], M = hdr[1], nlist = hdr[2];
  if (d <= 0 || M <= 0 || nlist <= 0 || d % M || nlist > AMP_MAX_NLIST || n < 0 || n >= (1ll << 31)) {
    return set_error(AMP_EFORMAT, "implausible header");
  }
  // the sections must fit the file before anything is allocated for them
  const double need = 4.0 * nlist * d + 4.0 * M * kKsub * (d / M) + 8.0 * (nlist + 1) + 8.0 * n + (double)n * M;
  if (fsize >= 0 && need > (double)fsize) return set_error(AMP_EFORMAT, "header sizes exceed the file");
  std::vector<float> C((size_t)nlist * d), CB((size_t)M * kKsub * (d / M));
  std::vector<int64_t> off(nlist + 1), ids(n);
  std::vector<uint8_t> codes((size_t)n * M);
  std::vector<int32_t> radq(nlist);
  amp_status s;
  if ((s = rsec(f, 1, C.data(), C.size() * 4)) || (s = rsec(f, 2, CB.data(), CB.size() * 4)) ||
      (s = rsec(f, 3, off.data(), off.size() * 8)) || (s = rsec(f, 4, ids.data(), ids.size() * 8)) ||
      (s = rsec(f, 5, codes.data(), codes.size())) || (s = rsec(f, 6, radq.data(), radq.size() * 4))) {
    return s;
  }
  if (off[nlist] != n) {
    return set_error(AMP_EFORMAT, "list offsets do not match n");
  }
  amp_index_arrays a{d, M, nlist, hdr[3], hdr[4], hdr[5], C.data(), CB.data(), off.data(), ids.data(), codes.data(),
                     radq.data()};
  amp_index*& ix = *pix;
  if ((s = amp_index_from_arrays(&a, &ix)) != AMP_OK) {
    return s == AMP_EINVAL ? set_error(AMP_EFORMAT, "index content invalid: %s", g_err) : s;
  }
  if (hm & ~7u) {
    return set_error(AMP_EFORMAT, "unknown section flags 0x%x", hm);
  }
  // a predictor's sections: scalars, g_mul, support vectors, weights, table
  auto read_model = [&](uint32_t tag0, amp_predictor_model& m, std::vector<int32_t>& sv, std::vector<int32_t>& beta,
                        std::vector<int32_t>& table) -> amp_status {
    int64_t scal[15];
    uint64_t gm = 0;
    amp_status st;
    if ((st = rsec(f, tag0, scal, sizeof scal)) || (st = rsec(f, tag0 + 1, &gm, 8))) return st;
    const int nsv = (int)scal[0];
    if (nsv < 0 || nsv > 4096) return set_error(AMP_EFORMAT, "bad model size");
    sv.resize(5 * (size_t)nsv);
    beta.resize(nsv);
    table.resize(kTableN);
    if ((st = rsec(f, tag0 + 2, sv.data(), sv.size() * 4)) || (st = rsec(f, tag0 + 3, beta.data(), beta.size() * 4)) ||
        (st = rsec(f, tag0 + 4, table.data(), table.size() * 4)))
      return st;
    m = amp_predictor_model{};
    m.n_sv = nsv;
    m.sv = sv.data();
    m.beta = beta.data();
    m.table = table.data();
    m.beta0 = scal[1];
    for (int i = 0; i < 5; ++i) m.feat_lo[i] = scal[2 + i], m.feat_mul[i] = scal[7 + i];
    for (int i = 0; i < 3; ++i) m.theta[i] = scal[12 + i];
    m.g_mul = gm;
    return AMP_OK;
  };
  if (hm & 1) {
    int64_t scal[15];
    uint64_t gm = 0;
    if ((s = rsec(f, 7, scal, sizeof scal)) || (s = rsec(f, 8, &gm, 8))) {
      return s;
    }
    const int nsv = (int)scal[0];
    if (nsv < 0 || nsv > 4096) {
      return set_error(AMP_EFORMAT, "bad model size");
    }
    std::vector<int32_t> sv(5 * (size_t)nsv), beta(nsv), table(kTableN);
    if ((s = rsec(f, 9, sv.data(), sv.size() * 4)) || (s = rsec(f, 10, beta.data(), beta.size() * 4)) ||
        (s = rsec(f, 11, table.data(), table.size() * 4))) {
      return s;
    }
    amp_predictor_model m{};
    m.n_sv = nsv;
    m.sv = sv.data();
    m.beta = beta.data();
    m.table = table.data();
    m.beta0 = scal[1];
    for (int i = 0; i < 5; ++i) m.feat_lo[i] = scal[2 + i], m.feat_mul[i] = scal[7 + i];
    m.theta[0] = scal[12];
    m.theta[1] = scal[13];
    m.theta[2] = scal[14];
    m.g_mul = gm;
    if ((s = amp_index_set_predictor(ix, &m)) != AMP_OK) {
      return s;
    }
  }
  if (hm & 2) {
    int32_t cs[5];
    if ((s = rsec(f, 12, cs, sizeof cs)) != AMP_OK) {
      return s;
    }
    const int S = cs[0], P = cs[1], w = cs[2];
    if (S < 1 || w < 1 || S * w != d || w > 64 || P < 1 || P > std::min(nlist, 1024)) {
      return set_error(AMP_EFORMAT, "implausible sub-space map");
    }
    std::vector<int8_t> codes((size_t)nlist * d);
    std::vector<int32_t> asg((size_t)nlist * S), cen((size_t)S * P * w), rad((size_t)S * P), cnt((size_t)S * P);
    if ((s = rsec(f, 13, codes.data(), codes.size())) || (s = rsec(f, 14, asg.data(), asg.size() * 4)) ||
        (s = rsec(f, 15, cen.data(), cen.size() * 4)) || (s = rsec(f, 16, rad.data(), rad.size() * 4)) ||
        (s = rsec(f, 17, cnt.data(), cnt.size() * 4))) {
      return s;
    }
    for (int32_t a : asg)
      if (a < 0 || a >= P) {
        return set_error(AMP_EFORMAT, "sub-space index out of range");
      }
    ix->has_clmap = true;
    ix->cl_S = S;
    ix->cl_P = P;
    ix->cl_w = w;
    ix->cl_ec = cs[3];
    std::memcpy(&ix->cl_o, &cs[4], 4);
    ix->cl_codes.swap(codes);
    ix->cl_assign.swap(asg);
    ix->cl_centre.swap(cen);
    ix->cl_radius.swap(rad);
    ix->cl_count.swap(cnt);
    ix->dev_cl_stale = true;
  }
  if (hm & 4) {
    amp_predictor_model m;
    std::vector<int32_t> sv, beta, table;
    if ((s = read_model(18, m, sv, beta, table)) != AMP_OK || (s = amp_index_set_cl_predictor(ix, &m)) != AMP_OK) {
      return s;
    }
  }
  return AMP_OK;
}

// ------------------------------------------------------------------ search
}  // extern "C"

namespace amp {

// the buffers of a search workspace for at most nq queries, np probes,
// k <= kmax, candidate capacity capq and `units` work units per phase;
// `take(&ptr, count)` hands out device memory for `count` elements (an
// allocation, or a bump pointer into the fixed scratch).  host_io adds the
// host-mode staging of BF16 query rows and of the outputs.
template <class Take>
static amp_status lay_out(const amp_index* ix, Workspace& w, size_t nq, size_t np, size_t kmax, size_t capq,
                          int64_t units, bool host_io, Take&& take) {
  const size_t NB = (size_t)kNCls * ix->nlist, npairs = nq * np;
  amp_status s;
#define AMP_TAKE(ptr, n) \
  if ((s = take(ptr, (size_t)(n))) != AMP_OK) return s
  AMP_TAKE(&w.queries, nq * ix->d);
  if (host_io) AMP_TAKE(&w.qraw, nq * ix->d);
  AMP_TAKE(&w.kq, nq);
  AMP_TAKE(&w.npq, nq);
  AMP_TAKE(&w.qnorm, nq);
  AMP_TAKE(&w.coarse, nq * ix->nlist);
  AMP_TAKE(&w.probes, npairs);
  AMP_TAKE(&w.pbits, npairs);
  AMP_TAKE(&w.xbits, npairs);
  AMP_TAKE(&w.tau, nq);
  AMP_TAKE(&w.pbase, npairs);
  {
    // inner-product tables (one LUT per query), else a token allocation
    const bool ip = ix->metric == AMP_IP;
    AMP_TAKE(&w.qi16, ip ? nq * ix->d : 1);
    AMP_TAKE(&w.iptab, ip ? nq * ix->M * kKsub : 1);
    AMP_TAKE(&w.iplo, ip ? nq * ix->M : 1);
    AMP_TAKE(&w.ipspan, ip ? nq : 1);
    AMP_TAKE(&w.iplsum, ip ? nq : 1);
    AMP_TAKE(&w.iptq, ip ? nq * 4 * ix->M * kKsub : 1);
    AMP_TAKE(&w.ipsh, ip ? nq * 4 : 1);
    AMP_TAKE(&w.ipmask, ip ? nq : 1);
  }
  {
    // integer cluster locating (indexes with a sub-space map), else a token
    const bool cl = ix->has_clmap;
    const size_t S = cl ? ix->cl_S : 0, kp = cl ? cl_kpad(ix->cl_w) : 0, pw = cl ? (ix->cl_P + 31) / 32 : 0;
    AMP_TAKE(&w.clq, cl ? nq * S * kp : 1);
    AMP_TAKE(&w.clqn, cl ? nq * S * 2 : 1);
    AMP_TAKE(&w.clmask, cl ? nq * S * pw : 1);
    AMP_TAKE(&w.clcn, cl ? (size_t)ix->nlist * S * 2 : 1);
    w.cap_cl = cl_layout_key(ix);
  }
  AMP_TAKE(&w.retry, nq);
  AMP_TAKE(&w.tau_id, nq);
  AMP_TAKE(&w.ccount, nq);
  AMP_TAKE(&w.ckey, nq * capq);
  AMP_TAKE(&w.cid, nq * capq);
  AMP_TAKE(&w.cnt, 2 * kQSub * NB);
  AMP_TAKE(&w.rank, 2 * npairs);
  AMP_TAKE(&w.units, 2 * (size_t)units);
  AMP_TAKE(&w.pairoff, 2 * (NB + 1));
  AMP_TAKE(&w.unitoff, 2 * (NB + 1));
  AMP_TAKE(&w.sorted, 2 * npairs);
  AMP_TAKE(&w.counters, 2 * (size_t)(kNCls + 1) * kQueueSlot);
  AMP_TAKE(&w.flags, 4);
  AMP_TAKE(&w.status, 1);
  AMP_TAKE(&w.work, 4);
  if (host_io) {
    AMP_TAKE(&w.o_ids, nq * kmax);
    AMP_TAKE(&w.o_dist, nq * kmax);
    AMP_TAKE(&w.o_qdist, nq * kmax);
  }
#undef AMP_TAKE
  w.cap_nq = nq;
  w.cap_np = np;
  w.cap_k = kmax;
  w.capq = capq;
  w.cap_units = units;
  return AMP_OK;
}

// grow a (non-fixed) workspace; the buffers move, so captured graphs go too
static amp_status ensure_workspace(amp_index* ix, Workspace& w, size_t nq, size_t np, size_t kmax, size_t capq,
                                   int64_t units) {
  if (nq <= w.cap_nq && np <= w.cap_np && kmax <= w.cap_k && capq == w.capq && units <= w.cap_units &&
      w.cap_cl == cl_layout_key(ix))
    return AMP_OK;
  if (w.fixed) return set_error(AMP_EINVAL, "search does not fit its fixed workspace");
  nq = std::max(nq, w.cap_nq);
  np = std::max(np, w.cap_np);
  kmax = std::max(kmax, w.cap_k);
  units = std::max(units, w.cap_units);
  // the scratch space may still be in use by an earlier search
  if (w.ev_done) AMP_HIP(hipEventSynchronize(w.ev_done));
  free_workspace(w);
  std::vector<void*>* t = &w.blocks;
  auto take = [&](auto** p, size_t n) { return dalloc(p, n, t); };
  amp_status s = lay_out(ix, w, nq, np, kmax, capq, units, true, take);
  if (s != AMP_OK) {
    free_workspace(w);
    return s;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&w.hstage), 2 * nq * sizeof(int32_t), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&w.ev_stage, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&w.ev_done, hipEventDisableTiming) != hipSuccess) {
    hipGetLastError();
    free_workspace(w);
    return set_error(AMP_ENOMEM, "pinned staging allocation failed");
  }
  return AMP_OK;
}

bool carve_workspace(const amp_index* ix, Workspace& w, char* base, size_t bytes, int64_t nq, int npmax, int kmax,
                     size_t capq, int64_t units) {
  Workspace c;
  c.fixed = true;
  size_t off = 0;
  auto take = [&](auto** p, size_t n) -> amp_status {
    using E = std::remove_pointer_t<std::remove_pointer_t<decltype(p)>>;
    const size_t at = (off + 255) & ~(size_t)255;
    const size_t need = std::max<size_t>(1, n) * sizeof(E);
    if (at > bytes || need > bytes - at) return AMP_ENOMEM;
    *p = reinterpret_cast<E*>(base + at);
    off = at + need;
    return AMP_OK;
  };
  if (lay_out(ix, c, (size_t)nq, (size_t)npmax, (size_t)kmax, capq, units, false, take) != AMP_OK) return false;
  w = c;
  return true;
}

size_t plan_capq(int kmax) {
  // a power of two (the merge sorts up to capq keys in place, 16 bytes each
  // in LDS: at most 8192), at least kmax
  size_t capq = 16;
  while ((capq < env_size("AMP_CAPQ", 4096) || capq < (size_t)kmax) && capq < (1u << 13)) capq <<= 1;
  return capq;
}

// capacity of the candidate buffer, list chunk lengths and the unit-table
// size of a search (shared by the search and by workspace reservation)
struct SearchPlan {
  size_t capq;
  int64_t chunk, chunk1, max_units;
};

static SearchPlan plan_search(const amp_index* ix, int64_t nq, int npmax, int kmax, bool worst_case,
                              int64_t tuned_chunk = 0, int64_t tuned_chunk1 = 0) {
  SearchPlan p;
  p.capq = plan_capq(kmax);
  // list chunk of a work unit, phase 2 and the phase-1 bound.  Whole lists
  // when the batch has enough units to fill the chip (each chunk rebuilds
  // its pairs' LUTs, and a chunked phase 1 gives a looser bound); otherwise
  // (few queries, long lists: the streaming case) chunks sized for about four
  // (phase 2) or two (phase 1) units per workgroup slot of the chip, at least
  // 4096 vectors.  AMP_CHUNK / AMP_CHUNK1 and the autotuner's table
  // override.  The worst case (any smaller batch) is the shortest automatic
  // chunk.
  const int64_t mean_list = std::max<int64_t>(1, ix->n / ix->nlist);
  const int64_t slots = 512;  // persistent workgroups: 256 CUs x 2
  auto pick_chunk = [&](int64_t pairs, int64_t per_slot, int64_t lo, const char* env, int64_t tuned) -> int64_t {
    const int64_t c = (int64_t)env_size(env, 0);
    if (c > 0) return c;
    if (worst_case) return lo;
    if (tuned > 0) return tuned;
    return std::min<int64_t>(1 << 16, std::max<int64_t>(lo, pairs * mean_list / (per_slot * slots)));
  };
  // (every phase-1 chunk adds its own minima to the query's bound, so
  // splitting a list does not loosen the bound; each chunk rebuilds its
  // LUTs, so the autotuner may go down to 1024 where that pays)
  p.chunk = pick_chunk(nq * npmax, 4, 4096, "AMP_CHUNK", tuned_chunk);
  p.chunk1 = pick_chunk(nq, 2, 4096, "AMP_CHUNK1", tuned_chunk1);
  const int64_t max_nch = std::max<int64_t>(1, (ix->max_list + p.chunk - 1) / p.chunk);
  const int64_t max_nch1 = std::max<int64_t>(1, (ix->max_list + p.chunk1 - 1) / p.chunk1);
  p.max_units = std::max<int64_t>(nq * npmax * max_nch, nq * max_nch1);
  return p;
}

// status of a search from its device flags (the same mapping as k_status)
static amp_status flags_status(int32_t f, size_t capq) {
  if (f & 16) return set_error(AMP_EDEVICE, "internal error: scan kernel with static LDS");
  if (f & 8) return set_error(AMP_EDEVICE, "internal error: a work unit exceeded the scan tile");
  if (f & 32) return set_error(AMP_EINVAL, "a device k / nprobe entry was outside its bound (clamped)");
  if (f & 4) return set_error(AMP_EOVERFLOW, "work-unit table overflowed");
  if (f) return set_error(AMP_EOVERFLOW, "candidate buffer of %zu entries overflowed", capq);
  return AMP_OK;
}

amp_status search_on(amp_index* ix, Workspace& w, const void* queries, int64_t nq, const int32_t* k,
                     const int32_t* nprobe, int32_t per_query, const amp_precision_policy* pol,
                     const amp_search_opts* opts, int64_t* out_ids, float* out_dist) {
  if (!ix || !queries || !k || !nprobe || !pol || !opts || !out_ids || !out_dist)
    return set_error(AMP_EINVAL, "null argument");
  if (nq <= 0 || nq > (1 << 24)) return set_error(AMP_EINVAL, "nq %lld out of range", (long long)nq);
  if (opts->mem != AMP_MEM_HOST && opts->mem != AMP_MEM_DEVICE) return set_error(AMP_EINVAL, "bad mem kind");
  if (opts->q_dtype != AMP_F32 && opts->q_dtype != AMP_BF16)
    return set_error(AMP_EINVAL, "bad query dtype %d", opts->q_dtype);
  if (opts->flags & ~(AMP_SEARCH_GRAPH | AMP_SEARCH_DEVICE_SIZES))
    return set_error(AMP_EINVAL, "unknown search flags 0x%x", opts->flags);
  const bool host = opts->mem == AMP_MEM_HOST;
  const bool dev_sizes = (opts->flags & AMP_SEARCH_DEVICE_SIZES) != 0;
  const int npmax_lim = std::min(ix->nlist, AMP_MAX_NPROBE);
  int kmax = 0, npmax = 0;
  if (dev_sizes) {
    if (host || !per_query)
      return set_error(AMP_EINVAL, "AMP_SEARCH_DEVICE_SIZES needs device memory and per_query = 1");
    if (opts->kmax < 1 || opts->kmax > AMP_MAX_K)
      return set_error(AMP_EINVAL, "opts.kmax = %d outside [1, %d]", opts->kmax, AMP_MAX_K);
    if (opts->npmax < 1 || opts->npmax > npmax_lim)
      return set_error(AMP_EINVAL, "opts.npmax = %d outside [1, %d]", opts->npmax, npmax_lim);
    kmax = opts->kmax;
    npmax = opts->npmax;
  } else {
    const int64_t nk = per_query ? nq : 1;
    for (int64_t i = 0; i < nk; ++i) {
      if (k[i] < 1 || k[i] > AMP_MAX_K) return set_error(AMP_EINVAL, "k = %d outside [1, %d]", k[i], AMP_MAX_K);
      if (nprobe[i] < 1 || nprobe[i] > npmax_lim)
        return set_error(AMP_EINVAL, "nprobe = %d outside [1, %d]", nprobe[i], npmax_lim);
      kmax = std::max(kmax, k[i]);
      npmax = std::max(npmax, nprobe[i]);
    }
  }
  switch (pol->kind) {
    case AMP_POLICY_FP32: break;
    case AMP_POLICY_FIXED:
      if (pol->fixed_bits != 4 && pol->fixed_bits != 8 && pol->fixed_bits != 12 && pol->fixed_bits != 16)
        return set_error(AMP_EINVAL, "fixed_bits must be 4, 8, 12 or 16");
      break;
    case AMP_POLICY_ADAPTIVE:
      if (!ix->has_model) return set_error(AMP_EINVAL, "adaptive policy needs a predictor");
      if (pol->allowed_bits_mask & ~((1u << 4) | (1u << 8) | (1u << 12) | (1u << 16)))
        return set_error(AMP_EINVAL, "allowed_bits_mask has widths outside {4,8,12,16}");
      break;
    case AMP_POLICY_EXPLICIT:
      if (!pol->explicit_bits) return set_error(AMP_EINVAL, "explicit policy needs explicit_bits");
      for (int64_t i = 0; i < nq * npmax; ++i) {
        int b = pol->explicit_bits[i];
        if (b != 4 && b != 8 && b != 12 && b != 16) return set_error(AMP_EINVAL, "explicit width %d", b);
      }
      break;
    default: return set_error(AMP_EINVAL, "bad policy kind %d", pol->kind);
  }
  if (pol->granularity != AMP_GRAN_PAIR && pol->granularity != AMP_GRAN_SUBSPACE)
    return set_error(AMP_EINVAL, "bad quantiser granularity %d", pol->granularity);
  if (pol->lut_dtype != 0 && pol->lut_dtype != AMP_LUT_BF16 && pol->lut_dtype != AMP_LUT_F16 &&
      pol->lut_dtype != AMP_LUT_F8E4M3)
    return set_error(AMP_EINVAL, "bad LUT build dtype %d", pol->lut_dtype);
  if (pol->lut_dtype == AMP_LUT_F8E4M3 && (ix->grid_kind != AMP_GRID_E4M3 || ix->metric == AMP_L1))
    return set_error(AMP_EINVAL, "the FP8 LUT build needs an index on the e4m3 operand grid, L2 or inner product");
  if (opts->lut_export) {
    const amp_lut_export* ex = opts->lut_export;
    if (opts->mem != AMP_MEM_DEVICE || pol->kind == AMP_POLICY_FP32 || ix->metric == AMP_L1 ||
        (opts->flags & AMP_SEARCH_GRAPH) || !ex->q || !ex->shift || !ex->base)
      return set_error(AMP_EINVAL, "the LUT export needs device memory, an integer policy, L2 or inner product, "
                                   "no graph replay, and q, shift and base buffers");
  }
  const int cl_policy = opts->cl_policy;
  int cl_lo = 8, cl_hi = 8;
  if (cl_policy != AMP_CL_FP32) {
    if (cl_policy != AMP_CL_FIXED && cl_policy != AMP_CL_ADAPTIVE)
      return set_error(AMP_EINVAL, "bad cluster-locating policy %d", cl_policy);
    if (!ix->has_clmap) return set_error(AMP_EINVAL, "integer cluster locating needs a sub-space map");
    if (cl_policy == AMP_CL_ADAPTIVE && !ix->has_cl_model)
      return set_error(AMP_EINVAL, "adaptive cluster locating needs a CL predictor");
    if (opts->out_coarse) return set_error(AMP_EINVAL, "out_coarse is FP32 cluster locating's output (out_cl_dist)");
    if (cl_policy == AMP_CL_FIXED) {
      if (opts->cl_bits < 1 || opts->cl_bits > 8) return set_error(AMP_EINVAL, "cl_bits must be 1..8");
      cl_lo = cl_hi = opts->cl_bits;
    } else {
      cl_lo = opts->cl_bits ? opts->cl_bits : 4;
      if (cl_lo < 1 || cl_lo > 7) return set_error(AMP_EINVAL, "adaptive cl_bits (low width) must be 1..7");
    }
  } else if (opts->out_cl_dist || opts->out_cl_bits) {
    return set_error(AMP_EINVAL, "out_cl_dist / out_cl_bits need an integer cluster-locating policy");
  }
  if (opts->out_cl_bits && cl_policy != AMP_CL_ADAPTIVE)
    return set_error(AMP_EINVAL, "out_cl_bits needs adaptive cluster locating");
  const bool use_graph = (opts->flags & AMP_SEARCH_GRAPH) != 0;
  if (use_graph && (host || (per_query && !dev_sizes) || opts->stage_ms || opts->work ||
                    pol->kind == AMP_POLICY_EXPLICIT))
    return set_error(AMP_EINVAL, "graph replay needs device memory, constant k and nprobe or device-resident "
                                 "per-query sizes, no stage timing or work counters, and a non-explicit policy");
  if (w.fixed) {
    if (host) return set_error(AMP_EINVAL, "a fixed-scratch search takes device memory");
    if (per_query && !dev_sizes)
      return set_error(AMP_EINVAL, "a fixed-scratch search takes per-query sizes as device arrays "
                                   "(AMP_SEARCH_DEVICE_SIZES)");
    if (pol->kind == AMP_POLICY_EXPLICIT || use_graph || opts->stage_ms || opts->work)
      return set_error(AMP_EINVAL, "a fixed-scratch search takes no explicit widths, graph replay, stage "
                                   "timing or work counters");
  }
  const bool bf16 = opts->q_dtype == AMP_BF16;
  if (!host && (reinterpret_cast<uintptr_t>(queries) & (bf16 ? 1 : 15)))
    return set_error(AMP_EINVAL, "device query buffer must be %d-byte aligned", bf16 ? 2 : 16);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    hipGetLastError();
    return set_error(AMP_EDEVICE, "no HIP device");
  }
  std::lock_guard<std::mutex> lk(ix->mu);
  amp_status s;
  if (w.fixed) {
    // nothing may be allocated: the index and its predictor must be resident
    if (ix->dev.device != dev || !ix->dev.centroids)
      return set_error(AMP_EINVAL, "index is not resident on device %d (amp_index_to_device first)", dev);
    if (pol->kind == AMP_POLICY_ADAPTIVE && ix->dev_model_stale)
      return set_error(AMP_EINVAL, "predictor changed since amp_index_to_device (call it again)");
    if (cl_policy != AMP_CL_FP32 && ix->dev_cl_stale)
      return set_error(AMP_EINVAL, "sub-space map or CL predictor changed since amp_index_to_device (call it again)");
  } else {
    if ((s = to_device_locked(ix, dev)) != AMP_OK) return s;
    if (pol->kind == AMP_POLICY_ADAPTIVE && ix->dev_model_stale && (s = upload_model(ix)) != AMP_OK) return s;
    if (cl_policy != AMP_CL_FP32 && ix->dev_cl_stale && (s = upload_cl(ix)) != AMP_OK) return s;
  }
  if (w.fixed && cl_policy != AMP_CL_FP32 && w.cap_cl != cl_layout_key(ix))
    return set_error(AMP_EINVAL, "search does not fit its fixed workspace");
  // the schedule: the autotuner's entry for this policy kind and batch size,
  // if any (results do not depend on it)
  amp_tune_entry tc{};
  tc.narrow = -1;
  if (ix->tune_forcing) {
    tc = ix->tune_force;
  } else {
    int lg = 0;
    while ((1ll << lg) < nq) ++lg;
    for (const amp_tune_entry& e : ix->tune)
      if (e.policy_kind == pol->kind && e.nq_log2 == lg) tc = e;
  }
  const int lut_dtype = pol->lut_dtype ? pol->lut_dtype
                                       : (pol->kind != AMP_POLICY_FP32 ? tc.lut_dtype : 0);
  SearchPlan plan;
  if (w.fixed) {
    // whole lists: the unit table then holds at most one unit per pair
    plan.capq = w.capq;
    plan.chunk = plan.chunk1 = std::max<int64_t>(1, ix->max_list);
    plan.max_units = whole_list_units(nq, npmax);
    if ((size_t)nq > w.cap_nq || (size_t)npmax > w.cap_np || (size_t)kmax > w.cap_k || w.capq < (size_t)kmax ||
        plan.max_units > w.cap_units)
      return set_error(AMP_EINVAL, "search does not fit its fixed workspace");
  } else {
    plan = plan_search(ix, nq, npmax, kmax, false, tc.chunk, tc.chunk1);
    if ((s = ensure_workspace(ix, w, nq, npmax, kmax, plan.capq, plan.max_units)) != AMP_OK) return s;
  }
  const size_t capq = plan.capq;
  const int64_t chunk = plan.chunk, chunk1 = plan.chunk1;
  hipStream_t st = reinterpret_cast<hipStream_t>(opts->stream);
  // the scratch space is reused: start after the previous search on it
  if (w.ev_done) AMP_HIP(hipStreamWaitEvent(st, w.ev_done, 0));
  const float* qdev = static_cast<const float*>(queries);
  const uint16_t* qbf = bf16 ? static_cast<const uint16_t*>(queries) : nullptr;
  if (host) {
    if (bf16) {
      AMP_HIP(hipMemcpyAsync(w.qraw, queries, (size_t)nq * ix->d * 2, hipMemcpyHostToDevice, st));
      qbf = w.qraw;
    } else {
      AMP_HIP(hipMemcpyAsync(w.queries, queries, (size_t)nq * ix->d * 4, hipMemcpyHostToDevice, st));
      qdev = w.queries;
    }
  }
  if (bf16) qdev = w.queries;  // widened there by the first kernel
  if (per_query && !dev_sizes) {
    // through pinned staging, so that the copy is stream-ordered and the call
    // need not wait for earlier work on the stream; the staging area is free
    // once the previous upload from it has run
    AMP_HIP(hipEventSynchronize(w.ev_stage));
    std::memcpy(w.hstage, k, nq * 4);
    std::memcpy(w.hstage + nq, nprobe, nq * 4);
    AMP_HIP(hipMemcpyAsync(w.kq, w.hstage, nq * 4, hipMemcpyHostToDevice, st));
    AMP_HIP(hipMemcpyAsync(w.npq, w.hstage + nq, nq * 4, hipMemcpyHostToDevice, st));
    AMP_HIP(hipEventRecord(w.ev_stage, st));
  }
  if (pol->kind == AMP_POLICY_EXPLICIT) {
    AMP_HIP(hipMemcpyAsync(w.xbits, pol->explicit_bits, (size_t)nq * npmax, hipMemcpyHostToDevice, st));
    if (!host) AMP_HIP(hipStreamSynchronize(st));  // the host array may go away after return
  }
  SearchDims sd;
  sd.nq = (int)nq;
  sd.d = ix->d;
  sd.M = ix->M;
  sd.dsub = ix->dsub;
  sd.nlist = ix->nlist;
  sd.npmax = npmax;
  sd.kmax = kmax;
  sd.metric = ix->metric;
  sd.grid_kind = ix->grid_kind;
  sd.grid_e = ix->grid_e;
  sd.kconst = per_query ? 0 : k[0];
  sd.npconst = per_query ? 0 : nprobe[0];
  // a batch with few pairs per list (a few queries: the streaming case) fills
  // one-word LUT rows: wider rows would multiply LDS traffic per vector
  // (AMP_NARROW=0/1 forces the choice)
  {
    const char* nv = getenv("AMP_NARROW");
    const bool narrow = nv && *nv ? nv[0] == '1'
                                  : (tc.narrow >= 0 ? tc.narrow == 1 : (int64_t)nq * npmax < 4 * (int64_t)ix->nlist);
    sd.wpr = scan_wpr(ix->M, pol->kind == AMP_POLICY_FP32, lut_dtype, narrow);
  }
  sd.chunk = chunk;
  sd.chunk1 = chunk1;
  sd.q_bf16 = qbf;
  sd.q_conv = w.queries;
  sd.want_work = opts->work != nullptr;
  sd.max_units = w.cap_units;
  sd.capq = capq;
  sd.policy = pol->kind;
  sd.lut_dtype = lut_dtype;
  sd.gran = pol->granularity;
  {
    // AMP_PAIR_SKIP=0 scans every pair in full (results unchanged: a pair
    // whose base exceeds its query's bound holds no top-k vector), to measure
    // the scan's traffic without the skip
    const char* pv = getenv("AMP_PAIR_SKIP");
    sd.noskip = pv && pv[0] == '0';
  }
  {
    // scan unit queue (AMP_QUEUE=0/1 forces the choice)
    const char* qv = getenv("AMP_QUEUE");
    sd.queue = qv && *qv ? (qv[0] == '1') : (tc.queue == 1);
  }
  sd.fixed_bits = pol->fixed_bits;
  sd.allowed_mask = pol->allowed_bits_mask ? pol->allowed_bits_mask
                                           : ((1u << 4) | (1u << 8) | (1u << 12) | (1u << 16));
  sd.margin = pol->margin_q40;
  sd.k_dev = dev_sizes ? k : nullptr;
  sd.np_dev = dev_sizes ? nprobe : nullptr;
  sd.out_status = host ? nullptr : opts->out_status;
  // AMP_RERUNS (0..2) lowers the number of phase-2 re-runs, so that tests can
  // force an unresolved candidate overflow
  sd.lut_export = opts->lut_export;
  sd.reruns = (int)std::min<size_t>(2, env_size("AMP_RERUNS", 2));
  if (const char* rv = getenv("AMP_RERUNS"))
    if (rv[0] == '0') sd.reruns = 0;
  sd.cl_policy = cl_policy;
  sd.cl_lo = cl_lo;
  sd.cl_hi = cl_hi;
  sd.cl_S = ix->cl_S;
  sd.cl_P = ix->cl_P;
  sd.cl_w = ix->cl_w;
  sd.cl_kp = ix->has_clmap ? cl_kpad(ix->cl_w) : 0;
  sd.cl_pw = (ix->cl_P + 31) / 32;
  sd.cl_ec = ix->cl_ec;
  sd.cl_o = ix->cl_o;
  sd.out_cl_dist = nullptr;
  sd.out_cl_bits = nullptr;
  // host mode: the CL outputs go through temporary device buffers
  std::vector<void*> cl_tmp;
  struct TmpFree {
    std::vector<void*>& v;
    ~TmpFree() {
      for (void* p : v) hipFree(p);
    }
  } cl_tmp_free{cl_tmp};
  if (opts->out_cl_dist) {
    if (host) {
      if ((s = dalloc(&sd.out_cl_dist, (size_t)nq * ix->nlist, &cl_tmp)) != AMP_OK) return s;
    } else {
      sd.out_cl_dist = opts->out_cl_dist;
    }
  }
  if (opts->out_cl_bits) {
    if (host) {
      if ((s = dalloc(&sd.out_cl_bits, (size_t)nq * ix->cl_S * ix->cl_P, &cl_tmp)) != AMP_OK) return s;
    } else {
      sd.out_cl_bits = opts->out_cl_bits;
    }
  }
  const ModelArgs clma = cl_model_args(ix);
  // AMP_CL_TABLE=0 evaluates the CL regressor directly (same widths)
  {
    const char* tv = getenv("AMP_CL_TABLE");
    sd.cl_tab = (tv && tv[0] == '0') ? nullptr : ix->dev.cltab;
  }
  ModelArgs ma{};
  if (ix->has_model) {
    ma.n_sv = ix->n_sv;
    ma.sv = ix->dev.model.sv;
    ma.beta = ix->dev.model.beta;
    ma.table = ix->dev.model.table;
    ma.beta0 = ix->beta0;
    for (int f = 0; f < 5; ++f) ma.feat_lo[f] = ix->feat_lo[f], ma.feat_mul[f] = ix->feat_mul[f];
    ma.g_mul = ix->g_mul;
    for (int i = 0; i < 3; ++i) ma.theta[i] = ix->theta[i];
  }
  if (use_graph && st == nullptr)
    return set_error(AMP_EINVAL, "graph replay needs a created stream (the null stream cannot be captured)");
  hipEvent_t ev[AMP_N_STAGES + 1];
  const bool timed = opts->stage_ms != nullptr;
  if (timed)
    for (auto& e : ev) AMP_HIP(hipEventCreate(&e));
  // a view with the per-query pointers nulled when k and nprobe are constant
  // (the kernels then take sd.kconst / sd.npconst)
  Workspace wv;
  {
    std::vector<GraphSlot> keep;
    keep.swap(w.graphs);  // (not copied into the view)
    wv = w;
    keep.swap(w.graphs);
  }
  if (!per_query) {
    wv.kq = nullptr;
    wv.npq = nullptr;
  }
  int64_t* oi = host ? w.o_ids : out_ids;
  float* od = host ? w.o_dist : out_dist;
  int64_t* oq = host ? (opts->out_qdist ? w.o_qdist : nullptr) : opts->out_qdist;
  float* oc = (!host && opts->out_coarse) ? opts->out_coarse : nullptr;
  const hipMemcpyKind out_kind = host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  auto enqueue = [&](hipEvent_t* evs) -> hipError_t {
    hipError_t e = launch_search(ix, wv, qdev, sd, ma, clma, oi, od, oq, oc, st, evs);
    if (e != hipSuccess) return e;
    if (opts->out_probes &&
        (e = hipMemcpyAsync(opts->out_probes, w.probes, (size_t)nq * npmax * 4, out_kind, st)) != hipSuccess)
      return e;
    if (opts->out_bits && (e = hipMemcpyAsync(opts->out_bits, w.pbits, (size_t)nq * npmax, out_kind, st)) != hipSuccess)
      return e;
    return hipSuccess;
  };
  hipError_t he = hipSuccess;
  if (use_graph) {
    // captured graphs per workspace, replayed while the launch key is
    // unchanged; the least recently used one goes when the cache is full
    GraphKey key{queries, out_ids, out_dist, opts->out_qdist, opts->out_probes, opts->out_bits, opts->out_coarse,
                 opts->out_status, dev_sizes ? k : nullptr, dev_sizes ? nprobe : nullptr,
                 st, nq, per_query ? kmax : k[0], per_query ? npmax : nprobe[0], pol->kind, pol->fixed_bits,
                 sd.allowed_mask, pol->margin_q40, lut_dtype, w.generation, ix->model_generation, chunk, chunk1,
                 capq, sd.wpr, opts->q_dtype, sd.queue, cl_policy, cl_lo, opts->out_cl_dist, opts->out_cl_bits,
                 pol->granularity};
    GraphSlot* hit = nullptr;
    for (GraphSlot& g : w.graphs)
      if (g.key == key) hit = &g;
    if (!hit) {
      if (w.graphs.size() >= kMaxGraphs) {
        auto old = std::min_element(w.graphs.begin(), w.graphs.end(),
                                    [](const GraphSlot& a, const GraphSlot& b) { return a.last_use < b.last_use; });
        hipGraphExecDestroy(old->exec);
        w.graphs.erase(old);
      }
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      AMP_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
      he = enqueue(nullptr);
      hipError_t ec = hipStreamEndCapture(st, &g);
      if (he == hipSuccess) he = ec;
      if (he == hipSuccess) he = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (g) hipGraphDestroy(g);
      if (he == hipSuccess) {
        w.graphs.push_back(GraphSlot{key, ex, 0});
        hit = &w.graphs.back();
      }
    }
    if (he == hipSuccess) {
      hit->last_use = ++ix->graph_clock;
      he = hipGraphLaunch(hit->exec, st);
    }
  } else {
    he = enqueue(timed ? ev : nullptr);
  }
  if (he != hipSuccess) {
    if (timed)
      for (auto& e : ev) hipEventDestroy(e);
    return set_error(AMP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(he));
  }
  if (host && opts->out_coarse)
    AMP_HIP(hipMemcpyAsync(opts->out_coarse, w.coarse, (size_t)nq * ix->nlist * 4, hipMemcpyDeviceToHost, st));
  if (host && opts->out_cl_dist)
    AMP_HIP(hipMemcpyAsync(opts->out_cl_dist, sd.out_cl_dist, (size_t)nq * ix->nlist * 4, hipMemcpyDeviceToHost, st));
  if (host && opts->out_cl_bits)
    AMP_HIP(hipMemcpyAsync(opts->out_cl_bits, sd.out_cl_bits, (size_t)nq * ix->cl_S * ix->cl_P, hipMemcpyDeviceToHost,
                           st));
  int32_t flags[4] = {0, 0, 0, 0};
  if (host) {
    AMP_HIP(hipMemcpyAsync(out_ids, w.o_ids, (size_t)nq * kmax * 8, hipMemcpyDeviceToHost, st));
    AMP_HIP(hipMemcpyAsync(out_dist, w.o_dist, (size_t)nq * kmax * 4, hipMemcpyDeviceToHost, st));
    if (opts->out_qdist)
      AMP_HIP(hipMemcpyAsync(opts->out_qdist, w.o_qdist, (size_t)nq * kmax * 8, hipMemcpyDeviceToHost, st));
    AMP_HIP(hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st));
  }
  if (w.ev_done) AMP_HIP(hipEventRecord(w.ev_done, st));
  if (host) AMP_HIP(hipStreamSynchronize(st));
  if (timed) {
    // stages: 0 CL, 1 top-nprobe, 2 predictor, 3 pair bases, 4 queue of the
    // phase-1 bound, 5 phase-1 scan + bound + queue of the full scan, 6 full
    // scan (phase 2), 7 re-runs + merge; the last slot holds the sum
    constexpr int NS = AMP_N_STAGES - 1;
    AMP_HIP(hipEventSynchronize(ev[NS]));
    float total = 0.f;
    for (int i = 0; i < NS; ++i) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
      opts->stage_ms[i] = ms;
      total += ms;
    }
    opts->stage_ms[NS] = total;
    for (auto& e : ev) hipEventDestroy(e);
  }
  if (opts->work) {
    uint64_t wk[4];
    AMP_HIP(hipStreamSynchronize(st));
    AMP_HIP(hipMemcpy(wk, w.work, sizeof wk, hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) opts->work[i] = (int64_t)wk[i];
  }
  if (getenv("AMP_STATS") && !w.fixed) {
    // debug: candidates forwarded to the merge per query
    std::vector<uint32_t> cc(nq);
    AMP_HIP(hipStreamSynchronize(st));
    AMP_HIP(hipMemcpy(cc.data(), w.ccount, nq * 4, hipMemcpyDeviceToHost));
    double sum = 0;
    uint32_t mx = 0;
    for (uint32_t c : cc) sum += c, mx = std::max(mx, c);
    fprintf(stderr, "[amp] candidates per query: mean %.1f max %u (capacity %zu)\n", sum / nq, mx, capq);
    if (host) fprintf(stderr, "[amp] phase-2 re-runs: %d %d\n", flags[1], flags[2]);
    // pairs, work units and scanned vectors per phase and lane class
    const int ncls = pol->kind == AMP_POLICY_FP32 ? 1 : kNCls;
    const size_t NB = (size_t)ncls * ix->nlist;
    std::vector<int64_t> po(2 * (NB + 1)), uo(2 * (NB + 1));
    AMP_HIP(hipMemcpy(po.data(), w.pairoff, po.size() * 8, hipMemcpyDeviceToHost));
    AMP_HIP(hipMemcpy(uo.data(), w.unitoff, uo.size() * 8, hipMemcpyDeviceToHost));
    std::vector<int32_t> order(ix->nlist);
    AMP_HIP(hipMemcpy(order.data(), ix->dev.lorder, order.size() * 4, hipMemcpyDeviceToHost));
    for (int ph = 0; ph < 2; ++ph)
      for (int c = 0; c < ncls; ++c) {
        const int64_t* P = po.data() + ph * (NB + 1);
        const int64_t* U = uo.data() + ph * (NB + 1);
        int64_t vec = 0, maxl = 0;
        for (int b = 0; b < ix->nlist; ++b) {
          const int64_t nu = U[c * ix->nlist + b + 1] - U[c * ix->nlist + b];
          const int32_t p = order[b];
          const int64_t len = ix->offsets[p + 1] - ix->offsets[p];
          vec += nu * len;
          if (nu) maxl = std::max(maxl, len);
        }
        fprintf(stderr, "[amp] phase %d class %d: pairs %lld units %lld unit-vectors %lld longest list %lld\n", ph + 1,
                c, (long long)(P[(c + 1) * ix->nlist] - P[c * ix->nlist]),
                (long long)(U[(c + 1) * ix->nlist] - U[c * ix->nlist]), (long long)vec, (long long)maxl);
      }
  }
  if (host) {
    const amp_status fs = flags_status(flags[0], capq);
    if (opts->out_status) *opts->out_status = fs;
    return fs;
  }
  return AMP_OK;
}

amp_status reserve_workspace(amp_index* ix, int64_t nq, int npmax, int kmax, Workspace* w) {
  std::lock_guard<std::mutex> lk(ix->mu);
  const SearchPlan p = plan_search(ix, nq, npmax, kmax, true);
  return ensure_workspace(ix, w ? *w : ix->ws, nq, npmax, kmax, p.capq, p.max_units);
}

}  // namespace amp

extern "C" {

static amp_status amp_search_body(amp_index* ix, const void* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                      int32_t per_query, const amp_precision_policy* pol, const amp_search_opts* opts,
                      int64_t* out_ids, float* out_dist);
amp_status amp_search(amp_index* ix, const void* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                      int32_t per_query, const amp_precision_policy* pol, const amp_search_opts* opts,
                      int64_t* out_ids, float* out_dist) {
  return host_guard([&] { return amp_search_body(ix, queries, nq, k, nprobe, per_query, pol, opts, out_ids, out_dist); });
}

static amp_status amp_search_body(amp_index* ix, const void* queries, int64_t nq, const int32_t* k, const int32_t* nprobe,
                      int32_t per_query, const amp_precision_policy* pol, const amp_search_opts* opts,
                      int64_t* out_ids, float* out_dist) {
  if (!ix) return set_error(AMP_EINVAL, "null argument");
  return search_on(ix, ix->ws, queries, nq, k, nprobe, per_query, pol, opts, out_ids, out_dist);
}

}  // extern "C"

