// IVF-PQ index construction (paper Sec. 2.1) on the GPU: k-means coarse
// quantiser, residual product quantiser with one 256-word codebook per
// subspace shared by all lists, PQ encoding, list-contiguous layout, per-list
// size and radius (the predictor's features, Sec. 3.3), operand grid step.
//
// Conventions (the paper leaves them open):
//  * k-means trains on at most 256 points per centroid, a seeded sample; the
//    initial centroids are the first distinct points of a seeded order; a
//    fixed number of Lloyd iterations; ties to the lowest centroid index; an
//    empty cluster takes the training point farthest from its centroid;
//  * integer data: centroids and codewords rounded after training, every
//    vector re-assigned (all distances exact integers);
//  * members of a list in increasing id order;
//  * grid step h = 2^e, the smallest power of two with the largest codeword
//    or residual magnitude (inner product: also centroid and vector
//    magnitudes) within the grid's largest value (255, or 448 for e4m3);
//    integer data: h = 1;  radius max ||x - c|| in grid units, rounded.
// Distances and assignments run on the GPU (FP32 MFMA); sums and the final
// layout on the host in FP64 / integers.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "amp_internal.h"

namespace amp {
namespace {

// counter-based generator (SplitMix64) for the seeded samples and orders
inline uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int n_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h ? h : 1u, 16u));
}

template <typename F>
void parallel_for(int64_t n, F&& f) {  // f(begin, end, thread)
  // a failed host allocation (in a worker, or starting one) is rethrown once
  // every started thread has been joined
  const int T = (int)std::min<int64_t>(n_threads(), std::max<int64_t>(1, n));
  std::vector<std::thread> th;
  std::atomic<bool> oom{false};
  try {
    th.reserve(T);
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        try {
          f(n * t / T, n * (t + 1) / T, t);
        } catch (const std::bad_alloc&) {
          oom = true;
        }
      });
  } catch (...) {
    for (auto& x : th) x.join();
    throw std::bad_alloc();
  }
  for (auto& x : th) x.join();
  if (oom) throw std::bad_alloc();
}

struct Dev {  // device scratch of the build, freed on scope exit
  std::vector<void*> blocks;
  ~Dev() {
    for (void* p : blocks) (void)hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t n) {
    void* v = nullptr;
    const hipError_t e = hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) blocks.push_back(v);
    *p = static_cast<T*>(v);
    return e;
  }
};

#define AMP_BHIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return set_error(AMP_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// k-means of rows [n][dd] (host, contiguous) into k centroids; returns FP32
// centroids [k][dd]
amp_status kmeans(const float* rows, int64_t n, int dd, int k, int iters, uint64_t seed, hipStream_t st,
                  std::vector<float>& out) {
  const int64_t ntrain = std::min<int64_t>(n, (int64_t)256 * k);
  // seeded sample: the ntrain rows of smallest hash, in row order
  std::vector<int64_t> sample(n);
  std::iota(sample.begin(), sample.end(), 0);
  if (ntrain < n) {
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) key[i] = mix64(seed * 0x100000001B3ull ^ (uint64_t)i);
    std::nth_element(sample.begin(), sample.begin() + ntrain, sample.end(),
                     [&](int64_t a, int64_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
    sample.resize(ntrain);
    std::sort(sample.begin(), sample.end());
  }
  std::vector<float> S((size_t)ntrain * dd);
  for (int64_t i = 0; i < ntrain; ++i) std::memcpy(&S[(size_t)i * dd], rows + sample[i] * dd, dd * sizeof(float));
  // initial centroids: first distinct rows in a seeded order of the sample
  std::vector<int64_t> perm(ntrain);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<uint64_t> pk(ntrain);
  for (int64_t i = 0; i < ntrain; ++i) pk[i] = mix64((seed + 0x5851F42D4C957F2Dull) ^ (uint64_t)i);
  std::sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return pk[a] < pk[b] || (pk[a] == pk[b] && a < b); });
  std::vector<int64_t> picked;
  std::unordered_set<std::string> seen;
  for (int64_t i : perm) {
    std::string b(reinterpret_cast<const char*>(&S[(size_t)i * dd]), dd * sizeof(float));
    if (!seen.insert(b).second) continue;
    picked.push_back(i);
    if ((int)picked.size() == k) break;
  }
  const size_t npk = picked.size();
  for (size_t i = npk; i < (size_t)k; ++i) picked.push_back(picked[i % npk]);  // fewer distinct rows than k
  std::vector<double> C((size_t)k * dd);
  for (int c = 0; c < k; ++c)
    for (int t = 0; t < dd; ++t) C[(size_t)c * dd + t] = S[(size_t)picked[c] * dd + t];
  Dev dv;
  float *dS, *dC, *dxn, *dcn, *dd_;
  int32_t* da;
  AMP_BHIP(dv.alloc(&dS, S.size()));
  AMP_BHIP(dv.alloc(&dC, (size_t)k * dd));
  AMP_BHIP(dv.alloc(&dxn, ntrain));
  AMP_BHIP(dv.alloc(&dcn, k));
  AMP_BHIP(dv.alloc(&dd_, ntrain));
  AMP_BHIP(dv.alloc(&da, ntrain));
  AMP_BHIP(hipMemcpyAsync(dS, S.data(), S.size() * sizeof(float), hipMemcpyHostToDevice, st));
  std::vector<float> Cf((size_t)k * dd);
  std::vector<int32_t> a(ntrain);
  std::vector<float> dist(ntrain);
  for (int it = 0; it < iters; ++it) {
    for (size_t i = 0; i < Cf.size(); ++i) Cf[i] = (float)C[i];
    AMP_BHIP(hipMemcpyAsync(dC, Cf.data(), Cf.size() * sizeof(float), hipMemcpyHostToDevice, st));
    AMP_BHIP(launch_assign(dS, ntrain, dd, dd, dC, k, dxn, dcn, da, dd_, st));
    AMP_BHIP(hipMemcpyAsync(a.data(), da, ntrain * 4, hipMemcpyDeviceToHost, st));
    AMP_BHIP(hipMemcpyAsync(dist.data(), dd_, ntrain * 4, hipMemcpyDeviceToHost, st));
    AMP_BHIP(hipStreamSynchronize(st));
    // members of each cluster (counting sort), then FP64 means per cluster
    std::vector<int64_t> cnt(k + 1, 0), mem(ntrain);
    for (int64_t i = 0; i < ntrain; ++i) ++cnt[a[i] + 1];
    for (int c = 0; c < k; ++c) cnt[c + 1] += cnt[c];
    {
      std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
      for (int64_t i = 0; i < ntrain; ++i) mem[pos[a[i]]++] = i;
    }
    std::vector<double> newC(C);
    parallel_for(k, [&](int64_t c0, int64_t c1, int) {
      std::vector<double> acc(dd);
      for (int64_t c = c0; c < c1; ++c) {
        if (cnt[c + 1] == cnt[c]) continue;
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int64_t j = cnt[c]; j < cnt[c + 1]; ++j) {
          const float* x = &S[(size_t)mem[j] * dd];
          for (int t = 0; t < dd; ++t) acc[t] += x[t];
        }
        const double inv = 1.0 / (double)(cnt[c + 1] - cnt[c]);
        for (int t = 0; t < dd; ++t) newC[(size_t)c * dd + t] = acc[t] * inv;
      }
    });
    // empty clusters: the training points farthest from their centroids
    std::vector<int> empty;
    for (int c = 0; c < k; ++c)
      if (cnt[c + 1] == cnt[c]) empty.push_back(c);
    if (!empty.empty()) {
      std::vector<int64_t> far(ntrain);
      std::iota(far.begin(), far.end(), 0);
      std::stable_sort(far.begin(), far.end(), [&](int64_t x, int64_t y) { return dist[x] > dist[y]; });
      for (size_t e = 0; e < empty.size(); ++e)
        for (int t = 0; t < dd; ++t) newC[(size_t)empty[e] * dd + t] = S[(size_t)far[e % far.size()] * dd + t];
    }
    C.swap(newC);
  }
  out.resize((size_t)k * dd);
  for (size_t i = 0; i < out.size(); ++i) out[i] = (float)C[i];
  return AMP_OK;
}

}  // namespace
}  // namespace amp

using namespace amp;

static amp_status amp_index_build_body(const void* base_in, int64_t n, int32_t d, const int64_t* ids,
                                      const amp_build_params* prm, amp_index** out);
extern "C" amp_status amp_index_build(const void* base_in, int64_t n, int32_t d, const int64_t* ids,
                                      const amp_build_params* prm, amp_index** out) {
  return host_guard([&] { return amp_index_build_body(base_in, n, d, ids, prm, out); });
}

static amp_status amp_index_build_body(const void* base_in, int64_t n, int32_t d, const int64_t* ids,
                                      const amp_build_params* prm, amp_index** out) {
  if (!base_in || !prm || !out) return set_error(AMP_EINVAL, "null argument");
  *out = nullptr;
  const int nlist = prm->nlist, M = prm->M;
  if (d <= 0 || M <= 0 || nlist <= 0 || n < 1) return set_error(AMP_EINVAL, "d, M, nlist, n must be positive");
  if (n < nlist) return set_error(AMP_EINVAL, "fewer vectors (%lld) than lists (%d)", (long long)n, nlist);
  if (n >= (1ll << 31)) return set_error(AMP_EUNSUPPORTED, "more than 2^31 vectors");
  if (d % M) return set_error(AMP_EINVAL, "d (%d) must be a multiple of M (%d)", d, M);
  if (d / M > kMaxDsub) return set_error(AMP_EUNSUPPORTED, "d/M = %d > %d", d / M, kMaxDsub);
  if (M % 4) return set_error(AMP_EUNSUPPORTED, "M (%d) must be a multiple of 4", M);
  if (nlist > AMP_MAX_NLIST) return set_error(AMP_EINVAL, "nlist %d > %d", nlist, AMP_MAX_NLIST);
  if (prm->kmeans_iters < 0 || prm->kmeans_iters > 1000) return set_error(AMP_EINVAL, "kmeans_iters out of range");
  if (prm->metric != AMP_L2 && prm->metric != AMP_IP && prm->metric != AMP_L1)
    return set_error(AMP_EINVAL, "bad metric %d", prm->metric);
  if (prm->grid_kind != AMP_GRID_U9 && prm->grid_kind != AMP_GRID_E4M3)
    return set_error(AMP_EINVAL, "bad grid kind %d", prm->grid_kind);
  if (prm->base_dtype != AMP_F32 && prm->base_dtype != AMP_BF16)
    return set_error(AMP_EINVAL, "bad base dtype %d", prm->base_dtype);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return set_error(AMP_EDEVICE, "no HIP device");
  }
  const int dsub = d / M, iters = prm->kmeans_iters;
  // BF16 rows widened once (exact: the bit pattern is the top half)
  std::vector<float> widened;
  const float* base = static_cast<const float*>(base_in);
  if (prm->base_dtype == AMP_BF16) {
    widened.resize((size_t)n * d);
    const uint16_t* b16 = static_cast<const uint16_t*>(base_in);
    parallel_for((int64_t)n * d, [&](int64_t i0, int64_t i1, int) {
      for (int64_t i = i0; i < i1; ++i) {
        const uint32_t u = (uint32_t)b16[i] << 16;
        std::memcpy(&widened[i], &u, 4);
      }
    });
    base = widened.data();
  }
  hipStream_t st = nullptr;
  AMP_BHIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sg{st};
  amp_status s;
  // coarse quantiser
  std::vector<float> C;
  if ((s = kmeans(base, n, d, nlist, iters, prm->seed, st, C)) != AMP_OK) return s;
  if (prm->integer_data)
    for (float& v : C) v = std::nearbyint(v);
  // assign every vector (chunks on the device) and keep its residual sample
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(1 << 28) / (4 * d)));
  std::vector<int32_t> a(n);
  {
    Dev dv;
    float *dX, *dC, *dxn, *dcn;
    int32_t* da;
    AMP_BHIP(dv.alloc(&dX, (size_t)chunk * d));
    AMP_BHIP(dv.alloc(&dC, C.size()));
    AMP_BHIP(dv.alloc(&dxn, chunk));
    AMP_BHIP(dv.alloc(&dcn, nlist));
    AMP_BHIP(dv.alloc(&da, chunk));
    AMP_BHIP(hipMemcpyAsync(dC, C.data(), C.size() * 4, hipMemcpyHostToDevice, st));
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
      const int64_t m = std::min(chunk, n - c0);
      AMP_BHIP(hipMemcpyAsync(dX, base + c0 * d, (size_t)m * d * 4, hipMemcpyHostToDevice, st));
      AMP_BHIP(launch_assign(dX, m, d, d, dC, nlist, dxn, dcn, da, nullptr, st));
      AMP_BHIP(hipMemcpyAsync(a.data() + c0, da, m * 4, hipMemcpyDeviceToHost, st));
    }
    AMP_BHIP(hipStreamSynchronize(st));
  }
  // residual codebook: k-means per subspace on a seeded sample of residuals
  const int64_t nr = std::min<int64_t>(n, (int64_t)256 * kKsub);
  std::vector<int64_t> rs(n);
  std::iota(rs.begin(), rs.end(), 0);
  if (nr < n) {
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) key[i] = mix64((prm->seed + 1) * 0x100000001B3ull ^ (uint64_t)i);
    std::nth_element(rs.begin(), rs.begin() + nr, rs.end(),
                     [&](int64_t x, int64_t y) { return key[x] < key[y] || (key[x] == key[y] && x < y); });
    rs.resize(nr);
    std::sort(rs.begin(), rs.end());
  }
  std::vector<float> CB((size_t)M * kKsub * dsub);
  {
    std::vector<float> sub((size_t)nr * dsub), cbm;
    for (int m = 0; m < M; ++m) {
      for (int64_t i = 0; i < nr; ++i) {
        const int64_t r = rs[i];
        for (int t = 0; t < dsub; ++t)
          sub[(size_t)i * dsub + t] = base[r * d + m * dsub + t] - C[(size_t)a[r] * d + m * dsub + t];
      }
      if ((s = kmeans(sub.data(), nr, dsub, kKsub, iters, prm->seed + 1000 + m, st, cbm)) != AMP_OK) return s;
      std::copy(cbm.begin(), cbm.end(), CB.begin() + (size_t)m * kKsub * dsub);
    }
  }
  if (prm->integer_data)
    for (float& v : CB) v = std::nearbyint(v);
  // encode (residuals on the device, nearest codeword per subspace), and
  // the largest residual magnitude for the grid step
  std::vector<uint8_t> codes((size_t)n * M);
  {
    Dev dv;
    float *dX, *dR, *dC, *dCB, *dxn, *dcn;
    int32_t *da, *dcode;
    AMP_BHIP(dv.alloc(&dX, (size_t)chunk * d));
    AMP_BHIP(dv.alloc(&dR, (size_t)chunk * d));
    AMP_BHIP(dv.alloc(&dC, C.size()));
    AMP_BHIP(dv.alloc(&dCB, CB.size()));
    AMP_BHIP(dv.alloc(&dxn, chunk));
    AMP_BHIP(dv.alloc(&dcn, kKsub));
    AMP_BHIP(dv.alloc(&da, chunk));
    AMP_BHIP(dv.alloc(&dcode, chunk));
    AMP_BHIP(hipMemcpyAsync(dC, C.data(), C.size() * 4, hipMemcpyHostToDevice, st));
    AMP_BHIP(hipMemcpyAsync(dCB, CB.data(), CB.size() * 4, hipMemcpyHostToDevice, st));
    std::vector<int32_t> cm(chunk);
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
      const int64_t m = std::min(chunk, n - c0);
      AMP_BHIP(hipMemcpyAsync(dX, base + c0 * d, (size_t)m * d * 4, hipMemcpyHostToDevice, st));
      AMP_BHIP(hipMemcpyAsync(da, a.data() + c0, m * 4, hipMemcpyHostToDevice, st));
      AMP_BHIP(launch_residual(dX, da, dC, m, d, dR, st));
      for (int sm = 0; sm < M; ++sm) {
        AMP_BHIP(launch_assign(dR + sm * dsub, m, dsub, d, dCB + (size_t)sm * kKsub * dsub, kKsub, dxn, dcn, dcode,
                               nullptr, st));
        AMP_BHIP(hipMemcpyAsync(cm.data(), dcode, m * 4, hipMemcpyDeviceToHost, st));
        AMP_BHIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < m; ++i) codes[(size_t)(c0 + i) * M + sm] = (uint8_t)cm[i];
      }
    }
  }
  // list layout: by list, ids increasing inside a list
  std::vector<int64_t> idv(n);
  for (int64_t i = 0; i < n; ++i) idv[i] = ids ? ids[i] : i;
  std::vector<int64_t> off(nlist + 1, 0), order(n);
  for (int64_t i = 0; i < n; ++i) ++off[a[i] + 1];
  for (int p = 0; p < nlist; ++p) off[p + 1] += off[p];
  {
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < n; ++i) order[pos[a[i]]++] = i;
  }
  parallel_for(nlist, [&](int64_t p0, int64_t p1, int) {
    for (int64_t p = p0; p < p1; ++p)
      std::sort(order.begin() + off[p], order.begin() + off[p + 1],
                [&](int64_t x, int64_t y) { return idv[x] < idv[y]; });
  });
  std::vector<int64_t> sid(n);
  std::vector<uint8_t> scodes((size_t)n * M);
  for (int64_t j = 0; j < n; ++j) {
    sid[j] = idv[order[j]];
    std::memcpy(&scodes[(size_t)j * M], &codes[(size_t)order[j] * M], M);
  }
  // radius (FP64) and the largest residual magnitude, per thread then merged
  const int T = n_threads();
  std::vector<std::vector<double>> radt(T, std::vector<double>(nlist, 0.0));
  std::vector<double> amax(T, 0.0);
  parallel_for(n, [&](int64_t i0, int64_t i1, int t) {
    for (int64_t i = i0; i < i1; ++i) {
      double s2 = 0.0;
      for (int u = 0; u < d; ++u) {
        const double r = (double)(base[i * d + u] - C[(size_t)a[i] * d + u]);  // FP32 residual
        s2 += r * r;
        amax[t] = std::max(amax[t], std::fabs(r));
        if (prm->metric == AMP_IP) amax[t] = std::max(amax[t], (double)std::fabs(base[i * d + u]));
      }
      radt[t][a[i]] = std::max(radt[t][a[i]], std::sqrt(s2));
    }
  });
  std::vector<double> rad(nlist, 0.0);
  double A = 0.0;
  for (int t = 0; t < T; ++t) {
    A = std::max(A, amax[t]);
    for (int p = 0; p < nlist; ++p) rad[p] = std::max(rad[p], radt[t][p]);
  }
  for (float v : CB) A = std::max(A, (double)std::fabs(v));
  if (prm->metric == AMP_IP)
    for (float v : C) A = std::max(A, (double)std::fabs(v));
  int e = 0;
  if (!prm->integer_data && A > 0) e = (int)std::ceil(std::log2(A / (prm->grid_kind == AMP_GRID_E4M3 ? 448.0 : 255.0)));
  const double h = std::ldexp(1.0, e);
  std::vector<int32_t> radq(nlist);
  for (int p = 0; p < nlist; ++p) radq[p] = (int32_t)std::nearbyint(rad[p] / h);
  amp_index_arrays arr{};
  arr.d = d;
  arr.M = M;
  arr.nlist = nlist;
  arr.metric = prm->metric;
  arr.grid_kind = prm->grid_kind;
  arr.grid_e = e;
  arr.centroids = C.data();
  arr.codebook = CB.data();
  arr.list_offsets = off.data();
  arr.ids = sid.data();
  arr.codes = scodes.data();
  arr.radq = radq.data();
  return amp_index_from_arrays(&arr, out);
}

extern "C" amp_status amp_index_get_arrays(const amp_index* ix, amp_index_arrays* out) {
  if (!ix || !out) return set_error(AMP_EINVAL, "null argument");
  out->d = ix->d;
  out->M = ix->M;
  out->nlist = ix->nlist;
  out->metric = ix->metric;
  out->grid_kind = ix->grid_kind;
  out->grid_e = ix->grid_e;
  out->centroids = ix->centroids.data();
  out->codebook = ix->codebook.data();
  out->list_offsets = ix->offsets.data();
  out->ids = ix->ids.data();
  out->codes = ix->codes.data();
  out->radq = ix->radq.data();
  return AMP_OK;
}
