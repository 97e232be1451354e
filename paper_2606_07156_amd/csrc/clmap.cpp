// Vector space division for reduced-precision cluster locating (paper
// Sec. 3.1): the 8-bit operand codes of the centroids, the dimension slices
// and the per-slice sub-spaces (clusters of the centroids' slice codes) with
// their centres, radii and member counts, and the CL predictor's model.
//
// Host code that runs once per index; the search kernels read the result.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <random>
#include <vector>

#include "amp_internal.h"

namespace amp {

// code offset and exponent: o = FP32 midpoint of the centroid value range
// (inner product: 0), ec = smallest exponent with every centroid value
// within 127 * 2^ec of o
void cl_params_host(const std::vector<float>& C, int metric, float* o, int* ec) {
  float lo = std::numeric_limits<float>::infinity(), hi = -lo;
  for (float v : C) lo = std::min(lo, v), hi = std::max(hi, v);
  *o = metric == AMP_IP ? 0.f : (float)(((double)lo + (double)hi) / 2.0);
  const double A = std::max((double)hi - (double)*o, (double)*o - (double)lo);
  int e = 0;
  if (A > 0) {
    e = -60;
    while (A > 127.0 * std::ldexp(1.0, e)) ++e;
  }
  *ec = e;
}

// 8-bit signed code of one value: x - o rounded to FP32, scaled by 2^-ec
// (exact), rounded half to even, clamped
int8_t cl_code_host(float x, float o, int ec) {
  volatile float diff = x - o;  // one FP32 rounding
  const double v = std::nearbyint(std::ldexp((double)diff, -ec));
  return (int8_t)std::min(127.0, std::max(-128.0, v));
}

}  // namespace amp

using namespace amp;

static amp_status build_cl_map_impl(amp_index* ix, int32_t S, int32_t P, int32_t iters, uint64_t seed) {
  if (!ix) return set_error(AMP_EINVAL, "null index");
  if (ix->metric != AMP_L2 && ix->metric != AMP_IP)
    return set_error(AMP_EUNSUPPORTED, "reduced-precision cluster locating supports L2 and inner product");
  if (S < 1 || ix->d % S) return set_error(AMP_EINVAL, "d (%d) must be a positive multiple of S (%d)", ix->d, S);
  const int w = ix->d / S;
  if (w > 64) return set_error(AMP_EUNSUPPORTED, "d / S = %d > 64", w);
  const int nl = ix->nlist;
  if (P < 1 || P > std::min(nl, 1024)) return set_error(AMP_EINVAL, "P = %d outside [1, min(nlist, 1024)]", P);
  if (iters < 0 || iters > 1000) return set_error(AMP_EINVAL, "iters outside [0, 1000]");
  float o;
  int ec;
  cl_params_host(ix->centroids, ix->metric, &o, &ec);
  const int d = ix->d;
  std::vector<int8_t> codes((size_t)nl * d);
  for (size_t i = 0; i < codes.size(); ++i) codes[i] = cl_code_host(ix->centroids[i], o, ec);
  std::vector<int32_t> assign((size_t)nl * S), centre((size_t)S * P * w), radius((size_t)S * P),
      count((size_t)S * P);
  std::mt19937_64 rng(seed);
  std::vector<double> X((size_t)nl * w), Z((size_t)P * w), acc((size_t)P * w);
  std::vector<int> a(nl), cnt(P);
  std::vector<double> dbest(nl);
  auto nearest = [&](const double* x, const double* Zc, double* dout) {
    int best = 0;
    double bd = std::numeric_limits<double>::infinity();
    for (int u = 0; u < P; ++u) {
      double s = 0;
      for (int t = 0; t < w; ++t) {
        const double df = x[t] - Zc[(size_t)u * w + t];
        s += df * df;
      }
      if (s < bd) bd = s, best = u;  // strict: ties keep the lower index
    }
    if (dout) *dout = bd;
    return best;
  };
  for (int s = 0; s < S; ++s) {
    for (int i = 0; i < nl; ++i)
      for (int t = 0; t < w; ++t) X[(size_t)i * w + t] = codes[(size_t)i * d + s * w + t];
    // starting points: the first P distinct slices of a seeded order (fewer
    // distinct slices than P: the remaining centres repeat the first one)
    std::vector<int> order(nl);
    std::iota(order.begin(), order.end(), 0);
    std::shuffle(order.begin(), order.end(), rng);
    int got = 0;
    for (int idx = 0; idx < nl && got < P; ++idx) {
      const double* x = &X[(size_t)order[idx] * w];
      bool dup = false;
      for (int u = 0; u < got && !dup; ++u)
        dup = std::equal(x, x + w, &Z[(size_t)u * w]);
      if (!dup) std::copy(x, x + w, &Z[(size_t)got++ * w]);
    }
    for (int u = got; u < P; ++u) std::copy(&Z[0], &Z[w], &Z[(size_t)u * w]);
    for (int it = 0; it < iters; ++it) {
      std::fill(acc.begin(), acc.end(), 0.0);
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int i = 0; i < nl; ++i) {
        a[i] = nearest(&X[(size_t)i * w], Z.data(), &dbest[i]);
        cnt[a[i]]++;
        for (int t = 0; t < w; ++t) acc[(size_t)a[i] * w + t] += X[(size_t)i * w + t];
      }
      for (int u = 0; u < P; ++u) {
        if (cnt[u]) {
          for (int t = 0; t < w; ++t) Z[(size_t)u * w + t] = acc[(size_t)u * w + t] / cnt[u];
        } else {
          // reseed from the point farthest from its centre (lowest index on ties)
          int far = 0;
          for (int i = 1; i < nl; ++i)
            if (dbest[i] > dbest[far]) far = i;
          std::copy(&X[(size_t)far * w], &X[(size_t)far * w] + w, &Z[(size_t)u * w]);
          dbest[far] = 0;
        }
      }
    }
    // integer centres (half away from zero), then the nearest-centre partition
    for (size_t i = 0; i < (size_t)P * w; ++i) Z[i] = std::round(Z[i]);
    std::fill(cnt.begin(), cnt.end(), 0);
    std::vector<int64_t> r2(P, 0);
    for (int i = 0; i < nl; ++i) {
      double dd;
      const int u = nearest(&X[(size_t)i * w], Z.data(), &dd);
      assign[(size_t)i * S + s] = u;
      cnt[u]++;
      r2[u] = std::max<int64_t>(r2[u], (int64_t)dd);  // exact: integer operands
    }
    for (int u = 0; u < P; ++u) {
      for (int t = 0; t < w; ++t) centre[((size_t)s * P + u) * w + t] = (int32_t)Z[(size_t)u * w + t];
      int64_t r = (int64_t)std::sqrt((double)r2[u]);
      while (r * r < r2[u]) ++r;
      while (r > 0 && (r - 1) * (r - 1) >= r2[u]) --r;
      radius[(size_t)s * P + u] = (int32_t)r;
      count[(size_t)s * P + u] = cnt[u];
    }
  }
  std::lock_guard<std::mutex> lk(ix->mu);
  ix->has_clmap = true;
  ix->cl_S = S;
  ix->cl_P = P;
  ix->cl_w = w;
  ix->cl_o = o;
  ix->cl_ec = ec;
  ix->cl_codes.swap(codes);
  ix->cl_assign.swap(assign);
  ix->cl_centre.swap(centre);
  ix->cl_radius.swap(radius);
  ix->cl_count.swap(count);
  ix->has_cl_model = false;
  ix->cl_n_sv = 0;
  ix->dev_cl_stale = true;
  ix->model_generation++;
  return AMP_OK;
}

static amp_status set_cl_predictor_impl(amp_index* ix, const amp_predictor_model* m);

extern "C" {

amp_status amp_index_build_cl_map(amp_index* ix, int32_t S, int32_t P, int32_t iters, uint64_t seed) {
  return host_guard([&] { return build_cl_map_impl(ix, S, P, iters, seed); });
}

amp_status amp_index_set_cl_predictor(amp_index* ix, const amp_predictor_model* m) {
  return host_guard([&] { return set_cl_predictor_impl(ix, m); });
}

amp_status amp_index_get_cl_map(const amp_index* ix, amp_cl_map* out) {
  if (!ix || !out) return set_error(AMP_EINVAL, "null argument");
  if (!ix->has_clmap) return set_error(AMP_EINVAL, "index has no sub-space map");
  out->S = ix->cl_S;
  out->P = ix->cl_P;
  out->w = ix->cl_w;
  out->o = ix->cl_o;
  out->ec = ix->cl_ec;
  out->assign = ix->cl_assign.data();
  out->centre = ix->cl_centre.data();
  out->radius = ix->cl_radius.data();
  out->count = ix->cl_count.data();
  return AMP_OK;
}

}  // extern "C"

static amp_status set_cl_predictor_impl(amp_index* ix, const amp_predictor_model* m) {
  if (!ix || !m) return set_error(AMP_EINVAL, "null argument");
  if (!ix->has_clmap) return set_error(AMP_EINVAL, "index has no sub-space map");
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
  ix->cl_n_sv = m->n_sv;
  ix->cl_sv.swap(sv);
  ix->cl_beta.swap(beta);
  ix->cl_table.swap(table);
  ix->cl_beta0 = m->beta0;
  for (int f = 0; f < 5; ++f) ix->cl_feat_lo[f] = m->feat_lo[f], ix->cl_feat_mul[f] = m->feat_mul[f];
  for (int i = 0; i < 3; ++i) ix->cl_theta[i] = m->theta[i];
  ix->cl_g_mul = m->g_mul;
  ix->has_cl_model = true;
  ix->dev_cl_stale = true;
  ix->model_generation++;
  return AMP_OK;
}

extern "C" amp_status amp_index_get_cl_predictor(const amp_index* ix, amp_predictor_model* m, int32_t* sv, int32_t* beta,
                                      int32_t* table, int32_t capacity) {
  if (!ix || !m) return set_error(AMP_EINVAL, "null argument");
  if (!ix->has_cl_model) return set_error(AMP_EINVAL, "index has no CL predictor");
  m->n_sv = ix->cl_n_sv;
  if (capacity < ix->cl_n_sv) return set_error(AMP_EINVAL, "capacity %d below n_sv %d", capacity, ix->cl_n_sv);
  if ((ix->cl_n_sv && (!sv || !beta)) || !table) return set_error(AMP_EINVAL, "null output buffer");
  std::copy(ix->cl_sv.begin(), ix->cl_sv.end(), sv);
  std::copy(ix->cl_beta.begin(), ix->cl_beta.end(), beta);
  std::copy(ix->cl_table.begin(), ix->cl_table.end(), table);
  m->sv = sv;
  m->beta = beta;
  m->table = table;
  m->beta0 = ix->cl_beta0;
  for (int f = 0; f < 5; ++f) m->feat_lo[f] = ix->cl_feat_lo[f], m->feat_mul[f] = ix->cl_feat_mul[f];
  for (int i = 0; i < 3; ++i) m->theta[i] = ix->cl_theta[i];
  m->g_mul = ix->cl_g_mul;
  return AMP_OK;
}
