// Offline training of the precision predictor (paper Sec. 3.3-3.4): features
// {d', r1, r2, n1, n2} of (query, probed cluster) pairs of a training query
// set, labels from the distance margin between the query's neighbours and
// non-neighbours in each probed cluster, an RBF epsilon-SVR fitted by SMO,
// and its export to the fixed-point model the search kernels evaluate.
//
// This is host code that runs once per index; it is not part of a search.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <random>
#include <thread>
#include <vector>

#include "amp_internal.h"

namespace amp {

namespace {

// operand grid (same definition as the search kernels): round half to even,
// then saturate to the 9-bit grid or round to the e4m3-representable integers
int e4m3_int_host(int v) {
  int a = v < 0 ? -v : v;
  if (a >= 16) {
    int E = 31 - __builtin_clz(a), sh = E - 3;
    int q = a >> sh, rem = a & ((1 << sh) - 1), half = 1 << (sh - 1);
    if (rem > half || (rem == half && (q & 1))) q++;
    a = q << sh;
  }
  a = std::min(a, 448);
  return v < 0 ? -a : a;
}
int grid_host(float r, int e, int kind) {
  float x = std::nearbyint(std::ldexp(r, -e));
  if (kind == AMP_GRID_U9) return (int)std::min(255.f, std::max(-255.f, x));
  x = std::min(65536.f, std::max(-65536.f, x));
  return e4m3_int_host((int)x);
}
int64_t mitchell_q8_host(int64_t x) {
  uint64_t y = (uint64_t)x + 1;
  int k = 63 - __builtin_clzll(y);
  return 256 * (int64_t)k + (int64_t)((y << 8) >> k) - 256;
}
// quantiser shift (the search kernels' rule): smallest s with
// (R + n hf(s)) >> s <= n (2^b - 1); n = 1 with R the largest subspace
// range (one width per pair), n = M with R the sum of the ranges
// (per-subspace widths)
int shift_for(int64_t R, int n, int b) {
  const int64_t top = (int64_t)n * ((1ll << b) - 1);
  int s = 0;
  while (((R + (s ? ((int64_t)n << (s - 1)) : 0)) >> s) > top) ++s;
  return s;
}

// T worker threads running f(t, stop); a failed host allocation in any of
// them (or in starting them) stops the others and is rethrown after every
// started thread has been joined
template <class F>
void run_workers(int T, F&& f) {
  std::vector<std::thread> th;
  std::atomic<bool> oom{false};
  try {
    th.reserve(T);
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        try {
          f(t, oom);
        } catch (const std::bad_alloc&) {
          oom = true;
        }
      });
  } catch (...) {
    oom = true;
    for (auto& x : th) x.join();
    throw std::bad_alloc();
  }
  for (auto& x : th) x.join();
  if (oom) throw std::bad_alloc();
}

struct Sample {
  int64_t x[5];
  int bits;
};

// epsilon-SVR dual solved by SMO with the maximal-violating-pair working set
// (Keerthi et al., 2001), written for the 2l-variable form
//   min 1/2 b'Qb + p'b,  z'b = 0,  0 <= b <= C,
// with b = [alpha; alpha*], z = [+1; -1], p = [eps - y; eps + y],
// Q_ij = z_i z_j K(i mod l, j mod l).  Returns coefficients alpha - alpha*
// and the bias of f(x) = sum_i coef_i K(x_i, x) + bias.
void svr_smo(const std::vector<double>& K, const std::vector<double>& y, double C, double eps, double tol,
             int max_iter, std::vector<double>& coef, double& bias, int& iters) {
  const int l = (int)y.size(), n = 2 * l;
  std::vector<double> beta(n, 0.0), G(n), z(n);
  for (int t = 0; t < n; ++t) {
    z[t] = t < l ? 1.0 : -1.0;
    G[t] = t < l ? eps - y[t] : eps + y[t - l];
  }
  auto Kt = [&](int a, int b) { return K[(size_t)(a % l) * l + (b % l)]; };
  iters = 0;
  for (; iters < max_iter; ++iters) {
    int i = -1, j = -1;
    double gmax = -1e300, gmin = 1e300;
    for (int t = 0; t < n; ++t) {
      const bool up = (z[t] > 0 && beta[t] < C) || (z[t] < 0 && beta[t] > 0);
      const bool low = (z[t] > 0 && beta[t] > 0) || (z[t] < 0 && beta[t] < C);
      const double v = -z[t] * G[t];
      if (up && v > gmax) gmax = v, i = t;
      if (low && v < gmin) gmin = v, j = t;
    }
    if (i < 0 || j < 0 || gmax - gmin < tol) break;
    // move along z_i d_i + z_j d_j = 0 minimising the quadratic
    const double Kii = Kt(i, i), Kjj = Kt(j, j), Kij = Kt(i, j);
    const double a = std::max(Kii + Kjj - 2.0 * Kij, 1e-12);
    double step = (gmax - gmin) / a;  // change of z_i*beta_i
    // box limits on beta_i (+z_i step) and beta_j (-z_j step)
    double lim_i = z[i] > 0 ? C - beta[i] : beta[i];
    double lim_j = z[j] > 0 ? beta[j] : C - beta[j];
    step = std::min(step, std::min(lim_i, lim_j));
    const double di = z[i] * step, dj = -z[j] * step;
    beta[i] += di;
    beta[j] += dj;
    beta[i] = std::min(C, std::max(0.0, beta[i]));
    beta[j] = std::min(C, std::max(0.0, beta[j]));
    for (int t = 0; t < n; ++t)
      G[t] += z[t] * (z[i] * Kt(t, i) * di + z[j] * Kt(t, j) * dj);
  }
  // bias from free variables (average of -z_t G_t), else the interval middle
  double sum = 0;
  int nf = 0;
  double ub = 1e300, lb = -1e300;
  for (int t = 0; t < n; ++t) {
    const double v = -z[t] * G[t];
    if (beta[t] > 1e-12 && beta[t] < C - 1e-12) sum += v, ++nf;
    const bool up = (z[t] > 0 && beta[t] < C) || (z[t] < 0 && beta[t] > 0);
    if (up) lb = std::max(lb, v);
    else ub = std::min(ub, v);
  }
  bias = nf ? sum / nf : 0.5 * (std::min(ub, 1e300) + std::max(lb, -1e300));
  coef.assign(l, 0.0);
  for (int t = 0; t < l; ++t) coef[t] = beta[t] - beta[t + l];
}

}  // namespace
}  // namespace amp

using namespace amp;

static amp_status svr_fit_impl(const double* K, const double* y, int32_t l, double C, double eps, double tol,
                                  int32_t max_iter, double* coef, double* bias, int32_t* iterations) {
  if (!K || !y || !coef || !bias || l < 1 || !(C > 0) || !(eps >= 0) || !(tol > 0) || max_iter < 1)
    return set_error(AMP_EINVAL, "bad SVR fit arguments");
  std::vector<double> Kv(K, K + (size_t)l * l), yv(y, y + l), cv;
  int it = 0;
  svr_smo(Kv, yv, C, eps, tol, max_iter, cv, *bias, it);
  std::copy(cv.begin(), cv.end(), coef);
  if (iterations) *iterations = it;
  return AMP_OK;
}

static amp_status train_predictor_impl(amp_index* ix, const float* tq, int64_t nq, int32_t k, int32_t nprobe,
                                                const amp_train_params* prm, amp_train_report* rep) {
  if (!ix || !tq || !prm) return set_error(AMP_EINVAL, "null argument");
  if (nq <= 0 || k < 1 || nprobe < 1 || nprobe > ix->nlist) return set_error(AMP_EINVAL, "bad nq / k / nprobe");
  if (prm->n_samples < 8 || prm->n_samples > 8192) return set_error(AMP_EINVAL, "n_samples outside [8, 8192]");
  if (!(prm->gamma > 0) || !(prm->C > 0) || !(prm->epsilon >= 0)) return set_error(AMP_EINVAL, "bad SVR parameters");
  if (prm->granularity != AMP_GRAN_PAIR && prm->granularity != AMP_GRAN_SUBSPACE)
    return set_error(AMP_EINVAL, "bad quantiser granularity %d", prm->granularity);
  uint32_t allowed = prm->allowed_bits_mask ? prm->allowed_bits_mask : ((1u << 4) | (1u << 8) | (1u << 12) | (1u << 16));
  std::vector<int> widths;
  for (int b = 4; b <= 16; b += 4)
    if (allowed & (1u << b)) widths.push_back(b);
  if (widths.empty() || (allowed & ~((1u << 4) | (1u << 8) | (1u << 12) | (1u << 16))))
    return set_error(AMP_EINVAL, "allowed_bits_mask must select widths among 4, 8, 12, 16");
  const int d = ix->d, M = ix->M, dsub = ix->dsub, nl = ix->nlist;
  // grid codebook (and, for inner product, grid centroids)
  const bool ip = ix->metric == AMP_IP, l1 = ix->metric == AMP_L1;
  std::vector<int32_t> cbi((size_t)M * kKsub * dsub);
  for (size_t i = 0; i < cbi.size(); ++i) cbi[i] = grid_host(ix->codebook[i], ix->grid_e, ix->grid_kind);
  std::vector<int32_t> cgi;
  if (ip) {
    cgi.resize((size_t)nl * d);
    for (size_t i = 0; i < cgi.size(); ++i) cgi[i] = grid_host(ix->centroids[i], ix->grid_e, ix->grid_kind);
  }
  // labelled pairs of one training query (queries run on worker threads;
  // their samples are concatenated in query order)
  auto label_query = [&](int64_t qi, std::vector<Sample>& out) {
    std::vector<double> D(nl);
    std::vector<int> order(nl);
    std::vector<int32_t> ri(d), qg(d);
    std::vector<int64_t> T((size_t)M * kKsub);
    const float* q = tq + (size_t)qi * d;
    // CL in FP64 (inner product: the negated dot product), probes by
    // (distance, list)
    for (int c = 0; c < nl; ++c) {
      double s = 0;
      for (int t = 0; t < d; ++t) {
        if (ip) {
          s -= (double)q[t] * (double)ix->centroids[(size_t)c * d + t];
        } else if (l1) {
          s += std::fabs((double)q[t] - (double)ix->centroids[(size_t)c * d + t]);
        } else {
          const double df = (double)q[t] - (double)ix->centroids[(size_t)c * d + t];
          s += df * df;
        }
      }
      D[c] = s;
    }
    std::iota(order.begin(), order.end(), 0);
    std::partial_sort(order.begin(), order.begin() + nprobe, order.end(),
                      [&](int a, int b) { return D[a] < D[b] || (D[a] == D[b] && a < b); });
    // the query-wide inner-product LUT -qi.cbi and its spread
    // mode 0: inner product, 1: L2, 2: L1
    const bool gsub = prm->granularity == AMP_GRAN_SUBSPACE;
    auto build_lut = [&](const int32_t* v, int mode) {
      int64_t Rp = 0;
      for (int m = 0; m < M; ++m) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int j = 0; j < kKsub; ++j) {
          int64_t s = 0;
          for (int t = 0; t < dsub; ++t) {
            const int64_t c = cbi[((size_t)m * kKsub + j) * dsub + t];
            if (mode == 1) {
              const int64_t df = v[m * dsub + t] - c;
              s += df * df;
            } else if (mode == 2) {
              s += std::llabs(v[m * dsub + t] - c);
            } else {
              s -= v[m * dsub + t] * c;
            }
          }
          T[(size_t)m * kKsub + j] = s;
          lo = std::min(lo, s);
          hi = std::max(hi, s);
        }
        Rp = gsub ? Rp + (hi - lo) : std::max(Rp, hi - lo);  // sum of the ranges or the largest
      }
      return Rp;
    };
    int64_t Rq = 0;
    if (ip) {
      for (int t = 0; t < d; ++t) qg[t] = grid_host(q[t], ix->grid_e, ix->grid_kind);
      Rq = build_lut(qg.data(), 0);
    }
    // exact integer ADC distances of every candidate, per probed list
    std::vector<int64_t> dq2(nprobe), R(nprobe);
    std::vector<std::vector<int64_t>> dist(nprobe);
    std::vector<std::pair<int64_t, int64_t>> cand;
    for (int r = 0; r < nprobe; ++r) {
      const int p = order[r];
      int64_t s2 = 0, extra = 0;
      for (int t = 0; t < d; ++t) {
        if (ip) {
          ri[t] = qg[t] - cgi[(size_t)p * d + t];  // d' of inner product: ||qi - ci||^2
          extra -= (int64_t)qg[t] * cgi[(size_t)p * d + t];
        } else {
          ri[t] = grid_host(q[t] - ix->centroids[(size_t)p * d + t], ix->grid_e, ix->grid_kind);
        }
        s2 += (int64_t)ri[t] * ri[t];
      }
      dq2[r] = s2;
      R[r] = ip ? Rq : build_lut(ri.data(), l1 ? 2 : 1);
      for (int64_t v = ix->offsets[p]; v < ix->offsets[p + 1]; ++v) {
        int64_t s = extra;
        for (int m = 0; m < M; ++m) s += T[(size_t)m * kKsub + ix->codes[(size_t)v * M + m]];
        dist[r].push_back(s);
        cand.emplace_back(s, ix->ids[v]);
      }
    }
    if ((int64_t)cand.size() <= k) return;
    std::nth_element(cand.begin(), cand.begin() + k, cand.end());
    std::sort(cand.begin(), cand.begin() + k + 1);
    const int64_t dk = cand[k - 1].first, dk1 = cand[k].first;
    const std::pair<int64_t, int64_t> kth = cand[k - 1];
    // C1 = probed list with the smallest d' (ties: lower list id)
    int c1 = 0;
    for (int r = 1; r < nprobe; ++r)
      if (dq2[r] < dq2[c1] || (dq2[r] == dq2[c1] && order[r] < order[c1])) c1 = r;
    for (int r = 0; r < nprobe; ++r) {
      const int p = order[r];
      // margin between neighbours and non-neighbours in this list
      int64_t delta = INT64_MAX;
      for (size_t i = 0; i < dist[r].size(); ++i) {
        const int64_t dv = dist[r][i], id = ix->ids[ix->offsets[p] + i];
        const bool nbr = std::make_pair(dv, id) <= kth;
        delta = std::min(delta, nbr ? dk1 - dv : dv - dk);
      }
      int bstar = widths.back();
      for (int b : widths) {
        const int s = shift_for(R[r], gsub ? M : 1, b);
        const int64_t err = (int64_t)M * (s ? (1ll << (s - 1)) : 0);
        if (err < delta || s == 0) {
          bstar = b;
          break;
        }
      }
      Sample smp;
      smp.x[0] = dq2[r];
      smp.x[1] = ix->radq[order[c1]];
      smp.x[2] = ix->radq[p];
      smp.x[3] = ix->offsets[order[c1] + 1] - ix->offsets[order[c1]];
      smp.x[4] = ix->offsets[p + 1] - ix->offsets[p];
      smp.bits = bstar;
      out.push_back(smp);
    }
  };
  std::vector<std::vector<Sample>> per_q(nq);
  {
    const unsigned hw = std::thread::hardware_concurrency();
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(nq, std::min(hw ? hw : 1u, 16u)));
    run_workers(T, [&](int t, const std::atomic<bool>& stop) {
      for (int64_t qi = t; qi < nq && !stop; qi += T) label_query(qi, per_q[qi]);
    });
  }
  std::vector<Sample> all;
  for (auto& v : per_q) all.insert(all.end(), v.begin(), v.end());
  if (all.size() < 8) return set_error(AMP_EINVAL, "too few training pairs");
  // integer feature map: fixed-point log2, then min-max onto 0..1023
  int64_t flo[5], fmul[5];
  for (int f = 0; f < 5; ++f) {
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (const Sample& s : all) {
      const int64_t L = mitchell_q8_host(s.x[f]);
      lo = std::min(lo, L);
      hi = std::max(hi, L);
    }
    flo[f] = lo;
    fmul[f] = (1023ll * 65536) / std::max<int64_t>(1, hi - lo);
  }
  auto to_u = [&](const Sample& s, int32_t* u) {
    for (int f = 0; f < 5; ++f) {
      int64_t v = ((mitchell_q8_host(s.x[f]) - flo[f]) * fmul[f]) >> 16;
      u[f] = (int32_t)std::min<int64_t>(1023, std::max<int64_t>(0, v));
    }
  };
  // stratified sample: round-robin over width classes
  std::mt19937_64 rng(prm->seed);
  std::vector<std::vector<int>> byb(17);
  for (size_t i = 0; i < all.size(); ++i) byb[all[i].bits].push_back((int)i);
  for (auto& v : byb) std::shuffle(v.begin(), v.end(), rng);
  std::vector<int> pick;
  const int want = std::min<int>(prm->n_samples, (int)all.size());
  std::vector<size_t> cur(17, 0);
  while ((int)pick.size() < want) {
    bool any = false;
    for (int b : widths)
      if (cur[b] < byb[b].size() && (int)pick.size() < want) pick.push_back(byb[b][cur[b]++]), any = true;
    if (!any) break;
  }
  const int l = (int)pick.size();
  std::vector<int32_t> U((size_t)l * 5);
  std::vector<double> y(l);
  for (int i = 0; i < l; ++i) {
    to_u(all[pick[i]], &U[(size_t)i * 5]);
    y[i] = (all[pick[i]].bits - 4) / 12.0;
  }
  std::vector<double> K((size_t)l * l);
  const double gs = prm->gamma / (1023.0 * 1023.0);
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < l; ++j) {
      double s = 0;
      for (int f = 0; f < 5; ++f) {
        const double df = U[(size_t)i * 5 + f] - U[(size_t)j * 5 + f];
        s += df * df;
      }
      K[(size_t)i * l + j] = std::exp(-gs * s);
    }
  std::vector<double> coef;
  double bias = 0;
  int iters = 0;
  const int max_iter = prm->max_iter > 0 ? prm->max_iter : 100000;
  svr_smo(K, y, prm->C, prm->epsilon, prm->tol > 0 ? prm->tol : 1e-3, max_iter, coef, bias, iters);
  // export the support vectors in fixed point
  std::vector<int32_t> sv, beta;
  for (int i = 0; i < l; ++i) {
    const double c = coef[i];
    if (std::fabs(c) < 1e-9) continue;
    for (int f = 0; f < 5; ++f) sv.push_back(U[(size_t)i * 5 + f]);
    beta.push_back((int32_t)std::llround(c * (1 << 20)));
  }
  std::vector<int32_t> table(kTableN);
  for (int i = 0; i < kTableN; ++i) table[i] = (int32_t)std::llround(std::exp(-(i + 0.5) / 64.0) * (1 << 20));
  amp_predictor_model m{};
  m.n_sv = (int32_t)beta.size();
  m.sv = sv.data();
  m.beta = beta.data();
  m.table = table.data();
  m.beta0 = (int64_t)std::llround(bias * 1099511627776.0);
  for (int f = 0; f < 5; ++f) m.feat_lo[f] = flo[f], m.feat_mul[f] = fmul[f];
  m.g_mul = (uint64_t)std::llround(prm->gamma * 64.0 / (1023.0 * 1023.0) * 4294967296.0);
  // thresholds halfway between the label values of consecutive widths
  const double mid[3] = {0.5 / 3.0, 1.5 / 3.0, 2.5 / 3.0};
  for (int i = 0; i < 3; ++i) m.theta[i] = (int64_t)std::llround(mid[i] * 1099511627776.0);
  if (m.n_sv > 4096) return set_error(AMP_EUNSUPPORTED, "%d support vectors exceed 4096", m.n_sv);
  amp_status st = amp_index_set_predictor(ix, &m);
  if (st != AMP_OK) return st;
  if (rep) {
    memset(rep, 0, sizeof *rep);
    rep->n_pairs = (int64_t)all.size();
    rep->n_samples = l;
    rep->n_sv = m.n_sv;
    rep->smo_iterations = iters;
    for (const Sample& s : all) rep->label_hist[s.bits / 4 - 1]++;
    // training error of the real-valued regressor on the sample
    double se = 0;
    for (int i = 0; i < l; ++i) {
      double f = bias;
      for (int j = 0; j < l; ++j) f += coef[j] * K[(size_t)j * l + i];
      se += (f - y[i]) * (f - y[i]);
    }
    rep->train_rmse = std::sqrt(se / l);
  }
  return AMP_OK;
}

// ------------------------------------------------------------------ CL predictor
// Labels per (training query, slice, sub-space) from the full-width integer
// coarse distances and the nprobe boundary; the same feature map, sampling,
// SMO fit and fixed-point export as the LUT predictor, with two classes (the
// low width, 8 bits) and one threshold.
static amp_status train_cl_predictor_impl(amp_index* ix, const float* tq, int64_t nq, int32_t nprobe,
                                                   int32_t low, const amp_train_params* prm,
                                                   amp_train_report* rep) {
  if (!ix || !tq || !prm) return set_error(AMP_EINVAL, "null argument");
  if (!ix->has_clmap) return set_error(AMP_EINVAL, "index has no sub-space map");
  if (nq <= 0 || nprobe < 1 || nprobe >= ix->nlist) return set_error(AMP_EINVAL, "bad nq / nprobe");
  if (low < 1 || low > 7) return set_error(AMP_EINVAL, "low width %d outside [1, 7]", low);
  if (prm->n_samples < 8 || prm->n_samples > 8192) return set_error(AMP_EINVAL, "n_samples outside [8, 8192]");
  if (!(prm->gamma > 0) || !(prm->C > 0) || !(prm->epsilon >= 0)) return set_error(AMP_EINVAL, "bad SVR parameters");
  const int d = ix->d, nl = ix->nlist, S = ix->cl_S, P = ix->cl_P, w = ix->cl_w;
  const bool ip = ix->metric == AMP_IP;
  const int klo = 8 - low;
  auto tr = [](int v, int k) { return v - (v & ((1 << k) - 1)); };  // floor to a multiple of 2^k
  auto label_query = [&](int64_t qi, std::vector<Sample>& out) {
    const float* q = tq + (size_t)qi * d;
    std::vector<int> vq(d);
    for (int t = 0; t < d; ++t) vq[t] = cl_code_host(q[t], ix->cl_o, ix->cl_ec);
    // partial distances per (centroid, slice) at full and low width
    std::vector<int64_t> p8((size_t)nl * S), plo((size_t)nl * S), D(nl, 0);
    for (int i = 0; i < nl; ++i)
      for (int s = 0; s < S; ++s) {
        int64_t a8 = 0, al = 0;
        for (int t = s * w; t < (s + 1) * w; ++t) {
          const int c = ix->cl_codes[(size_t)i * d + t];
          if (ip) {
            a8 -= (int64_t)vq[t] * c;
            al -= (int64_t)tr(vq[t], klo) * tr(c, klo);
          } else {
            const int64_t d8 = vq[t] - c, dl = tr(vq[t], klo) - tr(c, klo);
            a8 += d8 * d8;
            al += dl * dl;
          }
        }
        p8[(size_t)i * S + s] = a8;
        plo[(size_t)i * S + s] = al;
        D[i] += a8;
      }
    std::vector<int> order(nl);
    std::iota(order.begin(), order.end(), 0);
    std::partial_sort(order.begin(), order.begin() + nprobe + 1, order.end(),
                      [&](int a, int b) { return D[a] < D[b] || (D[a] == D[b] && a < b); });
    const int64_t dnp = D[order[nprobe - 1]], dnp1 = D[order[nprobe]];
    std::vector<char> nbr(nl, 0);
    for (int r = 0; r < nprobe; ++r) nbr[order[r]] = 1;
    for (int s = 0; s < S; ++s) {
      std::vector<int64_t> delta(P, INT64_MAX), err(P, 0), d2(P, 0);
      for (int i = 0; i < nl; ++i) {
        const int u = ix->cl_assign[(size_t)i * S + s];
        const int64_t m = nbr[i] ? dnp1 - D[i] : D[i] - dnp;
        delta[u] = std::min(delta[u], m);
        err[u] = std::max<int64_t>(err[u], std::llabs(plo[(size_t)i * S + s] - p8[(size_t)i * S + s]));
      }
      int c1 = 0;
      for (int u = 0; u < P; ++u) {
        int64_t a = 0;
        for (int t = 0; t < w; ++t) {
          const int64_t df = vq[s * w + t] - ix->cl_centre[((size_t)s * P + u) * w + t];
          a += df * df;
        }
        d2[u] = a;
        if (a < d2[c1]) c1 = u;
      }
      for (int u = 0; u < P; ++u) {
        if (ix->cl_count[(size_t)s * P + u] == 0) continue;
        Sample smp;
        smp.x[0] = d2[u];
        smp.x[1] = ix->cl_radius[(size_t)s * P + c1];
        smp.x[2] = ix->cl_radius[(size_t)s * P + u];
        smp.x[3] = ix->cl_count[(size_t)s * P + c1];
        smp.x[4] = ix->cl_count[(size_t)s * P + u];
        smp.bits = 2 * err[u] < delta[u] ? low : 8;
        out.push_back(smp);
      }
    }
  };
  std::vector<std::vector<Sample>> per_q(nq);
  {
    const unsigned hw = std::thread::hardware_concurrency();
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(nq, std::min(hw ? hw : 1u, 16u)));
    run_workers(T, [&](int t, const std::atomic<bool>& stop) {
      for (int64_t qi = t; qi < nq && !stop; qi += T) label_query(qi, per_q[qi]);
    });
  }
  std::vector<Sample> all;
  for (auto& v : per_q) all.insert(all.end(), v.begin(), v.end());
  if (all.size() < 8) return set_error(AMP_EINVAL, "too few training samples");
  int64_t flo[5], fmul[5];
  for (int f = 0; f < 5; ++f) {
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (const Sample& s : all) {
      const int64_t L = mitchell_q8_host(s.x[f]);
      lo = std::min(lo, L);
      hi = std::max(hi, L);
    }
    flo[f] = lo;
    fmul[f] = (1023ll * 65536) / std::max<int64_t>(1, hi - lo);
  }
  auto to_u = [&](const Sample& s, int32_t* u) {
    for (int f = 0; f < 5; ++f) {
      int64_t v = ((mitchell_q8_host(s.x[f]) - flo[f]) * fmul[f]) >> 16;
      u[f] = (int32_t)std::min<int64_t>(1023, std::max<int64_t>(0, v));
    }
  };
  // stratified sample: alternate between the two classes
  std::mt19937_64 rng(prm->seed);
  std::vector<int> cls[2];
  for (size_t i = 0; i < all.size(); ++i) cls[all[i].bits == low ? 0 : 1].push_back((int)i);
  for (auto& v : cls) std::shuffle(v.begin(), v.end(), rng);
  std::vector<int> pick;
  const int want = std::min<int>(prm->n_samples, (int)all.size());
  size_t cur[2] = {0, 0};
  while ((int)pick.size() < want) {
    bool any = false;
    for (int c = 0; c < 2; ++c)
      if (cur[c] < cls[c].size() && (int)pick.size() < want) pick.push_back(cls[c][cur[c]++]), any = true;
    if (!any) break;
  }
  const int l = (int)pick.size();
  std::vector<int32_t> U((size_t)l * 5);
  std::vector<double> y(l);
  for (int i = 0; i < l; ++i) {
    to_u(all[pick[i]], &U[(size_t)i * 5]);
    y[i] = all[pick[i]].bits == low ? 0.0 : 1.0;
  }
  std::vector<double> K((size_t)l * l);
  const double gs = prm->gamma / (1023.0 * 1023.0);
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < l; ++j) {
      double s = 0;
      for (int f = 0; f < 5; ++f) {
        const double df = U[(size_t)i * 5 + f] - U[(size_t)j * 5 + f];
        s += df * df;
      }
      K[(size_t)i * l + j] = std::exp(-gs * s);
    }
  std::vector<double> coef;
  double bias = 0;
  int iters = 0;
  const int max_iter = prm->max_iter > 0 ? prm->max_iter : 100000;
  svr_smo(K, y, prm->C, prm->epsilon, prm->tol > 0 ? prm->tol : 1e-3, max_iter, coef, bias, iters);
  std::vector<int32_t> sv, beta;
  for (int i = 0; i < l; ++i) {
    const double c = coef[i];
    if (std::fabs(c) < 1e-9) continue;
    for (int f = 0; f < 5; ++f) sv.push_back(U[(size_t)i * 5 + f]);
    beta.push_back((int32_t)std::llround(c * (1 << 20)));
  }
  std::vector<int32_t> table(kTableN);
  for (int i = 0; i < kTableN; ++i) table[i] = (int32_t)std::llround(std::exp(-(i + 0.5) / 64.0) * (1 << 20));
  amp_predictor_model m{};
  m.n_sv = (int32_t)beta.size();
  m.sv = sv.data();
  m.beta = beta.data();
  m.table = table.data();
  m.beta0 = (int64_t)std::llround(bias * 1099511627776.0);
  for (int f = 0; f < 5; ++f) m.feat_lo[f] = flo[f], m.feat_mul[f] = fmul[f];
  m.g_mul = (uint64_t)std::llround(prm->gamma * 64.0 / (1023.0 * 1023.0) * 4294967296.0);
  m.theta[0] = (int64_t)std::llround(0.5 * 1099511627776.0);
  if (m.n_sv > 4096) return set_error(AMP_EUNSUPPORTED, "%d support vectors exceed 4096", m.n_sv);
  amp_status st = amp_index_set_cl_predictor(ix, &m);
  if (st != AMP_OK) return st;
  if (rep) {
    memset(rep, 0, sizeof *rep);
    rep->n_pairs = (int64_t)all.size();
    rep->n_samples = l;
    rep->n_sv = m.n_sv;
    rep->smo_iterations = iters;
    for (const Sample& s : all) rep->label_hist[s.bits == low ? 0 : 1]++;
    double se = 0;
    for (int i = 0; i < l; ++i) {
      double f = bias;
      for (int j = 0; j < l; ++j) f += coef[j] * K[(size_t)j * l + i];
      se += (f - y[i]) * (f - y[i]);
    }
    rep->train_rmse = std::sqrt(se / l);
  }
  return AMP_OK;
}

// ------------------------------------------------------------------ C entry points
extern "C" amp_status amp_svr_fit(const double* K, const double* y, int32_t l, double C, double eps, double tol,
                                  int32_t max_iter, double* coef, double* bias, int32_t* iterations) {
  return host_guard([&] { return svr_fit_impl(K, y, l, C, eps, tol, max_iter, coef, bias, iterations); });
}

extern "C" amp_status amp_index_train_predictor(amp_index* ix, const float* tq, int64_t nq, int32_t k, int32_t nprobe,
                                                const amp_train_params* prm, amp_train_report* rep) {
  return host_guard([&] { return train_predictor_impl(ix, tq, nq, k, nprobe, prm, rep); });
}

extern "C" amp_status amp_index_train_cl_predictor(amp_index* ix, const float* tq, int64_t nq, int32_t nprobe,
                                                   int32_t low, const amp_train_params* prm,
                                                   amp_train_report* rep) {
  return host_guard([&] { return train_cl_predictor_impl(ix, tq, nq, nprobe, low, prm, rep); });
}
