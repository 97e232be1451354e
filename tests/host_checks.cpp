// Host-side checks of the C ABI under AddressSanitizer / UndefinedBehavior-
// Sanitizer (built and run by tests/test_host_sanitize.py, CPU only): index
// construction and validation, file round trip and corrupt files, the CL
// sub-space map, both predictor trainers, the SVR solver, the tuning table,
// and forced host allocation failures (a replaced operator new that fails
// after a given number of allocations): every call must return AMP_OK or
// AMP_ENOMEM, leave the index usable, and leak nothing.
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "../include/amp.h"

// ------------------------------------------------------- fault injection
static std::atomic<long> g_budget{-1};  // allocations left before failing (-1: never fail)

static void* take(size_t n) {
  long b = g_budget.load();
  while (b >= 0) {
    if (b == 0) return nullptr;
    if (g_budget.compare_exchange_weak(b, b - 1)) break;
  }
  return std::malloc(n ? n : 1);
}
void* operator new(size_t n) {
  if (void* p = take(n)) return p;
  throw std::bad_alloc();
}
void* operator new[](size_t n) {
  if (void* p = take(n)) return p;
  throw std::bad_alloc();
}
void* operator new(size_t n, const std::nothrow_t&) noexcept { return take(n); }
void* operator new[](size_t n, const std::nothrow_t&) noexcept { return take(n); }
void operator delete(void* p) noexcept { std::free(p); }
void operator delete[](void* p) noexcept { std::free(p); }
void operator delete(void* p, size_t) noexcept { std::free(p); }
void operator delete[](void* p, size_t) noexcept { std::free(p); }

static int g_fail = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "CHECK failed at line %d: %s (%s)\n", __LINE__, #c, \
                   amp_last_error());                                         \
      ++g_fail;                                                               \
    }                                                                         \
  } while (0)

// ------------------------------------------------------- a small index
struct Arrays {
  int d = 32, M = 8, nlist = 16;
  std::vector<float> C, CB;
  std::vector<int64_t> off, ids;
  std::vector<uint8_t> codes;
  std::vector<int32_t> radq;
  amp_index_arrays a{};
  Arrays() {
    std::mt19937 r(7);
    std::normal_distribution<float> nd;
    const int n = 3000;
    C.resize((size_t)nlist * d);
    for (auto& v : C) v = 4.f * nd(r);
    CB.resize((size_t)M * 256 * (d / M));
    for (auto& v : CB) v = nd(r);
    off.resize(nlist + 1);
    for (int p = 0; p <= nlist; ++p) off[p] = (int64_t)n * p / nlist;
    ids.resize(n);
    for (int i = 0; i < n; ++i) ids[i] = i;
    codes.resize((size_t)n * M);
    for (auto& c : codes) c = (uint8_t)(r() & 255);
    radq.assign(nlist, 40);
    a = amp_index_arrays{d, M, nlist, AMP_L2, AMP_GRID_U9, -4, C.data(), CB.data(), off.data(), ids.data(),
                         codes.data(), radq.data()};
  }
};

static std::vector<float> queries(int nq, int d, unsigned seed) {
  std::mt19937 r(seed);
  std::normal_distribution<float> nd;
  std::vector<float> q((size_t)nq * d);
  for (auto& v : q) v = 4.f * nd(r);
  return q;
}

static amp_train_params train_params() {
  amp_train_params p{};
  p.n_samples = 64;
  p.max_iter = 2000;
  p.gamma = 1.0;
  p.C = 1.0;
  p.epsilon = 0.1;
  p.tol = 1e-3;
  return p;
}

static void basic(const char* dir) {
  Arrays A;
  amp_index* ix = nullptr;
  CHECK(amp_index_from_arrays(&A.a, &ix) == AMP_OK);
  // validation
  amp_index* bad = nullptr;
  amp_index_arrays b = A.a;
  b.d = 30;
  CHECK(amp_index_from_arrays(&b, &bad) == AMP_EINVAL && !bad);
  b = A.a;
  b.metric = 7;
  CHECK(amp_index_from_arrays(&b, &bad) == AMP_EINVAL);
  std::vector<int64_t> ids2 = A.ids;
  std::swap(ids2[0], ids2[1]);
  b = A.a;
  b.ids = ids2.data();
  CHECK(amp_index_from_arrays(&b, &bad) == AMP_EINVAL);
  CHECK(amp_index_from_arrays(nullptr, &bad) == AMP_EINVAL);
  // the CL map and both trainers
  CHECK(amp_index_build_cl_map(ix, 4, 6, 5, 1) == AMP_OK);
  CHECK(amp_index_build_cl_map(ix, 5, 6, 5, 1) == AMP_EINVAL);
  amp_cl_map m{};
  CHECK(amp_index_get_cl_map(ix, &m) == AMP_OK && m.S == 4 && m.P == 6 && m.w == 8);
  const std::vector<float> tq = queries(24, A.d, 3);
  amp_train_params p = train_params();
  amp_train_report rep{};
  CHECK(amp_index_train_predictor(ix, tq.data(), 24, 10, 4, &p, &rep) == AMP_OK && rep.n_pairs == 96);
  p.granularity = AMP_GRAN_SUBSPACE;
  CHECK(amp_index_train_predictor(ix, tq.data(), 24, 10, 4, &p, &rep) == AMP_OK);
  p.granularity = 3;
  CHECK(amp_index_train_predictor(ix, tq.data(), 24, 10, 4, &p, &rep) == AMP_EINVAL);
  p.granularity = 0;
  CHECK(amp_index_train_cl_predictor(ix, tq.data(), 24, 4, 4, &p, &rep) == AMP_OK);
  CHECK(amp_index_train_cl_predictor(ix, tq.data(), 24, 4, 8, &p, &rep) == AMP_EINVAL);
  // the SVR solver
  {
    std::vector<double> K(16), y = {0, 1, 0, 1}, coef(4);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) K[i * 4 + j] = std::exp(-0.5 * (i - j) * (i - j));
    double bias = 0;
    CHECK(amp_svr_fit(K.data(), y.data(), 4, 1.0, 0.1, 1e-4, 1000, coef.data(), &bias, nullptr) == AMP_OK);
    CHECK(amp_svr_fit(K.data(), y.data(), 0, 1.0, 0.1, 1e-4, 1000, coef.data(), &bias, nullptr) == AMP_EINVAL);
  }
  // tuning table
  {
    amp_tune_entry e{};
    e.policy_kind = AMP_POLICY_ADAPTIVE;
    e.nq_log2 = 10;
    e.narrow = -1;
    CHECK(amp_index_set_tuning(ix, &e, 1) == AMP_OK);
    int32_t cnt = 0;
    CHECK(amp_index_get_tuning(ix, nullptr, 0, &cnt) == AMP_OK && cnt == 1);
    e.narrow = 5;
    CHECK(amp_index_set_tuning(ix, &e, 1) == AMP_EINVAL);
  }
  // file round trip and damaged files
  char path[512];
  std::snprintf(path, sizeof path, "%s/host_checks.ampidx", dir);
  CHECK(amp_index_save(ix, path) == AMP_OK);
  amp_index* ld = nullptr;
  CHECK(amp_index_load(path, &ld) == AMP_OK && ld);
  amp_cl_map m2{};
  CHECK(ld && amp_index_get_cl_map(ld, &m2) == AMP_OK && m2.P == 6 &&
        std::memcmp(m.assign, m2.assign, sizeof(int32_t) * A.nlist * 4) == 0);
  amp_index_free(ld);
  {
    FILE* f = std::fopen(path, "rb");
    std::vector<char> bytes;
    if (f) {
      std::fseek(f, 0, SEEK_END);
      bytes.resize((size_t)std::ftell(f));
      std::fseek(f, 0, SEEK_SET);
      CHECK(std::fread(bytes.data(), 1, bytes.size(), f) == bytes.size());
      std::fclose(f);
    }
    char bpath[600];
    std::snprintf(bpath, sizeof bpath, "%s.bad", path);
    std::mt19937 r(11);
    for (int trial = 0; trial < 40 && !bytes.empty(); ++trial) {
      std::vector<char> v = bytes;
      if (trial % 2) v.resize(r() % v.size());            // truncated
      else v[r() % v.size()] ^= (char)(1 + (r() % 255));  // one byte damaged
      FILE* g = std::fopen(bpath, "wb");
      std::fwrite(v.data(), 1, v.size(), g);
      std::fclose(g);
      amp_index* x = nullptr;
      const amp_status s = amp_index_load(bpath, &x);
      CHECK(s == AMP_OK || s == AMP_EFORMAT || s == AMP_EIO);
      CHECK((s == AMP_OK) == (x != nullptr));
      amp_index_free(x);
    }
    std::remove(bpath);
  }
  std::remove(path);
  amp_index_free(ix);
}

// every host entry point under forced allocation failures
static void injected(const char* dir) {
  Arrays A;
  const std::vector<float> tq = queries(16, A.d, 5);
  char path[512];
  std::snprintf(path, sizeof path, "%s/host_checks_inj.ampidx", dir);
  amp_index* base = nullptr;
  CHECK(amp_index_from_arrays(&A.a, &base) == AMP_OK);
  CHECK(amp_index_build_cl_map(base, 4, 6, 3, 1) == AMP_OK);
  amp_train_params p = train_params();
  CHECK(amp_index_train_cl_predictor(base, tq.data(), 16, 4, 4, &p, nullptr) == AMP_OK);
  CHECK(amp_index_train_predictor(base, tq.data(), 16, 10, 4, &p, nullptr) == AMP_OK);
  CHECK(amp_index_save(base, path) == AMP_OK);
  int ok_seen[6] = {0, 0, 0, 0, 0, 0}, oom_seen[6] = {0, 0, 0, 0, 0, 0};
  // budgets 0..59 one by one, then growing by half until every call succeeds
  for (long budget = 0; budget < 4000000; budget = budget < 60 ? budget + 1 : budget + budget / 2) {
    amp_status s[6];
    amp_index* ix = nullptr;
    g_budget = budget;
    s[0] = amp_index_from_arrays(&A.a, &ix);
    g_budget = -1;
    CHECK(s[0] == AMP_OK || s[0] == AMP_ENOMEM);
    CHECK((s[0] == AMP_OK) == (ix != nullptr));
    (s[0] == AMP_OK ? ok_seen : oom_seen)[0]++;
    amp_index_free(ix);
    // the other calls on an index made without failures
    ix = nullptr;
    CHECK(amp_index_from_arrays(&A.a, &ix) == AMP_OK);
    g_budget = budget;
    s[1] = amp_index_build_cl_map(ix, 4, 6, 3, 1);
    g_budget = -1;
    g_budget = budget;
    s[2] = amp_index_train_predictor(ix, tq.data(), 16, 10, 4, &p, nullptr);
    g_budget = -1;
    if (s[1] == AMP_OK) {
      g_budget = budget;
      s[3] = amp_index_train_cl_predictor(ix, tq.data(), 16, 4, 4, &p, nullptr);
      g_budget = -1;
    } else {
      s[3] = AMP_OK;
    }
    amp_index* ld = nullptr;
    g_budget = budget;
    s[4] = amp_index_load(path, &ld);
    g_budget = -1;
    CHECK((s[4] == AMP_OK) == (ld != nullptr));
    amp_index_free(ld);
    amp_predictor_model mdl{};
    std::vector<int32_t> sv(5 * 4096), beta(4096), table(1024);
    CHECK(amp_index_get_predictor(base, &mdl, sv.data(), beta.data(), table.data(), 4096) == AMP_OK);
    g_budget = budget;
    s[5] = amp_index_set_predictor(ix, &mdl);
    g_budget = -1;
    for (int i = 1; i < 6; ++i) {
      CHECK(s[i] == AMP_OK || s[i] == AMP_ENOMEM);
      (s[i] == AMP_OK ? ok_seen : oom_seen)[i]++;
    }
    // the index stays usable after any failure
    int32_t d = 0;
    CHECK(amp_index_info(ix, &d, nullptr, nullptr, nullptr) == AMP_OK && d == A.d);
    CHECK(amp_index_train_predictor(ix, tq.data(), 16, 10, 4, &p, nullptr) == AMP_OK);
    amp_index_free(ix);
  }
  for (int i = 0; i < 6; ++i) {
    if (!(ok_seen[i] > 0 && oom_seen[i] > 0))
      std::fprintf(stderr, "call %d: %d successes, %d allocation failures\n", i, ok_seen[i], oom_seen[i]);
    CHECK(ok_seen[i] > 0 && oom_seen[i] > 0);
  }
  std::remove(path);
  amp_index_free(base);
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : "/tmp";
  basic(dir);
  injected(dir);
  std::printf("host checks: %s (%d failures)\n", g_fail ? "FAILED" : "ok", g_fail);
  return g_fail ? 1 : 0;
}
