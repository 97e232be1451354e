// Serving loop: continuous batching of single-query requests onto the search
// path of one device.
//
// Requests are admitted into a fixed pool of pinned query slots (the memory
// bound of the queue: a full pool rejects with AMP_EBUSY), gathered into
// batches of requests sharing a precision policy, and each batch runs as one
// device-mode search with per-query k and nprobe.  Two batches may be in
// flight, each on an execution slot of its own (stream, search scratch,
// staging): the worker launches batch i+1 (query and size upload, search,
// result copies, all stream-ordered) before it waits for batch i, so the two
// searches overlap on the device and the host-side gather, scatter and
// callbacks overlap both.  A batch is padded to a size bucket and its search
// replays a HIP graph captured once per (slot, bucket, policy): the
// per-query k and nprobe travel in device memory, so one graph serves every
// mix of sizes.  A batch whose search reports an error on the device (a
// candidate overflow) fails its requests with that status.  Latency runs
// from a request's arrival stamp to the moment its results are in the
// caller's buffers.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "amp_internal.h"

namespace amp {
namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

bool same_policy(const amp_precision_policy& a, const amp_precision_policy& b) {
  return a.kind == b.kind && a.fixed_bits == b.fixed_bits && a.allowed_bits_mask == b.allowed_bits_mask &&
         a.lut_dtype == b.lut_dtype && a.margin_q40 == b.margin_q40;
}

struct Request {
  uint64_t ticket;
  int32_t k, nprobe, slot;
  int64_t* out_ids;
  float* out_dist;
  int64_t* out_qdist;
  void (*done)(void*, amp_status);
  void* user;
  int64_t arrival_ns;
  amp_precision_policy policy;
  bool cancelled;
};

struct Batch {  // one in-flight search and its staging set
  std::vector<Request*> reqs;
  int set = 0, kmax = 0;
  amp_status status = AMP_OK;
};

struct Staging {  // execution slot of an in-flight batch
  void* hq = nullptr;        // pinned [cap][d] query rows
  int32_t* hsz = nullptr;    // pinned [2][cap] per-query k, nprobe
  int64_t* hids = nullptr;   // pinned [cap][max_k]
  float* hdist = nullptr;
  int64_t* hqd = nullptr;
  int32_t* hstatus = nullptr;  // pinned: device status of the batch's search
  void* dq = nullptr;        // device copies
  int32_t* dsz = nullptr;
  int64_t* dids = nullptr;
  float* ddist = nullptr;
  int64_t* dqd = nullptr;
  int32_t* dstatus = nullptr;
  hipEvent_t ev = nullptr;   // results copied back
  hipStream_t stream = nullptr;
  Workspace ws;              // search scratch of this slot
};

// batch size bucket (graphs are captured per bucket): powers of two up to
// 128, then multiples of 128
int bucket_of(int n) {
  if (n <= 128) {
    int b = 1;
    while (b < n) b <<= 1;
    return b;
  }
  return (n + 127) / 128 * 128;
}

}  // namespace
}  // namespace amp

using namespace amp;

struct amp_server {
  amp_index* ix = nullptr;
  amp_server_config cfg{};
  int device = 0, d = 0, esize = 4;
  int cap = 0;  // rows of a padded batch (the largest bucket)
  // admission pool
  void* pool = nullptr;  // pinned [max_pending][d] query rows
  std::vector<int32_t> free_slots;
  Staging stg[2];
  std::mutex mu;
  std::condition_variable cv_work, cv_idle;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> live;  // pending or in flight
  std::deque<Batch> inflight;
  uint64_t next_ticket = 1;
  bool stopping = false;
  // statistics since creation or the last reset
  int64_t submitted = 0, rejected = 0, completed = 0, cancelled = 0, failed = 0, batches = 0, batched = 0;
  int64_t t0 = 0;
  std::vector<float> lat_ms;
  std::thread worker;

  ~amp_server();
  amp_status init();
  void run();
  void launch(Batch& b);
  void complete(Batch& b);
};

static constexpr size_t kMaxLatencySamples = 1u << 24;

amp_server::~amp_server() {
  (void)hipSetDevice(device);
  for (Staging& s : stg) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    release_workspace(s.ws);
    if (s.ev) (void)hipEventDestroy(s.ev);
    void* host[] = {s.hq, s.hsz, s.hids, s.hdist, s.hqd, s.hstatus};
    for (void* p : host)
      if (p) (void)hipHostFree(p);
    void* dev[] = {s.dq, s.dsz, s.dids, s.ddist, s.dqd, s.dstatus};
    for (void* p : dev)
      if (p) (void)hipFree(p);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  if (pool) (void)hipHostFree(pool);
}

amp_status amp_server::init() {
  cap = bucket_of(cfg.max_batch);
  const size_t B = cap, K = cfg.max_k, row = (size_t)d * esize;
  auto hfail = [](const char* what) {
    (void)hipGetLastError();
    return set_error(AMP_ENOMEM, "server: %s allocation failed", what);
  };
  if (hipHostMalloc(&pool, (size_t)cfg.max_pending * row, hipHostMallocDefault) != hipSuccess) return hfail("pool");
  amp_status s = amp_index_to_device(ix, device);
  for (Staging& g : stg) {
    if (s != AMP_OK) return s;
    // default-priority streams of their own: the two slots' searches overlap
    if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess) return hfail("stream");
    if (hipHostMalloc(&g.hq, B * row, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&g.hsz), 2 * B * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&g.hids), B * K * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&g.hdist), B * K * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&g.hqd), B * K * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&g.hstatus), 4, hipHostMallocDefault) != hipSuccess)
      return hfail("pinned staging");
    std::memset(g.hq, 0, B * row);  // padded rows stay zero
    if (hipMalloc(&g.dq, B * row) != hipSuccess || hipMalloc(reinterpret_cast<void**>(&g.dsz), 2 * B * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&g.dids), B * K * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&g.ddist), B * K * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&g.dqd), B * K * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&g.dstatus), 4) != hipSuccess)
      return hfail("device staging");
    if (hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess) return hfail("event");
    // the slot's search scratch, sized now for the largest batch: growing it
    // later would wait for the batch in flight
    s = reserve_workspace(ix, cap, cfg.max_nprobe, cfg.max_k, &g.ws);
  }
  if (s != AMP_OK) return s;
  free_slots.resize(cfg.max_pending);
  for (int32_t i = 0; i < cfg.max_pending; ++i) free_slots[i] = cfg.max_pending - 1 - i;
  return AMP_OK;
}

// gather the batch's queries and sizes into its slot's staging (padded to
// the bucket) and enqueue upload, search and result copies on the slot's
// stream
void amp_server::launch(Batch& b) {
  Staging& s = stg[b.set];
  const size_t row = (size_t)d * esize;
  const int n = (int)b.reqs.size();
  const int nb = bucket_of(n);
  int32_t* hk = s.hsz;
  int32_t* hnp = s.hsz + cap;
  for (int i = 0; i < n; ++i) {
    Request* r = b.reqs[i];
    std::memcpy(static_cast<char*>(s.hq) + i * row, static_cast<char*>(pool) + (size_t)r->slot * row, row);
    hk[i] = r->k;
    hnp[i] = r->nprobe;
    b.kmax = std::max(b.kmax, r->k);
  }
  // padding rows: zero queries with k = nprobe = 1 (their results are dropped)
  std::memset(static_cast<char*>(s.hq) + (size_t)n * row, 0, (size_t)(nb - n) * row);
  for (int i = n; i < nb; ++i) hk[i] = hnp[i] = 1;
  {
    std::lock_guard<std::mutex> lk(mu);  // the rows are copied: the slots take new requests
    for (Request* r : b.reqs) free_slots.push_back(r->slot);
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(s.dq, s.hq, nb * row, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(s.dsz, s.hsz, 2 * (size_t)cap * 4, hipMemcpyHostToDevice, s.stream)) != hipSuccess) {
    (void)hipGetLastError();
    b.status = set_error(AMP_EDEVICE, "server: query upload failed: %s", hipGetErrorString(e));
    return;
  }
  amp_search_opts o{};
  o.mem = AMP_MEM_DEVICE;
  o.stream = s.stream;
  o.out_qdist = s.dqd;
  o.q_dtype = cfg.q_dtype;
  o.flags = AMP_SEARCH_GRAPH | AMP_SEARCH_DEVICE_SIZES;
  o.kmax = cfg.max_k;
  o.npmax = cfg.max_nprobe;
  o.out_status = s.dstatus;
  b.status = search_on(ix, s.ws, s.dq, nb, s.dsz, s.dsz + cap, 1, &b.reqs[0]->policy, &o, s.dids, s.ddist);
  if (b.status != AMP_OK) return;
  const size_t nk = (size_t)n * cfg.max_k;
  if ((e = hipMemcpyAsync(s.hids, s.dids, nk * 8, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(s.hdist, s.ddist, nk * 4, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(s.hqd, s.dqd, nk * 8, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(s.hstatus, s.dstatus, 4, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
      (e = hipEventRecord(s.ev, s.stream)) != hipSuccess) {
    (void)hipGetLastError();
    b.status = set_error(AMP_EDEVICE, "server: result copy failed: %s", hipGetErrorString(e));
  }
}

// wait for the batch, hand each request its rows, run the callbacks
void amp_server::complete(Batch& b) {
  Staging& s = stg[b.set];
  if (b.status == AMP_OK) {
    const hipError_t e = hipEventSynchronize(s.ev);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.status = set_error(AMP_EDEVICE, "server: batch failed: %s", hipGetErrorString(e));
    } else if (*s.hstatus != AMP_OK) {
      // the device reported an error (a candidate overflow): the batch fails
      b.status = set_error(*s.hstatus, "server: the batch's search reported %s on the device",
                           amp_status_str(*s.hstatus));
    }
  }
  std::vector<std::pair<Request*, amp_status>> fin;
  fin.reserve(b.reqs.size());
  const int64_t t = now_ns();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < b.reqs.size(); ++i) {
      Request* r = b.reqs[i];
      live.erase(r->ticket);
      amp_status st = b.status;
      if (r->cancelled) {
        st = AMP_ECANCELED;
        ++cancelled;
      } else if (st == AMP_OK) {
        const size_t o = i * (size_t)cfg.max_k;
        std::memcpy(r->out_ids, s.hids + o, r->k * 8);
        std::memcpy(r->out_dist, s.hdist + o, r->k * 4);
        if (r->out_qdist) std::memcpy(r->out_qdist, s.hqd + o, r->k * 8);
        ++completed;
        if (lat_ms.size() < kMaxLatencySamples) lat_ms.push_back((float)((t - r->arrival_ns) * 1e-6));
      } else {
        ++failed;
      }
      fin.emplace_back(r, st);
    }
  }
  for (auto& [r, st] : fin) {
    if (r->done) r->done(r->user, st);
    delete r;
  }
}

void amp_server::run() {
  (void)hipSetDevice(device);
  int next_set = 0;
  for (;;) {
    Batch b;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (inflight.empty()) {
        cv_idle.notify_all();
        cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
        if (pending.empty()) break;  // stopping and drained
        // an idle device may wait a little for the batch to fill
        if (cfg.batch_window_us > 0 && !stopping && (int)pending.size() < cfg.max_batch) {
          const auto until = std::chrono::steady_clock::time_point(std::chrono::nanoseconds(
              pending.front()->arrival_ns + (int64_t)cfg.batch_window_us * 1000));
          cv_work.wait_until(lk, until, [&] { return stopping || (int)pending.size() >= cfg.max_batch; });
        }
      }
      // requests of the oldest one's policy, in arrival order
      const amp_precision_policy pol = pending.empty() ? amp_precision_policy{} : pending.front()->policy;
      for (auto it = pending.begin(); it != pending.end() && (int)b.reqs.size() < cfg.max_batch;) {
        if (same_policy((*it)->policy, pol)) {
          b.reqs.push_back(*it);
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      if (!b.reqs.empty()) {
        b.set = next_set;
        next_set ^= 1;
        ++batches;
        batched += (int64_t)b.reqs.size();
      }
    }
    if (!b.reqs.empty()) {
      launch(b);
      inflight.push_back(std::move(b));
    }
    // keep at most two batches in flight; with nothing new to launch, finish
    // the oldest
    if (inflight.size() == 2 || (b.reqs.empty() && !inflight.empty()) ||
        (!inflight.empty() && inflight.front().status != AMP_OK)) {
      complete(inflight.front());
      inflight.pop_front();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stopping && pending.empty() && inflight.empty()) break;
    }
  }
  while (!inflight.empty()) {
    complete(inflight.front());
    inflight.pop_front();
  }
  std::lock_guard<std::mutex> lk(mu);
  cv_idle.notify_all();
}

static amp_status check_policy(const amp_index* ix, const amp_precision_policy& p) {
  switch (p.kind) {
    case AMP_POLICY_FP32: break;
    case AMP_POLICY_FIXED:
      if (p.fixed_bits != 4 && p.fixed_bits != 8 && p.fixed_bits != 12 && p.fixed_bits != 16)
        return set_error(AMP_EINVAL, "fixed_bits must be 4, 8, 12 or 16");
      break;
    case AMP_POLICY_ADAPTIVE:
      if (!ix->has_model) return set_error(AMP_EINVAL, "adaptive policy needs a predictor");
      if (p.allowed_bits_mask & ~((1u << 4) | (1u << 8) | (1u << 12) | (1u << 16)))
        return set_error(AMP_EINVAL, "allowed_bits_mask has widths outside {4,8,12,16}");
      break;
    case AMP_POLICY_EXPLICIT: return set_error(AMP_EINVAL, "the server does not take the explicit policy");
    default: return set_error(AMP_EINVAL, "bad policy kind %d", p.kind);
  }
  if (p.lut_dtype != 0 && p.lut_dtype != AMP_LUT_BF16 && p.lut_dtype != AMP_LUT_F16 && p.lut_dtype != AMP_LUT_F8E4M3)
    return set_error(AMP_EINVAL, "bad LUT build dtype %d", p.lut_dtype);
  if (p.lut_dtype == AMP_LUT_F8E4M3 && (ix->grid_kind != AMP_GRID_E4M3 || ix->metric == AMP_L1))
    return set_error(AMP_EINVAL, "the FP8 LUT build needs an index on the e4m3 operand grid, L2 or inner product");
  return AMP_OK;
}

static amp_status amp_server_create_body(amp_index* ix, const amp_server_config* cfg_in, amp_server** out);
extern "C" amp_status amp_server_create(amp_index* ix, const amp_server_config* cfg_in, amp_server** out) {
  return host_guard([&] { return amp_server_create_body(ix, cfg_in, out); });
}

static amp_status amp_server_create_body(amp_index* ix, const amp_server_config* cfg_in, amp_server** out) {
  if (!ix || !cfg_in || !out) return set_error(AMP_EINVAL, "null argument");
  *out = nullptr;
  amp_server_config c = *cfg_in;
  if (c.max_batch == 0) c.max_batch = 1024;
  if (c.max_pending == 0) c.max_pending = 4 * c.max_batch;
  if (c.max_k == 0) c.max_k = 100;
  if (c.max_nprobe == 0) c.max_nprobe = std::min(ix->nlist, AMP_MAX_NPROBE);
  if (c.max_batch < 1 || c.max_batch > 65536) return set_error(AMP_EINVAL, "max_batch %d outside [1, 65536]", c.max_batch);
  if (c.max_pending < 1 || c.max_pending > (1 << 22))
    return set_error(AMP_EINVAL, "max_pending %d outside [1, 2^22]", c.max_pending);
  if (c.max_k < 1 || c.max_k > AMP_MAX_K) return set_error(AMP_EINVAL, "max_k %d outside [1, %d]", c.max_k, AMP_MAX_K);
  if (c.max_nprobe < 1 || c.max_nprobe > std::min(ix->nlist, AMP_MAX_NPROBE))
    return set_error(AMP_EINVAL, "max_nprobe %d outside [1, %d]", c.max_nprobe, std::min(ix->nlist, AMP_MAX_NPROBE));
  if (c.batch_window_us < 0 || c.batch_window_us > 1000000)
    return set_error(AMP_EINVAL, "batch_window_us %d outside [0, 1e6]", c.batch_window_us);
  if (c.q_dtype != AMP_F32 && c.q_dtype != AMP_BF16) return set_error(AMP_EINVAL, "bad query dtype %d", c.q_dtype);
  amp_status s = check_policy(ix, c.policy);
  if (s != AMP_OK) return s;
  c.policy.explicit_bits = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(AMP_EDEVICE, "no HIP device");
  }
  amp_server* sv = new (std::nothrow) amp_server;
  if (!sv) return set_error(AMP_ENOMEM, "server allocation failed");
  sv->ix = ix;
  sv->cfg = c;
  sv->device = dev;
  sv->d = ix->d;
  sv->esize = c.q_dtype == AMP_BF16 ? 2 : 4;
  if ((s = sv->init()) != AMP_OK) {
    delete sv;
    return s;
  }
  sv->t0 = now_ns();
  sv->worker = std::thread([sv] { sv->run(); });
  *out = sv;
  return AMP_OK;
}

static amp_status amp_server_submit_body(amp_server* sv, const amp_request* rq, uint64_t* ticket);
extern "C" amp_status amp_server_submit(amp_server* sv, const amp_request* rq, uint64_t* ticket) {
  return host_guard([&] { return amp_server_submit_body(sv, rq, ticket); });
}

static amp_status amp_server_submit_body(amp_server* sv, const amp_request* rq, uint64_t* ticket) {
  if (!sv || !rq || !rq->query || !rq->out_ids || !rq->out_dist) return set_error(AMP_EINVAL, "null argument");
  if (rq->k < 1 || rq->k > sv->cfg.max_k) return set_error(AMP_EINVAL, "k = %d outside [1, %d]", rq->k, sv->cfg.max_k);
  if (rq->nprobe < 1 || rq->nprobe > sv->cfg.max_nprobe)
    return set_error(AMP_EINVAL, "nprobe = %d outside [1, %d]", rq->nprobe, sv->cfg.max_nprobe);
  amp_precision_policy pol = sv->cfg.policy;
  if (rq->policy) {
    amp_status s = check_policy(sv->ix, *rq->policy);
    if (s != AMP_OK) return s;
    pol = *rq->policy;
    pol.explicit_bits = nullptr;
  }
  const int64_t t = now_ns();
  std::unique_lock<std::mutex> lk(sv->mu);
  ++sv->submitted;
  if (sv->stopping) {
    ++sv->rejected;
    return set_error(AMP_EBUSY, "server is shutting down");
  }
  if (sv->free_slots.empty()) {
    ++sv->rejected;
    return set_error(AMP_EBUSY, "admission: %d requests already queued", sv->cfg.max_pending);
  }
  Request* r = new (std::nothrow) Request;
  if (!r) return set_error(AMP_ENOMEM, "request allocation failed");
  r->slot = sv->free_slots.back();
  sv->free_slots.pop_back();
  const size_t row = (size_t)sv->d * sv->esize;
  std::memcpy(static_cast<char*>(sv->pool) + (size_t)r->slot * row, rq->query, row);
  r->ticket = sv->next_ticket++;
  r->k = rq->k;
  r->nprobe = rq->nprobe;
  r->out_ids = rq->out_ids;
  r->out_dist = rq->out_dist;
  r->out_qdist = rq->out_qdist;
  r->done = rq->done;
  r->user = rq->user;
  r->arrival_ns = rq->arrival_ns > 0 ? rq->arrival_ns : t;
  r->policy = pol;
  r->cancelled = false;
  sv->pending.push_back(r);
  sv->live.emplace(r->ticket, r);
  if (ticket) *ticket = r->ticket;
  lk.unlock();
  sv->cv_work.notify_one();
  return AMP_OK;
}

extern "C" amp_status amp_server_cancel(amp_server* sv, uint64_t ticket) {
  if (!sv) return set_error(AMP_EINVAL, "null server");
  Request* gone = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return set_error(AMP_EINVAL, "ticket %llu is not queued or in flight", (unsigned long long)ticket);
    Request* r = it->second;
    auto pit = std::find(sv->pending.begin(), sv->pending.end(), r);
    if (pit != sv->pending.end()) {  // not launched: remove it now
      sv->pending.erase(pit);
      sv->live.erase(it);
      sv->free_slots.push_back(r->slot);
      ++sv->cancelled;
      gone = r;
      if (sv->pending.empty() && sv->inflight.empty()) sv->cv_idle.notify_all();
    } else {  // in flight: its results are dropped on completion
      r->cancelled = true;
    }
  }
  if (gone) {
    if (gone->done) gone->done(gone->user, AMP_ECANCELED);
    delete gone;
  }
  return AMP_OK;
}

extern "C" amp_status amp_server_flush(amp_server* sv) {
  if (!sv) return set_error(AMP_EINVAL, "null server");
  if (std::this_thread::get_id() == sv->worker.get_id())
    return set_error(AMP_EINVAL, "flush from a completion callback would never return");
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_idle.wait(lk, [&] { return sv->live.empty(); });
  return AMP_OK;
}

extern "C" amp_status amp_server_stats(amp_server* sv, amp_server_report* out, int32_t reset) {
  if (!sv || !out) return set_error(AMP_EINVAL, "null argument");
  std::vector<float> lat;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    const int64_t t = now_ns();
    out->submitted = sv->submitted;
    out->rejected = sv->rejected;
    out->completed = sv->completed;
    out->cancelled = sv->cancelled;
    out->failed = sv->failed;
    out->batches = sv->batches;
    out->pending = (int64_t)sv->pending.size();
    out->in_flight = (int64_t)sv->live.size() - (int64_t)sv->pending.size();
    out->elapsed_s = (t - sv->t0) * 1e-9;
    out->qps = out->elapsed_s > 0 ? sv->completed / out->elapsed_s : 0.0;
    out->mean_batch = sv->batches ? (double)sv->batched / sv->batches : 0.0;
    lat.swap(sv->lat_ms);
    if (reset) {
      sv->submitted = sv->rejected = sv->completed = sv->cancelled = sv->failed = sv->batches = sv->batched = 0;
      sv->t0 = t;
    } else {
      sv->lat_ms = lat;
    }
  }
  out->p50_ms = out->p99_ms = out->max_ms = 0.0;
  if (!lat.empty()) {
    auto pct = [&](double q) {
      const size_t i = std::min(lat.size() - 1, (size_t)(q * (double)(lat.size() - 1) + 0.5));
      std::nth_element(lat.begin(), lat.begin() + i, lat.end());
      return (double)lat[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = *std::max_element(lat.begin(), lat.end());
  }
  return AMP_OK;
}

extern "C" void amp_server_destroy(amp_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  delete sv;
}
