// Allocation-free search entry point.  The scratch of the search lives in one
// fixed array of device memory (`scratch`, kScratchBytes per device, held by
// the loaded library until the process ends) instead of buffers the library
// allocates: for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid it).
#include <mutex>
#include <type_traits>

#include "amp_internal.h"

namespace amp {

constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// device address of `scratch` on each device, looked up once per device with
// that device current (each device holds its own copy of the array; the host
// name of the array is not a device address)
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

static amp_status scratch_of(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(AMP_EDEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(AMP_EDEVICE, "hipGetSymbolAddress of the search scratch failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return AMP_OK;
}

}  // namespace amp

using namespace amp;

extern "C" amp_status amp_search_noalloc(amp_index* ix, const void* queries, int64_t nq, const int32_t* k,
                                         const int32_t* nprobe, int32_t per_query, const amp_precision_policy* pol,
                                         const amp_search_opts* opts, int64_t* out_ids, float* out_dist) {
  if (!ix || !k || !nprobe || !opts) return set_error(AMP_EINVAL, "null argument");
  if (nq <= 0 || nq > (1 << 24)) return set_error(AMP_EINVAL, "nq %lld out of range", (long long)nq);
  // the sizes the scratch is laid out for (checked again by the search)
  int kmax, npmax;
  if (opts->flags & AMP_SEARCH_DEVICE_SIZES) {
    kmax = opts->kmax;
    npmax = opts->npmax;
  } else {
    if (per_query)
      return set_error(AMP_EINVAL, "amp_search_noalloc takes per-query sizes as device arrays "
                                   "(AMP_SEARCH_DEVICE_SIZES)");
    kmax = k[0];
    npmax = nprobe[0];
  }
  if (kmax < 1 || kmax > AMP_MAX_K) return set_error(AMP_EINVAL, "k = %d outside [1, %d]", kmax, AMP_MAX_K);
  if (npmax < 1 || npmax > std::min(ix->nlist, AMP_MAX_NPROBE))
    return set_error(AMP_EINVAL, "nprobe = %d outside [1, %d]", npmax, std::min(ix->nlist, AMP_MAX_NPROBE));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(AMP_EDEVICE, "no HIP device");
  }
  char* base = nullptr;
  amp_status s = scratch_of(dev, &base);
  if (s != AMP_OK) return s;
  // the search keeps every list whole (one work unit per pair at most); the
  // candidate buffer shrinks towards k if the batch does not fit otherwise
  // (overflows are then resolved by the re-runs, or reported)
  const int64_t units = whole_list_units(nq, npmax);
  size_t capq = plan_capq(kmax);
  size_t min_capq = 16;  // the smallest power of two that holds k results
  while (min_capq < (size_t)kmax) min_capq <<= 1;
  Workspace w;
  while (!carve_workspace(ix, w, base, kScratchBytes, nq, npmax, kmax, capq, units)) {
    if (capq <= min_capq)
      return set_error(AMP_EINVAL, "a search of %lld queries, nprobe %d, k %d does not fit the %zu MiB scratch",
                       (long long)nq, npmax, kmax, kScratchBytes >> 20);
    capq >>= 1;
  }
  return search_on(ix, w, queries, nq, k, nprobe, per_query, pol, opts, out_ids, out_dist);
}
