// miann_search_noalloc: the batched search for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// Every temporary buffer of a search (the path-extension hand-off, the
// per-stage results, the dense entry's query split, minima, bounds and
// candidate masks) is carved from one file-scope device array. Each GPU that
// loads the library holds its own copy of the array until the process ends.
// Host code never uses the array's name as an address: the device address is
// looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/miann.h"

miann_status miann_fail(miann_status st, const char* fmt, ...);
miann_status miann_search_impl(const miann_index* ix, const void* queries, int64_t nq, int32_t k, int32_t itopk,
                               int32_t max_iters, const miann_search_params* spp, uint32_t* ids, void* dists,
                               int64_t* counters, void* stream, void* ext, size_t ext_bytes);

namespace {

constexpr size_t kScratchBytes = (size_t)MIANN_NOALLOC_SCRATCH_MB << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex dev_mu;
void* dev_scratch[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (looked up on the first call on the device).
miann_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return miann_fail(MIANN_EDEVICE, "miann_search_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return miann_fail(MIANN_EUNSUPPORTED, "miann_search_noalloc: device %d", dev);
  std::lock_guard<std::mutex> lk(dev_mu);
  if (!dev_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return miann_fail(MIANN_EDEVICE, "miann_search_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    dev_scratch[dev] = p;
  }
  *out = dev_scratch[dev];
  return MIANN_OK;
}

}  // namespace

extern "C" {

miann_status miann_search_noalloc(const miann_index* idx, const void* queries_dev, int64_t nq, int32_t k,
                                  int32_t itopk, int32_t max_iters, const miann_search_params* sp, uint32_t* ids_dev,
                                  void* dists_dev, int64_t* counters_dev, void* stream) {
  void* p = nullptr;
  const miann_status st = scratch_ptr(&p);
  if (st != MIANN_OK) return st;
  return miann_search_impl(idx, queries_dev, nq, k, itopk, max_iters, sp, ids_dev, dists_dev, counters_dev, stream, p,
                           kScratchBytes);
}

size_t miann_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
