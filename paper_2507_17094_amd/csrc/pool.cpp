// The library's memory pools (one per device).
#include "pool.hpp"

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

namespace miann {

hipMemPool_t lib_pool() {
  static std::mutex mu;
  static hipMemPool_t pools[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!pools[dev]) {
    hipMemPoolProps props = {};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t p = nullptr;
    if (hipMemPoolCreate(&p, &props) != hipSuccess) return nullptr;
    uint64_t keep = UINT64_MAX;
    hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
    pools[dev] = p;
  }
  return pools[dev];
}

namespace {
struct Kept {
  void* p = nullptr;
  size_t cap = 0;
  bool busy = false;
};
std::mutex kept_mu;
std::map<std::tuple<int, hipStream_t, int>, Kept> kept;
}  // namespace

hipError_t scratch_lease(int slot, size_t bytes, hipStream_t st, ScratchLease* out) {
  out->p = nullptr;
  out->kept = false;
  if (bytes == 0) bytes = 16;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (st == hipStreamPerThread) return pool_malloc_async(&out->p, bytes, st);
  {
    std::lock_guard<std::mutex> lk(kept_mu);
    Kept& k = kept[std::make_tuple(dev, st, slot)];
    if (!k.busy) {
      if (k.cap < bytes) {
        // a larger block: the old one goes back to the pool in stream order
        if (k.p) hipFreeAsync(k.p, st);
        k.p = nullptr;
        k.cap = 0;
        // power-of-two sizes: a stream whose requests grow reallocates a few times, not at every new maximum
        size_t cap = 65536;
        while (cap < bytes) cap <<= 1;
        void* p = nullptr;
        const hipError_t e = pool_malloc_async(&p, cap, st);
        if (e != hipSuccess) return e;
        k.p = p;
        k.cap = cap;
      }
      k.busy = true;
      out->p = k.p;
      out->kept = true;
      return hipSuccess;
    }
  }
  return pool_malloc_async(&out->p, bytes, st);
}

void scratch_release(int slot, const ScratchLease& l, hipStream_t st) {
  if (!l.p) return;
  if (!l.kept) {
    hipFreeAsync(l.p, st);
    return;
  }
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(kept_mu);
  kept[std::make_tuple(dev, st, slot)].busy = false;
}

hipError_t scratch_drop_stream(hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  hipError_t rc = hipSuccess;
  std::lock_guard<std::mutex> lk(kept_mu);
  for (auto it = kept.begin(); it != kept.end();) {
    if (std::get<0>(it->first) == dev && std::get<1>(it->first) == st && !it->second.busy) {
      if (it->second.p) {
        const hipError_t e = hipFreeAsync(it->second.p, st);
        if (e != hipSuccess) rc = e;
      }
      it = kept.erase(it);
    } else {
      ++it;
    }
  }
  return rc;
}

}  // namespace miann
