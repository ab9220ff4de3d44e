// Stream-ordered device allocations of the library.
//
// Every temporary buffer of a search or build comes from one memory pool per
// device owned by the library. The pool keeps freed blocks (release threshold
// = unlimited), so repeated searches of similar sizes reuse memory instead of
// going back to the driver; the host application's default pool is left as
// it is.
#pragma once
#include <hip/hip_runtime.h>

namespace miann {

// The library's pool of the current device (created on first use).
hipMemPool_t lib_pool();

template <typename T>
inline hipError_t pool_malloc_async(T** p, size_t bytes, hipStream_t st) {
  hipMemPool_t pool = lib_pool();
  if (!pool) return hipErrorOutOfMemory;
  return hipMallocFromPoolAsync((void**)p, bytes, pool, st);
}

}  // namespace miann
