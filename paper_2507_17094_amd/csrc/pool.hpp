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

// Scratch that stays with a stream. The hot paths (search scratch, dense entry buffers) lease one block per
// (device, stream, slot); a released block is kept for the next lease on the same stream, whose work the stream
// orders after the previous user's, so back-to-back calls skip the stream-ordered allocator and the markers it
// queues. A lease whose block is held by another host thread on the same stream gets a block of its own from the
// pool instead. A kept block grows in powers of two to cover the largest size asked for and is held until
// scratch_drop_stream (miann_release_scratch) or the end of the process. hipStreamPerThread names a different
// stream in every thread, so its leases are never kept.
enum ScratchSlot { kSlotSearch = 0, kSlotDenseQueries = 1, kSlotDenseWork = 2, kNumSlots = 3 };
struct ScratchLease {
  void* p = nullptr;
  bool kept = false;  // the stream's kept block (else a block of its own)
};
hipError_t scratch_lease(int slot, size_t bytes, hipStream_t st, ScratchLease* out);
void scratch_release(int slot, const ScratchLease& l, hipStream_t st);
// Returns the stream's kept blocks to the pool (stream-ordered frees on `st`, so work already queued on it keeps
// its buffers); blocks leased at the moment stay kept. Call before destroying a stream that searched.
hipError_t scratch_drop_stream(hipStream_t st);

}  // namespace miann
