// Random-row gather probe: the memory ceiling of the stage kernel's access
// pattern (random rows of a table much larger than the caches), measured with
// the same 8-lane, 16-byte gather the distance evaluation uses.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace miann {

// Random-row gather probe: the HBM ceiling of the stage kernel's access pattern for rows of 128 * CPL bytes.
// 8-lane teams gather rows in 16-byte chunks, two rows per team at a time with all of a lane's chunk loads
// issued before the first is used (as the distance gathers do), fold each row into one word and write it.
// Ids at or beyond n_rows read row 0.
template <int CPL>
__global__ __launch_bounds__(256) void gather_probe_kernel(const void* __restrict__ table, int64_t n_rows,
                                                           const uint32_t* __restrict__ ids, int64_t n,
                                                           uint32_t* __restrict__ out) {
  const int lane = lane_id(), team = lane >> 3, tl = lane & 7;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), nw = (int64_t)gridDim.x * 4;
  const int row16 = 8 * CPL;
  for (int64_t r0 = wave * 16; r0 < n; r0 += nw * 16) {
    const int64_t ra = r0 + team, rb = r0 + 8 + team;
    uint32_t ia = ra < n ? ids[ra] : 0u, ib = rb < n ? ids[rb] : 0u;
    ia = ia < n_rows ? ia : 0u;
    ib = ib < n_rows ? ib : 0u;
    const gptr<u32x4_t> pa = as_global((const u32x4_t*)table + (size_t)ia * row16);
    const gptr<u32x4_t> pb = as_global((const u32x4_t*)table + (size_t)ib * row16);
    uint4 a[CPL], b[CPL];
#pragma unroll
    for (int m = 0; m < CPL; m++) {
      a[m] = load16(pa, tl + 8 * m);
      b[m] = load16(pb, tl + 8 * m);
    }
    uint32_t xa = 0, xb = 0;
#pragma unroll
    for (int m = 0; m < CPL; m++) {
      xa += a[m].x ^ a[m].y ^ a[m].z ^ a[m].w;
      xb += b[m].x ^ b[m].y ^ b[m].z ^ b[m].w;
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      xa += xor_lane_u32(xa, o);
      xb += xor_lane_u32(xb, o);
    }
    if (tl == 0 && ra < n) out[ra] = xa;
    if (tl == 0 && rb < n) out[rb] = xb;
  }
}

hipError_t launch_gather_probe(const void* table, int64_t n_rows, int row_bytes, const uint32_t* ids, int64_t n,
                               uint32_t* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t waves = (n + 15) / 16;
  const unsigned blocks = (unsigned)std::min<int64_t>((waves + 3) / 4, 256 * 16);
  switch (row_bytes / 128) {
#define MIANN_PROBE(C)                                                                                           \
  case C:                                                                                                        \
    hipLaunchKernelGGL(gather_probe_kernel<C>, dim3(blocks), dim3(256), 0, st, table, n_rows, ids, n, out);       \
    break;
    MIANN_PROBE(1)
    MIANN_PROBE(2)
    MIANN_PROBE(3)
    MIANN_PROBE(4)
    MIANN_PROBE(6)
    MIANN_PROBE(8)
#undef MIANN_PROBE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace miann
