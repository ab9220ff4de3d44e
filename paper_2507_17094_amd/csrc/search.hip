// Stage dispatch over vector types and the reduction over shards; the stage
// kernel itself lives in search_impl.hpp, instantiated once per type by
// search_f32.hip, search_f16.hip, search_fp8.hip and search_u8.hip so that
// the four compile in parallel.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace miann {

template <int DT>
hipError_t launch_dt(int cpl, const StageArgs& a, hipStream_t st);
extern template hipError_t launch_dt<DT_F32>(int, const StageArgs&, hipStream_t);
extern template hipError_t launch_dt<DT_F16>(int, const StageArgs&, hipStream_t);
extern template hipError_t launch_dt<DT_FP8>(int, const StageArgs&, hipStream_t);
extern template hipError_t launch_dt<DT_U8>(int, const StageArgs&, hipStream_t);

// Reduction over shards (Sec. 3.1.2): first k of the union of the S sorted
// per-stage lists, by (dist, global id). One wave per query.
__global__ __launch_bounds__(256) void merge_kernel(const uint64_t* so, int64_t nq, int S, int k, int is_u8,
                                                    uint32_t* ids, void* dists) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  const int lane = lane_id();
  const uint64_t* row = so + (size_t)q * S * k;
  int head = 0;
  uint64_t cur = lane < S ? row[(size_t)lane * k] : kDummy;
  for (int i = 0; i < k; i++) {
    uint64_t m = cur;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t other = xor_lane_u64(m, o);
      m = other < m ? other : m;
    }
    if (lane == 0) {
      const bool ok = m != kDummy;
      ids[(size_t)q * k + i] = ok ? (uint32_t)m : kNone;
      if (is_u8) ((int32_t*)dists)[(size_t)q * k + i] = ok ? (int32_t)(m >> 32) : 0x7FFFFFFF;
      else ((uint32_t*)dists)[(size_t)q * k + i] = ok ? (uint32_t)(m >> 32) : 0x7F800000u;
    }
    if (m != kDummy && cur == m && lane < S) {
      head++;
      cur = head < k ? row[(size_t)lane * k + head] : kDummy;
    }
  }
}

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

int stage_lds_bytes(const StageArgs& a) {
  int b = 2 * a.lp_pow2 * 8 + 64 * 8 + kNumCtr * 8 + 64 * 4 + (4 << a.hash_log2) + a.d_pad * 4 + kMaxR * a.W * 4 + 2 * kMaxR * 4;
  return (b + 15) & ~15;
}

hipError_t launch_stage(int dtype, int cpl, const StageArgs& a, hipStream_t st) {
  if (a.nq == 0) return hipSuccess;
  switch (dtype) {
    case DT_F32: return launch_dt<DT_F32>(cpl, a, st);
    case DT_F16: return launch_dt<DT_F16>(cpl, a, st);
    case DT_FP8: return launch_dt<DT_FP8>(cpl, a, st);
    case DT_U8: return launch_dt<DT_U8>(cpl, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_merge(const uint64_t* stage_out, int64_t nq, int S, int k, int is_u8, uint32_t* ids, void* dists,
                        hipStream_t st) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(merge_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, stage_out, nq, S, k, is_u8, ids,
                     dists);
  return hipGetLastError();
}

}  // namespace miann
