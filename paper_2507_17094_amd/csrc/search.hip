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
  auto put = [&](int i, uint64_t m) {
    const bool ok = m != kDummy;
    ids[(size_t)q * k + i] = ok ? (uint32_t)m : kNone;
    if (is_u8) ((int32_t*)dists)[(size_t)q * k + i] = ok ? (int32_t)(m >> 32) : 0x7FFFFFFF;
    else ((uint32_t*)dists)[(size_t)q * k + i] = ok ? (uint32_t)(m >> 32) : 0x7F800000u;
  };
  const int nk = S * k;
  if (nk <= 128) {
    // all the stages' keys at once (distinct: the shards hold distinct nodes), sorted in registers
    uint64_t v[2] = {lane < nk ? row[lane] : kDummy, 64 + lane < nk ? row[64 + lane] : kDummy};
    if (nk <= 64) {
      v[0] = bitonic_sort_u64<64>(v[0]);
    } else {
      bitonic_sort_regs<2>(v);
    }
    if (lane < k) put(lane, v[0]);
    if (64 + lane < k) put(64 + lane, v[1]);
    return;
  }
  // longer lists: k rounds of the smallest head of the S lists
  int head = 0;
  uint64_t cur = lane < S ? row[(size_t)lane * k] : kDummy;
  for (int i = 0; i < k; i++) {
    uint64_t m = cur;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t other = xor_lane_u64(m, o);
      m = other < m ? other : m;
    }
    if (lane == 0) put(i, m);
    if (m != kDummy && cur == m && lane < S) {
      head++;
      cur = head < k ? row[(size_t)lane * k + head] : kDummy;
    }
  }
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
