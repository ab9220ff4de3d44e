// Host-callable launchers of the index-preparation kernels (build.hip, knn.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miann {

hipError_t pad_rows(const void* src, int64_t n, int d, int esize, void* dst, int d_pad, const uint32_t* rows,
                    hipStream_t st);
hipError_t quantize(const float* src, int64_t n, int d, int store, void* dst, int d_pad, float* scale,
                    const uint32_t* rows, hipStream_t st);
hipError_t sign_table(const void* orig, int in_dtype, int64_t n, int d, int d_pad, const uint32_t* graph, int deg,
                      uint32_t* out, hipStream_t st);
hipError_t gather_rows(const void* src, const uint32_t* ids, int64_t m, int row_bytes, void* dst, hipStream_t st);
hipError_t gather_f32(const float* src, const uint32_t* ids, int64_t m, float* dst, hipStream_t st);
hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t iota_u32(uint32_t* p, int64_t n, uint32_t base, hipStream_t st);
hipError_t count_out_of_range(const uint32_t* ids, int64_t n, uint32_t limit, int allow_none, int64_t* host_bad,
                              hipStream_t st);
hipError_t u8_to_f32(const uint8_t* src, int64_t total, float* dst, hipStream_t st);
// dead[u] = 1 for every u whose gmap[u] is in sorted_ids[0..m) (other flags unchanged).
hipError_t mark_dead(const uint32_t* gmap, int64_t n, const uint32_t* sorted_ids, int64_t m, uint8_t* dead,
                     hipStream_t st);
hipError_t fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st);
// iters[i] = counter 7 of query i ([n][8] counters), budget[i] = log(1 + iters[i]).
hipError_t budget_labels(const int64_t* ctr, int64_t n, int32_t* iters, float* budget, hipStream_t st);
// dst [n][d] (row length d) from src rows of d_pad elements, `esize` bytes each.
hipError_t unpad_rows(const void* src, int64_t n, int d_pad, int esize, void* dst, int d, hipStream_t st);

}  // namespace miann
