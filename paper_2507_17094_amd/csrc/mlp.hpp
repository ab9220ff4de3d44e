// Host-callable launchers of the predictor kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miann {

hipError_t gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sar, int64_t sac, const uint16_t* B, int64_t sbr,
                     int64_t sbc, const float* bias, int relu, const uint16_t* mask, float* Cf, uint16_t* Cb, int ldc,
                     hipStream_t st);
hipError_t to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st);
// out[j][k] = in[k][j] for a [K][N] bf16 matrix; rows N .. n_pad - 1 of out are zero.
hipError_t transpose_bf16(const uint16_t* in, int K, int N, int n_pad, uint16_t* out, hipStream_t st);
hipError_t gather_batch(const float* x, int d, const uint32_t* idx, int B, const int32_t* lab, const float* y,
                        uint16_t* xb, int32_t* lb, float* yb, hipStream_t st);
hipError_t loss_grad(const float* Z, int B, int R, const int32_t* lab, const float* y, float lambda, uint16_t* dZ,
                     float* loss, hipStream_t st);
hipError_t colsum(const uint16_t* G, int B, int N, float* db, hipStream_t st);
hipError_t adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* wb, hipStream_t st);
hipError_t readout(const float* Z, int n, int R, int t, float tau, const uint32_t* gmap, int t_min, int t_max,
                   float budget_scale,
                   uint32_t* seeds, int32_t* iters, float* conf, uint32_t* top_idx, hipStream_t st);
hipError_t zero_f32(float* p, int64_t n, hipStream_t st);
// Output layer and read-out in one pass (no logits stored): the read-out's outputs from H2 [n][hidden] bf16 and
// the output layer's weights column by column (W3t [no_pad][hidden], no_pad a multiple of 64 with zero rows past
// R + 1). hidden in {64, 128, 256}; lists: out_readout_lists_bytes(n) of scratch.
bool out_readout_supported(int hidden);
size_t out_readout_lists_bytes(int n);
hipError_t out_readout(const uint16_t* H2, int n, int hidden, const uint16_t* W3t, const float* b3, int R, int t,
                       float tau, const uint32_t* gmap, int t_min, int t_max, float budget_scale, uint64_t* lists,
                       uint32_t* seeds, int32_t* iters, float* conf, uint32_t* top_idx, hipStream_t st);

}  // namespace miann
