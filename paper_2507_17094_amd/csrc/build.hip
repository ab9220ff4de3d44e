// Index-preparation kernels: padded copies, per-vector quantisation, the
// direction sign table (Sec. 3.3.2 (a), Sec. 4), row gathers, small fills.
#include "build.hpp"
#include "pool.hpp"
#include "common.hpp"

namespace miann {

// ---------------------------------------------------------------------------
// Padded copy: dst[v][0..d_pad) = src[v][0..d), zero padding. One wave per row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void pad_rows_kernel(const T* __restrict__ src, int64_t n, int d, T* __restrict__ dst, int d_pad,
                                const uint32_t* __restrict__ rows) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t sv = rows ? (int64_t)rows[v] : v;
  for (int i = lane; i < d_pad; i += 64) dst[v * d_pad + i] = i < d ? src[sv * d + i] : (T)0;
}

hipError_t pad_rows(const void* src, int64_t n, int d, int esize, void* dst, int d_pad, const uint32_t* rows,
                    hipStream_t st) {
  if (n == 0) return hipSuccess;
  dim3 g((unsigned)((n + 3) / 4)), b(256);
  if (esize == 4)
    hipLaunchKernelGGL(pad_rows_kernel<float>, g, b, 0, st, (const float*)src, n, d, (float*)dst, d_pad, rows);
  else
    hipLaunchKernelGGL(pad_rows_kernel<uint8_t>, g, b, 0, st, (const uint8_t*)src, n, d, (uint8_t*)dst, d_pad, rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Quantisation. FP8 E4M3 (OCP "fn"): s = max|x| / 448 (1 if x = 0), code =
// RNE(x / s) saturating at 448. FP16: s = 1, code = RNE(x).
// ---------------------------------------------------------------------------
__device__ uint32_t fp8_encode_rne(float x) {
  if (x != x) return 0x7Fu;
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (a >= 448.f) return sign | 0x7Eu;
  if (a < 0.015625f) {  // below 2^-6: subnormal steps of 2^-9 (m = 8 is the first normal code)
    const uint32_t m = (uint32_t)__builtin_rintf(a * 512.f);
    return sign | m;
  }
  int e;
  const float fr = frexpf(a, &e);  // a = fr * 2^e, fr in [0.5, 1)
  int ex = e - 1;                  // a = (2 fr) * 2^ex, 2 fr in [1, 2)
  uint32_t m = (uint32_t)__builtin_rintf((2.f * fr - 1.f) * 8.f);
  if (m == 8) { m = 0; ex++; }
  uint32_t code = ((uint32_t)(ex + 7) << 3) | m;
  if (code > 0x7Eu) code = 0x7Eu;
  return sign | code;
}

template <int STORE>
__global__ void quantize_kernel(const float* __restrict__ src, int64_t n, int d, void* __restrict__ dst, int d_pad,
                                float* __restrict__ scale, const uint32_t* __restrict__ rows) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t sv = rows ? (int64_t)rows[v] : v;
  const float* x = src + sv * d;
  if (STORE == DT_F16) {
    uint16_t* o = (uint16_t*)dst + v * d_pad;
    for (int i = lane; i < d_pad; i += 64) {
      const _Float16 h = i < d ? (_Float16)x[i] : (_Float16)0.f;
      o[i] = __builtin_bit_cast(uint16_t, h);
    }
    if (lane == 0) scale[v] = 1.f;
  } else {
    float mx = 0.f;
    for (int i = lane; i < d; i += 64) mx = fmaxf(mx, fabsf(x[i]));
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    const float s = mx == 0.f ? 1.f : mx / 448.f;
    uint8_t* o = (uint8_t*)dst + v * d_pad;
    for (int i = lane; i < d_pad; i += 64) o[i] = i < d ? (uint8_t)fp8_encode_rne(x[i] / s) : (uint8_t)0;
    if (lane == 0) scale[v] = s;
  }
}

hipError_t quantize(const float* src, int64_t n, int d, int store, void* dst, int d_pad, float* scale,
                    const uint32_t* rows, hipStream_t st) {
  if (n == 0) return hipSuccess;
  dim3 g((unsigned)((n + 3) / 4)), b(256);
  if (store == DT_F16)
    hipLaunchKernelGGL(quantize_kernel<DT_F16>, g, b, 0, st, src, n, d, dst, d_pad, scale, rows);
  else
    hipLaunchKernelGGL(quantize_kernel<DT_FP8>, g, b, 0, st, src, n, d, dst, d_pad, scale, rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Direction table: for edge (u, slot j, v), bit i of word i/32 (LSB first) is
// [x_v[i] > x_u[i]] on the originals. Layout [n][W][deg] so that the deg
// slots of one word are contiguous (one coalesced read per word at search
// time). One wave per node; one ballot covers 64 coordinates.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void sign_table_kernel(const T* __restrict__ x, int64_t n, int d, int d_pad, const uint32_t* __restrict__ graph,
                                  int deg, int W, uint32_t* __restrict__ out) {
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= n) return;
  const int lane = threadIdx.x & 63;
  const T* xu = x + u * d_pad;
  for (int j = 0; j < deg; j++) {
    const uint32_t v = graph[u * deg + j];
    const T* xv = x + (int64_t)(v == kNone ? 0 : v) * d_pad;
    for (int w2 = 0; w2 < W; w2 += 2) {
      const int i = w2 * 32 + lane;
      const bool gt = v != kNone && i < d && xv[i] > xu[i];
      const uint64_t bits = __ballot(gt);
      if (lane == 0) {
        out[(u * W + w2) * deg + j] = (uint32_t)bits;
        if (w2 + 1 < W) out[(u * W + w2 + 1) * deg + j] = (uint32_t)(bits >> 32);
      }
    }
  }
}

hipError_t sign_table(const void* orig, int in_dtype, int64_t n, int d, int d_pad, const uint32_t* graph, int deg,
                      uint32_t* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int W = (d + 31) / 32;
  dim3 g((unsigned)((n + 3) / 4)), b(256);
  if (in_dtype == DT_U8)
    hipLaunchKernelGGL(sign_table_kernel<uint8_t>, g, b, 0, st, (const uint8_t*)orig, n, d, d_pad, graph, deg, W, out);
  else
    hipLaunchKernelGGL(sign_table_kernel<float>, g, b, 0, st, (const float*)orig, n, d, d_pad, graph, deg, W, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row gather: dst[i] = src[ids[i]] for rows of `row_bytes` (multiple of 16).
// ---------------------------------------------------------------------------
__global__ void gather_rows_kernel(const uint4* __restrict__ src, const uint32_t* __restrict__ ids, int64_t m,
                                   int row16, uint4* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  const int lane = threadIdx.x & 63;
  const int64_t s = ids[r];
  for (int i = lane; i < row16; i += 64) dst[r * row16 + i] = src[s * row16 + i];
}

hipError_t gather_rows(const void* src, const uint32_t* ids, int64_t m, int row_bytes, void* dst, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, (const uint4*)src, ids, m,
                     row_bytes / 16, (uint4*)dst);
  return hipGetLastError();
}

__global__ void gather_f32_kernel(const float* __restrict__ src, const uint32_t* __restrict__ ids, int64_t m,
                                  float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) dst[i] = src[ids[i]];
}

hipError_t gather_f32(const float* src, const uint32_t* ids, int64_t m, float* dst, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_f32_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, src, ids, m, dst);
  return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

__global__ void iota_u32_kernel(uint32_t* p, int64_t n, uint32_t base) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = base + (uint32_t)i;
}

hipError_t iota_u32(uint32_t* p, int64_t n, uint32_t base, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, base);
  return hipGetLastError();
}

// u8 -> f32 padded copy (for the MFMA distance tiles, which work in f32).
__global__ void u8_to_f32_kernel(const uint8_t* __restrict__ src, int64_t total, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < total) dst[i] = (float)src[i];
}

hipError_t u8_to_f32(const uint8_t* src, int64_t total, float* dst, hipStream_t st) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(u8_to_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, total, dst);
  return hipGetLastError();
}

// Counts entries of ids[0..n) that are >= limit (kNone allowed when allow_none).
__global__ void count_bad_kernel(const uint32_t* __restrict__ ids, int64_t n, uint32_t limit, int allow_none,
                                 unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = ids[i];
  if (v >= limit && !(allow_none && v == kNone)) atomicAdd(bad, 1ull);
}

hipError_t count_out_of_range(const uint32_t* ids, int64_t n, uint32_t limit, int allow_none, int64_t* host_bad,
                              hipStream_t st) {
  *host_bad = 0;
  if (n == 0) return hipSuccess;
  unsigned long long* d = nullptr;
  hipError_t e = pool_malloc_async((void**)&d, 8, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, st, (uint32_t*)d, 2, 0u);
  hipLaunchKernelGGL(count_bad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ids, n, limit, allow_none, d);
  unsigned long long h = 0;
  e = hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFreeAsync(d, st);
  *host_bad = (int64_t)h;
  return e;
}

// Unpadded copy: dst [n][d] from src rows of d_pad elements of `esize` bytes.
__global__ void unpad_rows_kernel(const uint8_t* __restrict__ src, int64_t n, int row_src, int row_dst,
                                  uint8_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * row_dst) return;
  const int64_t r = i / row_dst, c = i % row_dst;
  dst[i] = src[r * row_src + c];
}

hipError_t unpad_rows(const void* src, int64_t n, int d_pad, int esize, void* dst, int d, hipStream_t st) {
  const int64_t total = n * (int64_t)d * esize;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(unpad_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, (const uint8_t*)src,
                     n, d_pad * esize, d * esize, (uint8_t*)dst);
  return hipGetLastError();
}

// Predictor labels from per-query counters [n][8]: iters = the last iteration in which the top-k changed
// (counter 7), budget = log(1 + iters) (the regression target).
__global__ void budget_labels_kernel(const int64_t* __restrict__ ctr, int64_t n, int32_t* __restrict__ iters,
                                     float* __restrict__ budget) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t it = ctr[i * 8 + 7];
  iters[i] = (int32_t)it;
  budget[i] = log1pf((float)it);
}

hipError_t budget_labels(const int64_t* ctr, int64_t n, int32_t* iters, float* budget, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(budget_labels_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ctr, n, iters, budget);
  return hipGetLastError();
}

// Deletion flags (Sec. 6.2): dead[u] |= 1 when gmap[u] is one of the m sorted global ids.
__global__ void mark_dead_kernel(const uint32_t* __restrict__ gmap, int64_t n, const uint32_t* __restrict__ ids,
                                 int64_t m, uint8_t* __restrict__ dead) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= n) return;
  const uint32_t g = gmap[u];
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ids[mid] < g) lo = mid + 1;
    else hi = mid;
  }
  if (lo < m && ids[lo] == g) dead[u] = 1;
}

hipError_t mark_dead(const uint32_t* gmap, int64_t n, const uint32_t* sorted_ids, int64_t m, uint8_t* dead,
                     hipStream_t st) {
  if (n == 0 || m == 0) return hipSuccess;
  hipLaunchKernelGGL(mark_dead_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gmap, n, sorted_ids, m,
                     dead);
  return hipGetLastError();
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace miann
