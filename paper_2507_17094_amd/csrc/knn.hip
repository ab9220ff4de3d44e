// Dense distance tiles on the MFMA units with fused top-K selection.
//
// Work that really is a dense contraction -- queries x ghost nodes for the
// dense ghost entry, the exact k-NN of a shard against itself during graph
// construction, the inter-shard 1-NN map I(u) (Sec. 3.1.2), and exact ground
// truth (Sec. 2.1 Eq. 1) -- runs here. A 256-thread workgroup owns 64 query
// rows; each step computes a 64 x 64 tile of |q|^2 + |x|^2 - 2 q.x with
// v_mfma_f32_32x32x2_f32 (one 32 x 32 block per wave), and each wave then
// filters 16 rows of the tile against that row's current K'-th best key and
// merges survivors into the row's sorted list in LDS. The selected K' = K + 16
// candidates are rescored in direct form (the search kernel's definition: float
// differences, squares summed in double, rounded once), sorted by (dist, id) and
// cut to K, so the result is the exact
// top-K unless the GEMM-form error exceeds the distance gap across 16 ranks.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <map>
#include <mutex>

#include "common.hpp"
#include "pool.hpp"
#include "knn.hpp"

namespace miann {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int TQ = 64;   // query rows per workgroup
constexpr int TX = 64;   // base rows per step
constexpr int KC = 32;   // k-chunk (floats) staged in LDS
constexpr int BSTR = KC + 1;
constexpr int DSTR = TX + 1;

__global__ void fill_cnt_kernel(int* c) { *c = 0; }

__global__ void pad_u8_kernel(const uint8_t* __restrict__ q, int64_t nq, int d, int dp, uint8_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nq * dp) return;
  const int64_t r = i / dp;
  const int c = (int)(i % dp);
  out[i] = c < d ? q[r * d + c] : 0;
}

// Merge sorted candidate keys (one per lane, kDummy = none; keys unique) into
// the sorted list L[0..n). ck: 64-entry scratch.
__device__ void merge_list(uint64_t* L, int n, uint64_t c, uint64_t* ck) {
  const int lane = lane_id();
  const bool real = c != kDummy;
  int pos = 0;
  if (real) {
    int step = 1;
    while (step * 2 <= n) step <<= 1;
    for (; step > 0; step >>= 1)
      if (pos + step <= n && L[pos + step - 1] < c) pos += step;
  } else {
    pos = n;
  }
  const uint64_t vm = __ballot(real && pos < n);
  if (vm == 0) return;
  const int nv = __popcll(vm);
  const int rank = lanes_below(vm);
  if (real && pos < n) ck[rank] = c;
  wsync();
  uint64_t pv[4];
  int np[4];
#pragma unroll
  for (int m = 0; m < 4; m++) {
    const int i = lane + 64 * m;
    np[m] = -1;
    pv[m] = kDummy;
    if (i < n) {
      pv[m] = L[i];
      int p = 0;
      int step = 1;
      while (step * 2 <= nv) step <<= 1;
      for (; step > 0; step >>= 1)
        if (p + step <= nv && ck[p + step - 1] < pv[m]) p += step;
      np[m] = i + p;
    }
  }
  wsync();
#pragma unroll
  for (int m = 0; m < 4; m++) {
    const int i = lane + 64 * m;
    if (np[m] >= 0 && np[m] < n && np[m] != i) L[np[m]] = pv[m];
  }
  if (real && pos < n && pos + rank < n) L[pos + rank] = c;
  wsync();
}

// Sorts the f keys of the row's tail (L[kp..kp+f)), merges them into the
// sorted head L[0..kp), and sets *thr to the head's last key.
__device__ __forceinline__ void compact_tail(uint64_t* L, int kp, int f, uint64_t* thr, uint64_t* ck) {
  const int lane = lane_id();
  uint64_t c = lane < f ? L[kp + lane] : kDummy;
  wsync();
  c = bitonic_sort_u64<64>(c);
  merge_list(L, kp, c, ck);
  if (lane == 0) *thr = L[kp - 1];
  wsync();
}

template <typename TIN>
__global__ __launch_bounds__(256) void tile_select_kernel(const TIN* __restrict__ A, const float* __restrict__ an,
                                                          int64_t na, const int* __restrict__ na_dev,
                                                          const uint32_t* __restrict__ qlist,
                                                          const TIN* __restrict__ B, const float* __restrict__ bn,
                                                          int64_t nb, int dpf, int kp, int tail_cap,
                                                          int exclude_self, uint64_t* __restrict__ out) {
  extern __shared__ __align__(16) char smem[];
  const int ASTR = dpf + 1;
  float* As = (float*)smem;
  float* Bs = As + TQ * ASTR;
  float* Dt = Bs + TX * BSTR;
  // per row: the sorted best kp keys, then a tail of tail_cap (<= 64) entries
  // that collects keys passing the row's threshold until it is full (then it
  // is sorted and merged into the head)
  const int LS = kp + tail_cap;
  uint64_t* lists = (uint64_t*)(((uintptr_t)(Dt + TQ * DSTR) + 15) & ~(uintptr_t)15);
  uint64_t* thr = lists + (size_t)TQ * LS;
  uint64_t* cks = thr + TQ;
  float* anl = (float*)(cks + 4 * 64);
  int* tfill = (int*)(anl + TQ);
  int64_t* qrow = (int64_t*)(((uintptr_t)(tfill + TQ) + 7) & ~(uintptr_t)7);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n_rows = na_dev ? (int64_t)*na_dev : na;
  const int64_t r0 = (int64_t)blockIdx.x * TQ;
  if (r0 >= n_rows) return;

  for (int r = tid; r < TQ; r += 256) {
    const int64_t gr = r0 + r;
    qrow[r] = gr < n_rows ? (qlist ? (int64_t)qlist[gr] : gr) : -1;
  }
  __syncthreads();
  for (int e = tid; e < TQ * dpf; e += 256) {
    const int r = e / dpf, c = e % dpf;
    const int64_t q = qrow[r];
    As[r * ASTR + c] = q >= 0 ? (float)A[q * dpf + c] : 0.f;
  }
  for (int r = tid; r < TQ; r += 256) anl[r] = qrow[r] >= 0 ? an[qrow[r]] : 0.f;
  for (int e = tid; e < TQ * LS; e += 256) lists[e] = kDummy;
  for (int r = tid; r < TQ; r += 256) {
    thr[r] = kDummy;
    tfill[r] = 0;
  }
  __syncthreads();

  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 31, lk = lane >> 5;
  uint64_t* ck = cks + wave * 64;

  for (int64_t j0 = 0; j0 < nb; j0 += TX) {
    floatx16 acc;
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = 0.f;
    for (int kc = 0; kc < dpf; kc += KC) {
      __syncthreads();
      for (int e = tid; e < TX * KC; e += 256) {
        const int r = e / KC, c = e % KC;
        const int64_t gb = j0 + r;
        Bs[r * BSTR + c] = gb < nb ? (float)B[gb * dpf + kc + c] : 0.f;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < KC; kk += 2) {
        const float av = As[(wr + li) * ASTR + kc + kk + lk];
        const float bv = Bs[(wc + li) * BSTR + kk + lk];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const int row = wr + 8 * (j >> 2) + 4 * lk + (j & 3);
      const int col = wc + li;
      const int64_t gb = j0 + col;
      float dv = INFINITY;
      if (gb < nb && qrow[row] >= 0 && !(exclude_self && qrow[row] == gb)) {
        dv = anl[row] + bn[gb] - 2.f * acc[j];
        dv = dv < 0.f ? 0.f : dv;
      }
      Dt[row * DSTR + col] = dv;
    }
    __syncthreads();
    for (int rr = 0; rr < TQ / 4; rr++) {
      const int row = wave * (TQ / 4) + rr;
      if (qrow[row] < 0) continue;
      const float dv = Dt[row * DSTR + lane];
      const uint64_t key = dv < INFINITY ? (((uint64_t)__float_as_uint(dv) << 32) | (uint64_t)(j0 + lane)) : kDummy;
      bool pass = key < thr[row];
      uint64_t m = __ballot(pass);
      if (m == 0) continue;
      int f = tfill[row];
      if (f + __popcll(m) > tail_cap) {
        // tail full: fold it into the sorted head, tighten the threshold, filter again
        if (f > 0) compact_tail(lists + (size_t)row * LS, kp, f, thr + row, ck);
        f = 0;
        pass = key < thr[row];
        m = __ballot(pass);
        if (__popcll(m) > tail_cap) {
          // more survivors than the tail holds: merge them into the head directly
          uint64_t c = pass ? key : kDummy;
          c = bitonic_sort_u64<64>(c);
          merge_list(lists + (size_t)row * LS, kp, c, ck);
          if (lane == 0) thr[row] = lists[(size_t)row * LS + kp - 1];
          wsync();
          continue;
        }
      }
      uint64_t* tail = lists + (size_t)row * LS + kp;
      if (pass) tail[f + lanes_below(m)] = key;
      wsync();
      if (lane == 0) tfill[row] = f + __popcll(m);
      wsync();
    }
  }
  __syncthreads();
  for (int rr = 0; rr < TQ / 4; rr++) {
    const int row = wave * (TQ / 4) + rr;
    const int f = tfill[row];
    if (qrow[row] >= 0 && f > 0) compact_tail(lists + (size_t)row * LS, kp, f, thr + row, ck);
  }
  __syncthreads();
  for (int e = tid; e < TQ * kp; e += 256) {
    const int r = e / kp;
    const int64_t gr = r0 + r;
    if (gr < n_rows) out[gr * kp + (e % kp)] = lists[(size_t)r * LS + (e % kp)];
  }
}

// Row norms |x|^2 in f32 (GEMM-form selection only).
template <typename TIN>
__global__ void norms_kernel(const TIN* __restrict__ X, int64_t n, int dpf, float* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < dpf; i += 64) {
    const double x = (double)X[v * dpf + i];
    s += x * x;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += xor_lane_f64(s, o);
  if (lane == 0) out[v] = (float)s;
}

// Direct-form rescoring of K' candidates per row, sort, keep k.
// Base rows in representation DT ([nb][bpad] codes (+scale)); query rows are
// f32 ([.][bpad]) for float bases or u8 ([.][bpad]) for u8 bases.
template <int DT>
__global__ __launch_bounds__(256) void rescore_kernel(const uint64_t* __restrict__ cand, int64_t nrows,
                                                      const int* __restrict__ nrows_dev, int kp,
                                                      const uint32_t* __restrict__ qlist, const void* __restrict__ Q,
                                                      const void* __restrict__ Bv, const float* __restrict__ bscale,
                                                      int bpad, int k, uint64_t* __restrict__ out) {
  extern __shared__ __align__(16) char smem[];
  constexpr int P16 = Fmt<DT>::per16;
  constexpr int ESZ = Fmt<DT>::esize;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, team = lane >> 3, tl = lane & 7;
  const int64_t r = (int64_t)blockIdx.x * 4 + wave;
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows;
  if (r >= n_rows) return;
  int np2 = 1;
  while (np2 < kp) np2 <<= 1;
  uint64_t* buf = (uint64_t*)smem + (size_t)wave * np2;
  const int64_t qi = qlist ? (int64_t)qlist[r] : r;
  const int row16 = bpad * ESZ / 16;
  for (int c0 = 0; c0 < kp; c0 += 8) {
    const int ci = c0 + team;
    const uint64_t key = ci < kp ? cand[r * kp + ci] : kDummy;
    const bool ok = key != kDummy;
    const uint32_t id = ok ? (uint32_t)key : 0u;
    const uint4* brow = (const uint4*)((const char*)Bv + (size_t)id * bpad * ESZ);
    uint32_t dbits = 0;
    if constexpr (DT == DT_U8) {
      const uint4* qrow = (const uint4*)((const uint8_t*)Q + (size_t)qi * bpad);
      int acc = 0;
      if (ok)
        for (int c = tl; c < row16; c += 8) {
          const uint4 xb = brow[c], qb = qrow[c];
          const uint32_t xw[4] = {xb.x, xb.y, xb.z, xb.w}, qw[4] = {qb.x, qb.y, qb.z, qb.w};
#pragma unroll
          for (int e = 0; e < 16; e++) {
            const int t = (int)((qw[e >> 2] >> (8 * (e & 3))) & 0xFF) - (int)((xw[e >> 2] >> (8 * (e & 3))) & 0xFF);
            acc += t * t;
          }
        }
      acc += xor_lane_i32(acc, 1);
      acc += xor_lane_i32(acc, 2);
      acc += xor_lane_i32(acc, 4);
      dbits = (uint32_t)acc;
    } else {
      const float* qrow = (const float*)Q + (size_t)qi * bpad;
      const float s = (DT == DT_F16 || DT == DT_FP8) ? (ok ? bscale[id] : 0.f) : 1.f;
      double acc = 0.0;
      if (ok)
        for (int c = tl; c < row16; c += 8) {
          float x[P16];
          decode16<DT>(brow[c], x);
#pragma unroll
          for (int e = 0; e < P16; e++) {
            const float xe = (DT == DT_F16 || DT == DT_FP8) ? s * x[e] : x[e];
            const float t = qrow[c * P16 + e] - xe;
            acc = __builtin_fma((double)t, (double)t, acc);
          }
        }
      acc += xor_lane_f64(acc, 1);
      acc += xor_lane_f64(acc, 2);
      acc += xor_lane_f64(acc, 4);
      dbits = __float_as_uint((float)acc);
    }
    if (tl == 0 && ci < kp) buf[ci] = ok ? (((uint64_t)dbits << 32) | id) : kDummy;
  }
  for (int i = kp + lane; i < np2; i += 64) buf[i] = kDummy;
  wsync();
  for (int kk = 2; kk <= np2; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < np2; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = buf[i], y = buf[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) { buf[i] = y; buf[ixj] = x; }
        }
      }
      wsync();
    }
  for (int i = lane; i < k; i += 64) out[qi * k + i] = i < kp ? buf[i] : kDummy;
}

// f32 copy of (f32 | u8) query rows, padded.
__global__ void queries_f32_kernel(const void* __restrict__ q, int q_dt, int64_t nq, int d, int dpf,
                                   float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nq * dpf) return;
  const int64_t r = i / dpf;
  const int c = (int)(i % dpf);
  float v = 0.f;
  if (c < d) v = q_dt == DT_U8 ? (float)((const uint8_t*)q)[r * d + c] : ((const float*)q)[r * d + c];
  out[i] = v;
}

hipError_t queries_to_f32(const void* q, int q_dt, int64_t nq, int d, int dpf, float* out, hipStream_t st) {
  if (nq == 0) return hipSuccess;
  const int64_t tot = nq * dpf;
  hipLaunchKernelGGL(queries_f32_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, q, q_dt, nq, d, dpf,
                     out);
  return hipGetLastError();
}

__global__ void dequant_kernel(const void* __restrict__ store, const float* __restrict__ scale, int dt, int64_t n,
                               int d_pad, int dpf, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * dpf) return;
  const int64_t r = i / dpf;
  const int c = (int)(i % dpf);
  float v = 0.f;
  if (c < d_pad) {
    const void* row = (const char*)store + (size_t)r * d_pad * (dt == DT_F32 ? 4 : dt == DT_F16 ? 2 : 1);
    switch (dt) {
      case DT_F32: v = load_elem<DT_F32>(row, c); break;
      case DT_F16: v = scale[r] * load_elem<DT_F16>(row, c); break;
      case DT_FP8: v = scale[r] * load_elem<DT_FP8>(row, c); break;
      default: v = load_elem<DT_U8>(row, c); break;
    }
  }
  out[i] = v;
}

hipError_t dequant_rows(const void* store, const float* scale, int dt, int64_t n, int d_pad, int dpf, float* out,
                        hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t tot = n * dpf;
  hipLaunchKernelGGL(dequant_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, store, scale, dt, n, d_pad,
                     dpf, out);
  return hipGetLastError();
}

static size_t tile_lds(int dpf, int kp, int tail_cap) {
  size_t b = (size_t)TQ * (dpf + 1) * 4 + (size_t)TX * BSTR * 4 + (size_t)TQ * DSTR * 4 + 16;
  b += (size_t)TQ * (kp + tail_cap) * 8 + TQ * 8 + 4 * 64 * 8 + TQ * 4 + TQ * 4 + 8 + TQ * 8;
  return b;
}

template <typename TIN>
static hipError_t launch_tiles(const TIN* A, const float* an, int64_t na, const int* na_dev, const uint32_t* qlist,
                               const TIN* B, const float* bn, int64_t nb, int dpf, int kp, int exclude_self,
                               uint64_t* out, hipStream_t st) {
  // the largest tail (up to 64 keys per row) that fits the 160 KB of LDS
  int tail_cap = 64;
  while (tail_cap > 0 && tile_lds(dpf, kp, tail_cap) > 160 * 1024) tail_cap -= 8;
  const size_t lds = tile_lds(dpf, kp, tail_cap);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool set = false;
  if (!set) {
    hipFuncSetAttribute((const void*)tile_select_kernel<TIN>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    set = true;
  }
  hipLaunchKernelGGL(tile_select_kernel<TIN>, dim3((unsigned)((na + TQ - 1) / TQ)), dim3(256), lds, st, A, an, na,
                     na_dev, qlist, B, bn, nb, dpf, kp, tail_cap, exclude_self, out);
  return hipGetLastError();
}

static hipError_t launch_rescore(int dt, const uint64_t* cand, int64_t nrows, const int* nrows_dev, int kp,
                                 const uint32_t* qlist, const void* Q, const void* Bv, const float* bscale, int bpad,
                                 int k, uint64_t* out, hipStream_t st) {
  int np2 = 1;
  while (np2 < kp) np2 <<= 1;
  const size_t lds = (size_t)4 * np2 * 8;
  dim3 g((unsigned)((nrows + 3) / 4)), b(256);
  switch (dt) {
    case DT_F32:
      hipLaunchKernelGGL(rescore_kernel<DT_F32>, g, b, lds, st, cand, nrows, nrows_dev, kp, qlist, Q, Bv, bscale, bpad, k, out);
      break;
    case DT_F16:
      hipLaunchKernelGGL(rescore_kernel<DT_F16>, g, b, lds, st, cand, nrows, nrows_dev, kp, qlist, Q, Bv, bscale, bpad, k, out);
      break;
    case DT_FP8:
      hipLaunchKernelGGL(rescore_kernel<DT_FP8>, g, b, lds, st, cand, nrows, nrows_dev, kp, qlist, Q, Bv, bscale, bpad, k, out);
      break;
    default:
      hipLaunchKernelGGL(rescore_kernel<DT_U8>, g, b, lds, st, cand, nrows, nrows_dev, kp, qlist, Q, Bv, bscale, bpad, k, out);
      break;
  }
  return hipGetLastError();
}

hipError_t knn_exact(const float* A_f32, int64_t na, const float* B_f32, int64_t nb, int dpf, int d, int raw_dt,
                     const void* A_raw, int a_raw_pad, const void* B_raw, const float* B_scale, int b_raw_pad, int k,
                     int exclude_self, const uint32_t* qlist, uint64_t* out, hipStream_t st) {
  (void)d;
  (void)a_raw_pad;
  if (na == 0) return hipSuccess;
  int kp = k + 16;
  if (kp > nb - (exclude_self ? 1 : 0)) kp = (int)nb - (exclude_self ? 1 : 0);
  if (kp < k) kp = k;
  float *an = nullptr, *bn = nullptr;
  uint64_t* cand = nullptr;
  hipError_t e = pool_malloc_async(&an, (size_t)na * 4, st);
  if (e == hipSuccess) e = pool_malloc_async(&bn, (size_t)nb * 4, st);
  if (e == hipSuccess) e = pool_malloc_async(&cand, (size_t)na * kp * 8, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(norms_kernel<float>, dim3((unsigned)((na + 3) / 4)), dim3(256), 0, st, A_f32, na, dpf, an);
    hipLaunchKernelGGL(norms_kernel<float>, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, st, B_f32, nb, dpf, bn);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int u8 = raw_dt == DT_U8;
    if (knn_split_supported(dpf, kp, u8))
      e = knn_split_select(A_f32, na, B_f32, nb, dpf, kp, exclude_self, u8, cand, st);
    else
      e = launch_tiles<float>(A_f32, an, na, nullptr, nullptr, B_f32, bn, nb, dpf, kp, exclude_self, cand, st);
  }
  // rows of `cand` are indexed by position; rescoring reads query row qlist[r] (or r)
  if (e == hipSuccess) e = launch_rescore(raw_dt, cand, na, nullptr, kp, qlist, A_raw, B_raw, B_scale, b_raw_pad, k, out, st);
  if (an) hipFreeAsync(an, st);
  if (bn) hipFreeAsync(bn, st);
  if (cand) hipFreeAsync(cand, st);
  return e;
}

// ---------------------------------------------------------------------------
// Dense ghost entry. The queries-by-ghosts contraction is a plain GEMM: tiles
// of 64 query rows x 64 ghosts on v_mfma_f32_32x32x2_f32 write the GEMM-form
// distances |q|^2 + |g|^2 - 2 q.g of a block of rows to D. One wave per row
// then selects the kp smallest (dist, ghost) keys of its row: the kp-th
// smallest of the two smallest keys of each lane's columns bounds the row's
// kp-th smallest key from above, the keys at or below the bound are collected
// and sorted, and if more than CAP pass, the bound is lowered to the kp-th
// smallest of the first CAP collected and the row scanned again.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dense_gemm_kernel(const float* __restrict__ Q, const float* __restrict__ qn,
                                                         const int* __restrict__ nrows_dev, int64_t nrows_max,
                                                         const uint32_t* __restrict__ qlist, int64_t row0,
                                                         int64_t rows_chunk, const float* __restrict__ G,
                                                         const float* __restrict__ gn, int64_t R, int dpf,
                                                         int64_t ldd, float* __restrict__ D) {
  __shared__ float As[64 * BSTR];
  __shared__ float Bs[64 * BSTR];
  __shared__ int64_t qrow[64];
  __shared__ float qnl[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows_max;
  const int64_t rl0 = (int64_t)blockIdx.y * 64;  // first row of the tile within the chunk
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  if (row0 + rl0 >= n_rows || rl0 >= rows_chunk) return;
  for (int r = tid; r < 64; r += 256) {
    const int64_t gr = row0 + rl0 + r;
    const bool ok = gr < n_rows && rl0 + r < rows_chunk;
    qrow[r] = ok ? (qlist ? (int64_t)qlist[gr] : gr) : -1;
    qnl[r] = ok ? qn[qrow[r]] : 0.f;
  }
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 31, lk = lane >> 5;
  floatx16 acc;
#pragma unroll
  for (int j = 0; j < 16; j++) acc[j] = 0.f;
  for (int kc = 0; kc < dpf; kc += KC) {
    __syncthreads();
    for (int e = tid; e < 64 * KC; e += 256) {
      const int r = e / KC, c = e % KC;
      const int64_t q = qrow[r];
      As[r * BSTR + c] = (q >= 0 && kc + c < dpf) ? Q[q * dpf + kc + c] : 0.f;
      const int64_t g = c0 + r;
      Bs[r * BSTR + c] = (g < R && kc + c < dpf) ? G[g * dpf + kc + c] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; kk += 2) {
      const float av = As[(wr + li) * BSTR + kk + lk];
      const float bv = Bs[(wc + li) * BSTR + kk + lk];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const int row = wr + 8 * (j >> 2) + 4 * lk + (j & 3);
    const int64_t col = c0 + wc + li;
    if (qrow[row] >= 0 && col < R) {
      float dv = qnl[row] + gn[col] - 2.f * acc[j];
      D[(rl0 + row) * ldd + col] = dv < 0.f ? 0.f : dv;
    }
  }
}

template <int CAP>
__global__ __launch_bounds__(256) void dense_select_kernel(const float* __restrict__ D, int64_t ldd, int64_t R,
                                                           const int* __restrict__ nrows_dev, int64_t nrows_max,
                                                           int64_t row0, int64_t rows_chunk, int kp,
                                                           uint64_t* __restrict__ out) {
  constexpr int NR = CAP / 64;
  __shared__ uint64_t bufs[4 * CAP];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t rl = (int64_t)blockIdx.x * 4 + wave;
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows_max;
  if (rl >= rows_chunk || row0 + rl >= n_rows) return;
  uint64_t* buf = bufs + wave * CAP;
  const float* d = D + rl * ldd;
  auto mk = [](float v, int64_t j) { return ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)j; };
  // the two smallest keys of this lane's columns
  uint64_t m[2] = {kDummy, kDummy};
  for (int64_t j = lane; j < R; j += 64) {
    const uint64_t key = mk(d[j], j);
    if (key < m[0]) {
      m[1] = m[0];
      m[0] = key;
    } else if (key < m[1]) {
      m[1] = key;
    }
  }
  bitonic_sort_regs<2>(m);
  const int rb = (kp - 1) >> 6, lb = (kp - 1) & 63;
  uint64_t bound = shfl_u64(rb == 0 ? m[0] : m[1], lb);
  uint64_t v[NR];
  for (;;) {
    int cnt = 0;
    for (int64_t j0 = 0; j0 < R; j0 += 64) {
      const int64_t j = j0 + lane;
      const uint64_t key = j < R ? mk(d[j], j) : kDummy;
      const bool pass = key != kDummy && key <= bound;
      const uint64_t bm = ballot(pass);
      const int pos = cnt + lanes_below(bm);
      if (pass && pos < CAP) buf[pos] = key;
      cnt += __popcll(bm);
    }
    wsync();
#pragma unroll
    for (int r = 0; r < NR; r++) {
      const int i = r * 64 + lane;
      v[r] = i < cnt && i < CAP ? buf[i] : kDummy;
    }
    wsync();
    bitonic_sort_regs<NR>(v);
    if (cnt <= CAP) break;
    // more than CAP keys at or below the bound: the kp-th smallest of the first CAP is a lower bound
    uint64_t x = v[0];
#pragma unroll
    for (int r = 1; r < NR; r++)
      if (r == rb) x = v[r];
    bound = shfl_u64(x, lb);
  }
  uint64_t* o = out + (row0 + rl) * kp;
#pragma unroll
  for (int r = 0; r < NR; r++) {
    const int i = r * 64 + lane;
    if (i < kp) o[i] = v[r];
  }
}

__global__ void shard_qlist_kernel(int64_t nq, const uint64_t* __restrict__ qkeys, int S, int shard, int all,
                                   uint32_t* __restrict__ list, int* __restrict__ count) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  const uint64_t key = qkeys ? qkeys[q] : (uint64_t)q;
  if (all || (int)(key % (uint64_t)S) == shard) list[atomicAdd(count, 1)] = (uint32_t)q;
}

__global__ void dense_out_kernel(const uint64_t* __restrict__ best, const uint32_t* __restrict__ list,
                                 const int* __restrict__ count, int t, const uint32_t* __restrict__ g_map, int S,
                                 int shard, uint64_t* __restrict__ out) {
  // g_map == nullptr: emit ghost indices instead of the nodes they copy
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = i / t;
  const int j = (int)(i % t);
  if (r >= *count) return;
  const uint32_t q = list[r];
  const uint64_t key = best[(size_t)q * t + j];
  const uint32_t g = (uint32_t)key;
  out[((size_t)q * S + shard) * t + j] =
      key == kDummy ? kDummy : ((key & 0xFFFFFFFF00000000ull) | (g_map ? g_map[g] : g));
}

hipError_t dense_entry(int store_dt, const void* queries, int64_t nq, int d, const uint64_t* qkeys, int S, int shard,
                       int ppe, const float* g_f32, const void* g_store, const float* g_scale, const uint32_t* g_map,
                       int64_t R, int d_pad, int d_pad_f32, int t, uint64_t* out, hipStream_t st) {
  if (nq == 0) return hipSuccess;
  const int qdt = store_dt == DT_U8 ? DT_U8 : DT_F32;
  int kp = t + 16;
  if (kp > R) kp = (int)R;
  if (kp < t) kp = t;
  char* buf = nullptr;
  const size_t sz_list = ((size_t)nq * 4 + 255) & ~(size_t)255;
  const size_t sz_cnt = 256;
  const size_t sz_qf = ((size_t)nq * d_pad_f32 * 4 + 255) & ~(size_t)255;
  const size_t sz_qraw = ((size_t)nq * d_pad * (qdt == DT_U8 ? 1 : 4) + 255) & ~(size_t)255;
  const size_t sz_qn = ((size_t)nq * 4 + 255) & ~(size_t)255;
  const size_t sz_gn = ((size_t)R * 4 + 255) & ~(size_t)255;
  const size_t sz_cand = ((size_t)nq * kp * 8 + 255) & ~(size_t)255;
  const size_t sz_best = (size_t)nq * t * 8;
  const size_t total = sz_list + sz_cnt + sz_qf + sz_qraw + sz_qn + sz_gn + sz_cand + sz_best;
  hipError_t e = pool_malloc_async((void**)&buf, total, st);
  if (e != hipSuccess) return e;
  char* p = buf;
  uint32_t* list = (uint32_t*)p; p += sz_list;
  int* cnt = (int*)p; p += sz_cnt;
  float* qf = (float*)p; p += sz_qf;
  void* qraw = p; p += sz_qraw;
  float* qn = (float*)p; p += sz_qn;
  float* gn = (float*)p; p += sz_gn;
  uint64_t* cand = (uint64_t*)p; p += sz_cand;
  uint64_t* best = (uint64_t*)p;
  hipLaunchKernelGGL(fill_cnt_kernel, dim3(1), dim3(1), 0, st, cnt);
  hipLaunchKernelGGL(shard_qlist_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, nq, qkeys, S, shard,
                     ppe ? 0 : 1, list, cnt);
  e = queries_to_f32(queries, qdt, nq, d, d_pad_f32, qf, st);
  if (e == hipSuccess) {
    if (qdt == DT_U8) {
      hipLaunchKernelGGL(pad_u8_kernel, dim3((unsigned)((nq * d_pad + 255) / 256)), dim3(256), 0, st,
                         (const uint8_t*)queries, nq, d, d_pad, (uint8_t*)qraw);
    } else {
      e = queries_to_f32(queries, DT_F32, nq, d, d_pad, (float*)qraw, st);
    }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(norms_kernel<float>, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, qf, nq, d_pad_f32, qn);
    hipLaunchKernelGGL(norms_kernel<float>, dim3((unsigned)((R + 3) / 4)), dim3(256), 0, st, g_f32, R, d_pad_f32, gn);
    e = hipGetLastError();
  }
  // GEMM-form distances of blocks of rows against all ghosts, then per-row selection of kp candidates
  const int64_t ldd = (R + 63) / 64 * 64;
  int64_t chunk = ((int64_t)1 << 27) / ldd;  // at most 512 MB of distances at a time
  chunk = chunk < 64 ? 64 : chunk / 64 * 64;
  if (chunk > (nq + 63) / 64 * 64) chunk = (nq + 63) / 64 * 64;
  float* D = nullptr;
  if (e == hipSuccess) e = pool_malloc_async((void**)&D, (size_t)chunk * ldd * 4, st);
  for (int64_t row0 = 0; row0 < nq && e == hipSuccess; row0 += chunk) {
    hipLaunchKernelGGL(dense_gemm_kernel, dim3((unsigned)(ldd / 64), (unsigned)(chunk / 64)), dim3(256), 0, st, qf,
                       qn, cnt, nq, list, row0, chunk, g_f32, gn, R, d_pad_f32, ldd, D);
    hipLaunchKernelGGL(dense_select_kernel<256>, dim3((unsigned)((chunk + 3) / 4)), dim3(256), 0, st, D, ldd, R, cnt,
                       nq, row0, chunk, kp, cand);
    e = hipGetLastError();
  }
  if (D) hipFreeAsync(D, st);
  if (e == hipSuccess)
    e = launch_rescore(store_dt, cand, nq, cnt, kp, list, qraw, g_store, g_scale, d_pad, t, best, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(dense_out_kernel, dim3((unsigned)((nq * t + 255) / 256)), dim3(256), 0, st, best, list, cnt, t,
                       g_map, S, shard, out);
    e = hipGetLastError();
  }
  hipFreeAsync(buf, st);
  return e;
}

// ---------------------------------------------------------------------------
// Dense ghost entry over the ghosts of several shards at once. The ghost rows
// of every shard are concatenated (each shard's block padded to a multiple of
// 64 columns) and their traversal values split as x = hi + lo with hi, lo in
// bf16, so q.x ~ qh.xh + qh.xl + ql.xh on the bf16 matrix cores with f32
// accumulation (relative error about 2^-16 of |q||x|, far below the distance
// gaps the 16 extra candidates absorb; the candidates are rescored exactly).
// The distances are never stored: pass 1 keeps the smallest key of every 8
// columns, a bound kernel takes for each (query, shard) the kp-th smallest of a
// subset of those minima (so at least kp keys lie at or below it), pass 2
// recomputes the tiles and appends only the keys at or below the bound to a
// short per-(query, shard) list, and one wave per list sorts it, rescores the
// kp smallest exactly and writes the exact top-t seeds.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// hi/lo bf16 split and f32 norm of n rows of x ([n][dk] f32); rows n..n_pad get zeros and norm +inf.
__global__ void split_rows_kernel(const float* __restrict__ x, int64_t n, int64_t n_pad, int dk,
                                  uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, float* __restrict__ norm) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n_pad) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int c = lane; c < dk; c += 64) {
    const float v = r < n ? x[r * dk + c] : 0.f;
    const uint16_t h = f32_to_bf16(v);
    hi[r * dk + c] = h;
    lo[r * dk + c] = f32_to_bf16(v - bf16_to_f32(h));
    s += (double)v * (double)v;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += xor_lane_f64(s, o);
  if (lane == 0) norm[r] = r < n ? (float)s : INFINITY;
}

hipError_t split_rows(const float* x, int64_t n, int64_t n_pad, int dk, uint16_t* hi, uint16_t* lo, float* norm,
                      hipStream_t st) {
  if (n_pad == 0) return hipSuccess;
  hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)((n_pad + 3) / 4)), dim3(256), 0, st, x, n, n_pad, dk, hi, lo,
                     norm);
  return hipGetLastError();
}

// Query preparation of the dense entry in one pass, one wave per row: the hi/lo bf16 split and f32 norm over dk
// columns (as split_rows_kernel computes them from the f32 row padded to dk), and the exact-distance copy of the
// row padded to d_pad (f32, or u8 for u8 queries).
__global__ __launch_bounds__(256) void dense_queries_kernel(const void* __restrict__ q, int q_dt, int64_t nq, int d,
                                                            int dk, int d_pad, uint16_t* __restrict__ hi,
                                                            uint16_t* __restrict__ lo, float* __restrict__ norm,
                                                            void* __restrict__ qraw) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nq) return;
  const int lane = threadIdx.x & 63;
  const int cmax = dk > d_pad ? dk : d_pad;
  double s = 0.0;
  for (int c = lane; c < cmax; c += 64) {
    float v = 0.f;
    uint8_t b = 0;
    if (c < d) {
      if (q_dt == DT_U8) {
        b = ((const uint8_t*)q)[r * d + c];
        v = (float)b;
      } else {
        v = ((const float*)q)[r * d + c];
      }
    }
    if (c < dk) {
      const uint16_t h = f32_to_bf16(v);
      hi[r * dk + c] = h;
      lo[r * dk + c] = f32_to_bf16(v - bf16_to_f32(h));
      s += (double)v * (double)v;
    }
    if (c < d_pad) {
      if (q_dt == DT_U8) ((uint8_t*)qraw)[r * d_pad + c] = b;
      else ((float*)qraw)[r * d_pad + c] = v;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += xor_lane_f64(s, o);
  if (lane == 0) norm[r] = (float)s;
}

constexpr int CAPG = 256; // candidates sorted per (query, shard); more fall back to an exact scan
// Pass 1 keeps, per lane slot and block, KEEP of the GEMM-form distances of its 16 register classes: the 4 smallest
// (t <= 8) or all 16, in a row of mcap values per (row, shard) (at least 2 t where the split of the tiles allows).

// LDS rows of the tile kernel: hi and lo bf16 copies of 64 ghost columns, each row padded by 8 elements (16 bytes)
// against bank conflicts.
__host__ __device__ constexpr int dense_lds_stride(int dk) { return dk + 8; }

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// 64 rows x DK bf16 (hi and lo) staged by 256 threads: thread t owns row t / 4
// and the 16-byte chunks c = t % 4 + 4 m of it (DK / 32 chunks per array).
template <int DK>
struct Stage64 {
  static constexpr int NCH = DK / 32;
  u32x4_t h[NCH], l[NCH];  // ext-vector registers (a struct-typed uint4 array would live in scratch)
  __device__ __forceinline__ void load(const uint16_t* __restrict__ H, const uint16_t* __restrict__ L, int64_t row,
                                       int c0) {
    const u32x4_t* hp = (const u32x4_t*)(H + row * DK) + c0;
    const u32x4_t* lp = (const u32x4_t*)(L + row * DK) + c0;
#pragma unroll
    for (int m = 0; m < NCH; m++) {
      h[m] = hp[4 * m];
      l[m] = lp[4 * m];
    }
  }
  __device__ __forceinline__ void store(uint16_t* Sh, uint16_t* Sl, int r, int c0) const {
    constexpr int P = dense_lds_stride(DK);
#pragma unroll
    for (int m = 0; m < NCH; m++) {
      *(u32x4_t*)&Sh[r * P + (c0 + 4 * m) * 8] = h[m];
      *(u32x4_t*)&Sl[r * P + (c0 + 4 * m) * 8] = l[m];
    }
  }
};

// The accumulators of a 32-ghost half tile start at -gn/2 of their ghosts: register j of the lanes of half
// h = lane / 32 holds ghost 8 (j / 4) + 4 h + j % 4 of the half, four consecutive ghosts per 16-byte LDS read.
__device__ __forceinline__ void init_acc(f32x16_t& acc, const float* ngl, int h) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const f32x4_t v = *(const f32x4_t*)&ngl[8 * q + 4 * h];
#pragma unroll
    for (int r = 0; r < 4; r++) acc[4 * q + r] = v[r];
  }
}

// Inserts x into k, kept in descending order.
template <int KEEP>
__device__ __forceinline__ void keep_largest(float (&k)[KEEP], float x) {
#pragma unroll
  for (int i = 0; i < KEEP - 1; i++) {
    const float hi = fmaxf(k[i], x);
    x = fminf(k[i], x);
    k[i] = hi;
  }
  k[KEEP - 1] = fmaxf(k[KEEP - 1], x);
}

// Writes a lane's KEEP smallest GEMM-form distances G = qn - 2 a (clamped at 0) from its per-register maxima of a
// (all 16 when KEEP is 16; 16-byte aligned destination).
template <int KEEP>
__device__ __forceinline__ void write_kept(float* __restrict__ dst, const float (&mx)[16], float qv) {
  if constexpr (KEEP == 16) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      f32x4_t o;
#pragma unroll
      for (int i = 0; i < 4; i++) o[i] = fmaxf(qv - 2.f * mx[4 * q + i], 0.f);
      ((f32x4_t*)dst)[q] = o;
    }
  } else {
    static_assert(KEEP == 4, "KEEP");
    float k[KEEP];
#pragma unroll
    for (int i = 0; i < KEEP; i++) k[i] = -INFINITY;
#pragma unroll
    for (int j = 0; j < 16; j++) keep_largest<KEEP>(k, mx[j]);
    f32x4_t o;
#pragma unroll
    for (int i = 0; i < KEEP; i++) o[i] = fmaxf(qv - 2.f * k[i], 0.f);
    *(f32x4_t*)dst = o;
  }
}

// Work item of a tile-pass block: (shard, row block, column group), numbered shard-major, and handed out so that
// the blocks the dispatcher sends to one XCD (block ids congruent mod nxcd) take one contiguous run of items: a
// run spans few shards and row blocks, so an XCD's L2 holds those shards' ghost tiles and those rows' queries.
struct TileItem {
  int sl, grp;
  int64_t rb;
};
__device__ __forceinline__ bool tile_item(int nxcd, int64_t rtiles, int nseg, int gps, TileItem& it) {
  const int64_t nitems = rtiles * nseg * gps;
  const int64_t per = (nitems + nxcd - 1) / nxcd;
  const int64_t b = blockIdx.x;
  const int64_t item = (b % nxcd) * per + b / nxcd;
  if (item >= nitems) return false;
  it.sl = (int)(item / (rtiles * gps));
  const int64_t r = item % (rtiles * gps);
  it.rb = r / gps;
  it.grp = (int)(r % gps);
  return true;
}

// Query row sets of 32 a wave of the tile kernel keeps in registers for rows of dk elements, and the ghost tile
// buffers in LDS (two where two blocks per CU still fit: the next tile is stored while this one is multiplied, one
// barrier per tile).
__host__ __device__ constexpr int dense_wide_sets(int dk) { return dk <= 96 ? 2 : 1; }
__host__ __device__ constexpr int dense_wide_bufs(int dk) { return dk <= 96 ? 2 : 1; }
// Dynamic LDS of the tile kernel: NBUF x (hi and lo tiles of 64 padded rows, 64 floats of -gn/2).
inline size_t dense_wide_lds(int dk) {
  return (size_t)dense_wide_bufs(dk) * ((size_t)2 * 64 * dense_lds_stride(dk) * 2 + 64 * 4);
}

// GEMM-form distances G = qn - 2 a with a = q.x - gn/2 (three bf16 products hi.hi + hi.lo + lo.hi accumulated in
// float32 onto -gn/2) of a block's query rows against a run of 64-column ghost tiles of one shard. Each wave keeps
// NS sets of 32 rows' hi and lo fragments in registers for the whole run of tiles (a block of 4 waves owns 128 NS
// rows) and multiplies them with the two 32-ghost halves of every tile in turn, ghosts as the first operand, so an
// accumulator leaves one query per lane (lane & 31), each ghost fragment read from LDS feeds 3 NS MFMAs, and
// register j of half c holds ghost 32 c + 8 (j / 4) + 4 (lane / 32) + j % 4. Only the ghost tile goes through LDS.
//   MODE 0: one maximum of a per register over the block's tiles; each lane writes KEEP of the G of each set's
//   row (the smallest; clamped at 0), each the GEMM form of a distinct ghost, to
//   M[row][shard][group][lane / 32][KEEP] (mcap values per row and shard);
//   MODE 1: the mask word of (row, shard, tile, lane / 32) of each set's row: bit 16 c + j for a at or above the
//   row's threshold.
// The next tile's columns are loaded into registers while the current one is multiplied. Padding columns carry
// norm +inf, so their a is -inf: never a maximum or a candidate (thresholds are finite). Rows without a query get
// a NaN threshold and never qualify; their pass-1 values land in the chunk's buffers and are never read.
// (two sets and 2 waves per SIMD up to 96-element rows; one set above, at most 256 registers)
template <int MODE, int DK, int KEEP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void dense_tiles_wide_kernel(
    const uint16_t* __restrict__ Qh, const uint16_t* __restrict__ Ql, const float* __restrict__ qn,
    const uint32_t* __restrict__ list, const int* __restrict__ nrows_dev, int64_t nrows_max, int64_t row0,
    int64_t rows_chunk, const uint16_t* __restrict__ Gh, const uint16_t* __restrict__ Gl,
    const float* __restrict__ gn, const int64_t* __restrict__ off, int s0, int nseg, int gps, int cg, int nht,
    int nxcd, int64_t rtiles, int mcap, float* __restrict__ M, const float* __restrict__ thr,
    uint32_t* __restrict__ cmask) {
  static_assert(DK % 32 == 0 && DK <= 256, "DK");
  constexpr int P = dense_lds_stride(DK);
  constexpr int KB = DK / 16;
  constexpr int NS = dense_wide_sets(DK);
  constexpr int NBUF = dense_wide_bufs(DK);
  extern __shared__ __align__(16) char dsm[];
  uint16_t(*Bh)[64 * P] = (uint16_t(*)[64 * P])dsm;
  uint16_t(*Bl)[64 * P] = Bh + NBUF;
  float(*ngl)[64] = (float(*)[64])(Bl + NBUF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows_max;
  TileItem it;
  if (!tile_item(nxcd, rtiles, nseg, gps, it)) return;
  const int64_t rl0 = it.rb * (128 * NS);
  const int sl = it.sl, grp = it.grp;
  const int s = s0 + sl;
  const int64_t cb = off[s];  // first column of the shard's block
  const int ntiles = (int)((off[s + 1] - cb) / 64);
  const int tt0 = grp * cg, tt1 = tt0 + cg < ntiles ? tt0 + cg : ntiles;
  if (row0 + rl0 >= n_rows || rl0 >= rows_chunk || tt0 >= tt1) return;
  const int h = lane >> 5, col = lane & 31;
  int64_t rl[NS];  // this lane's rows of the chunk, one per set
  float qv[NS];    // MODE 0: the row's norm; MODE 1: its threshold on a (NaN for rows without a query)
  bf16x8_t qh[NS][KB], ql[NS][KB];
#pragma unroll
  for (int si = 0; si < NS; si++) {
    rl[si] = rl0 + (wave * NS + si) * 32 + col;
    const int64_t gr = row0 + rl[si];
    const int64_t qa = gr < n_rows && rl[si] < rows_chunk ? (list ? (int64_t)list[gr] : gr) : -1;
    qv[si] = qa < 0 ? __builtin_nanf("") : (MODE == 0 ? qn[qa] : thr[rl[si] * nseg + sl]);
    const int64_t q = qa < 0 ? 0 : qa;  // rows without a query read row 0
    const bf16x8_t* hp = (const bf16x8_t*)(Qh + q * DK + h * 8);
    const bf16x8_t* lp = (const bf16x8_t*)(Ql + q * DK + h * 8);
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
      qh[si][kb] = hp[2 * kb];
      ql[si][kb] = lp[2 * kb];
    }
  }
  const int sr = tid >> 2, sc0 = tid & 3;
  Stage64<DK> nb;
  nb.load(Gh, Gl, cb + (int64_t)tt0 * 64 + sr, sc0);
  float ng = sc0 == 0 ? -0.5f * gn[cb + (int64_t)tt0 * 64 + sr] : 0.f;
  float mx[NS][16];
#pragma unroll
  for (int si = 0; si < NS; si++)
#pragma unroll
    for (int j = 0; j < 16; j++) mx[si][j] = -INFINITY;
  if constexpr (NBUF == 2) {
    nb.store(Bh[0], Bl[0], sr, sc0);
    if (sc0 == 0) ngl[0][sr] = ng;
    if (tt0 + 1 < tt1) {
      const int64_t nxt = cb + (int64_t)(tt0 + 1) * 64 + sr;
      nb.load(Gh, Gl, nxt, sc0);
      if (sc0 == 0) ng = -0.5f * gn[nxt];
    }
  }
  for (int tt = tt0; tt < tt1; tt++) {
    const int cur = NBUF == 2 ? (tt - tt0) & 1 : 0;
    if constexpr (NBUF == 2) {
      __syncthreads();  // tile tt is stored in buffer cur, and the other buffer's tile is consumed
      if (tt + 1 < tt1) {
        nb.store(Bh[cur ^ 1], Bl[cur ^ 1], sr, sc0);
        if (sc0 == 0) ngl[cur ^ 1][sr] = ng;
        if (tt + 2 < tt1) {
          const int64_t nxt = cb + (int64_t)(tt + 2) * 64 + sr;
          nb.load(Gh, Gl, nxt, sc0);
          if (sc0 == 0) ng = -0.5f * gn[nxt];
        }
      }
    } else {
      __syncthreads();  // the previous tile is consumed
      nb.store(Bh[0], Bl[0], sr, sc0);
      if (sc0 == 0) ngl[0][sr] = ng;
      {
        const int64_t nxt = cb + (int64_t)(tt + 1 < tt1 ? tt + 1 : tt) * 64 + sr;  // (the last tile reloads itself)
        nb.load(Gh, Gl, nxt, sc0);
        if (sc0 == 0) ng = -0.5f * gn[nxt];
      }
      __syncthreads();
    }
    const uint16_t* bh = Bh[cur];
    const uint16_t* bl = Bl[cur];
    uint32_t w[NS];
#pragma unroll
    for (int si = 0; si < NS; si++) w[si] = 0;
    // the tile's two 32-ghost halves one after the other (half the accumulator registers, left to fragment reads)
#pragma unroll
    for (int c = 0; c < 2; c++) {
      f32x16_t acc[NS];
      init_acc(acc[0], ngl[cur] + 32 * c, h);
#pragma unroll
      for (int si = 1; si < NS; si++) acc[si] = acc[0];
#pragma unroll
      for (int kb = 0; kb < KB; kb++) {
        const int rb = (32 * c + col) * P + kb * 16 + h * 8;
        const bf16x8_t gh = *(const bf16x8_t*)&bh[rb], gl = *(const bf16x8_t*)&bl[rb];
#pragma unroll
        for (int si = 0; si < NS; si++) {
          acc[si] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gh, qh[si][kb], acc[si], 0, 0, 0);
          acc[si] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gl, qh[si][kb], acc[si], 0, 0, 0);
          acc[si] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gh, ql[si][kb], acc[si], 0, 0, 0);
        }
      }
#pragma unroll
      for (int si = 0; si < NS; si++) {
        if constexpr (MODE == 0) {
#pragma unroll
          for (int j = 0; j < 16; j++) mx[si][j] = fmaxf(mx[si][j], acc[si][j]);
        } else {
#pragma unroll
          for (int j = 0; j < 16; j++) w[si] |= acc[si][j] >= qv[si] ? 1u << (16 * c + j) : 0u;
        }
      }
    }
    if constexpr (MODE == 1) {
#pragma unroll
      for (int si = 0; si < NS; si++) cmask[(rl[si] * nseg + sl) * nht + 2 * tt + h] = w[si];
    }
  }
  if constexpr (MODE == 0) {
#pragma unroll
    for (int si = 0; si < NS; si++)
      write_kept<KEEP>(M + (rl[si] * nseg + sl) * mcap + (grp * 2 + h) * KEEP, mx[si], qv[si]);
  }
}

template <int MODE, int KEEP>
static void launch_dense_tiles(int dk, dim3 grid, hipStream_t st, const uint16_t* qh, const uint16_t* ql,
                               const float* qn, const uint32_t* rl, const int* rc, int64_t nq, int64_t row0,
                               int64_t chunk, const DenseGhosts& G, int s0, int nseg, int gps, int cg, int nht,
                               int nxcd, int64_t rtiles, int mcap, float* Mg, const float* thr, uint32_t* cmask) {
  const size_t lds = dense_wide_lds(dk);
#define MIANN_DENSE_WIDE(KC)                                                                                         \
  case KC: {                                                                                                         \
    static std::once_flag set;                                                                                       \
    std::call_once(set, [] {                                                                                         \
      (void)hipFuncSetAttribute((const void*)dense_tiles_wide_kernel<MODE, 32 * KC, KEEP>,                           \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)dense_wide_lds(32 * KC));            \
    });                                                                                                              \
    hipLaunchKernelGGL((dense_tiles_wide_kernel<MODE, 32 * KC, KEEP>), grid, dim3(256), lds, st, qh, ql, qn, rl, rc, \
                       nq, row0, chunk, G.hi, G.lo, G.norm, G.off_dev, s0, nseg, gps, cg, nht, nxcd, rtiles, mcap, Mg, \
                       thr, cmask);                                                                                  \
    break;                                                                                                           \
  }
  switch (dk / 32) {
    MIANN_DENSE_WIDE(1)
    MIANN_DENSE_WIDE(2)
    MIANN_DENSE_WIDE(3)
    MIANN_DENSE_WIDE(4)
    MIANN_DENSE_WIDE(5)
    MIANN_DENSE_WIDE(6)
    MIANN_DENSE_WIDE(7)
    MIANN_DENSE_WIDE(8)
    default: break;
  }
#undef MIANN_DENSE_WIDE
}

// Blocks of the pass-1 tile kernel for rows of dk elements one CU holds at once, times the device's CUs (per device
// and dk, from the occupancy query).
static int64_t dense_tile_slots(int dk) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({dev, dk});
  if (it != cache.end()) return it->second;
  int ncu = 0, per = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
  hipError_t e = hipErrorInvalidValue;
#define MIANN_SLOTS_WIDE(KC)                                                                                         \
  case KC:                                                                                                           \
    (void)hipFuncSetAttribute((const void*)dense_tiles_wide_kernel<0, 32 * KC, 4>,                                   \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)dense_wide_lds(32 * KC));              \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, dense_tiles_wide_kernel<0, 32 * KC, 4>, 256,             \
                                                     dense_wide_lds(32 * KC));                                       \
    break;
  switch (dk / 32) {
    MIANN_SLOTS_WIDE(1)
    MIANN_SLOTS_WIDE(2)
    MIANN_SLOTS_WIDE(3)
    MIANN_SLOTS_WIDE(4)
    MIANN_SLOTS_WIDE(5)
    MIANN_SLOTS_WIDE(6)
    MIANN_SLOTS_WIDE(7)
    MIANN_SLOTS_WIDE(8)
    default: break;
  }
#undef MIANN_SLOTS_WIDE
  if (e != hipSuccess || per < 1) per = 1;
  const int64_t slots = (int64_t)ncu * per;
  cache[{dev, dk}] = slots;
  return slots;
}

// The current device's XCDs (dies with their own L2), 1 if the runtime does not say.
static int device_xcds() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || n < 1) n = 1;
  cache[dev] = n;
  return n;
}

// Column groups per shard for the tile passes over rtiles row blocks and nseg shards of at most ntmax tiles, between
// g_min and g_max groups: the split with the least time by rounds of blocks over the chip's slots times the tiles
// per block (plus one for the block's prologue). Returns gps and sets cg, the tiles per group.
static int64_t dense_groups(int64_t rtiles, int nseg, int64_t ntmax, int64_t slots, int64_t g_min, int64_t g_max,
                            int* cg_out) {
  g_max = std::max<int64_t>(1, std::min(g_max, ntmax));
  g_min = std::max<int64_t>(1, std::min(g_min, g_max));
  int64_t best_g = g_min, best_cost = INT64_MAX;
  for (int64_t g = g_min; g <= g_max; g++) {
    const int64_t cg = (ntmax + g - 1) / g;
    const int64_t gg = (ntmax + cg - 1) / cg;
    if (gg != g || gg < g_min) continue;  // the same split as a smaller g
    const int64_t blocks = rtiles * nseg * gg;
    const int64_t cost = (blocks + slots - 1) / slots * (cg + 1);
    if (cost < best_cost) best_cost = cost, best_g = gg;
  }
  *cg_out = (int)((ntmax + best_g - 1) / best_g);
  return best_g;
}

// Rows per block of the tile passes for rows of dk elements, and the values pass 1 keeps per row and block.
static int dense_block_rows(int dk) { return 128 * dense_wide_sets(dk); }
// Lane slots (query sets x lane halves, per row) of a block of the pass-1 kernel for rows of dk elements.
static int dense_slots_per_block(int) { return 2; }

__device__ __forceinline__ float dense_threshold(float b, float qf, float gf, float eps);

// One wave per (row, shard): the threshold of pass 2, which keeps every exact top-t ghost of the shard.
// G_j = qn + gn_j - 2 q.x_j is the GEMM form of the distance to ghost j, computed as qn - 2 a_j with
// a_j = q.x_j - gn_j / 2 (split-bf16 products accumulated in float32), D_j the exact distance (the search's
// definition), E >= |G_j - D_j|. Pass 1 left, per block of the shard's tiles, KEEP G per lane slot (its smallest), each
// the G of a distinct ghost; so the t-th smallest b_t of those values has t ghosts with G <= b_t, hence D <= b_t + E
// for t ghosts and tau_D (the t-th smallest D) <= b_t + E; an exact top-t ghost j then has
// G_j <= D_j + E <= tau_D + E <= b_t + 2E, that is a_j >= (qn - b_t - 2E) / 2, the threshold (rounded down).
// Fewer than t values (a shard with fewer than t ghosts, or t above what pass 1 keeps) give -FLT_MAX: every real
// ghost qualifies, and no padding column (a = -inf). E = eps (qn + max_j gn_j), see dense_eps.
__global__ __launch_bounds__(256) void dense_bound_kernel(const float* __restrict__ M, int nvb, int mcap, int cg,
                                                          const int64_t* __restrict__ off,
                                                          const int64_t* __restrict__ Rs, int s0, int nseg,
                                                          const int* __restrict__ nrows_dev, int64_t nrows_max,
                                                          int64_t row0, int64_t rows_chunk, int t,
                                                          const uint32_t* __restrict__ list,
                                                          const float* __restrict__ qn,
                                                          const float* __restrict__ gmax, float eps,
                                                          float* __restrict__ thr) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t item = (int64_t)blockIdx.x * 4 + wave;
  const int64_t rl = item / nseg;
  const int sl = (int)(item % nseg);
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows_max;
  if (rl >= rows_chunk || row0 + rl >= n_rows) return;
  const int s = s0 + sl;
  const int64_t R = Rs[s];
  const int kp = (int)(t < R ? t : R);
  const int ntiles = (int)((off[s + 1] - off[s]) / 64);
  const int64_t nv = (int64_t)((ntiles + cg - 1) / cg) * nvb;  // the values of the blocks that ran
  const float* m = M + (rl * nseg + sl) * mcap;
  // the row's norm and the shard's largest ghost norm, loaded before the values are sorted
  const int64_t qi = list ? (int64_t)list[row0 + rl] : row0 + rl;
  const float qf = qn[qi], gf = gmax[s];
  // float bits of non-negative values order like the values; 0xFFFFFFFF = none
  // all of a lane's loads of one round are issued before the first is consumed (one memory latency per round)
  constexpr int U = 8;
  uint32_t v0 = 0xFFFFFFFFu, v1 = 0xFFFFFFFFu;
  for (int64_t g0 = lane; g0 < nv; g0 += 64 * U) {
    uint32_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t g = g0 + (int64_t)u * 64;
      x[u] = g < nv ? __float_as_uint(m[g]) : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t lo = x[u] < v0 ? x[u] : v0;
      v1 = x[u] < v0 ? v0 : (x[u] < v1 ? x[u] : v1);
      v0 = lo;
    }
  }
  uint32_t b;
  if (kp <= 32) {
    const uint32_t srt = bitonic_sort_u32<64>(v0);
    b = (uint32_t)__builtin_amdgcn_readlane((int)srt, kp - 1);
  } else {
    uint64_t w[2] = {(uint64_t)v0, (uint64_t)v1};
    bitonic_sort_regs<2>(w);
    const uint64_t x = (kp - 1) >= 64 ? w[1] : w[0];
    b = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (kp - 1) & 63);
  }
  const float th = dense_threshold(b < 0x7F800000u ? __uint_as_float(b) : INFINITY, qf, gf, eps);
  if (lane == 0) thr[rl * nseg + sl] = th;
}

// Threshold of pass 2 from a finite b_t (see dense_bound_kernel), rounded down; -FLT_MAX without one.
__device__ __forceinline__ float dense_threshold(float b, float qf, float gf, float eps) {
  float th = -FLT_MAX;
  if (b < INFINITY) {
    const double qd = (double)qf;
    const double E = (double)eps * (qd + (double)gf);
    const double x = 0.5 * (qd - ((double)b + 2.0 * E));
    th = (float)x;
    if ((double)th > x) th = nextafterf(th, -INFINITY);
  }
  return th;
}

// The same threshold with one (row, shard) per lane, for t <= KMAX: the lane streams the values pass 1 kept for
// the row and shard (16-byte loads) through an ascending list of its KMAX smallest, and b_t is the t-th of them.
template <int KMAX>
__global__ __launch_bounds__(64) void dense_bound_lanes_kernel(const float* __restrict__ M, int nvb, int mcap, int cg,
                                                               const int64_t* __restrict__ off,
                                                               const int64_t* __restrict__ Rs, int s0, int nseg,
                                                               const int* __restrict__ nrows_dev, int64_t nrows_max,
                                                               int64_t row0, int64_t rows_chunk, int t,
                                                               const uint32_t* __restrict__ list,
                                                               const float* __restrict__ qn,
                                                               const float* __restrict__ gmax, float eps,
                                                               float* __restrict__ thr) {
  const int64_t item = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t rl = item / nseg;
  const int sl = (int)(item % nseg);
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows_max;
  if (rl >= rows_chunk || row0 + rl >= n_rows) return;
  const int s = s0 + sl;
  const int64_t R = Rs[s];
  const int kp = (int)(t < R ? t : R);
  const int ntiles = (int)((off[s + 1] - off[s]) / 64);
  const int n4 = ((ntiles + cg - 1) / cg) * nvb / 4;  // 16-byte groups of the blocks that ran
  const f32x4_t* m4 = (const f32x4_t*)(M + (rl * nseg + sl) * mcap);
  const int64_t qi = list ? (int64_t)list[row0 + rl] : row0 + rl;
  const float qf = qn[qi], gf = gmax[s];
  float top[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; i++) top[i] = INFINITY;
#pragma unroll 4
  for (int g = 0; g < n4; g++) {
    const f32x4_t x = m4[g];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      float v = x[r];
#pragma unroll
      for (int i = 0; i < KMAX; i++) {
        const float lo = fminf(top[i], v);
        v = fmaxf(top[i], v);
        top[i] = lo;
      }
    }
  }
  float b = INFINITY;
#pragma unroll
  for (int i = 0; i < KMAX; i++) b = i == kp - 1 ? top[i] : b;
  thr[rl * nseg + sl] = dense_threshold(b, qf, gf, eps);
}

// Exact distance (the search's definition) of query row q to a stored row, by an 8-lane team; every lane of the
// team returns the team's result.
template <int DT>
__device__ __forceinline__ uint32_t exact_dist_team(const void* __restrict__ Q, int64_t qi, const void* __restrict__ brow,
                                                    float bscale, int bpad, int tl) {
  constexpr int P16 = Fmt<DT>::per16;
  constexpr int ESZ = Fmt<DT>::esize;
  const int row16 = bpad * ESZ / 16;
  const uint4* b4 = (const uint4*)brow;
  if constexpr (DT == DT_U8) {
    const uint4* q4 = (const uint4*)((const uint8_t*)Q + (size_t)qi * bpad);
    int acc = 0;
    for (int c = tl; c < row16; c += 8) {
      const uint4 xb = b4[c], qb = q4[c];
      const uint32_t xw[4] = {xb.x, xb.y, xb.z, xb.w}, qw[4] = {qb.x, qb.y, qb.z, qb.w};
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const int t = (int)((qw[e >> 2] >> (8 * (e & 3))) & 0xFF) - (int)((xw[e >> 2] >> (8 * (e & 3))) & 0xFF);
        acc += t * t;
      }
    }
    acc += xor_lane_i32(acc, 1);
    acc += xor_lane_i32(acc, 2);
    acc += xor_lane_i32(acc, 4);
    return (uint32_t)acc;
  } else {
    const float* qrow = (const float*)Q + (size_t)qi * bpad;
    double acc = 0.0;
    for (int c = tl; c < row16; c += 8) {
      float x[P16];
      decode16<DT>(b4[c], x);
#pragma unroll
      for (int e = 0; e < P16; e++) {
        const float xe = (DT == DT_F16 || DT == DT_FP8) ? bscale * x[e] : x[e];
        const float t = qrow[c * P16 + e] - xe;
        acc = __builtin_fma((double)t, (double)t, acc);
      }
    }
    acc += xor_lane_f64(acc, 1);
    acc += xor_lane_f64(acc, 2);
    acc += xor_lane_f64(acc, 4);
    return __float_as_uint((float)acc);
  }
}

// Exact distances of two stored rows to query row qi by an 8-lane team (every lane of the team returns both).
template <int DT>
__device__ __forceinline__ void exact_dist_team2(const void* __restrict__ Q, int64_t qi, const void* __restrict__ brow0,
                                                 float sc0, const void* __restrict__ brow1, float sc1, int bpad, int tl,
                                                 uint32_t& d0, uint32_t& d1) {
  constexpr int P16 = Fmt<DT>::per16;
  constexpr int ESZ = Fmt<DT>::esize;
  const int row16 = bpad * ESZ / 16;
  const uint4* b0 = (const uint4*)brow0;
  const uint4* b1 = (const uint4*)brow1;
  if constexpr (DT == DT_U8) {
    const uint4* q4 = (const uint4*)((const uint8_t*)Q + (size_t)qi * bpad);
    int a0 = 0, a1 = 0;
    for (int c = tl; c < row16; c += 8) {
      const uint4 x0 = b0[c], x1 = b1[c], qb = q4[c];
      const uint32_t w0[4] = {x0.x, x0.y, x0.z, x0.w}, w1[4] = {x1.x, x1.y, x1.z, x1.w};
      const uint32_t qw[4] = {qb.x, qb.y, qb.z, qb.w};
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const int qe = (int)((qw[e >> 2] >> (8 * (e & 3))) & 0xFF);
        const int t0 = qe - (int)((w0[e >> 2] >> (8 * (e & 3))) & 0xFF);
        const int t1 = qe - (int)((w1[e >> 2] >> (8 * (e & 3))) & 0xFF);
        a0 += t0 * t0;
        a1 += t1 * t1;
      }
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      a0 += xor_lane_i32(a0, o);
      a1 += xor_lane_i32(a1, o);
    }
    d0 = (uint32_t)a0;
    d1 = (uint32_t)a1;
  } else {
    const float* qrow = (const float*)Q + (size_t)qi * bpad;
    double a0 = 0.0, a1 = 0.0;
    for (int c = tl; c < row16; c += 8) {
      float x0[P16], x1[P16];
      decode16<DT>(b0[c], x0);
      decode16<DT>(b1[c], x1);
#pragma unroll
      for (int e = 0; e < P16; e++) {
        const float qe = qrow[c * P16 + e];
        const float t0 = qe - ((DT == DT_F16 || DT == DT_FP8) ? sc0 * x0[e] : x0[e]);
        const float t1 = qe - ((DT == DT_F16 || DT == DT_FP8) ? sc1 * x1[e] : x1[e]);
        a0 = __builtin_fma((double)t0, (double)t0, a0);
        a1 = __builtin_fma((double)t1, (double)t1, a1);
      }
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      a0 += xor_lane_f64(a0, o);
      a1 += xor_lane_f64(a1, o);
    }
    d0 = __float_as_uint((float)a0);
    d1 = __float_as_uint((float)a1);
  }
}

// Candidate column of bit b of mask word i of a (row, shard): word i covers tile i / 2 and lane half i % 2.
__device__ __forceinline__ uint32_t mask_col(int i, int b) {
  return (uint32_t)((i >> 1) * 64 + 32 * (b >> 4) + 8 * ((b >> 2) & 3) + 4 * (i & 1) + (b & 3));
}

// One wave per (row, shard) item: expand the candidate masks of the shard's tiles into a column list, compute every
// candidate's exact distance, sort, and write the exact top-t seeds (dist bits << 32 | node id) to
// out[(q * S + s) * t + i]. A list longer than CAPG is replaced by an exact scan of all the shard's ghosts; both
// give the exact top-t. (The path of lists too long for an 8-lane team.)
template <int DT>
__device__ __forceinline__ void final_item_wave(const uint32_t* __restrict__ cmask, int nht, const uint32_t* __restrict__ list,
                                int64_t row0, int64_t rl, int sl, const int64_t* __restrict__ Rs, int s0, int nseg,
                                int t, const DenseShardDev* __restrict__ shd, const void* __restrict__ qraw,
                                int d_pad, int S, uint64_t* __restrict__ out, uint64_t* ebuf) {
  constexpr int ESZ = Fmt<DT>::esize;
  constexpr bool kScaled = DT == DT_F16 || DT == DT_FP8;
  const int lane = lane_id(), team = lane >> 3, tl = lane & 7;
  const int s = s0 + sl;
  const int64_t R = Rs[s];
  const int64_t qi = list ? (int64_t)list[row0 + rl] : row0 + rl;
  const DenseShardDev sh = shd[s];
  const size_t row_bytes = (size_t)d_pad * ESZ;
  // candidate columns: mask word i (one per lane and round) of tile i / 2 contributes the set bits of its lane
  // half i % 2: bit b is column 64 (i / 2) + 32 (b / 16) + 8 (b / 4 % 4) + 4 (i % 2) + b % 4
  const int nt = (int)(2 * ((R + 63) / 64));
  const uint32_t* mrow = cmask + (rl * nseg + sl) * nht;
  int n = 0;
  for (int i0 = 0; i0 < nt; i0 += 64) {
    const int i = i0 + lane;
    uint32_t m = i < nt ? mrow[i] : 0u;
    const int c = __popc(m);
    int pre = c;  // inclusive prefix over the lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = (int)shfl_u32((uint32_t)pre, lane >= o ? lane - o : lane);
      pre += lane >= o ? y : 0;
    }
    int at = n + pre - c;
    while (m) {
      const int b = __ffs(m) - 1;
      m &= m - 1;
      if (at < CAPG) ebuf[at] = (uint64_t)mask_col(i, b);
      at++;
    }
    n += (int)shfl_u32((uint32_t)pre, 63);
  }
  wsync();
  uint64_t best;  // exact keys, ascending, one per lane (the first t are the result)
  if (n <= CAPG) {
    // exact distances, two candidates per 8-lane team and round
    for (int r0 = 0; r0 < n; r0 += 16) {
      const int c0 = r0 + team, c1 = r0 + 8 + team;
      const uint32_t j0 = c0 < n ? (uint32_t)ebuf[c0] : 0u, j1 = c1 < n ? (uint32_t)ebuf[c1] : 0u;
      const float sc0 = kScaled ? sh.g_scale[j0] : 1.f, sc1 = kScaled ? sh.g_scale[j1] : 1.f;
      uint32_t d0, d1;
      exact_dist_team2<DT>(qraw, qi, (const char*)sh.g_store + (size_t)j0 * row_bytes, sc0,
                           (const char*)sh.g_store + (size_t)j1 * row_bytes, sc1, d_pad, tl, d0, d1);
      wsync();
      if (tl == 0 && c0 < n) ebuf[c0] = ((uint64_t)d0 << 32) | j0;
      if (tl == 0 && c1 < n) ebuf[c1] = ((uint64_t)d1 << 32) | j1;
      wsync();
    }
    uint64_t v[4];
#pragma unroll
    for (int r = 0; r < 4; r++) v[r] = r * 64 + lane < n ? ebuf[r * 64 + lane] : kDummy;
    if (n <= 64) {
      v[0] = bitonic_sort_u64<64>(v[0]);
    } else if (n <= 128) {
      uint64_t w[2] = {v[0], v[1]};
      bitonic_sort_regs<2>(w);
      v[0] = w[0];
    } else {
      bitonic_sort_regs<4>(v);
    }
    best = v[0];
  } else {
    // too many candidates: exact scan, 64 ghosts per round, merged into the running 64 best
    best = kDummy;
    for (int64_t g0 = 0; g0 < R; g0 += 64) {
      for (int r0 = 0; r0 < 64; r0 += 8) {
        const int64_t j = g0 + r0 + team;
        const bool ok = j < R;
        const uint32_t jj = ok ? (uint32_t)j : 0u;
        const float sc = kScaled ? sh.g_scale[jj] : 1.f;
        const uint32_t db = exact_dist_team<DT>(qraw, qi, (const char*)sh.g_store + (size_t)jj * row_bytes, sc, d_pad, tl);
        if (tl == 0) ebuf[r0 + team] = ok ? (((uint64_t)db << 32) | jj) : kDummy;
      }
      wsync();
      uint64_t c = bitonic_sort_u64<64>(ebuf[lane]);
      wsync();
      const uint64_t cr = reverse_lanes_u64(c);
      best = bitonic_merge_u64(best < cr ? best : cr);
    }
  }
  if (lane < t) {
    out[((size_t)qi * S + s) * t + lane] =
        best == kDummy ? kDummy : ((best & 0xFFFFFFFF00000000ull) | sh.g_map[(uint32_t)best]);
  }
}

constexpr int CAPT = 64;  // candidates an 8-lane team rescores; longer lists go to the block's waves

// Exact rescoring: 32 (row, shard) items per block, one 8-lane team each. The team expands the candidate masks of
// its item into a column list in LDS (lane l takes words l, l + 8, ...; a team prefix sum places its bits),
// computes the candidates' exact distances two at a time, and writes each candidate whose rank among the keys
// (dist bits << 32 | ghost) is below t to out[(q * S + s) * t + rank] (slots from the list's length to t get no
// seed). Lists longer than CAPT are collected and then rescored one per wave (final_item_wave). Both give the exact
// top-t. With TEAM false (t above 16: lists of t and more, which a team rescores in too many dependent rounds)
// each wave rescores one item of the block's four directly.
template <int DT, bool TEAM>
__global__ __launch_bounds__(256) void dense_final_kernel(
    const uint32_t* __restrict__ cmask, int nht, const uint32_t* __restrict__ list,
    const int* __restrict__ nrows_dev, int64_t nrows_max, int64_t row0, int64_t rows_chunk,
    const int64_t* __restrict__ Rs, int s0, int nseg, int t, const DenseShardDev* __restrict__ shd,
    const void* __restrict__ qraw, int d_pad, int S, uint64_t* __restrict__ out) {
  constexpr int ESZ = Fmt<DT>::esize;
  constexpr bool kScaled = DT == DT_F16 || DT == DT_FP8;
  __shared__ uint64_t tbuf[32 * CAPT];
  __shared__ uint64_t ebufs[4 * CAPG];
  __shared__ int nover;
  __shared__ int64_t over[32];
  const int tid = threadIdx.x, wave = tid >> 6, team = tid >> 3, tl = tid & 7;
  const int64_t n_rows = nrows_dev ? (int64_t)*nrows_dev : nrows_max;
  if constexpr (!TEAM) {
    const int64_t it = (int64_t)blockIdx.x * 4 + wave;
    if (it / nseg < rows_chunk && row0 + it / nseg < n_rows)
      final_item_wave<DT>(cmask, nht, list, row0, it / nseg, (int)(it % nseg), Rs, s0, nseg, t, shd, qraw, d_pad, S,
                          out, ebufs + wave * CAPG);
    return;
  }
  if (tid == 0) nover = 0;
  __syncthreads();
  const int64_t item = (int64_t)blockIdx.x * 32 + team;
  const int64_t rl = item / nseg;
  const int sl = (int)(item % nseg);
  if (rl < rows_chunk && row0 + rl < n_rows) {  // uniform over the team
    const int s = s0 + sl;
    const int64_t R = Rs[s];
    const int64_t qi = list ? (int64_t)list[row0 + rl] : row0 + rl;
    const DenseShardDev sh = shd[s];
    const size_t row_bytes = (size_t)d_pad * ESZ;
    uint64_t* tb = tbuf + team * CAPT;
    const int nt = (int)(2 * ((R + 63) / 64));
    const uint32_t* mrow = cmask + (rl * nseg + sl) * nht;
    int c = 0;
    for (int i = tl; i < nt; i += 8) c += __popc(mrow[i]);
    int pre = c;  // inclusive prefix over the team
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      const int y = (int)shfl_u32((uint32_t)pre, tl >= o ? (int)threadIdx.x % 64 - o : (int)threadIdx.x % 64);
      pre += tl >= o ? y : 0;
    }
    const int n = (int)shfl_u32((uint32_t)pre, ((int)threadIdx.x % 64) | 7);
    if (n > CAPT) {
      if (tl == 0) over[atomicAdd(&nover, 1)] = item;
    } else {
      int at = pre - c;
      for (int i = tl; i < nt; i += 8) {
        uint32_t m = mrow[i];
        while (m) {
          const int b = __ffs(m) - 1;
          m &= m - 1;
          tb[at++] = (uint64_t)mask_col(i, b);
        }
      }
      wsync();
      // exact distances, two candidates per round
      for (int r0 = 0; r0 < n; r0 += 2) {
        const uint32_t j0 = (uint32_t)tb[r0], j1 = r0 + 1 < n ? (uint32_t)tb[r0 + 1] : j0;
        const float sc0 = kScaled ? sh.g_scale[j0] : 1.f, sc1 = kScaled ? sh.g_scale[j1] : 1.f;
        uint32_t d0, d1;
        exact_dist_team2<DT>(qraw, qi, (const char*)sh.g_store + (size_t)j0 * row_bytes, sc0,
                             (const char*)sh.g_store + (size_t)j1 * row_bytes, sc1, d_pad, tl, d0, d1);
        wsync();
        if (tl == 0) {
          tb[r0] = ((uint64_t)d0 << 32) | j0;
          if (r0 + 1 < n) tb[r0 + 1] = ((uint64_t)d1 << 32) | j1;
        }
        wsync();
      }
      // rank of each candidate among the item's keys (all distinct: one key per ghost)
      uint64_t* o = out + ((size_t)qi * S + s) * t;
      for (int r = tl; r < n; r += 8) {
        const uint64_t key = tb[r];
        int rank = 0;
        for (int i = 0; i < n; i++) rank += tb[i] < key;
        if (rank < t) o[rank] = (key & 0xFFFFFFFF00000000ull) | sh.g_map[(uint32_t)key];
      }
      for (int r = n + tl; r < t; r += 8) o[r] = kDummy;
    }
  }
  __syncthreads();
  for (int k = wave; k < nover; k += 4) {
    const int64_t it = over[k];
    final_item_wave<DT>(cmask, nht, list, row0, it / nseg, (int)(it % nseg), Rs, s0, nseg, t, shd, qraw, d_pad, S,
                        out, ebufs + wave * CAPG);
  }
}

namespace {
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
// eps of the dense entry's error bound E = eps (qn + max gn) for rows of dk elements (see dense_bound_kernel).
// E bounds |G - D| with G = qn - 2 a computed from a = q.x - gn/2 and D the exact distance. It covers the dropped
// lo.lo term and the residual of the two-term bf16 split (about 3.03 2^-16 |q||x|, and 2 |q||x| <= qn + gn), the
// float32 accumulation of 3 dk products onto -gn/2 (partial sums at most qn + gn; 2^-23 per addition in case the
// matrix cores truncate: (3 dk + 1) 2^-23 (qn + gn) in a, twice that in G), the rounding of the norms, of G and of
// the exact distance (12 2^-24 (qn + gn)), with a factor of 2 on the whole.
float dense_eps(int dk) {
  return (float)(2.0 * (3.03 * std::ldexp(1.0, -16) + (12.0 * dk + 16.0) * std::ldexp(1.0, -24)));
}
// Bytes of the per-query buffers (split query rows, norms, raw rows, start-shard list, counter).
size_t dense_query_bytes(int store_dt, int64_t nq, int d_pad, int dk) {
  const size_t raw = store_dt == DT_U8 ? 1 : 4;
  return 2 * al256((size_t)nq * dk * 2) + al256((size_t)nq * 4) + al256((size_t)nq * d_pad * raw) +
         al256((size_t)nq * 4) + 256;
}
// Tiles of the largest shard in [s0, s1).
int64_t dense_max_tiles(const DenseGhosts& G, int s0, int s1) {
  int64_t ntmax = 0;
  for (int sx = s0; sx < s1; sx++) ntmax = std::max<int64_t>(ntmax, (G.off[sx + 1] - G.off[sx]) / 64);
  return ntmax;
}
// Scratch bytes per row of a chunk in the pass over shards [s0, s1): candidate masks, the mcap values pass 1 keeps
// per shard, and thresholds. (mcap < 0: the most any split can keep, 16 per lane slot and tile.)
size_t dense_row_bytes(const DenseGhosts& G, int s0, int s1, int dk, int64_t mcap) {
  const int64_t ntmax = dense_max_tiles(G, s0, s1);
  if (mcap < 0) mcap = std::max<int64_t>(4, ntmax * dense_slots_per_block(dk) * 16);
  return (size_t)(s1 - s0) * ((size_t)(2 * ntmax) * 4 + (size_t)mcap * 4 + 4);
}
}  // namespace

size_t dense_entry_min_scratch(int store_dt, int64_t nq, int d_pad, int dk, int S, int start_only,
                               const DenseGhosts& G) {
  size_t per_row = 0;
  const int npass = start_only ? S : 1;
  for (int ps = 0; ps < npass; ps++) {
    const int s0 = start_only ? ps : 0, s1 = start_only ? ps + 1 : S;
    per_row = std::max(per_row, dense_row_bytes(G, s0, s1, dk, -1));
  }
  return dense_query_bytes(store_dt, nq, d_pad, dk) + (size_t)dense_block_rows(dk) * per_row + 4096;
}

hipError_t dense_entry_split(int store_dt, const void* queries, int64_t nq, int d, int d_pad, int dk,
                             const uint64_t* qkeys, int S, int start_only, const DenseGhosts& G, int t, uint64_t* out,
                             hipStream_t st, void* ext, size_t ext_bytes) {
  if (nq == 0) return hipSuccess;
  const int qdt = store_dt == DT_U8 ? DT_U8 : DT_F32;
  auto al = al256;
  const size_t sz_qb = al((size_t)nq * dk * 2), sz_qn = al((size_t)nq * 4);
  const size_t sz_qraw = al((size_t)nq * d_pad * (qdt == DT_U8 ? 1 : 4));
  const size_t sz_list = al((size_t)nq * 4), sz_cnt = 256;
  const size_t total = 2 * sz_qb + sz_qn + sz_qraw + sz_list + sz_cnt;
  // a caller's buffer holds the query buffers first and the chunk work area after them
  if (ext && ext_bytes < dense_entry_min_scratch(store_dt, nq, d_pad, dk, S, start_only, G))
    return hipErrorInvalidValue;
  ScratchLease lq;
  hipError_t e = hipSuccess;
  if (ext) lq.p = ext;
  else e = scratch_lease(kSlotDenseQueries, total, st, &lq);
  if (e != hipSuccess) return e;
  char* buf = (char*)lq.p;
  char* p = buf;
  uint16_t* qh = (uint16_t*)p; p += sz_qb;
  uint16_t* ql = (uint16_t*)p; p += sz_qb;
  float* qn = (float*)p; p += sz_qn;
  void* qraw = p; p += sz_qraw;
  uint32_t* list = (uint32_t*)p; p += sz_list;
  int* qcnt = (int*)p;
  hipLaunchKernelGGL(dense_queries_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, queries, qdt, nq, d, dk,
                     d_pad, qh, ql, qn, qraw);
  e = hipGetLastError();
  // (rows, shard range) passes: every query against every shard, or each shard against the queries starting there
  const int npass = start_only ? S : 1;
  for (int ps = 0; ps < npass && e == hipSuccess; ps++) {
    const int s0 = start_only ? ps : 0, s1 = start_only ? ps + 1 : S;
    const int nseg = s1 - s0;
    const int64_t ncols = G.off[s1] - G.off[s0];
    if (ncols == 0) continue;
    const uint32_t* rl = nullptr;
    const int* rc = nullptr;
    if (start_only) {
      hipLaunchKernelGGL(fill_cnt_kernel, dim3(1), dim3(1), 0, st, qcnt);
      hipLaunchKernelGGL(shard_qlist_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, nq, qkeys, S, s0,
                         0, list, qcnt);
      rl = list;
      rc = qcnt;
    }
    // per chunk of rows: candidate masks [rows][nseg][nht], kept values [rows][nseg][mcap], thresholds
    // [rows][nseg]
    const int64_t ntmax = dense_max_tiles(G, s0, s1);
    const int64_t nht = 2 * ntmax;
    const int brows = dense_block_rows(dk);
    // pass 1 keeps the 4 smallest values per lane slot for t <= 8, else all 16, and at least 2 t values per (row,
    // shard) where the tiles allow; the column groups of cg tiles per block are split to keep the chip's block
    // slots busy (dense_groups). The split for all rows in one chunk fixes mcap; a smaller chunk splits within it.
    const int keep = t <= 8 || dk > 224 ? 4 : 16;  // (rows of 256 elements leave no registers for 16)
    const int nvb = dense_slots_per_block(dk) * keep;
    const int64_t g_min = (2 * t + nvb - 1) / nvb;
    const int64_t tslots = dense_tile_slots(dk);
    // (a pass over the queries that start on one shard holds about nq / S of them)
    const int64_t rows_exp = start_only ? (nq + S - 1) / S : nq;
    const int64_t rows_all = (rows_exp + brows - 1) / brows * brows;
    int cg = 1;
    const int64_t g_all = dense_groups(rows_all / brows, nseg, ntmax, tslots, g_min, ntmax, &cg);
    const int mcap = (int)((g_all * nvb + 3) / 4 * 4);
    const size_t per_row = dense_row_bytes(G, s0, s1, dk, mcap);
    // at most 512 MB of scratch, or what the caller's buffer leaves after the query buffers
    const size_t work_cap = ext ? ext_bytes - total - 4096 : ((size_t)1 << 29);
    int64_t chunk = (int64_t)(work_cap / per_row);
    chunk = chunk < brows ? brows : chunk / brows * brows;
    if (chunk > (nq + brows - 1) / brows * brows) chunk = (nq + brows - 1) / brows * brows;
    char* wb = nullptr;
    ScratchLease lw;
    if (ext) lw.p = buf + total;
    else e = scratch_lease(kSlotDenseWork, (size_t)chunk * per_row + 4096, st, &lw);
    wb = (char*)lw.p;
    if (e != hipSuccess) break;
    const int64_t rtiles = chunk / brows;
    const int64_t gps =
        dense_groups(std::min(rtiles, rows_all / brows), nseg, ntmax, tslots, g_min, mcap / nvb, &cg);
    uint32_t* cmask = (uint32_t*)wb;
    float* Mg = (float*)(cmask + (size_t)chunk * nseg * nht);
    float* thr = Mg + (size_t)chunk * nseg * mcap;
    // (rows counted on the device fill only the first row blocks: plain block order spreads them over the XCDs)
    const int nxcd = rc ? 1 : device_xcds();
    const int64_t nitems = rtiles * nseg * gps;
    const dim3 gg((unsigned)((nitems + nxcd - 1) / nxcd * nxcd));
    const unsigned gw = (unsigned)((chunk * nseg + 3) / 4);
    const unsigned gf = (unsigned)((chunk * nseg + 31) / 32);
    const int nh = (int)nht;
    for (int64_t row0 = 0; row0 < nq && e == hipSuccess; row0 += chunk) {
      if (keep == 16)
        launch_dense_tiles<0, 16>(dk, gg, st, qh, ql, qn, rl, rc, nq, row0, chunk, G, s0, nseg, (int)gps, cg, nh,
                                  nxcd, rtiles, mcap, Mg, thr, cmask);
      else
        launch_dense_tiles<0, 4>(dk, gg, st, qh, ql, qn, rl, rc, nq, row0, chunk, G, s0, nseg, (int)gps, cg, nh,
                                 nxcd, rtiles, mcap, Mg, thr, cmask);
      {
        const float eps = dense_eps(dk);
        const dim3 gl((unsigned)((chunk * nseg + 63) / 64));
        // one item per lane while its values are few; the wave per item (a few values per lane) otherwise
        const bool lanes = (int64_t)gps * nvb <= 128;
        if (lanes && t <= 8)
          hipLaunchKernelGGL(dense_bound_lanes_kernel<8>, gl, dim3(64), 0, st, Mg, nvb, mcap, cg, G.off_dev,
                             G.R_dev, s0, nseg, rc, nq, row0, chunk, t, rl, qn, G.gmax_dev, eps, thr);
        else if (lanes && t <= 16)
          hipLaunchKernelGGL(dense_bound_lanes_kernel<16>, gl, dim3(64), 0, st, Mg, nvb, mcap, cg, G.off_dev,
                             G.R_dev, s0, nseg, rc, nq, row0, chunk, t, rl, qn, G.gmax_dev, eps, thr);
        else if (lanes && t <= 32)
          hipLaunchKernelGGL(dense_bound_lanes_kernel<32>, gl, dim3(64), 0, st, Mg, nvb, mcap, cg, G.off_dev,
                             G.R_dev, s0, nseg, rc, nq, row0, chunk, t, rl, qn, G.gmax_dev, eps, thr);
        else
          hipLaunchKernelGGL(dense_bound_kernel, dim3(gw), dim3(256), 0, st, Mg, nvb, mcap, cg, G.off_dev,
                             G.R_dev, s0, nseg, rc, nq, row0, chunk, t, rl, qn, G.gmax_dev, eps, thr);
      }
      launch_dense_tiles<1, 4>(dk, gg, st, qh, ql, qn, rl, rc, nq, row0, chunk, G, s0, nseg, (int)gps, cg, nh,
                               nxcd, rtiles, mcap, Mg, thr, cmask);
      // exact rescoring: one 8-lane team per item for t <= 16, one wave per item above
#define MIANN_DENSE_FINAL(DTV)                                                                                       \
  if (t <= 16)                                                                                                       \
    hipLaunchKernelGGL((dense_final_kernel<DTV, true>), dim3(gf), dim3(256), 0, st, cmask, nh, rl, rc, nq, row0,     \
                       chunk, G.R_dev, s0, nseg, t, G.shards_dev, qraw, d_pad, S, out);                               \
  else                                                                                                               \
    hipLaunchKernelGGL((dense_final_kernel<DTV, false>), dim3(gw), dim3(256), 0, st, cmask, nh, rl, rc, nq, row0,    \
                       chunk, G.R_dev, s0, nseg, t, G.shards_dev, qraw, d_pad, S, out);
      switch (store_dt) {
        case DT_F32: MIANN_DENSE_FINAL(DT_F32) break;
        case DT_F16: MIANN_DENSE_FINAL(DT_F16) break;
        case DT_FP8: MIANN_DENSE_FINAL(DT_FP8) break;
        default: MIANN_DENSE_FINAL(DT_U8) break;
      }
#undef MIANN_DENSE_FINAL
      e = hipGetLastError();
    }
    if (!ext) scratch_release(kSlotDenseWork, lw, st);
  }
  if (!ext) scratch_release(kSlotDenseQueries, lq, st);
  return e;
}

// ---------------------------------------------------------------------------
// Graph pruning: nearest ceil(deg/2) of the K0 list, then reverse neighbours
// (nearest first), then the rest of the K0 list; duplicates skipped; the row
// is finally sorted by (dist, id).
// ---------------------------------------------------------------------------
__global__ void rev_count_kernel(const uint64_t* __restrict__ knn, int64_t n, int K0, int h, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * h) return;
  const int64_t v = i / h;
  const int j = (int)(i % h);
  atomicAdd(&cnt[(uint32_t)knn[v * K0 + j]], 1);
}

__global__ void rev_fill_kernel(const uint64_t* __restrict__ knn, int64_t n, int K0, int h,
                                const int64_t* __restrict__ off, int* __restrict__ fill, uint64_t* __restrict__ rev) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * h) return;
  const int64_t v = i / h;
  const int j = (int)(i % h);
  const uint64_t key = knn[v * K0 + j];
  const uint32_t u = (uint32_t)key;
  const int pos = atomicAdd(&fill[u], 1);
  rev[off[u] + pos] = (key & 0xFFFFFFFF00000000ull) | (uint32_t)v;
}

__global__ __launch_bounds__(256) void prune_kernel(const uint64_t* __restrict__ knn, int64_t n, int K0, int deg,
                                                    int h, const int64_t* __restrict__ off,
                                                    const uint64_t* __restrict__ rev, uint32_t* __restrict__ graph) {
  extern __shared__ __align__(16) char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + wave;
  if (u >= n) return;
  const int LMAX = 64 + 64 + 256;
  uint64_t* seq = (uint64_t*)smem + (size_t)wave * (LMAX + 64);
  // smallest 64 reverse keys, sorted
  uint64_t best = kDummy;
  const int64_t b0 = off[u], b1 = off[u + 1];
  for (int64_t c0 = b0; c0 < b1; c0 += 64) {
    uint64_t x = c0 + lane < b1 ? rev[c0 + lane] : kDummy;
    x = bitonic_sort_u64<64>(x);
    // merge two sorted 64-lists, keep the lower 64: pair best[i] with x[63 - i]
    const uint64_t xr = shfl_u64(x, 63 - lane);
    best = xr < best ? xr : best;
    best = bitonic_sort_u64<64>(best);
  }
  int L = 0;
  for (int j = lane; j < h; j += 64) seq[j] = knn[u * K0 + j];
  L = h;
  const int nrev = (int)((b1 - b0) < 64 ? (b1 - b0) : 64);
  if (lane < nrev) seq[L + lane] = best;
  L += nrev;
  for (int j = lane; j < K0 - h; j += 64) seq[L + j] = knn[u * K0 + h + j];
  L += K0 - h;
  wsync();
  // first occurrence of each id, in priority order; keep the first deg
  uint64_t* rowbuf = seq + LMAX;
  int taken = 0;
  for (int c0 = 0; c0 < L && taken < deg; c0 += 64) {
    const int i = c0 + lane;
    bool ok = false;
    uint64_t key = kDummy;
    if (i < L) {
      key = seq[i];
      ok = key != kDummy;
      const uint32_t id = (uint32_t)key;
      for (int j = 0; j < i && ok; j++)
        if ((uint32_t)seq[j] == id) ok = false;
    }
    const uint64_t m = __ballot(ok);
    const int pos = taken + lanes_below(m);
    if (ok && pos < deg) rowbuf[pos] = key;
    taken += __popcll(m);
  }
  wsync();
  uint64_t rowkey = lane < deg && lane < taken ? rowbuf[lane] : kDummy;
  rowkey = lane < deg ? rowkey : kDummy;
  rowkey = bitonic_sort_u64<64>(rowkey);
  if (lane < deg) graph[u * deg + lane] = rowkey == kDummy ? kNone : (uint32_t)rowkey;
}

__global__ void zero_i32_kernel(int* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void widen_kernel(const int* __restrict__ c, int64_t n, int64_t* __restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) o[i] = c[i];
}

hipError_t prune_graph(const uint64_t* knn, int64_t n, int K0, int deg, uint32_t* graph, hipStream_t st) {
  const int h = (deg + 1) / 2;
  int* cnt = nullptr;
  int* fill = nullptr;
  int64_t* off = nullptr;
  uint64_t* rev = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  const int64_t nh = n * h;
  hipError_t e = pool_malloc_async((void**)&cnt, (size_t)(n + 1) * 4, st);
  if (e == hipSuccess) e = pool_malloc_async((void**)&fill, (size_t)(n + 1) * 4, st);
  if (e == hipSuccess) e = pool_malloc_async((void**)&off, (size_t)(n + 1) * 8, st);
  if (e == hipSuccess) e = pool_malloc_async((void**)&rev, (size_t)(nh ? nh : 1) * 8, st);
  if (e != hipSuccess) return e;
  const unsigned gn = (unsigned)((n + 1 + 255) / 256);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(gn), dim3(256), 0, st, cnt, n + 1);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(gn), dim3(256), 0, st, fill, n + 1);
  hipLaunchKernelGGL(rev_count_kernel, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, st, knn, n, K0, h, cnt);
  // exclusive prefix over n + 1 counts (the last count is 0) -> off[0..n]
  int64_t* cnt64 = nullptr;
  e = pool_malloc_async((void**)&cnt64, (size_t)(n + 1) * 8, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(widen_kernel, dim3(gn), dim3(256), 0, st, cnt, n + 1, cnt64);
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt64, off, (int)(n + 1), st);
  }
  if (e == hipSuccess) e = pool_malloc_async(&tmp, tmp_bytes ? tmp_bytes : 16, st);
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt64, off, (int)(n + 1), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(rev_fill_kernel, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, st, knn, n, K0, h, off, fill,
                       rev);
    const size_t lds = (size_t)4 * (64 + 64 + 256 + 64) * 8;
    hipLaunchKernelGGL(prune_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), lds, st, knn, n, K0, deg, h, off, rev,
                       graph);
    e = hipGetLastError();
  }
  hipFreeAsync(cnt, st);
  hipFreeAsync(fill, st);
  hipFreeAsync(off, st);
  hipFreeAsync(rev, st);
  if (cnt64) hipFreeAsync(cnt64, st);
  if (tmp) hipFreeAsync(tmp, st);
  return e;
}

// ---------------------------------------------------------------------------
// Seeded orders and small conversions.
// ---------------------------------------------------------------------------
__global__ void sm_keys_kernel(uint64_t seed, int64_t n, uint64_t* __restrict__ keys, uint32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  keys[i] = sm_at(seed, (uint64_t)i + 1);
  ids[i] = (uint32_t)i;
}

hipError_t keyed_order(uint64_t seed, int64_t n, uint32_t* out, hipStream_t st) {
  uint64_t *k0 = nullptr, *k1 = nullptr;
  uint32_t* v0 = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  hipError_t e = pool_malloc_async((void**)&k0, (size_t)n * 8, st);
  if (e == hipSuccess) e = pool_malloc_async((void**)&k1, (size_t)n * 8, st);
  if (e == hipSuccess) e = pool_malloc_async((void**)&v0, (size_t)n * 4, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sm_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, seed, n, k0, v0);
  // radix sort is stable and the ids enter in increasing order: ties in the key keep id order
  e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k1, v0, out, (int)n, 0, 64, st);
  if (e == hipSuccess) e = pool_malloc_async(&tmp, tb ? tb : 16, st);
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, k0, k1, v0, out, (int)n, 0, 64, st);
  hipFreeAsync(k0, st);
  hipFreeAsync(k1, st);
  hipFreeAsync(v0, st);
  if (tmp) hipFreeAsync(tmp, st);
  return e;
}

hipError_t sort_u32(uint32_t* v, int64_t n, hipStream_t st) {
  uint32_t* o = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  hipError_t e = pool_malloc_async((void**)&o, (size_t)n * 4, st);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortKeys(nullptr, tb, v, o, (int)n, 0, 32, st);
  if (e == hipSuccess) e = pool_malloc_async(&tmp, tb ? tb : 16, st);
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortKeys(tmp, tb, v, o, (int)n, 0, 32, st);
  if (e == hipSuccess) e = hipMemcpyAsync(v, o, (size_t)n * 4, hipMemcpyDeviceToDevice, st);
  hipFreeAsync(o, st);
  if (tmp) hipFreeAsync(tmp, st);
  return e;
}

__global__ void keys_out_kernel(const uint64_t* __restrict__ keys, int64_t total, const uint32_t* __restrict__ gmap,
                                int is_u8, uint32_t* __restrict__ ids, void* __restrict__ dists) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const uint64_t k = keys[i];
  const bool ok = k != kDummy;
  ids[i] = ok ? (gmap ? gmap[(uint32_t)k] : (uint32_t)k) : kNone;
  if (is_u8) ((int32_t*)dists)[i] = ok ? (int32_t)(k >> 32) : 0x7FFFFFFF;
  else ((uint32_t*)dists)[i] = ok ? (uint32_t)(k >> 32) : 0x7F800000u;
}

hipError_t keys_to_output(const uint64_t* keys, int64_t nq, int k, const uint32_t* gmap, int is_u8, uint32_t* ids,
                          void* dists, hipStream_t st) {
  const int64_t tot = nq * k;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_out_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, keys, tot, gmap, is_u8,
                     ids, dists);
  return hipGetLastError();
}

__global__ void keys_ids_kernel(const uint64_t* __restrict__ keys, int64_t n, int k, int col, uint32_t* __restrict__ out,
                                int stride) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = keys[i * k + col];
  out[i * stride] = key == kDummy ? kNone : (uint32_t)key;
}

hipError_t keys_to_ids(const uint64_t* keys, int64_t n, int k, int col, uint32_t* out, int out_stride, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_ids_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, n, k, col, out,
                     out_stride);
  return hipGetLastError();
}

__global__ void keys_stage_kernel(const uint64_t* keys, int64_t nq, int k, const uint32_t* __restrict__ gmap,
                                  int S, int s, uint64_t* so) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nq * k) return;
  const int64_t q = i / k;
  const int j = (int)(i % k);
  const uint64_t key = keys[i];
  so[((size_t)q * S + s) * k + j] = key == kDummy ? kDummy : ((key & 0xFFFFFFFF00000000ull) | gmap[(uint32_t)key]);
}

hipError_t keys_to_stage(const uint64_t* keys, int64_t nq, int k, const uint32_t* gmap, int S, int s, uint64_t* so,
                         hipStream_t st) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_stage_kernel, dim3((unsigned)((nq * k + 255) / 256)), dim3(256), 0, st, keys, nq, k, gmap, S,
                     s, so);
  return hipGetLastError();
}

// Sorts each row of `rows` u64 keys (length k <= 256) ascending; one wave per row.
__global__ __launch_bounds__(256) void sort_rows_kernel(uint64_t* __restrict__ keys, int64_t rows, int k) {
  __shared__ uint64_t buf[4][256];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + wave;
  if (r >= rows) return;
  int n = 1;
  while (n < k) n <<= 1;
  uint64_t* b = buf[wave];
  for (int i = lane; i < n; i += 64) b[i] = i < k ? keys[r * k + i] : kDummy;
  wsync();
  for (int kk = 2; kk <= n; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < n; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = b[i], y = b[ixj];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) { b[i] = y; b[ixj] = x; }
        }
      }
      wsync();
    }
  for (int i = lane; i < k; i += 64) keys[r * k + i] = b[i];
}

hipError_t sort_rows(uint64_t* keys, int64_t rows, int k, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  if (k > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sort_rows_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, keys, rows, k);
  return hipGetLastError();
}

}  // namespace miann
