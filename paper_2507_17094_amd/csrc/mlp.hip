// Kernels of the learned entry / iteration-budget predictor: a BF16 MLP
// d_in -> hidden -> hidden -> (R entry logits + 1 budget) trained on traces of
// the search itself. GEMMs run on the gfx950 BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation and FP32 master weights.
#include <type_traits>

#include "common.hpp"
#include "mlp.hpp"
#include "pool.hpp"

namespace miann {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GT = 64;   // output tile (rows and columns) per workgroup
constexpr int GK = 32;   // k-chunk staged in LDS
constexpr int GKP = GK + 8;  // padded LDS row (16-byte aligned, fewer bank conflicts)

// C[i][j] = sum_k A(i,k) B(k,j); A(i,k) = A[i*sar + k*sac], B(k,j) = B[k*sbr + j*sbc].
// Epilogue: + bias[j], ReLU, mask by (mask[i][j] > 0), store f32 and/or bf16.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A,
                                                        int64_t sar, int64_t sac, const uint16_t* __restrict__ B,
                                                        int64_t sbr, int64_t sbc, const float* __restrict__ bias,
                                                        int relu, const uint16_t* __restrict__ mask,
                                                        float* __restrict__ Cf, uint16_t* __restrict__ Cb, int ldc) {
  __shared__ __align__(16) uint16_t As[GT * GKP];
  __shared__ __align__(16) uint16_t Bs[GT * GKP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; j++) acc[j] = 0.f;
  // 16-byte staging where the operand is contiguous along the staged dimension (row-major A along K,
  // row-major B along N) and the tile lies inside the matrix; element-wise staging otherwise
  const bool a_vec = sac == 1 && (sar & 7) == 0 && (K & 7) == 0 && i0 + GT <= M;
  const bool b_vec = sbc == 1 && (sbr & 7) == 0 && (N & 7) == 0 && j0 + GT <= N;
  // B stored column by column ([N][K], contiguous along K): staged like A
  const bool b_kvec = sbr == 1 && (sbc & 7) == 0 && (K & 7) == 0 && j0 + GT <= N;
  for (int k0 = 0; k0 < K; k0 += GK) {
    __syncthreads();
    const bool kfull = k0 + GK <= K;
    if (a_vec && kfull) {
      const int r = tid >> 2, c = (tid & 3) * 8;  // 64 rows x 32 k: one 8-element vector per thread
      *(uint4*)&As[r * GKP + c] = *(const uint4*)&A[(int64_t)(i0 + r) * sar + k0 + c];
    } else {
      for (int e = tid; e < GT * GK; e += 256) {
        const int r = sac == 1 ? e / GK : e % GT, c = sac == 1 ? e % GK : e / GT;
        const int gi = i0 + r, gk = k0 + c;
        As[r * GKP + c] = (gi < M && gk < K) ? A[(int64_t)gi * sar + (int64_t)gk * sac] : (uint16_t)0;
      }
    }
    if (b_kvec && kfull) {
      const int r = tid >> 2, c = (tid & 3) * 8;  // 64 columns x 32 k: one 8-element vector per thread
      *(uint4*)&Bs[r * GKP + c] = *(const uint4*)&B[(int64_t)(j0 + r) * sbc + k0 + c];
    } else if (b_vec && kfull) {
      // 32 k x 64 columns: thread -> (k = tid / 8, 8 consecutive columns), stored transposed
      const int kk = tid >> 3, c = (tid & 7) * 8;
      const uint4 v = *(const uint4*)&B[(int64_t)(k0 + kk) * sbr + j0 + c];
      const uint16_t* h = (const uint16_t*)&v;
#pragma unroll
      for (int q = 0; q < 8; q++) Bs[(c + q) * GKP + kk] = h[q];
    } else {
      // consecutive threads walk the operand's contiguous dimension
      for (int e = tid; e < GT * GK; e += 256) {
        const int r = sbc == 1 ? e % GT : e / GK, c = sbc == 1 ? e / GT : e % GK;
        const int gk = k0 + c, gj = j0 + r;
        Bs[r * GKP + c] = (gj < N && gk < K) ? B[(int64_t)gk * sbr + (int64_t)gj * sbc] : (uint16_t)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 16) {
      const bf16x8 av = *(const bf16x8*)&As[(wr + (lane & 31)) * GKP + kk + (lane >> 5) * 8];
      const bf16x8 bv = *(const bf16x8*)&Bs[(wc + (lane & 31)) * GKP + kk + (lane >> 5) * 8];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const int i = i0 + wr + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    const int c = j0 + wc + (lane & 31);
    if (i >= M || c >= N) continue;
    float v = acc[j];
    if (bias) v += bias[c];
    if (relu) v = v > 0.f ? v : 0.f;
    if (mask) v = bf2f(mask[(int64_t)i * ldc + c]) > 0.f ? v : 0.f;
    if (Cf) Cf[(int64_t)i * ldc + c] = v;
    if (Cb) Cb[(int64_t)i * ldc + c] = f2bf(v);
  }
}

hipError_t gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sar, int64_t sac, const uint16_t* B, int64_t sbr,
                     int64_t sbc, const float* bias, int relu, const uint16_t* mask, float* Cf, uint16_t* Cb, int ldc,
                     hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  dim3 g((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT));
  hipLaunchKernelGGL(gemm_bf16_kernel, g, dim3(256), 0, st, M, N, K, A, sar, sac, B, sbr, sbc, bias, relu, mask, Cf, Cb,
                     ldc);
  return hipGetLastError();
}

// out[j][k] = in[k][j] for a [K][N] bf16 matrix, rows j in [N, n_pad) of out zero.
__global__ void transpose_bf16_kernel(const uint16_t* __restrict__ in, int K, int N, int n_pad,
                                      uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)n_pad * K) return;
  const int j = (int)(i / K), k = (int)(i % K);
  out[i] = j < N ? in[(int64_t)k * N + j] : (uint16_t)0;
}

hipError_t transpose_bf16(const uint16_t* in, int K, int N, int n_pad, uint16_t* out, hipStream_t st) {
  const int64_t n = (int64_t)n_pad * K;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, K, N, n_pad, out);
  return hipGetLastError();
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

hipError_t to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, y);
  return hipGetLastError();
}

// Gathers rows idx[b] of x ([n][d] f32) into bf16 ([B][d]) and their labels.
__global__ void gather_batch_kernel(const float* __restrict__ x, int d, const uint32_t* __restrict__ idx, int B,
                                    const int32_t* __restrict__ lab, const float* __restrict__ y,
                                    uint16_t* __restrict__ xb, int32_t* __restrict__ lb, float* __restrict__ yb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * d) return;
  const int b = (int)(e / d), c = (int)(e % d);
  const int64_t r = idx ? (int64_t)idx[b] : b;
  xb[e] = f2bf(x[r * d + c]);
  if (c == 0) {
    if (lb) lb[b] = lab[r];
    if (yb) yb[b] = y[r];
  }
}

hipError_t gather_batch(const float* x, int d, const uint32_t* idx, int B, const int32_t* lab, const float* y,
                        uint16_t* xb, int32_t* lb, float* yb, hipStream_t st) {
  if (B == 0) return hipSuccess;
  const int64_t tot = (int64_t)B * d;
  hipLaunchKernelGGL(gather_batch_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x, d, idx, B, lab, y,
                     xb, lb, yb);
  return hipGetLastError();
}

// Loss and its gradient per row: softmax cross-entropy over the first R
// outputs (entry region) + lambda * (z_R - y)^2 (log-budget regression).
// dZ = (softmax - onehot, 2 lambda (z_R - y)) / B, stored in bf16.
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* __restrict__ Z, int B, int R,
                                                        const int32_t* __restrict__ lab, const float* __restrict__ y,
                                                        float lambda, uint16_t* __restrict__ dZ,
                                                        float* __restrict__ loss) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  const int lane = threadIdx.x & 63;
  const int N = R + 1;
  const float* z = Z + (int64_t)b * N;
  float mx = -INFINITY;
  for (int j = lane; j < R; j += 64) mx = fmaxf(mx, z[j]);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  float s = 0.f;
  for (int j = lane; j < R; j += 64) s += expf(z[j] - mx);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
  const float invB = 1.f / (float)B;
  int L = lab[b];
  L = L < 0 ? 0 : (L >= R ? R - 1 : L);  // labels outside [0, R) are clamped
  for (int j = lane; j < R; j += 64) {
    const float p = expf(z[j] - mx) / s;
    dZ[(int64_t)b * N + j] = f2bf((p - (j == L ? 1.f : 0.f)) * invB);
  }
  if (lane == 0) {
    const float diff = z[R] - y[b];
    dZ[(int64_t)b * N + R] = f2bf(2.f * lambda * diff * invB);
    const float ce = logf(s) + mx - z[L];
    atomicAdd(loss, (ce + lambda * diff * diff) * invB);
  }
}

hipError_t loss_grad(const float* Z, int B, int R, const int32_t* lab, const float* y, float lambda, uint16_t* dZ,
                     float* loss, hipStream_t st) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(loss_grad_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, Z, B, R, lab, y, lambda, dZ,
                     loss);
  return hipGetLastError();
}

// db[j] = sum_b G[b][j] (bf16 gradient rows -> f32 column sums).
// Column sums of a [B][N] bf16 matrix (bias gradients), deterministic: block (x, y) sums columns
// 64 x .. 64 x + 63 over the rows y, y + CS, y + 2 CS, ... (four row lanes per column, reduced in LDS in a
// fixed order) into partial[y][N]; a second kernel adds the CS partials of every column in order.
constexpr int CS = 16;  // row splits
__global__ __launch_bounds__(256) void colsum_part_kernel(const uint16_t* __restrict__ G, int B, int N,
                                                          float* __restrict__ partial) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  float s = 0.f;
  if (j < N)
    for (int b = blockIdx.y + CS * q; b < B; b += 4 * CS) s += bf2f(G[(int64_t)b * N + j]);
  red[q][c] = s;
  __syncthreads();
  if (q == 0 && j < N) partial[(int64_t)blockIdx.y * N + j] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void colsum_final_kernel(const float* __restrict__ partial, int N, float* __restrict__ db) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
#pragma unroll
  for (int y = 0; y < CS; y++) s += partial[(int64_t)y * N + j];
  db[j] = s;
}

hipError_t colsum(const uint16_t* G, int B, int N, float* db, hipStream_t st) {
  if (N == 0) return hipSuccess;
  float* partial = nullptr;
  hipError_t e = pool_malloc_async(&partial, (size_t)CS * N * 4, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)((N + 63) / 64), CS), dim3(256), 0, st, G, B, N, partial);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, partial, N, db);
  e = hipGetLastError();
  (void)hipFreeAsync(partial, st);
  return e;
}

// Adam (Kingma and Ba, 2015) on FP32 master weights; refreshes the bf16 copy.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2, uint16_t* __restrict__ wb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
}

hipError_t adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* wb, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps,
                     c1, c2, wb);
  return hipGetLastError();
}

// Inference read-out per row: confidence = max softmax probability over the R
// entry logits; seeds = ghost map of the t largest logits (ties -> smaller
// index); budget = clamp(ceil(budget_scale (exp(z_R) - 1)), t_min, t_max). Rows whose
// confidence is below tau get seeds[0] = none (fall back to ghost staging) and
// the budget t_max.
template <int NPL>
__global__ __launch_bounds__(256) void readout_kernel(const float* __restrict__ Z, int n, int R, int t, float tau,
                                                      const uint32_t* __restrict__ gmap, int t_min, int t_max,
                                                      float budget_scale,
                                                      uint32_t* __restrict__ seeds, int32_t* __restrict__ iters,
                                                      float* __restrict__ conf, uint32_t* __restrict__ top_idx) {
  __shared__ uint64_t sels[4 * 256];
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= n) return;
  const int lane = threadIdx.x & 63;
  uint64_t* sel = sels + (threadIdx.x >> 6) * 256;
  const float* zg = Z + (int64_t)b * (R + 1);
  // NPL > 0: the row's R logits are read once into registers (logit j = lane + 64 i in zr[i]); every pass below
  // reads them through zv(), in the same per-lane order either way
  float zr[NPL > 0 ? NPL : 1];
  if constexpr (NPL > 0) {
#pragma unroll
    for (int i = 0; i < NPL; i++) {
      const int j = lane + 64 * i;
      zr[i] = j < R ? zg[j] : 0.f;
    }
  }
  // f(j, z_j) for this lane's logits j = lane, lane + 64, ... < R, in increasing j
  auto each = [&](auto&& f) {
    if constexpr (NPL > 0) {
#pragma unroll
      for (int i = 0; i < NPL; i++)
        if (lane + 64 * i < R) f(lane + 64 * i, zr[i]);
    } else {
      for (int j = lane; j < R; j += 64) f(j, zg[j]);
    }
  };
  float mx = -INFINITY;
  each([&](int, float v) { mx = fmaxf(mx, v); });
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  float s = 0.f;
  each([&](int, float v) { s += expf(v - mx); });
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
  const float c = 1.f / s;
  // the t largest logits by (value desc, index asc), as ascending keys ((~ord(value)) << 32 | index)
  auto key_of = [&](int j, float v) {
    const uint32_t fb = __float_as_uint(v);
    const uint32_t ord = (fb & 0x80000000u) ? ~fb : (fb | 0x80000000u);  // order-preserving
    return ((uint64_t)(~ord) << 32) | (uint64_t)j;
  };
  // bound: the t-th smallest of the two smallest keys of every lane (a subset of the keys)
  uint64_t m2[2] = {~0ull, ~0ull};
  each([&](int j, float v) {
    uint64_t x = key_of(j, v);
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const uint64_t lo = x < m2[i] ? x : m2[i];
      x = x < m2[i] ? m2[i] : x;
      m2[i] = lo;
    }
  });
  uint64_t bound;
  if (t <= 32) {
    // the t-th smallest of the 64 lane minima (a subset of the keys, so at least t keys are at or below it)
    const uint64_t srt = bitonic_sort_u64<64>(m2[0]);
    bound = shfl_u64(srt, t - 1);
  } else {
    bitonic_sort_regs<2>(m2);
    bound = shfl_u64(t > 64 ? m2[1] : m2[0], (t - 1) & 63);
  }
  // collect the keys at or below the bound (at least t of them) and sort them
  int cnt = 0;
  auto collect = [&](int j, float v) {
    const uint64_t key = j < R ? key_of(j, v) : ~0ull;
    const bool pass = j < R && key <= bound;
    const uint64_t bm = __ballot(pass);
    const int pos = cnt + lanes_below(bm);
    if (pass && pos < 256) sel[pos] = key;
    cnt += __popcll(bm);
  };
  if constexpr (NPL > 0) {
    // every lane takes part in each round's ballot (rounds beyond R carry no keys)
#pragma unroll
    for (int i = 0; i < NPL; i++) collect(lane + 64 * i, zr[i]);
  } else {
    for (int j0 = 0; j0 < R; j0 += 64) collect(j0 + lane, j0 + lane < R ? zg[j0 + lane] : 0.f);
  }
  __builtin_amdgcn_wave_barrier();
  uint64_t v[4];
#pragma unroll
  for (int r = 0; r < 4; r++) v[r] = r * 64 + lane < cnt && r * 64 + lane < 256 ? sel[r * 64 + lane] : ~0ull;
  if (cnt <= 64) v[0] = bitonic_sort_u64<64>(v[0]);  // the usual case: one register
  else bitonic_sort_regs<4>(v);
  if (cnt > 256) {
    // more than 256 keys at the bound: t rounds of argmax instead
    uint64_t prev = 0;  // keys strictly increase
    for (int r = 0; r < t; r++) {
      uint64_t best = ~0ull;
      each([&](int j, float v) {
        const uint64_t key = key_of(j, v);
        if ((r == 0 || key > prev) && key < best) best = key;
      });
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint64_t other = shfl_xor_u64(best, o);
        best = other < best ? other : best;
      }
      prev = best;
      if (lane == 0) sel[r] = best;
    }
    __builtin_amdgcn_wave_barrier();
    v[0] = lane < t ? sel[lane] : ~0ull;
  }
  if (lane < t) {
    const uint32_t j = (uint32_t)v[0];
    if (top_idx) top_idx[(int64_t)b * t + lane] = j;
    seeds[(int64_t)b * t + lane] = (lane == 0 && c < tau) ? kNone : gmap[j];
  }
  if (lane == 0) {
    const float yb = zg[R];
    float tb = ceilf(budget_scale * (expf(yb) - 1.f));
    if (!(tb >= (float)t_min)) tb = (float)t_min;
    if (tb > (float)t_max) tb = (float)t_max;
    iters[b] = c < tau ? t_max : (int32_t)tb;  // a fallback query keeps the full budget
    conf[b] = c;
  }
}

hipError_t readout(const float* Z, int n, int R, int t, float tau, const uint32_t* gmap, int t_min, int t_max,
                   float budget_scale, uint32_t* seeds, int32_t* iters, float* conf, uint32_t* top_idx, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g((unsigned)((n + 3) / 4));
  if (R <= 1024)
    hipLaunchKernelGGL(readout_kernel<16>, g, dim3(256), 0, st, Z, n, R, t, tau, gmap, t_min, t_max, budget_scale,
                       seeds, iters, conf, top_idx);
  else if (R <= 4096)
    hipLaunchKernelGGL(readout_kernel<64>, g, dim3(256), 0, st, Z, n, R, t, tau, gmap, t_min, t_max, budget_scale,
                       seeds, iters, conf, top_idx);
  else
    hipLaunchKernelGGL(readout_kernel<0>, g, dim3(256), 0, st, Z, n, R, t, tau, gmap, t_min, t_max, budget_scale,
                       seeds, iters, conf, top_idx);
  return hipGetLastError();
}

// The output layer and the read-out without storing the logits (inference): Z = H2 W3 + b3 is formed tile by
// tile on the matrix cores (the same products, in the same order, as the output-layer GEMM) and consumed in
// registers. A block owns 128 rows (a wave 32, with their H2 fragments in registers) and sweeps the output
// columns twice in tiles of 64 through LDS (the next tile read while the current one is multiplied). The
// first sweep keeps, per row, the maximum entry logit and a list of candidate keys (value descending, index
// ascending) in global memory: a logit joins when it is above the t-th largest kept so far (later columns
// have larger indices, so an equal logit never ranks above it), and a list within 64 keys of its 256 is cut.
// The second sweep sums exp(z - maximum) (confidence = 1 / sum). Columns past the entry logits get bias
// -inf (so they drop out of both); column R's logit sets the budget. The outputs are those of the read-out
// kernel. lists: [blocks * 128][256] scratch.
__device__ __forceinline__ uint64_t logit_key(uint32_t j, float v) {
  const uint32_t fb = __float_as_uint(v);
  const uint32_t ord = (fb & 0x80000000u) ? ~fb : (fb | 0x80000000u);  // order-preserving
  return ((uint64_t)(~ord) << 32) | (uint64_t)j;
}
__device__ __forceinline__ float key_logit(uint64_t key) {
  const uint32_t ord = ~(uint32_t)(key >> 32);
  return __uint_as_float((ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Cuts one row's list (n <= 256 keys, written by this wave) without sorting it: the t-th best of the 64 lanes'
// best keys bounds the t-th best key of the list from below in rank, so every key at or before it in key order
// is kept (the true t best among them, at most 4 t keys in all); when more than 128 stay, the list is sorted
// and cut to its t best. The kept keys are written back in place; returns their number, and the key a new
// logit must beat (in kth).
__device__ __forceinline__ int cut_logits(uint64_t* __restrict__ L, int n, int t, int lane, uint64_t& kth) {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");  // the wave's own appends are visible
  uint64_t v[4];
#pragma unroll
  for (int r = 0; r < 4; r++) v[r] = r * 64 + lane < n ? L[r * 64 + lane] : ~0ull;
  uint64_t mk = v[0];
#pragma unroll
  for (int r = 1; r < 4; r++) mk = v[r] < mk ? v[r] : mk;
  const uint64_t srt = bitonic_sort_u64<64>(mk);
  uint64_t bound = t <= 64 ? readlane64(srt, t - 1) : ~0ull;
  int keep = 0;
#pragma unroll
  for (int r = 0; r < 4; r++) keep += __popcll(__ballot(v[r] <= bound && v[r] != ~0ull));
  if (keep > 128) {
    bitonic_sort_regs<4>(v);
    bound = ~0ull;
#pragma unroll
    for (int r = 0; r < 4; r++)
      if (((t - 1) >> 6) == r) bound = readlane64(v[r], (t - 1) & 63);
    keep = n < t ? n : t;
  }
  int at = 0;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const bool in = v[r] <= bound && v[r] != ~0ull;
    const uint64_t bm = __ballot(in);
    if (in) L[at + lanes_below(bm)] = v[r];
    at += __popcll(bm);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  kth = n < t ? ~0ull : bound;
  return at;
}

// The t best of one row's list (n <= 256 keys), ascending, to lanes 0 .. t - 1 (one key per lane).
__device__ __forceinline__ uint64_t best_logits(const uint64_t* __restrict__ L, int n, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  if (n <= 64) return bitonic_sort_u64<64>(lane < n ? L[lane] : ~0ull);
  if (n <= 128) {
    uint64_t w[2] = {L[lane], 64 + lane < n ? L[64 + lane] : ~0ull};
    bitonic_sort_regs<2>(w);
    return w[0];
  }
  uint64_t v[4];
#pragma unroll
  for (int r = 0; r < 4; r++) v[r] = r * 64 + lane < n ? L[r * 64 + lane] : ~0ull;
  bitonic_sort_regs<4>(v);
  return v[0];
}

template <int H>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void out_readout_kernel(
    const uint16_t* __restrict__ H2, int n, const uint16_t* __restrict__ W3t, const float* __restrict__ b3, int R,
    int no_tiles, int t, float tau, const uint32_t* __restrict__ gmap, int t_min, int t_max, float budget_scale,
    uint64_t* __restrict__ lists, uint32_t* __restrict__ seeds, int32_t* __restrict__ iters,
    float* __restrict__ conf, uint32_t* __restrict__ top_idx) {
  constexpr int P = H + 8;
  constexpr int KB = H / 16;
  constexpr int NCH = H / 32;
  constexpr int LCAP = 256;
  extern __shared__ __align__(16) char osm[];
  uint16_t* Sw = (uint16_t*)osm;
  float* thr_s = (float*)(Sw + 64 * P);
  int* cnt_s = (int*)(thr_s + 128);
  float* zr_s = (float*)(cnt_s + 128);
  float* mx_s = zr_s + 128;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int h = lane >> 5, col = lane & 31, wr = wave * 32;
  const int64_t r0 = (int64_t)blockIdx.x * 128;
  uint64_t* wl = lists + (r0 + wr) * LCAP;  // the wave's row r: wl + r * LCAP
  bf16x8 a[KB];
  {
    const bf16x8* ap = (const bf16x8*)(H2 + (r0 + wr + col) * H + h * 8);
#pragma unroll
    for (int kb = 0; kb < KB; kb++) a[kb] = ap[2 * kb];
  }
  if (tid < 128) {
    thr_s[tid] = -INFINITY;
    cnt_s[tid] = 0;
    zr_s[tid] = 0.f;
  }
  const int sr = tid >> 2, c0 = tid & 3;
  auto bias_of = [&](int j) { return j < R ? b3[j] : -INFINITY; };
  // one sweep over the output tiles; f(tt, acc) consumes each tile's two 32 x 32 accumulator blocks
  auto sweep = [&](auto&& f) {
    u32x4_t wst[NCH];
    {
      const u32x4_t* wp = (const u32x4_t*)(W3t + (int64_t)sr * H) + c0;
#pragma unroll
      for (int q = 0; q < NCH; q++) wst[q] = wp[4 * q];
    }
    float bnx[2] = {bias_of(col), bias_of(32 + col)};
    for (int tt = 0; tt < no_tiles; tt++) {
      const float bias[2] = {bnx[0], bnx[1]};
      const int nt = tt + 1 < no_tiles ? tt + 1 : tt;  // (the last tile reloads itself)
      bnx[0] = bias_of(nt * 64 + col);
      bnx[1] = bias_of(nt * 64 + 32 + col);
      __syncthreads();  // the previous tile is consumed
#pragma unroll
      for (int q = 0; q < NCH; q++) *(u32x4_t*)&Sw[sr * P + (c0 + 4 * q) * 8] = wst[q];
      {
        const u32x4_t* wp = (const u32x4_t*)(W3t + ((int64_t)nt * 64 + sr) * H) + c0;
#pragma unroll
        for (int q = 0; q < NCH; q++) wst[q] = wp[4 * q];
      }
      __syncthreads();
      f32x16 acc[2];
#pragma unroll
      for (int c = 0; c < 2; c++)
#pragma unroll
        for (int j = 0; j < 16; j++) acc[c][j] = 0.f;
#pragma unroll
      for (int kb = 0; kb < KB; kb++) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
          const bf16x8 bv = *(const bf16x8*)&Sw[(32 * c + col) * P + kb * 16 + h * 8];
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], bv, acc[c], 0, 0, 0);
        }
      }
      f(tt, acc, bias);
    }
  };
  // sweep 1: maxima, candidate lists, the budget logit
  float mx[16], tz[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    mx[j] = -INFINITY;
    tz[j] = -INFINITY;
  }
  sweep([&](int tt, const f32x16 (&acc)[2], const float (&bias)[2]) {
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const int jc = tt * 64 + 32 * c + col;
#pragma unroll
      for (int j = 0; j < 16; j++) {
        const int r = 8 * (j >> 2) + 4 * h + (j & 3);  // row within the wave
        const float z = acc[c][j] + bias[c];
        mx[j] = fmaxf(mx[j], z);
        const bool cand = z > tz[j];
        const uint64_t bm = __ballot(cand);
        if (bm) {
          const uint32_t hm = h ? (uint32_t)(bm >> 32) : (uint32_t)bm;
          const int base = cnt_s[wr + r];
          if (cand) wl[r * LCAP + base + __popc(hm & ((1u << col) - 1u))] = logit_key((uint32_t)jc, z);
          if (col == 0) cnt_s[wr + r] = base + __popc(hm);
        }
      }
    }
    if (tt == R / 64) {
      // column R (its bias was replaced by -inf above): the budget logit
#pragma unroll
      for (int c = 0; c < 2; c++)
#pragma unroll
        for (int j = 0; j < 16; j++)
          if (tt * 64 + 32 * c + col == R) zr_s[wr + 8 * (j >> 2) + 4 * h + (j & 3)] = acc[c][j] + b3[R];
    }
    // lists that could overflow in the next tile (64 more keys at most) are cut
    const int cr = cnt_s[wr + (lane & 31)];
    uint64_t need = __ballot(lane < 32 && cr > LCAP - 64);
    if (need) {
      while (need) {
        const int rr = __builtin_ctzll(need);
        need &= need - 1;
        uint64_t kth;
        const int nn = cut_logits(wl + rr * LCAP, cnt_s[wr + rr], t, lane, kth);
        if (lane == 0) {
          cnt_s[wr + rr] = nn;
          thr_s[wr + rr] = kth == ~0ull ? -INFINITY : key_logit(kth);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; j++) tz[j] = thr_s[wr + 8 * (j >> 2) + 4 * h + (j & 3)];
    }
  });
  // the rows' maxima over the 32 lanes of each half
#pragma unroll
  for (int j = 0; j < 16; j++) {
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) mx[j] = fmaxf(mx[j], __shfl_xor(mx[j], o, 64));
  }
  // sweep 2: the sums of exp(z - maximum)
  float sm[16];
#pragma unroll
  for (int j = 0; j < 16; j++) sm[j] = 0.f;
  sweep([&](int, const f32x16 (&acc)[2], const float (&bias)[2]) {
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
      for (int j = 0; j < 16; j++) sm[j] += __expf(acc[c][j] + bias[c] - mx[j]);
  });
#pragma unroll
  for (int j = 0; j < 16; j++) {
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) sm[j] += __shfl_xor(sm[j], o, 64);
    if (col == 0) mx_s[wr + 8 * (j >> 2) + 4 * h + (j & 3)] = 1.f / sm[j];  // the confidence
  }
  __builtin_amdgcn_wave_barrier();
  // every row of the wave: its t best, the confidence and the budget
  for (int rr = 0; rr < 32; rr++) {
    const int64_t b = r0 + wr + rr;
    if (b >= n) break;
    const uint64_t best = best_logits(wl + rr * LCAP, cnt_s[wr + rr], lane);
    const float c = mx_s[wr + rr];
    if (lane < t) {
      // a row whose logits are not numbers holds fewer than t keys: its missing seeds are none
      const bool ok = best != ~0ull;
      const uint32_t j = ok ? (uint32_t)best : kNone;
      if (top_idx) top_idx[b * t + lane] = j;
      seeds[b * t + lane] = (!ok || (lane == 0 && c < tau)) ? kNone : gmap[j];
    }
    if (lane == 0) {
      float tb = ceilf(budget_scale * (expf(zr_s[wr + rr]) - 1.f));
      if (!(tb >= (float)t_min)) tb = (float)t_min;
      if (tb > (float)t_max) tb = (float)t_max;
      iters[b] = c < tau ? t_max : (int32_t)tb;  // a fallback query keeps the full budget
      conf[b] = c;
    }
  }
}

bool out_readout_supported(int hidden) { return hidden == 64 || hidden == 128 || hidden == 256; }

size_t out_readout_lists_bytes(int n) { return (size_t)((n + 127) / 128) * 128 * 256 * 8; }

hipError_t out_readout(const uint16_t* H2, int n, int hidden, const uint16_t* W3t, const float* b3, int R, int t,
                       float tau, const uint32_t* gmap, int t_min, int t_max, float budget_scale, uint64_t* lists,
                       uint32_t* seeds, int32_t* iters, float* conf, uint32_t* top_idx, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!out_readout_supported(hidden) || t < 1 || t > 64 || t > R) return hipErrorInvalidValue;
  const int no_tiles = (R + 1 + 63) / 64;
  const dim3 g((unsigned)((n + 127) / 128));
  const size_t lds = (size_t)64 * (hidden + 8) * 2 + 128 * 16;
  switch (hidden) {
#define MIANN_OUT_READOUT(HH)                                                                                         \
  case HH:                                                                                                           \
    hipLaunchKernelGGL(out_readout_kernel<HH>, g, dim3(256), lds, st, H2, n, W3t, b3, R, no_tiles, t, tau, gmap, t_min, \
                       t_max, budget_scale, lists, seeds, iters, conf, top_idx);                                      \
    break;
    MIANN_OUT_READOUT(64)
    MIANN_OUT_READOUT(128)
    MIANN_OUT_READOUT(256)
#undef MIANN_OUT_READOUT
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

hipError_t zero_f32(float* p, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// Random permutation for shuffling: keys = splitmix(seed, i + 1), sorted elsewhere.

}  // namespace miann
