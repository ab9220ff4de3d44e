// Kernels of the learned entry / iteration-budget predictor: a BF16 MLP
// d_in -> hidden -> hidden -> (R entry logits + 1 budget) trained on traces of
// the search itself. GEMMs run on the gfx950 BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation and FP32 master weights.
#include "common.hpp"
#include "mlp.hpp"

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
__global__ void colsum_kernel(const uint16_t* __restrict__ G, int B, int N, float* __restrict__ db) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; b++) s += bf2f(G[(int64_t)b * N + j]);
  db[j] = s;
}

hipError_t colsum(const uint16_t* G, int B, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, G, B, N, db);
  return hipGetLastError();
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
