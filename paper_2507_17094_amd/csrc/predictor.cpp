// C-ABI of the learned entry / iteration-budget predictor: a BF16 MLP trained
// by the library's own forward and backward kernels (mlp.hip) on traces of the
// plain search, used to seed the search and set a per-query iteration budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/miann.h"
#include "common.hpp"
#include "pool.hpp"
#include "knn.hpp"
#include "mlp.hpp"

using namespace miann;

// shared with capi.cpp
miann_status miann_fail(miann_status st, const char* fmt, ...);

#define PTRY(expr)                                                                                         \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess) return miann_fail(MIANN_EDEVICE, "%s: %s (%s)", __func__, #expr, hipGetErrorString(e_)); \
  } while (0)

struct miann_predictor {
  int d_in = 0, hidden = 0, R = 0, n_out = 0;
  float* w[6] = {};   // W1 [d][h], b1 [h], W2 [h][h], b2 [h], W3 [h][n_out], b3 [n_out]
  float* g[6] = {};   // gradients
  float* m[6] = {};   // Adam moments
  float* v[6] = {};
  uint16_t* wb[3] = {};  // bf16 copies of W1, W2, W3
  int64_t sz[6] = {};
  int step = 0;
  std::vector<void*> allocs;
  ~miann_predictor() {
    for (void* p : allocs) hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e == hipSuccess) { allocs.push_back(q); *p = (T*)q; }
    return e;
  }
};

namespace {

struct Work {
  hipStream_t st;
  std::vector<void*> v;
  explicit Work(hipStream_t s) : st(s) {}
  template <typename T>
  hipError_t get(T** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = pool_malloc_async(&q, bytes ? bytes : 16, st);
    if (e == hipSuccess) { v.push_back(q); *p = (T*)q; }
    return e;
  }
  ~Work() { for (void* p : v) hipFreeAsync(p, st); }
};

// Forward over B rows of bf16 inputs xb: H1, H2 (bf16), Z (f32).
hipError_t forward(const miann_predictor* P, const uint16_t* xb, int B, uint16_t* H1, uint16_t* H2, float* Z,
                   hipStream_t st) {
  const int d = P->d_in, h = P->hidden, no = P->n_out;
  hipError_t e = gemm_bf16(B, h, d, xb, d, 1, P->wb[0], h, 1, P->w[1], 1, nullptr, nullptr, H1, h, st);
  if (e == hipSuccess) e = gemm_bf16(B, h, h, H1, h, 1, P->wb[1], h, 1, P->w[3], 1, nullptr, nullptr, H2, h, st);
  if (e == hipSuccess) e = gemm_bf16(B, no, h, H2, h, 1, P->wb[2], no, 1, P->w[5], 0, nullptr, Z, nullptr, no, st);
  return e;
}

// Loss, backward into P->g, optional Adam update.
miann_status fwd_bwd(miann_predictor* P, const uint16_t* xb, const int32_t* lab, const float* y, int B, float lambda,
                     float lr, int update, float* loss_dev, hipStream_t st) {
  const int d = P->d_in, h = P->hidden, no = P->n_out;
  Work w(st);
  uint16_t *H1, *H2, *dZ, *dH2, *dH1;
  float* Z;
  PTRY(w.get(&H1, (size_t)B * h * 2));
  PTRY(w.get(&H2, (size_t)B * h * 2));
  PTRY(w.get(&Z, (size_t)B * no * 4));
  PTRY(w.get(&dZ, (size_t)B * no * 2));
  PTRY(w.get(&dH2, (size_t)B * h * 2));
  PTRY(w.get(&dH1, (size_t)B * h * 2));
  PTRY(forward(P, xb, B, H1, H2, Z, st));
  PTRY(loss_grad(Z, B, P->R, lab, y, lambda, dZ, loss_dev, st));
  // dW3 = H2^T dZ, db3 = colsum(dZ), dH2 = (dZ W3^T) * [H2 > 0]
  PTRY(gemm_bf16(h, no, B, H2, 1, h, dZ, no, 1, nullptr, 0, nullptr, P->g[4], nullptr, no, st));
  PTRY(colsum(dZ, B, no, P->g[5], st));
  PTRY(gemm_bf16(B, h, no, dZ, no, 1, P->wb[2], 1, no, nullptr, 0, H2, nullptr, dH2, h, st));
  // dW2 = H1^T dH2, db2, dH1 = (dH2 W2^T) * [H1 > 0]
  PTRY(gemm_bf16(h, h, B, H1, 1, h, dH2, h, 1, nullptr, 0, nullptr, P->g[2], nullptr, h, st));
  PTRY(colsum(dH2, B, h, P->g[3], st));
  PTRY(gemm_bf16(B, h, h, dH2, h, 1, P->wb[1], 1, h, nullptr, 0, H1, nullptr, dH1, h, st));
  // dW1 = X^T dH1, db1
  PTRY(gemm_bf16(d, h, B, xb, 1, d, dH1, h, 1, nullptr, 0, nullptr, P->g[0], nullptr, h, st));
  PTRY(colsum(dH1, B, h, P->g[1], st));
  if (update) {
    P->step++;
    for (int i = 0; i < 6; i++)
      PTRY(adam(P->w[i], P->g[i], P->m[i], P->v[i], P->sz[i], lr, 0.9f, 0.999f, 1e-8f, P->step,
                (i % 2 == 0) ? P->wb[i / 2] : nullptr, st));
  }
  return MIANN_OK;
}

}  // namespace

extern "C" {

miann_status miann_predictor_create(int32_t d_in, int32_t hidden, int32_t n_entry, uint64_t seed,
                                    miann_predictor** out) {
  if (!out) return miann_fail(MIANN_EINVAL, "miann_predictor_create: null output");
  if (d_in < 1 || d_in > 4096 || hidden < 1 || hidden > 4096 || n_entry < 2 || n_entry > (1 << 20))
    return miann_fail(MIANN_EINVAL, "miann_predictor_create: sizes out of range");
  miann_predictor* P = new miann_predictor();
  P->d_in = d_in;
  P->hidden = hidden;
  P->R = n_entry;
  P->n_out = n_entry + 1;
  const int64_t sz[6] = {(int64_t)d_in * hidden, hidden, (int64_t)hidden * hidden, hidden,
                         (int64_t)hidden * P->n_out, P->n_out};
  const int64_t fan_in[6] = {d_in, d_in, hidden, hidden, hidden, hidden};
  // a non-blocking stream of its own: creating a predictor waits for its own copies only, not for the work
  // other streams (a server, say) have queued
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  std::vector<std::vector<float>> host(6);
  for (int i = 0; i < 6 && e == hipSuccess; i++) {
    P->sz[i] = sz[i];
    e = P->alloc(&P->w[i], sz[i] * 4);
    if (e == hipSuccess) e = P->alloc(&P->g[i], sz[i] * 4);
    if (e == hipSuccess) e = P->alloc(&P->m[i], sz[i] * 4);
    if (e == hipSuccess) e = P->alloc(&P->v[i], sz[i] * 4);
    if (e == hipSuccess && i % 2 == 0) e = P->alloc(&P->wb[i / 2], sz[i] * 2);
    if (e != hipSuccess) break;
    // weights U(-a, a), a = sqrt(6 / fan_in) from SplitMix64; biases zero
    std::vector<float>& h = host[i];
    h.assign(sz[i], 0.f);
    if (i % 2 == 0) {
      const double a = std::sqrt(6.0 / (double)fan_in[i]);
      for (int64_t j = 0; j < sz[i]; j++) {
        const double u = (double)(sm_at(seed + (uint64_t)i, (uint64_t)j + 1) >> 11) * (1.0 / 9007199254740992.0);
        h[j] = (float)(a * (2.0 * u - 1.0));
      }
    }
    e = hipMemcpyAsync(P->w[i], h.data(), sz[i] * 4, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipMemsetAsync(P->m[i], 0, sz[i] * 4, cs);
    if (e == hipSuccess) e = hipMemsetAsync(P->v[i], 0, sz[i] * 4, cs);
    if (e == hipSuccess) e = hipMemsetAsync(P->g[i], 0, sz[i] * 4, cs);
    if (e == hipSuccess && i % 2 == 0) e = to_bf16(P->w[i], sz[i], P->wb[i / 2], cs);
  }
  if (cs) {
    const hipError_t e2 = hipStreamSynchronize(cs);  // the host copies must outlive the transfers
    if (e == hipSuccess) e = e2;
    hipStreamDestroy(cs);
  }
  if (e != hipSuccess) {
    delete P;
    return miann_fail(MIANN_EDEVICE, "miann_predictor_create: %s", hipGetErrorString(e));
  }
  *out = P;
  return MIANN_OK;
}

void miann_predictor_free(miann_predictor* p) { delete p; }

miann_status miann_predictor_view_get(miann_predictor* P, miann_predictor_view* o) {
  if (!P || !o) return miann_fail(MIANN_EINVAL, "miann_predictor_view_get: null argument");
  o->d_in = P->d_in;
  o->hidden = P->hidden;
  o->n_entry = P->R;
  o->W1 = P->w[0]; o->b1 = P->w[1]; o->W2 = P->w[2]; o->b2 = P->w[3]; o->W3 = P->w[4]; o->b3 = P->w[5];
  o->gW1 = P->g[0]; o->gb1 = P->g[1]; o->gW2 = P->g[2]; o->gb2 = P->g[3]; o->gW3 = P->g[4]; o->gb3 = P->g[5];
  return MIANN_OK;
}

miann_status miann_predictor_sync_weights(miann_predictor* P, void* stream) {
  if (!P) return miann_fail(MIANN_EINVAL, "miann_predictor_sync_weights: null predictor");
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < 3; i++) PTRY(to_bf16(P->w[2 * i], P->sz[2 * i], P->wb[i], st));
  PTRY(hipStreamSynchronize(st));
  return MIANN_OK;
}

miann_status miann_predictor_step(miann_predictor* P, const float* x, const int32_t* entry, const float* budget,
                                  int32_t n, float lambda, float lr, int32_t update, float* loss_host, void* stream) {
  if (!P || !x || !entry || !budget) return miann_fail(MIANN_EINVAL, "miann_predictor_step: null argument");
  if (n < 1) return miann_fail(MIANN_EINVAL, "miann_predictor_step: n = %d", n);
  hipStream_t st = (hipStream_t)stream;
  Work w(st);
  uint16_t* xb;
  float* loss;
  PTRY(w.get(&xb, (size_t)n * P->d_in * 2));
  PTRY(w.get(&loss, 4));
  PTRY(zero_f32(loss, 1, st));
  PTRY(gather_batch(x, P->d_in, nullptr, n, nullptr, nullptr, xb, nullptr, nullptr, st));
  miann_status rc = fwd_bwd(P, xb, entry, budget, n, lambda, lr, update, loss, st);
  if (rc) return rc;
  float h = 0.f;
  PTRY(hipMemcpyAsync(&h, loss, 4, hipMemcpyDeviceToHost, st));
  PTRY(hipStreamSynchronize(st));
  if (loss_host) *loss_host = h;
  return MIANN_OK;
}

miann_status miann_predictor_train(miann_predictor* P, const float* x, const int32_t* entry, const float* budget,
                                   int64_t n, int32_t epochs, int32_t batch, float lr, float lambda, uint64_t seed,
                                   float* epoch_loss, void* stream) {
  if (!P || !x || !entry || !budget) return miann_fail(MIANN_EINVAL, "miann_predictor_train: null argument");
  if (n < 1 || epochs < 1 || batch < 1 || batch > (1 << 20))
    return miann_fail(MIANN_EINVAL, "miann_predictor_train: n, epochs, batch must be positive");
  hipStream_t st = (hipStream_t)stream;
  Work w(st);
  uint32_t* order;
  uint16_t* xb;
  int32_t* lb;
  float *yb, *loss;
  PTRY(w.get(&order, (size_t)n * 4));
  PTRY(w.get(&xb, (size_t)batch * P->d_in * 2));
  PTRY(w.get(&lb, (size_t)batch * 4));
  PTRY(w.get(&yb, (size_t)batch * 4));
  PTRY(w.get(&loss, 4));
  for (int ep = 0; ep < epochs; ep++) {
    PTRY(keyed_order(sm_at(seed, (uint64_t)ep + 1), n, order, st));
    PTRY(zero_f32(loss, 1, st));
    int nb = 0;
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
      const int B = (int)std::min<int64_t>(batch, n - b0);
      PTRY(gather_batch(x, P->d_in, order + b0, B, entry, budget, xb, lb, yb, st));
      miann_status rc = fwd_bwd(P, xb, lb, yb, B, lambda, lr, 1, loss, st);
      if (rc) return rc;
      nb++;
    }
    if (epoch_loss) {
      float h = 0.f;
      PTRY(hipMemcpyAsync(&h, loss, 4, hipMemcpyDeviceToHost, st));
      PTRY(hipStreamSynchronize(st));
      epoch_loss[ep] = h / (float)nb;
    }
  }
  PTRY(hipStreamSynchronize(st));
  return MIANN_OK;
}

miann_status miann_predictor_predict(const miann_predictor* P, const float* x, int64_t n, int32_t t, float tau,
                                     const uint32_t* ghost_map, int32_t t_min, int32_t t_max, float budget_scale,
                                     uint32_t* seeds, int32_t* iters, float* conf, uint32_t* top_entry,
                                     void* stream) {
  if (!P || (n > 0 && (!x || !ghost_map || !seeds || !iters || !conf)))
    return miann_fail(MIANN_EINVAL, "miann_predictor_predict: null argument");
  if (t < 1 || t > 64 || t > P->R) return miann_fail(MIANN_EINVAL, "miann_predictor_predict: t = %d out of range", t);
  if (t_min < 0 || t_max < t_min) return miann_fail(MIANN_EINVAL, "miann_predictor_predict: bad budget bounds");
  if (!(budget_scale > 0.f) || budget_scale > 1000.f)
    return miann_fail(MIANN_EINVAL, "miann_predictor_predict: budget_scale must be in (0, 1000]");
  hipStream_t st = (hipStream_t)stream;
  Work w(st);
  uint16_t *xb, *H1, *H2, *W3t;
  const int h = P->hidden, no = P->n_out, no_pad = (no + 63) / 64 * 64;
  // hidden widths the fused output layer covers: the logits are consumed where they are formed; others write
  // them to memory and read them back
  const bool fused = out_readout_supported(h);
  const int64_t chunk = fused ? 65536 : 16384;
  PTRY(w.get(&xb, (size_t)chunk * P->d_in * 2));
  PTRY(w.get(&H1, (size_t)chunk * h * 2));
  PTRY(w.get(&H2, (size_t)chunk * h * 2));
  // the output layer's weights column by column, so its tiles are staged in 16-byte vectors (the same products)
  PTRY(w.get(&W3t, (size_t)no_pad * h * 2));
  PTRY(transpose_bf16(P->wb[2], h, no, no_pad, W3t, st));
  float* Z = nullptr;
  uint64_t* lists = nullptr;
  if (fused) PTRY(w.get(&lists, out_readout_lists_bytes((int)chunk)));
  else PTRY(w.get(&Z, (size_t)chunk * no * 4));
  for (int64_t b0 = 0; b0 < n; b0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n - b0);
    PTRY(gather_batch(x + b0 * P->d_in, P->d_in, nullptr, B, nullptr, nullptr, xb, nullptr, nullptr, st));
    PTRY(gemm_bf16(B, h, P->d_in, xb, P->d_in, 1, P->wb[0], h, 1, P->w[1], 1, nullptr, nullptr, H1, h, st));
    PTRY(gemm_bf16(B, h, h, H1, h, 1, P->wb[1], h, 1, P->w[3], 1, nullptr, nullptr, H2, h, st));
    if (fused) {
      PTRY(out_readout(H2, B, h, W3t, P->w[5], P->R, t, tau, ghost_map, t_min, t_max, budget_scale, lists,
                       seeds + b0 * t, iters + b0, conf + b0, top_entry ? top_entry + b0 * t : nullptr, st));
    } else {
      PTRY(gemm_bf16(B, no, h, H2, h, 1, W3t, 1, h, P->w[5], 0, nullptr, Z, nullptr, no, st));
      PTRY(readout(Z, B, P->R, t, tau, ghost_map, t_min, t_max, budget_scale, seeds + b0 * t, iters + b0, conf + b0,
                   top_entry ? top_entry + b0 * t : nullptr, st));
    }
  }
  return MIANN_OK;
}

}  // extern "C"
