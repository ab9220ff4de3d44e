// C-ABI of libmiann: index objects, argument validation, error reporting and
// the host side of build / search. Every compute step runs in the HIP kernels
// of search.hip, build.hip and knn.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/miann.h"
#include "build.hpp"
#include "pool.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "knn.hpp"

using namespace miann;

namespace {

thread_local std::string g_err;

miann_status fail(miann_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MIANN_EDEVICE, "%s: %s (%s)", __func__, #expr, hipGetErrorString(e_)); \
  } while (0)

int esize_of(int dt) { return dt == MIANN_F32 ? 4 : dt == MIANN_F16 ? 2 : 1; }
int round_up(int x, int m) { return (x + m - 1) / m * m; }
// Stored row length in elements: rows padded to a multiple of 128 bytes.
int pad_elems(int d, int esize) { return round_up(d * esize, 128) / esize; }
int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

struct Shard {
  int64_t n = 0, R = 0;
  void* store = nullptr;      // [n][d_pad] traversal codes
  float* scale = nullptr;     // [n]
  void* orig = nullptr;       // [n][d_pad_in] originals (== store when not quantised)
  uint32_t* graph = nullptr;  // [n][deg]
  uint32_t* sign = nullptr;   // [n][W][deg]
  uint32_t* gmap = nullptr;   // [n]
  uint32_t* next = nullptr;   // [n]
  void* g_store = nullptr;    // [R][d_pad]
  float* g_scale = nullptr;   // [R]
  uint32_t* g_graph = nullptr;// [R][deg_g]
  uint32_t* g_map = nullptr;  // [R]
  float* g_f32 = nullptr;     // [R][d_pad_f32] traversal values in f32 (MFMA dense entry)
  uint8_t* dead = nullptr;    // [n] deletion flags, or null when nothing was deleted
};

}  // namespace

// Error reporting shared with the predictor translation unit.
miann_status miann_fail(miann_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

struct miann_index;
int miann_index_input_esize(const miann_index* idx, int32_t* d_out);

struct miann_index {
  int S = 1, d = 0, deg = 0, deg_g = 0, W = 0;
  int store_dtype = MIANN_F32, in_dtype = MIANN_F32, dgs = 0;
  int d_pad = 0;      // store row length (elements)
  int d_pad_in = 0;   // originals row length
  int d_pad_f32 = 0;  // f32 row length (rerank originals / MFMA copies)
  int64_t n_total = 0;
  int knn_k0 = 0;           // K0 of the graph build (0 = 2 * degree), reused when a shard is rebuilt
  uint64_t ghost_seed = 0;  // seed of the last ghost sample, reused when a shard is rebuilt
  // host seconds of the build steps: [graph (k-NN and pruning), direction table, inter-shard map, ghost shards]
  double build_s[4] = {0, 0, 0, 0};
  std::vector<Shard> sh;
  DenseGhosts dg;  // all shards' ghosts, bf16-split, for the dense entry
  std::vector<void*> allocs;
  std::vector<void*> ghost_allocs;
  ShardDev* dev_shards = nullptr;  // [S] descriptors read by the search kernels

  template <typename T>
  hipError_t alloc(T** p, size_t bytes, bool ghost = false) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
    if (e != hipSuccess) return e;
    (ghost ? ghost_allocs : allocs).push_back(v);
    *p = (T*)v;
    return hipSuccess;
  }
  // Frees one array of `allocs` (the caller has synchronised the streams that used it).
  void release(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it == allocs.end()) return;
    allocs.erase(it);
    hipFree(p);
  }
  void free_ghost() {
    for (void* p : ghost_allocs) hipFree(p);
    ghost_allocs.clear();
    for (auto& s : sh) {
      s.R = 0;
      s.g_store = nullptr; s.g_scale = nullptr; s.g_graph = nullptr; s.g_map = nullptr; s.g_f32 = nullptr;
    }
    dg = DenseGhosts();
  }
  ~miann_index() {
    free_ghost();
    for (void* p : allocs) hipFree(p);
  }
  // Uploads the shard descriptors (after any change of the shard arrays).
  hipError_t refresh(hipStream_t st) {
    std::vector<ShardDev> h(S);
    const bool lp = store_dtype == 1 || store_dtype == 2;
    for (int s = 0; s < S; s++) {
      const Shard& x = sh[s];
      ShardDev& o = h[s];
      o.store = x.store; o.scale = x.scale; o.orig = lp ? (const float*)x.orig : nullptr;
      o.graph = x.graph; o.sign = x.sign; o.gmap = x.gmap; o.next = x.next;
      o.g_store = x.g_store; o.g_scale = x.g_scale; o.g_graph = x.g_graph; o.g_map = x.g_map;
      o.dead = x.dead;
      o.n = (uint32_t)x.n; o.R = (uint32_t)x.R;
    }
    hipError_t e = hipSuccess;
    if (!dev_shards) e = alloc(&dev_shards, sizeof(ShardDev) * S);
    if (e == hipSuccess) e = hipMemcpyAsync(dev_shards, h.data(), sizeof(ShardDev) * S, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  }
};

namespace {

bool lowp(int dt) { return dt == MIANN_F16 || dt == MIANN_FP8E4M3; }

// Fills the store / originals / f32 copies of shard `s` from `src` rows.
miann_status fill_vectors(miann_index* ix, Shard& sh, const void* src, const uint32_t* rows, hipStream_t st) {
  const int64_t n = sh.n;
  const int ein = esize_of(ix->in_dtype);
  HIP_TRY(ix->alloc(&sh.orig, (size_t)n * ix->d_pad_in * ein));
  HIP_TRY(pad_rows(src, n, ix->d, ein, sh.orig, ix->d_pad_in, rows, st));
  if (lowp(ix->store_dtype)) {
    HIP_TRY(ix->alloc(&sh.store, (size_t)n * ix->d_pad * esize_of(ix->store_dtype)));
    HIP_TRY(ix->alloc(&sh.scale, (size_t)n * 4));
    HIP_TRY(quantize((const float*)src, n, ix->d, ix->store_dtype, sh.store, ix->d_pad, sh.scale, rows, st));
  } else {
    sh.store = sh.orig;
  }
  return MIANN_OK;
}

miann_status build_ghost_store(miann_index* ix, Shard& sh, hipStream_t st) {
  const int64_t R = sh.R;
  const int rb = ix->d_pad * esize_of(ix->store_dtype);
  HIP_TRY(ix->alloc(&sh.g_store, (size_t)R * rb, true));
  HIP_TRY(gather_rows(sh.store, sh.g_map, R, rb, sh.g_store, st));
  if (sh.scale) {
    HIP_TRY(ix->alloc(&sh.g_scale, (size_t)R * 4, true));
    HIP_TRY(gather_f32(sh.scale, sh.g_map, R, sh.g_scale, st));
  }
  HIP_TRY(ix->alloc(&sh.g_f32, (size_t)R * ix->d_pad_f32 * 4, true));
  HIP_TRY(dequant_rows(sh.g_store, sh.g_scale, ix->store_dtype, R, ix->d_pad, ix->d_pad_f32, sh.g_f32, st));
  return MIANN_OK;
}

// Concatenates the ghost rows of every shard (each block padded to 64 columns)
// as bf16 hi / lo halves with f32 norms, for the dense entry of all shards.
miann_status build_dense_ghosts(miann_index* ix, hipStream_t st) {
  DenseGhosts& G = ix->dg;
  G = DenseGhosts();
  G.dk = ix->d_pad_f32;
  G.off.assign(ix->S + 1, 0);
  G.R.assign(ix->S, 0);
  for (int s = 0; s < ix->S; s++) {
    if (ix->sh[s].R == 0) return MIANN_OK;  // the dense entry needs every shard's ghosts
    G.R[s] = ix->sh[s].R;
    G.off[s + 1] = G.off[s] + (G.R[s] + 63) / 64 * 64;
  }
  G.cols = G.off[ix->S];
  HIP_TRY(ix->alloc(&G.hi, (size_t)G.cols * G.dk * 2, true));
  HIP_TRY(ix->alloc(&G.lo, (size_t)G.cols * G.dk * 2, true));
  HIP_TRY(ix->alloc(&G.norm, (size_t)G.cols * 4, true));
  HIP_TRY(ix->alloc(&G.off_dev, (size_t)(ix->S + 1) * 8, true));
  HIP_TRY(ix->alloc(&G.R_dev, (size_t)ix->S * 8, true));
  HIP_TRY(ix->alloc(&G.shards_dev, sizeof(DenseShardDev) * ix->S, true));
  std::vector<DenseShardDev> sd(ix->S);
  for (int s = 0; s < ix->S; s++) sd[s] = DenseShardDev{ix->sh[s].g_store, ix->sh[s].g_scale, ix->sh[s].g_map};
  HIP_TRY(hipMemcpyAsync(G.shards_dev, sd.data(), sizeof(DenseShardDev) * ix->S, hipMemcpyHostToDevice, st));
  for (int s = 0; s < ix->S; s++) {
    const size_t o = (size_t)G.off[s];
    HIP_TRY(split_rows(ix->sh[s].g_f32, G.R[s], G.off[s + 1] - G.off[s], G.dk, G.hi + o * G.dk, G.lo + o * G.dk,
                       G.norm + o, st));
  }
  HIP_TRY(hipMemcpyAsync(G.off_dev, G.off.data(), (size_t)(ix->S + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G.R_dev, G.R.data(), (size_t)ix->S * 8, hipMemcpyHostToDevice, st));
  // each shard's largest ghost norm (the dense entry's error bound scales with it)
  std::vector<float> norms((size_t)G.cols), gmax((size_t)ix->S, 0.f);
  HIP_TRY(hipMemcpyAsync(norms.data(), G.norm, (size_t)G.cols * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int s = 0; s < ix->S; s++)
    for (int64_t j = 0; j < G.R[s]; j++) gmax[s] = std::max(gmax[s], norms[(size_t)(G.off[s] + j)]);
  HIP_TRY(ix->alloc(&G.gmax_dev, (size_t)ix->S * 4, true));
  HIP_TRY(hipMemcpyAsync(G.gmax_dev, gmax.data(), (size_t)ix->S * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return MIANN_OK;
}

miann_status check_common_dims(int d, int in_dtype, int store_dtype, int degree) {
  if (d < 1 || d > 4096) return fail(MIANN_EINVAL, "d = %d out of range [1, 4096]", d);
  if (in_dtype != MIANN_F32 && in_dtype != MIANN_U8) return fail(MIANN_EINVAL, "in_dtype must be F32 or U8");
  if (in_dtype == MIANN_U8 && store_dtype != MIANN_U8) return fail(MIANN_EINVAL, "u8 input needs the U8 store");
  if (in_dtype == MIANN_F32 && store_dtype == MIANN_U8) return fail(MIANN_EINVAL, "float input cannot use the U8 store");
  if (store_dtype < 0 || store_dtype > 3) return fail(MIANN_EINVAL, "store_dtype %d invalid", store_dtype);
  if (degree < 2 || degree > 64) return fail(MIANN_EINVAL, "degree = %d out of range [2, 64]", degree);
  const int row = pad_elems(d, esize_of(store_dtype)) * esize_of(store_dtype);
  if (row / 128 > 8) return fail(MIANN_EUNSUPPORTED, "stored rows of %d bytes exceed 1024", row);
  return MIANN_OK;
}

void init_dims(miann_index* ix, int d, int in_dtype, int store_dtype, int degree, int ghost_degree, int dgs) {
  ix->d = d;
  ix->in_dtype = in_dtype;
  ix->store_dtype = store_dtype;
  ix->deg = degree;
  ix->deg_g = ghost_degree;
  ix->dgs = dgs;
  ix->W = (d + 31) / 32;
  ix->d_pad = pad_elems(d, esize_of(store_dtype));
  ix->d_pad_in = pad_elems(d, esize_of(in_dtype));
  ix->d_pad_f32 = pad_elems(d, 4);
}

}  // namespace

// Element size of the index's input type (for the serving layer).
int miann_index_input_esize(const miann_index* idx, int32_t* d_out) {
  if (d_out) *d_out = idx->d;
  return idx->in_dtype == MIANN_U8 ? 1 : 4;
}

extern "C" {

const char* miann_last_error(void) { return g_err.c_str(); }
const char* miann_version(void) { return "miann 0.1 (gfx950)"; }

void miann_index_free(miann_index* idx) { delete idx; }

miann_status miann_index_build_times(const miann_index* idx, double* seconds4) {
  if (!idx || !seconds4) return fail(MIANN_EINVAL, "miann_index_build_times: null argument");
  for (int i = 0; i < 4; i++) seconds4[i] = idx->build_s[i];
  return MIANN_OK;
}

miann_status miann_index_info(const miann_index* idx, int32_t* num_shards, int64_t* n_total, int32_t* d,
                              int32_t* degree, int32_t* store_dtype) {
  if (!idx) return fail(MIANN_EINVAL, "miann_index_info: null index");
  if (num_shards) *num_shards = idx->S;
  if (n_total) *n_total = idx->n_total;
  if (d) *d = idx->d;
  if (degree) *degree = idx->deg;
  if (store_dtype) *store_dtype = idx->store_dtype;
  return MIANN_OK;
}

miann_status miann_index_shard(const miann_index* idx, int32_t s, miann_shard_view* o) {
  if (!idx || !o) return fail(MIANN_EINVAL, "miann_index_shard: null argument");
  if (s < 0 || s >= idx->S) return fail(MIANN_EINVAL, "miann_index_shard: shard %d out of range", s);
  const Shard& h = idx->sh[s];
  o->n = h.n;
  o->n_ghost = h.R;
  o->d = idx->d;
  o->d_pad = idx->d_pad;
  o->degree = idx->deg;
  o->ghost_degree = idx->deg_g;
  o->W = idx->W;
  o->store_dtype = idx->store_dtype;
  o->in_dtype = idx->in_dtype;
  o->store = h.store;
  o->scale = h.scale;
  o->originals = h.orig;
  o->graph = h.graph;
  o->sign = h.sign;
  o->global_ids = h.gmap;
  o->next_map = h.next;
  o->ghost_ids = h.g_map;
  o->ghost_graph = h.g_graph;
  return MIANN_OK;
}

miann_status miann_index_import(const miann_shard_desc* shards, int32_t S, int32_t d, int32_t in_dtype,
                                int32_t store_dtype, int32_t degree, int32_t ghost_degree, int32_t dgs_table,
                                void* stream, miann_index** out) {
  if (!shards || !out) return fail(MIANN_EINVAL, "miann_index_import: null argument");
  if (S < 1 || S > kMaxShards) return fail(MIANN_EINVAL, "num_shards = %d out of range [1, %d]", S, kMaxShards);
  miann_status rc = check_common_dims(d, in_dtype, store_dtype, degree);
  if (rc) return rc;
  int64_t total = 0;
  for (int s = 0; s < S; s++) {
    const miann_shard_desc& sd = shards[s];
    if (sd.n < degree + 1) return fail(MIANN_EINVAL, "shard %d has %lld nodes, needs >= degree + 1", s, (long long)sd.n);
    if (!sd.vectors || !sd.graph) return fail(MIANN_EINVAL, "shard %d: vectors and graph are required", s);
    if (S > 1 && !sd.next_map) return fail(MIANN_EINVAL, "shard %d: next_map required when S > 1", s);
    if (sd.n_ghost < 0 || (sd.n_ghost > 0 && (!sd.ghost_ids || !sd.ghost_graph)))
      return fail(MIANN_EINVAL, "shard %d: ghost arrays missing", s);
    if (sd.n_ghost > 0 && (ghost_degree < 2 || ghost_degree > 64 || sd.n_ghost < ghost_degree + 1))
      return fail(MIANN_EINVAL, "shard %d: ghost_degree %d invalid for %lld ghosts", s, ghost_degree,
                  (long long)sd.n_ghost);
    total += sd.n;
  }
  if (total >= (1ll << 30)) return fail(MIANN_EINVAL, "total nodes %lld exceed 2^30 - 1", (long long)total);
  hipStream_t st = (hipStream_t)stream;
  // every id the search will follow must lie inside its target array
  for (int s = 0; s < S; s++) {
    const miann_shard_desc& sd = shards[s];
    struct { const uint32_t* p; int64_t n; int64_t lim; int none; const char* what; } chk[] = {
        {sd.graph, sd.n * degree, sd.n, 1, "graph"},
        {sd.next_map, sd.next_map ? sd.n : 0, shards[(s + 1) % S].n, 0, "next_map"},
        {sd.ghost_ids, sd.n_ghost, sd.n, 0, "ghost_ids"},
        {sd.ghost_graph, sd.n_ghost * ghost_degree, sd.n_ghost, 1, "ghost_graph"},
        {sd.global_ids, sd.global_ids ? sd.n : 0, 1ll << 30, 0, "global_ids"}};
    for (auto& c : chk) {
      int64_t bad = 0;
      hipError_t e = count_out_of_range(c.p, c.n, (uint32_t)std::min<int64_t>(c.lim, 0xFFFFFFFFll), c.none, &bad, st);
      if (e != hipSuccess) return fail(MIANN_EDEVICE, "miann_index_import: %s", hipGetErrorString(e));
      if (bad) return fail(MIANN_EINVAL, "miann_index_import: shard %d: %lld %s entries out of range", s, (long long)bad, c.what);
    }
  }
  miann_index* ix = new miann_index();
  init_dims(ix, d, in_dtype, store_dtype, degree, ghost_degree, dgs_table);
  ix->S = S;
  ix->n_total = total;
  ix->sh.resize(S);
  int64_t off = 0;
  for (int s = 0; s < S && rc == MIANN_OK; s++) {
    const miann_shard_desc& sd = shards[s];
    Shard& h = ix->sh[s];
    h.n = sd.n;
    if ((rc = fill_vectors(ix, h, sd.vectors, nullptr, st))) break;
    hipError_t e = ix->alloc(&h.graph, (size_t)h.n * degree * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(h.graph, sd.graph, (size_t)h.n * degree * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = ix->alloc(&h.gmap, (size_t)h.n * 4);
    if (e == hipSuccess)
      e = sd.global_ids ? hipMemcpyAsync(h.gmap, sd.global_ids, (size_t)h.n * 4, hipMemcpyDeviceToDevice, st)
                        : iota_u32(h.gmap, h.n, (uint32_t)off, st);
    if (e == hipSuccess && sd.next_map) {
      e = ix->alloc(&h.next, (size_t)h.n * 4);
      if (e == hipSuccess) e = hipMemcpyAsync(h.next, sd.next_map, (size_t)h.n * 4, hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess && dgs_table) {
      e = ix->alloc(&h.sign, (size_t)h.n * ix->W * degree * 4);
      if (e == hipSuccess) e = sign_table(h.orig, in_dtype, h.n, d, ix->d_pad_in, h.graph, degree, h.sign, st);
    }
    if (e == hipSuccess && sd.n_ghost > 0) {
      h.R = sd.n_ghost;
      e = ix->alloc(&h.g_map, (size_t)h.R * 4, true);
      if (e == hipSuccess) e = hipMemcpyAsync(h.g_map, sd.ghost_ids, (size_t)h.R * 4, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = ix->alloc(&h.g_graph, (size_t)h.R * ghost_degree * 4, true);
      if (e == hipSuccess)
        e = hipMemcpyAsync(h.g_graph, sd.ghost_graph, (size_t)h.R * ghost_degree * 4, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) rc = build_ghost_store(ix, h, st);
    }
    if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_index_import: %s", hipGetErrorString(e));
    off += h.n;
  }
  if (rc == MIANN_OK) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = ix->refresh(st);
    if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_index_import: %s", hipGetErrorString(e));
  }
  if (rc == MIANN_OK) rc = build_dense_ghosts(ix, st);
  if (rc != MIANN_OK) {
    hipStreamSynchronize(st);  // queued copies and kernels may still use the index's buffers
    delete ix;
    return rc;
  }
  *out = ix;
  return MIANN_OK;
}

void miann_search_params_default(miann_search_params* sp) {
  if (!sp) return;
  std::memset(sp, 0, sizeof *sp);
  sp->search_width = 1;
  sp->n_init = 0;
  sp->entry = MIANN_ENTRY_RANDOM;
  sp->ghost_itopk = 32;
  sp->ghost_iters = 8;
  sp->t_seeds = 0;
  sp->dgs = 0;
  sp->discard_permille = 500;
  sp->cooldown_permille = 300;
  sp->random_discard = 0;
  sp->ppe = 1;
  sp->forward_f = 1;
  sp->rerank_mult = 4;
  sp->stop_on_no_change = 0;
  sp->hash_log2 = 0;
  sp->n_seeds = 0;
  sp->seed = 6;
}

}  // extern "C"

// The search of miann_search. With `ext` (device memory of ext_bytes, 256-byte aligned) every temporary
// buffer is carved from it and nothing is allocated; the call fails with EINVAL if it does not fit.
miann_status miann_search_impl(const miann_index* ix, const void* queries, int64_t nq, int32_t k, int32_t itopk,
                               int32_t max_iters, const miann_search_params* spp, uint32_t* ids, void* dists,
                               int64_t* counters, void* stream, void* ext, size_t ext_bytes) {
  if (!ix) return fail(MIANN_EINVAL, "miann_search: null index");
  miann_search_params sp;
  if (spp) sp = *spp; else miann_search_params_default(&sp);
  if (nq < 0) return fail(MIANN_EINVAL, "miann_search: nq = %lld < 0", (long long)nq);
  if (k < 1 || itopk < k || itopk > kMaxL)
    return fail(MIANN_EINVAL, "miann_search: need 1 <= k (%d) <= itopk (%d) <= %d", k, itopk, kMaxL);
  if (max_iters < 0) return fail(MIANN_EINVAL, "miann_search: max_iters = %d < 0", max_iters);
  const int degp = pow2_ceil(ix->deg);
  const int r = sp.search_width;
  if (r < 1 || r > kMaxR || r * degp > 64)
    return fail(MIANN_EINVAL, "miann_search: search_width %d invalid (r * pow2(degree) must be <= 64)", r);
  const int n_init = sp.n_init ? sp.n_init : ix->deg;
  if (n_init < 1 || n_init > 4096) return fail(MIANN_EINVAL, "miann_search: n_init = %d out of [1, 4096]", n_init);
  if (sp.entry < 0 || sp.entry > 4) return fail(MIANN_EINVAL, "miann_search: entry %d invalid", sp.entry);
  const bool ghost = sp.entry == MIANN_ENTRY_GHOST_GRAPH || sp.entry == MIANN_ENTRY_GHOST_DENSE ||
                     sp.entry == MIANN_ENTRY_PREDICTED;
  const bool ghost_graph = sp.entry == MIANN_ENTRY_GHOST_GRAPH || sp.entry == MIANN_ENTRY_PREDICTED;
  const int l_g = sp.ghost_itopk;
  const int t_seeds = sp.t_seeds ? sp.t_seeds : std::min(l_g, itopk);
  int degp_g = 0;
  if (ghost) {
    for (int s = 0; s < ix->S; s++)
      if (ix->sh[s].R == 0) return fail(MIANN_ESTATE, "miann_search: ghost entry needs miann_build_ghost first");
    if (sp.entry == MIANN_ENTRY_GHOST_DENSE && ix->dg.cols == 0)
      return fail(MIANN_ESTATE, "miann_search: dense ghost arrays missing (rebuild the ghost shards)");
    degp_g = pow2_ceil(ix->deg_g);
    if (l_g < 1 || l_g > kMaxL) return fail(MIANN_EINVAL, "miann_search: ghost_itopk %d out of [1, %d]", l_g, kMaxL);
    if (sp.ghost_iters < 0) return fail(MIANN_EINVAL, "miann_search: ghost_iters < 0");
    if (t_seeds < 1 || t_seeds > 64 || (ghost_graph && t_seeds > l_g))
      return fail(MIANN_EINVAL, "miann_search: t_seeds %d out of range", t_seeds);
    if (ghost_graph && r * degp_g > 64)
      return fail(MIANN_EINVAL, "miann_search: search_width too large for the ghost degree");
  }
  if ((sp.entry == MIANN_ENTRY_SEEDS || sp.entry == MIANN_ENTRY_PREDICTED) &&
      (!sp.seeds || sp.n_seeds < 1 || sp.n_seeds > 4096))
    return fail(MIANN_EINVAL, "miann_search: seed entry needs seeds and 1 <= n_seeds <= 4096");
  if (sp.dgs && !ix->dgs) return fail(MIANN_ESTATE, "miann_search: the index has no direction table");
  if (sp.discard_permille < 0 || sp.discard_permille > 1000 || sp.cooldown_permille < 0 || sp.cooldown_permille > 1000)
    return fail(MIANN_EINVAL, "miann_search: discard/cooldown permille out of [0, 1000]");
  if (sp.stage_waves != 0 && (sp.stage_waves < 4 || sp.stage_waves > 6))
    return fail(MIANN_EINVAL, "miann_search: stage_waves = %d (0, 4, 5 or 6)", sp.stage_waves);
  if (sp.dgs_threshold_permille < 0 || sp.dgs_threshold_permille > 1000 ||
      (sp.dgs_threshold_permille > 0 && sp.random_discard))
    return fail(MIANN_EINVAL, "miann_search: dgs_threshold_permille out of [0, 1000] or combined with random_discard");
  const int f = sp.forward_f;
  if (ix->S > 1 && sp.ppe && (f < 1 || f > 16 || f > itopk))
    return fail(MIANN_EINVAL, "miann_search: forward_f %d out of [1, min(16, itopk)]", f);
  const bool lp = lowp(ix->store_dtype);
  if (lp && sp.rerank_mult < 1) return fail(MIANN_EINVAL, "miann_search: rerank_mult must be >= 1");
  const int lp_max = std::max(itopk, ghost ? l_g : 1);
  int hlog = sp.hash_log2;
  if (hlog == 0) {
    hlog = 10;
    while ((1 << hlog) < 4 * (lp_max + 64) && hlog < 13) hlog++;
  }
  if (hlog < 8 || hlog > 13 || (1 << hlog) < 2 * (lp_max + 64))
    return fail(MIANN_EINVAL, "miann_search: hash_log2 %d too small for itopk %d (need 2^h >= 2 (itopk + 64))", hlog,
                lp_max);
  if (nq == 0) return MIANN_OK;
  if (!queries || !ids || !dists) return fail(MIANN_EINVAL, "miann_search: null queries or outputs");
  if (nq > (int64_t)1 << 31) return fail(MIANN_EINVAL, "miann_search: nq too large");

  hipStream_t st = (hipStream_t)stream;
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.sh = ix->dev_shards;
  a.seed = sp.seed;
  a.queries = queries;
  a.nq = nq;
  a.d = ix->d;
  a.d_pad = ix->d_pad;
  a.d_pad_f32 = ix->d_pad_f32;
  a.W = ix->W;
  a.deg = ix->deg;
  a.degp = degp;
  a.deg_g = ix->deg_g;
  a.degp_g = degp_g ? degp_g : 1;
  a.k = k;
  a.l = itopk;
  a.r = r;
  a.T = max_iters;
  a.n_init = n_init;
  a.l_g = l_g;
  a.T_g = sp.ghost_iters;
  a.t_seeds = t_seeds;
  a.entry = sp.entry;
  a.dgs = sp.dgs;
  a.n_keep = ix->deg - (sp.discard_permille * ix->deg) / 1000;
  a.stage_waves = sp.stage_waves;
  a.dgs_thr = sp.dgs_threshold_permille > 0 ? (int)(((int64_t)sp.dgs_threshold_permille * ix->d) / 1000) : -1;
  a.cooldown_pm = sp.cooldown_permille;
  a.random_discard = sp.random_discard;
  a.stop_on_no_change = sp.stop_on_no_change;
  a.ghost_every = sp.ghost_every_stage;
  a.S = ix->S;
  a.ppe = sp.ppe;
  a.f = f;
  a.rerank_m = sp.rerank_mult;
  a.lowp = lp;
  a.hash_log2 = hlog;
  a.lp_pow2 = std::max(64, pow2_ceil(lp_max));
  // queries (waves) per workgroup: 1, or MIANN_WAVES_PER_BLOCK (1..4) read once when the library first searches
  static const int wpb_env = [] {
    const char* w = getenv("MIANN_WAVES_PER_BLOCK");
    return w ? std::max(1, std::min(4, atoi(w))) : 1;
  }();
  a.waves_per_block = wpb_env;
  a.per_wave_lds = stage_lds_bytes(a);
  if ((int64_t)a.per_wave_lds * a.waves_per_block > 160 * 1024)
    return fail(MIANN_EUNSUPPORTED, "miann_search: %d bytes of LDS per query exceed the CU", a.per_wave_lds);
  a.qkeys = sp.qkeys;
  a.seeds = sp.seeds;
  a.n_seeds = sp.n_seeds;
  a.Tq = sp.max_iters_per_query;
  a.ctr = counters;
  const int cpl = ix->d_pad * esize_of(ix->store_dtype) / 128;

  // stream-ordered scratch for multi-stage searches and the dense entry
  void* scratch = nullptr;
  size_t off_hand = 0, off_stage = 0, off_dense = 0, total = 0;
  if (ix->S > 1) {
    off_hand = total;
    total += (size_t)2 * nq * f * 4;
    total = (total + 255) & ~(size_t)255;
    off_stage = total;
    total += (size_t)nq * ix->S * k * 8;
    total = (total + 255) & ~(size_t)255;
  }
  if (sp.entry == MIANN_ENTRY_GHOST_DENSE) {
    off_dense = total;
    total += (size_t)nq * ix->S * t_seeds * 8;
  }
  total = (total + 255) & ~(size_t)255;
  // a caller's buffer: the search's part first, the dense entry's after it
  const int start_only = ix->S > 1 && sp.ppe && !sp.ghost_every_stage;
  if (ext) {
    if (sp.phase_ms) return fail(MIANN_EINVAL, "miann_search: phase_ms creates events; use phase_events");
    size_t need = total;
    if (sp.entry == MIANN_ENTRY_GHOST_DENSE)
      need += dense_entry_min_scratch(ix->store_dtype, nq, ix->d_pad, ix->d_pad_f32, ix->S, start_only, ix->dg);
    if (need > ext_bytes)
      return fail(MIANN_EINVAL, "miann_search: %lld queries need %zu bytes of scratch, more than the %zu available",
                  (long long)nq, need, ext_bytes);
  }
  ScratchLease lease;
  if (ext) lease.p = ext;
  else if (total) HIP_TRY(scratch_lease(kSlotSearch, total, st, &lease));
  struct LeaseGuard {
    const ScratchLease& l;
    hipStream_t st;
    bool own;
    ~LeaseGuard() { if (own) scratch_release(kSlotSearch, l, st); }
  } lease_guard{lease, st, ext == nullptr};
  scratch = lease.p;
  char* sb = (char*)scratch;
  miann_status rc = MIANN_OK;
  // optional timing: events around [dense, stage 0..S-1, merge]
  const int nph = 2 + ix->S;
  std::vector<hipEvent_t> ev;
  if (sp.phase_ms) {
    ev.resize(2 * nph);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    for (int i = 0; i < nph; i++) sp.phase_ms[i] = 0.f;
  }
  auto mark = [&](int phase, int end) {
    if (!ev.empty()) hipEventRecord(ev[2 * phase + end], st);
  };
  // the caller's events: recorded in stream order, never waited on here
  auto mark_caller = [&](int i) {
    if (!sp.phase_events || !sp.phase_events[i]) return;
    const hipError_t e = hipEventRecord((hipEvent_t)sp.phase_events[i], st);
    if (e != hipSuccess && rc == MIANN_OK)
      rc = fail(MIANN_EINVAL, "miann_search: phase_events[%d]: %s", i, hipGetErrorString(e));
  };
  mark_caller(0);
  if (rc == MIANN_OK && sp.entry == MIANN_ENTRY_GHOST_DENSE) {
    a.dense = (const uint64_t*)(sb + off_dense);
    mark(0, 0);
    // dense seeds are needed for the start shard only, unless every stage takes a ghost entry
    hipError_t e = dense_entry_split(ix->store_dtype, queries, nq, ix->d, ix->d_pad, ix->d_pad_f32, sp.qkeys, ix->S,
                                     start_only, ix->dg, t_seeds, (uint64_t*)(sb + off_dense), st,
                                     ext ? sb + total : nullptr, ext ? ext_bytes - total : 0);
    if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_search: dense entry: %s", hipGetErrorString(e));
    mark(0, 1);
  }
  for (int t = 0; t < ix->S && rc == MIANN_OK; t++) {
    a.stage = t;
    if (ix->S > 1) {
      a.hand_in = (const uint32_t*)(sb + off_hand) + (size_t)(t & 1) * nq * f;
      a.hand_out = (uint32_t*)(sb + off_hand) + (size_t)((t + 1) & 1) * nq * f;
      a.stage_out = (uint64_t*)(sb + off_stage);
    } else {
      a.out_ids = ids;
      a.out_d = dists;
    }
    if (t == 0) mark_caller(1);
    mark(1 + t, 0);
    hipError_t e = launch_stage(ix->store_dtype, cpl, a, st);
    mark(1 + t, 1);
    if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_search: stage %d launch: %s", t, hipGetErrorString(e));
  }
  if (rc == MIANN_OK) mark_caller(2);
  if (rc == MIANN_OK && ix->S > 1) {
    mark(nph - 1, 0);
    hipError_t e = launch_merge((const uint64_t*)(sb + off_stage), nq, ix->S, k, ix->store_dtype == MIANN_U8, ids, dists, st);
    mark(nph - 1, 1);
    if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_search: merge launch: %s", hipGetErrorString(e));
  }
  if (rc == MIANN_OK) mark_caller(3);
  if (!ev.empty()) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess && rc == MIANN_OK) rc = fail(MIANN_EDEVICE, "miann_search: %s", hipGetErrorString(e));
    const bool used[3] = {sp.entry == MIANN_ENTRY_GHOST_DENSE, true, ix->S > 1};
    for (int i = 0; i < nph; i++) {
      const bool u = i == 0 ? used[0] : (i == nph - 1 ? used[2] : true);
      float ms = 0.f;
      if (u && hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) sp.phase_ms[i] = ms;
    }
    for (auto& e2 : ev) hipEventDestroy(e2);
  }
  return rc;
}

// Device bytes of a search's temporary buffers (hand-off, per-stage results, dense seeds, and the dense entry's
// query split and work area), as the stream-kept blocks hold them (each rounded up to a power of two): what a
// batch of nq queries with these parameters keeps on its stream. Used by the server's admission control.
size_t miann_search_scratch_bytes(const miann_index* ix, int64_t nq, int32_t k, int32_t itopk,
                                  const miann_search_params* spp) {
  if (!ix || nq <= 0) return 0;
  miann_search_params sp;
  if (spp) sp = *spp; else miann_search_params_default(&sp);
  auto p2 = [](size_t b) {
    size_t c = 65536;
    while (c < b) c <<= 1;
    return b ? c : 0;
  };
  const int t = sp.t_seeds ? sp.t_seeds : std::min(sp.ghost_itopk, itopk);
  size_t search = 0;
  if (ix->S > 1) search += (size_t)2 * nq * std::max(1, sp.forward_f) * 4 + (size_t)nq * ix->S * k * 8 + 512;
  size_t dense = 0;
  if (sp.entry == MIANN_ENTRY_GHOST_DENSE && ix->dg.cols) {
    search += (size_t)nq * ix->S * t * 8;
    const int start_only = ix->S > 1 && sp.ppe && !sp.ghost_every_stage;
    const size_t qpart = (size_t)nq * ((size_t)ix->d_pad_f32 * 4 + (size_t)ix->d_pad * 4 + 8) + 2048;
    const size_t one = dense_entry_min_scratch(ix->store_dtype, 1, ix->d_pad, ix->d_pad_f32, ix->S, start_only, ix->dg);
    // the work area: every row of the batch, up to the 512 MB chunk limit
    const size_t work = std::min((size_t)nq * one, (size_t)1 << 29);
    dense = p2(qpart) + p2(work);
  }
  return p2(search) + dense;
}

extern "C" {

miann_status miann_gather_probe(const void* table, int64_t n_rows, int32_t row_bytes, const uint32_t* ids, int64_t n,
                                uint32_t* out, void* stream) {
  if (n < 0 || n_rows < 1 || n_rows > (1ll << 32)) return fail(MIANN_EINVAL, "miann_gather_probe: sizes out of range");
  if (row_bytes % 128 || row_bytes < 128 || row_bytes > 1024 || row_bytes == 640 || row_bytes == 896)
    return fail(MIANN_EINVAL, "miann_gather_probe: row_bytes %d not in {128, 256, 384, 512, 768, 1024}", row_bytes);
  if (n > 0 && (!table || !ids || !out)) return fail(MIANN_EINVAL, "miann_gather_probe: null pointer");
  const hipError_t e = launch_gather_probe(table, n_rows, row_bytes, ids, n, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(MIANN_EDEVICE, "miann_gather_probe: %s", hipGetErrorString(e));
  return MIANN_OK;
}

miann_status miann_release_scratch(void* stream) {
  const hipError_t e = scratch_drop_stream((hipStream_t)stream);
  if (e != hipSuccess) return fail(MIANN_EDEVICE, "miann_release_scratch: %s", hipGetErrorString(e));
  return MIANN_OK;
}

miann_status miann_search(const miann_index* ix, const void* queries, int64_t nq, int32_t k, int32_t itopk,
                          int32_t max_iters, const miann_search_params* spp, uint32_t* ids, void* dists,
                          int64_t* counters, void* stream) {
  return miann_search_impl(ix, queries, nq, k, itopk, max_iters, spp, ids, dists, counters, stream, nullptr, 0);
}

}  // extern "C"

namespace {

// RAII list of stream-ordered temporaries.
struct Temps {
  hipStream_t st;
  std::vector<void*> v;
  explicit Temps(hipStream_t s) : st(s) {}
  template <typename T>
  hipError_t get(T** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = pool_malloc_async(&q, bytes ? bytes : 16, st);
    if (e == hipSuccess) { v.push_back(q); *p = (T*)q; }
    return e;
  }
  ~Temps() { for (void* p : v) hipFreeAsync(p, st); }
};

// f32 rows for the MFMA selection: the originals themselves for float input,
// a converted copy for u8 (row length d_pad_in in both cases).
miann_status gemm_rows(miann_index* ix, const Shard& h, Temps& tmp, const float** out) {
  if (ix->in_dtype == MIANN_F32) { *out = (const float*)h.orig; return MIANN_OK; }
  float* f = nullptr;
  HIP_TRY(tmp.get(&f, (size_t)h.n * ix->d_pad_in * 4));
  HIP_TRY(queries_to_f32(h.orig, MIANN_U8, h.n, ix->d_pad_in, ix->d_pad_in, f, tmp.st));
  *out = f;
  return MIANN_OK;
}

miann_status build_ghosts(miann_index* ix, const std::vector<int64_t>& R, int deg_g, uint64_t seed, hipStream_t st);

// Exact K0-NN of `n` rows (f32 copy `xf`, raw `xr`) among themselves, pruned to `deg`.
miann_status knn_graph(miann_index* ix, const float* xf, const void* xr, int64_t n, int deg, int K0, uint32_t* graph,
                       hipStream_t st) {
  Temps tmp(st);
  uint64_t* keys = nullptr;
  HIP_TRY(tmp.get(&keys, (size_t)n * K0 * 8));
  HIP_TRY(knn_exact(xf, n, xf, n, ix->d_pad_in, ix->d, ix->in_dtype, xr, ix->d_pad_in, xr, nullptr, ix->d_pad_in, K0, 1,
                    nullptr, keys, st));
  HIP_TRY(prune_graph(keys, n, K0, deg, graph, st));
  return MIANN_OK;
}

}  // namespace

extern "C" {

miann_status miann_build_graph(const void* base, int64_t n, int32_t d, int32_t in_dtype, const miann_build_params* bp,
                               void* stream, miann_index** out) {
  if (!base || !bp || !out) return fail(MIANN_EINVAL, "miann_build_graph: null argument");
  miann_status rc = check_common_dims(d, in_dtype, bp->store_dtype, bp->degree);
  if (rc) return rc;
  const int S = bp->num_shards;
  if (S < 1 || S > kMaxShards) return fail(MIANN_EINVAL, "miann_build_graph: num_shards %d out of [1, %d]", S, kMaxShards);
  if (n < (int64_t)S * (bp->degree + 1) || n >= (1ll << 30))
    return fail(MIANN_EINVAL, "miann_build_graph: n = %lld must be in [S * (degree + 1), 2^30)", (long long)n);
  const int K0 = bp->knn_k0 ? bp->knn_k0 : 2 * bp->degree;
  if (K0 < bp->degree || K0 > 240) return fail(MIANN_EINVAL, "miann_build_graph: knn_k0 %d out of [degree, 240]", K0);
  if ((int64_t)K0 >= n / S) return fail(MIANN_EINVAL, "miann_build_graph: knn_k0 %d too large for shards of %lld", K0, (long long)(n / S));
  hipStream_t st = (hipStream_t)stream;
  miann_index* ix = new miann_index();
  init_dims(ix, d, in_dtype, bp->store_dtype, bp->degree, 0, bp->dgs_table);
  ix->S = S;
  ix->knn_k0 = K0;
  ix->n_total = n;
  ix->sh.resize(S);
  {
    Temps tmp(st);
    uint32_t* perm = nullptr;
    if (S > 1) {
      hipError_t e = tmp.get(&perm, (size_t)n * 4);
      if (e == hipSuccess) e = keyed_order(bp->seed, n, perm, st);
      if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_build_graph: partition: %s", hipGetErrorString(e));
    }
    std::vector<const float*> xf(S, nullptr);
    for (int s = 0; s < S && rc == MIANN_OK; s++) {
      Shard& h = ix->sh[s];
      const int64_t lo = s * n / S, hi = (s + 1) * n / S;
      h.n = hi - lo;
      hipError_t e = ix->alloc(&h.gmap, (size_t)h.n * 4);
      if (e == hipSuccess)
        e = perm ? hipMemcpyAsync(h.gmap, perm + lo, (size_t)h.n * 4, hipMemcpyDeviceToDevice, st) : iota_u32(h.gmap, h.n, 0, st);
      if (e != hipSuccess) { rc = fail(MIANN_EDEVICE, "miann_build_graph: %s", hipGetErrorString(e)); break; }
      if ((rc = fill_vectors(ix, h, base, perm ? h.gmap : nullptr, st))) break;
      if ((rc = gemm_rows(ix, h, tmp, &xf[s]))) break;
      e = ix->alloc(&h.graph, (size_t)h.n * ix->deg * 4);
      if (e != hipSuccess) { rc = fail(MIANN_ENOMEM, "miann_build_graph: graph: %s", hipGetErrorString(e)); break; }
      hipStreamSynchronize(st);
      auto t0 = std::chrono::steady_clock::now();
      if ((rc = knn_graph(ix, xf[s], h.orig, h.n, ix->deg, K0, h.graph, st))) break;
      hipStreamSynchronize(st);
      auto t1 = std::chrono::steady_clock::now();
      ix->build_s[0] += std::chrono::duration<double>(t1 - t0).count();
      if (ix->dgs) {
        e = ix->alloc(&h.sign, (size_t)h.n * ix->W * ix->deg * 4);
        if (e == hipSuccess) e = sign_table(h.orig, in_dtype, h.n, d, ix->d_pad_in, h.graph, ix->deg, h.sign, st);
        if (e != hipSuccess) { rc = fail(MIANN_EDEVICE, "miann_build_graph: sign table: %s", hipGetErrorString(e)); break; }
        hipStreamSynchronize(st);
        ix->build_s[1] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
      }
    }
    // inter-shard map I_s(u) = argmin over shard (s+1) mod S (Sec. 3.1.2)
    hipStreamSynchronize(st);
    const auto t_map = std::chrono::steady_clock::now();
    for (int s = 0; S > 1 && s < S && rc == MIANN_OK; s++) {
      Shard& h = ix->sh[s];
      const Shard& nx = ix->sh[(s + 1) % S];
      uint64_t* keys = nullptr;
      hipError_t e = tmp.get(&keys, (size_t)h.n * 8);
      if (e == hipSuccess) e = ix->alloc(&h.next, (size_t)h.n * 4);
      if (e == hipSuccess)
        e = knn_exact(xf[s], h.n, xf[(s + 1) % S], nx.n, ix->d_pad_in, d, in_dtype, h.orig, ix->d_pad_in, nx.orig,
                      nullptr, ix->d_pad_in, 1, 0, nullptr, keys, st);
      if (e == hipSuccess) e = keys_to_ids(keys, h.n, 1, 0, h.next, 1, st);
      if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_build_graph: inter-shard map: %s", hipGetErrorString(e));
    }
    if (rc == MIANN_OK) {
      hipError_t e = hipStreamSynchronize(st);
      ix->build_s[2] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_map).count();
      if (e == hipSuccess) e = ix->refresh(st);
      if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_build_graph: %s", hipGetErrorString(e));
    }
  }
  if (rc != MIANN_OK) {
    hipStreamSynchronize(st);
    delete ix;
    return rc;
  }
  *out = ix;
  return MIANN_OK;
}

miann_status miann_build_ghost(miann_index* ix, double ratio, int64_t num_ghost, int32_t deg_g, uint64_t seed,
                               void* stream) {
  if (!ix) return fail(MIANN_EINVAL, "miann_build_ghost: null index");
  if (deg_g < 2 || deg_g > 64) return fail(MIANN_EINVAL, "miann_build_ghost: ghost_degree %d out of [2, 64]", deg_g);
  if (num_ghost < 0 || (num_ghost == 0 && !(ratio > 0.0 && ratio <= 1.0)))
    return fail(MIANN_EINVAL, "miann_build_ghost: need num_ghost > 0 or 0 < ratio <= 1");
  std::vector<int64_t> R(ix->S);
  for (int s = 0; s < ix->S; s++) {
    const int64_t n_s = ix->sh[s].n;
    R[s] = num_ghost ? num_ghost : (int64_t)std::floor(ratio * (double)n_s + 0.5);
    if (R[s] < 2 * deg_g + 1 || R[s] > n_s)
      return fail(MIANN_EINVAL, "miann_build_ghost: shard %d: %lld ghosts invalid (need 2 * ghost_degree < R <= n)", s,
                    (long long)R[s]);
  }
  return build_ghosts(ix, R, deg_g, seed, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// The ghost shards of every shard with R[s] ghosts (Sec. 3.2.2): a SplitMix64-keyed sample without replacement,
// its own exact-k-NN graph and the ghost store, then the dense entry's arrays.
miann_status build_ghosts(miann_index* ix, const std::vector<int64_t>& R, int deg_g, uint64_t seed, hipStream_t st) {
  hipStreamSynchronize(st);
  const auto t_ghost = std::chrono::steady_clock::now();
  ix->free_ghost();
  ix->deg_g = deg_g;
  ix->ghost_seed = seed;
  miann_status rc = MIANN_OK;
  for (int s = 0; s < ix->S && rc == MIANN_OK; s++) {
    Shard& h = ix->sh[s];
    Temps tmp(st);
    uint32_t* order = nullptr;
    hipError_t e = tmp.get(&order, (size_t)h.n * 4);
    if (e == hipSuccess) e = keyed_order(sm_at(seed, (uint64_t)(0x100 + s)), h.n, order, st);
    if (e == hipSuccess) e = ix->alloc(&h.g_map, (size_t)R[s] * 4, true);
    if (e == hipSuccess) e = hipMemcpyAsync(h.g_map, order, (size_t)R[s] * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = sort_u32(h.g_map, R[s], st);
    if (e != hipSuccess) { rc = fail(MIANN_EDEVICE, "miann_build_ghost: sample: %s", hipGetErrorString(e)); break; }
    h.R = R[s];
    // ghost graph over the ghost nodes' originals
    const int ein = esize_of(ix->in_dtype);
    void* gr = nullptr;
    float* gf = nullptr;
    e = tmp.get(&gr, (size_t)h.R * ix->d_pad_in * ein);
    if (e == hipSuccess) e = gather_rows(h.orig, h.g_map, h.R, ix->d_pad_in * ein, gr, st);
    if (e == hipSuccess) {
      if (ix->in_dtype == MIANN_F32) gf = (float*)gr;
      else {
        e = tmp.get(&gf, (size_t)h.R * ix->d_pad_in * 4);
        if (e == hipSuccess) e = queries_to_f32(gr, MIANN_U8, h.R, ix->d_pad_in, ix->d_pad_in, gf, st);
      }
    }
    if (e == hipSuccess) e = ix->alloc(&h.g_graph, (size_t)h.R * deg_g * 4, true);
    if (e != hipSuccess) { rc = fail(MIANN_EDEVICE, "miann_build_ghost: %s", hipGetErrorString(e)); break; }
    if ((rc = knn_graph(ix, gf, gr, h.R, deg_g, 2 * deg_g, h.g_graph, st))) break;
    rc = build_ghost_store(ix, h, st);
    if (rc == MIANN_OK) {
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_build_ghost: %s", hipGetErrorString(e));
    }
  }
  if (rc == MIANN_OK) rc = build_dense_ghosts(ix, st);
  if (rc != MIANN_OK) {
    hipStreamSynchronize(st);
    ix->free_ghost();
  }
  ix->build_s[3] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_ghost).count();
  hipError_t e = ix->refresh(st);
  if (rc == MIANN_OK && e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_build_ghost: %s", hipGetErrorString(e));
  return rc;
}

}  // namespace

extern "C" {

miann_status miann_exact_knn(const miann_index* cix, const void* queries, int64_t nq, int32_t k, uint32_t* ids,
                             void* dists, void* stream) {
  miann_index* ix = const_cast<miann_index*>(cix);
  if (!ix) return fail(MIANN_EINVAL, "miann_exact_knn: null index");
  if (nq < 0 || k < 1 || k > 240) return fail(MIANN_EINVAL, "miann_exact_knn: need nq >= 0 and 1 <= k <= 240");
  // rows are re-sorted by (dist, global id) with one wave per row (k <= 256)
  for (int s = 0; s < ix->S; s++)
    if (ix->sh[s].n < k) return fail(MIANN_EINVAL, "miann_exact_knn: k = %d exceeds shard %d size", k, s);
  if (nq == 0) return MIANN_OK;
  if (!queries || !ids || !dists) return fail(MIANN_EINVAL, "miann_exact_knn: null pointer");
  hipStream_t st = (hipStream_t)stream;
  Temps tmp(st);
  const int dpi = ix->d_pad_in;
  float* qf = nullptr;
  void* qraw = nullptr;
  uint64_t* keys = nullptr;
  uint64_t* so = nullptr;
  HIP_TRY(tmp.get(&qf, (size_t)nq * dpi * 4));
  HIP_TRY(queries_to_f32(queries, ix->in_dtype, nq, ix->d, dpi, qf, st));
  if (ix->in_dtype == MIANN_F32) qraw = qf;
  else {
    HIP_TRY(tmp.get(&qraw, (size_t)nq * dpi));
    HIP_TRY(pad_rows(queries, nq, ix->d, 1, qraw, dpi, nullptr, st));
  }
  HIP_TRY(tmp.get(&keys, (size_t)nq * k * 8));
  if (ix->S > 1) HIP_TRY(tmp.get(&so, (size_t)nq * ix->S * k * 8));
  for (int s = 0; s < ix->S; s++) {
    const Shard& h = ix->sh[s];
    const float* xf = nullptr;
    miann_status rc = gemm_rows(ix, h, tmp, &xf);
    if (rc) return rc;
    HIP_TRY(knn_exact(qf, nq, xf, h.n, dpi, ix->d, ix->in_dtype, qraw, dpi, h.orig, nullptr, dpi, k, 0, nullptr, keys, st));
    // per-shard lists in global ids, ordered by (dist, global id)
    if (ix->S == 1) {
      HIP_TRY(keys_to_stage(keys, nq, k, h.gmap, 1, 0, keys, st));
      HIP_TRY(sort_rows(keys, nq, k, st));
      HIP_TRY(keys_to_output(keys, nq, k, nullptr, ix->in_dtype == MIANN_U8, ids, dists, st));
    } else {
      HIP_TRY(keys_to_stage(keys, nq, k, h.gmap, ix->S, s, so, st));
    }
  }
  if (ix->S > 1) {
    HIP_TRY(sort_rows(so, nq * ix->S, k, st));
    HIP_TRY(launch_merge(so, nq, ix->S, k, ix->in_dtype == MIANN_U8, ids, dists, st));
  }
  return MIANN_OK;
}

miann_status miann_nearest_ghost(const miann_index* ix, int32_t shard, const void* vectors, int64_t n,
                                 uint32_t* ghost_idx, void* stream) {
  if (!ix) return fail(MIANN_EINVAL, "miann_nearest_ghost: null index");
  if (shard < 0 || shard >= ix->S) return fail(MIANN_EINVAL, "miann_nearest_ghost: shard %d out of range", shard);
  const Shard& h = ix->sh[shard];
  if (h.R == 0) return fail(MIANN_ESTATE, "miann_nearest_ghost: no ghost shard (call miann_build_ghost)");
  if (n < 0) return fail(MIANN_EINVAL, "miann_nearest_ghost: n < 0");
  if (n == 0) return MIANN_OK;
  if (!vectors || !ghost_idx) return fail(MIANN_EINVAL, "miann_nearest_ghost: null pointer");
  hipStream_t st = (hipStream_t)stream;
  Temps tmp(st);
  uint64_t* keys = nullptr;
  HIP_TRY(tmp.get(&keys, (size_t)n * 8));
  HIP_TRY(dense_entry(ix->store_dtype, vectors, n, ix->d, nullptr, 1, 0, 0, h.g_f32, h.g_store, h.g_scale, nullptr,
                      h.R, ix->d_pad, ix->d_pad_f32, 1, keys, st));
  HIP_TRY(keys_to_ids(keys, n, 1, 0, ghost_idx, 1, st));
  return MIANN_OK;
}


miann_status miann_predictor_labels(const miann_index* cix, const float* queries, int64_t n, int32_t k, int32_t itopk,
                                    int32_t max_iters, const miann_search_params* sp, int32_t* entry, float* budget,
                                    int32_t* iters, void* stream) {
  miann_index* ix = const_cast<miann_index*>(cix);
  if (!ix) return fail(MIANN_EINVAL, "miann_predictor_labels: null index");
  if (ix->S != 1) return fail(MIANN_EINVAL, "miann_predictor_labels: the learned entry is defined for one shard");
  if (ix->in_dtype != MIANN_F32) return fail(MIANN_EUNSUPPORTED, "miann_predictor_labels: float queries only");
  if (ix->sh[0].R == 0) return fail(MIANN_ESTATE, "miann_predictor_labels: no ghost shard");
  if (n < 0) return fail(MIANN_EINVAL, "miann_predictor_labels: n < 0");
  if (n == 0) return MIANN_OK;
  if (!queries || !entry || !budget || !iters) return fail(MIANN_EINVAL, "miann_predictor_labels: null pointer");
  hipStream_t st = (hipStream_t)stream;
  const Shard& h = ix->sh[0];
  Temps tmp(st);
  // budget: the search's trace (counter 7, the last iteration in which its top-k changed)
  int64_t* ctr = nullptr;
  uint32_t* ids = nullptr;
  float* ds = nullptr;
  HIP_TRY(tmp.get(&ctr, (size_t)n * kNumCtr * 8));
  HIP_TRY(tmp.get(&ids, (size_t)n * k * 4));
  HIP_TRY(tmp.get(&ds, (size_t)n * k * 4));
  miann_status rc = miann_search(ix, queries, n, k, itopk, max_iters, sp, ids, ds, ctr, stream);
  if (rc) return rc;
  HIP_TRY(budget_labels(ctr, n, iters, budget, st));
  // entry: the ghost nearest to the query's exact nearest node (local ids of the one shard)
  const int dpi = ix->d_pad_in;
  float* qf = nullptr;
  uint64_t* keys = nullptr;
  uint32_t* nn = nullptr;
  float* rows = nullptr;
  float* vec = nullptr;
  HIP_TRY(tmp.get(&qf, (size_t)n * dpi * 4));
  HIP_TRY(queries_to_f32(queries, MIANN_F32, n, ix->d, dpi, qf, st));
  HIP_TRY(tmp.get(&keys, (size_t)n * 8));
  HIP_TRY(knn_exact(qf, n, (const float*)h.orig, h.n, dpi, ix->d, ix->in_dtype, qf, dpi, h.orig, nullptr, dpi, 1, 0,
                    nullptr, keys, st));
  HIP_TRY(tmp.get(&nn, (size_t)n * 4));
  HIP_TRY(keys_to_ids(keys, n, 1, 0, nn, 1, st));
  HIP_TRY(tmp.get(&rows, (size_t)n * dpi * 4));
  HIP_TRY(gather_rows(h.orig, nn, n, dpi * 4, rows, st));
  HIP_TRY(tmp.get(&vec, (size_t)n * ix->d * 4));
  HIP_TRY(unpad_rows(rows, n, dpi, 4, vec, ix->d, st));
  return miann_nearest_ghost(ix, 0, vec, n, (uint32_t*)entry, stream);
}

miann_status miann_index_delete(miann_index* ix, const uint32_t* global_ids, int64_t m, void* stream) {
  if (!ix) return fail(MIANN_EINVAL, "miann_index_delete: null index");
  if (m < 0 || (m > 0 && !global_ids)) return fail(MIANN_EINVAL, "miann_index_delete: need m >= 0 and ids");
  if (m == 0) return MIANN_OK;
  hipStream_t st = (hipStream_t)stream;
  Temps tmp(st);
  uint32_t* ids = nullptr;
  HIP_TRY(tmp.get(&ids, (size_t)m * 4));
  HIP_TRY(hipMemcpyAsync(ids, global_ids, (size_t)m * 4, hipMemcpyDeviceToDevice, st));
  HIP_TRY(sort_u32(ids, m, st));
  bool fresh = false;
  for (int s = 0; s < ix->S; s++) {
    Shard& h = ix->sh[s];
    if (!h.dead) {
      HIP_TRY(ix->alloc(&h.dead, (size_t)h.n));
      HIP_TRY(fill_u8(h.dead, h.n, 0, st));
      fresh = true;
    }
    HIP_TRY(mark_dead(h.gmap, h.n, ids, m, h.dead, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (fresh) HIP_TRY(ix->refresh(st));
  return MIANN_OK;
}

miann_status miann_index_append(miann_index* ix, int32_t shard, const void* vectors, int64_t n_new, uint64_t ghost_seed,
                                void* stream) {
  if (!ix) return fail(MIANN_EINVAL, "miann_index_append: null index");
  if (shard < 0 || shard >= ix->S) return fail(MIANN_EINVAL, "miann_index_append: shard %d out of range", shard);
  if (n_new < 0 || (n_new > 0 && !vectors)) return fail(MIANN_EINVAL, "miann_index_append: need n >= 0 and rows");
  if (n_new == 0) return MIANN_OK;
  if (ix->n_total + n_new >= (1ll << 30))
    return fail(MIANN_EINVAL, "miann_index_append: %lld nodes would exceed 2^30 - 1", (long long)(ix->n_total + n_new));
  const int K0 = ix->knn_k0 ? ix->knn_k0 : 2 * ix->deg;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(st));
  Shard& h = ix->sh[shard];
  const int64_t n0 = h.n, n = n0 + n_new;
  if (K0 >= n) return fail(MIANN_EINVAL, "miann_index_append: shard too small for K0 = %d", K0);
  const int ein = esize_of(ix->in_dtype);
  const bool lp = lowp(ix->store_dtype);
  const size_t row_in = (size_t)ix->d_pad_in * ein, row_st = (size_t)ix->d_pad * esize_of(ix->store_dtype);
  Shard nh = h;  // the rebuilt shard; the old arrays are released once it is complete
  nh.n = n;
  hipError_t e = ix->alloc(&nh.orig, (size_t)n * row_in);
  if (e == hipSuccess) e = hipMemcpyAsync(nh.orig, h.orig, (size_t)n0 * row_in, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = pad_rows(vectors, n_new, ix->d, ein, (char*)nh.orig + n0 * row_in, ix->d_pad_in, nullptr, st);
  if (e == hipSuccess && lp) {
    // per-vector quantisation: the old rows' codes stay valid
    e = ix->alloc(&nh.store, (size_t)n * row_st);
    if (e == hipSuccess) e = ix->alloc(&nh.scale, (size_t)n * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(nh.store, h.store, (size_t)n0 * row_st, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(nh.scale, h.scale, (size_t)n0 * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = quantize((const float*)vectors, n_new, ix->d, ix->store_dtype, (char*)nh.store + n0 * row_st, ix->d_pad,
                   nh.scale + n0, nullptr, st);
  } else if (e == hipSuccess) {
    nh.store = nh.orig;
  }
  // the new rows take the next global ids
  if (e == hipSuccess) e = ix->alloc(&nh.gmap, (size_t)n * 4);
  if (e == hipSuccess) e = hipMemcpyAsync(nh.gmap, h.gmap, (size_t)n0 * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = iota_u32(nh.gmap + n0, n_new, (uint32_t)ix->n_total, st);
  if (e == hipSuccess && h.dead) {
    e = ix->alloc(&nh.dead, (size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(nh.dead, h.dead, (size_t)n0, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = fill_u8(nh.dead + n0, n_new, 0, st);
  }
  if (e == hipSuccess) e = ix->alloc(&nh.graph, (size_t)n * ix->deg * 4);
  if (e == hipSuccess && ix->dgs) e = ix->alloc(&nh.sign, (size_t)n * ix->W * ix->deg * 4);
  if (e != hipSuccess) return fail(MIANN_EDEVICE, "miann_index_append: %s", hipGetErrorString(e));
  miann_status rc = MIANN_OK;
  {
    Temps tmp(st);
    const float* xf = nullptr;
    // the shard's graph and direction table over all its rows (Sec. 6.2: an insertion rebuilds the affected shard)
    if ((rc = gemm_rows(ix, nh, tmp, &xf))) return rc;
    if ((rc = knn_graph(ix, xf, nh.orig, n, ix->deg, K0, nh.graph, st))) return rc;
    if (ix->dgs) HIP_TRY(sign_table(nh.orig, ix->in_dtype, n, ix->d, ix->d_pad_in, nh.graph, ix->deg, nh.sign, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  // swap in the rebuilt shard, then release the arrays it replaced
  Shard old = h;
  h = nh;
  ix->n_total += n_new;
  ix->release(old.orig);
  if (lp) { ix->release(old.store); ix->release(old.scale); }
  ix->release(old.gmap);
  ix->release(old.dead);
  ix->release(old.graph);
  ix->release(old.sign);
  // inter-shard maps into and out of the shard (Sec. 3.1.2), exact 1-NN as at build time
  if (ix->S > 1) {
    Temps tmp(st);
    std::vector<const float*> xf(ix->S, nullptr);
    for (int t : {(shard + ix->S - 1) % ix->S, shard, (shard + 1) % ix->S})
      if (!xf[t] && (rc = gemm_rows(ix, ix->sh[t], tmp, &xf[t]))) return rc;
    for (int s : {(shard + ix->S - 1) % ix->S, shard}) {
      Shard& a = ix->sh[s];
      const Shard& b = ix->sh[(s + 1) % ix->S];
      uint64_t* keys = nullptr;
      uint32_t* next = nullptr;
      HIP_TRY(tmp.get(&keys, (size_t)a.n * 8));
      HIP_TRY(ix->alloc(&next, (size_t)a.n * 4));
      HIP_TRY(knn_exact(xf[s], a.n, xf[(s + 1) % ix->S], b.n, ix->d_pad_in, ix->d, ix->in_dtype, a.orig, ix->d_pad_in,
                        b.orig, nullptr, ix->d_pad_in, 1, 0, nullptr, keys, st));
      HIP_TRY(keys_to_ids(keys, a.n, 1, 0, next, 1, st));
      HIP_TRY(hipStreamSynchronize(st));
      ix->release(a.next);
      a.next = next;
    }
  }
  // ghost shards: the same counts, sampled with ghost_seed (the seed of the earlier sample keeps the other
  // shards' samples unchanged)
  if (h.R > 0) {
    std::vector<int64_t> R(ix->S);
    for (int s = 0; s < ix->S; s++) R[s] = ix->sh[s].R;
    if (R[shard] > n) R[shard] = n;
    return build_ghosts(ix, R, ix->deg_g, ghost_seed, st);
  }
  hipError_t e2 = ix->refresh(st);
  if (e2 != hipSuccess) return fail(MIANN_EDEVICE, "miann_index_append: %s", hipGetErrorString(e2));
  return MIANN_OK;
}

miann_status miann_build_next_map(miann_index* ix, int32_t itopk, int32_t max_iters, const miann_search_params* spp,
                                  void* stream) {
  if (!ix) return fail(MIANN_EINVAL, "miann_build_next_map: null index");
  if (ix->S < 2) return fail(MIANN_EINVAL, "miann_build_next_map: needs S >= 2 shards");
  miann_search_params sp;
  if (spp) sp = *spp; else miann_search_params_default(&sp);
  if (sp.entry != MIANN_ENTRY_RANDOM && sp.entry != MIANN_ENTRY_GHOST_GRAPH)
    return fail(MIANN_EUNSUPPORTED, "miann_build_next_map: entry must be random or the ghost graph");
  if (sp.qkeys || sp.seeds || sp.max_iters_per_query || sp.phase_ms || sp.phase_events)
    return fail(MIANN_EINVAL, "miann_build_next_map: qkeys, seeds, per-query budgets and timing must be NULL");
  sp.ppe = 0;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(st));
  const int ein = esize_of(ix->in_dtype);
  std::vector<uint32_t*> nexts(ix->S, nullptr);
  miann_status rc = MIANN_OK;
  for (int s = 0; s < ix->S && rc == MIANN_OK; s++) {
    const Shard& h = ix->sh[s];
    // shard (s+1) mod S alone, results in its local ids, no deletion flags
    miann_index v;
    v.S = 1;
    v.d = ix->d; v.deg = ix->deg; v.deg_g = ix->deg_g; v.W = ix->W;
    v.store_dtype = ix->store_dtype; v.in_dtype = ix->in_dtype; v.dgs = ix->dgs;
    v.d_pad = ix->d_pad; v.d_pad_in = ix->d_pad_in; v.d_pad_f32 = ix->d_pad_f32;
    Shard nx = ix->sh[(s + 1) % ix->S];
    nx.gmap = nullptr;
    nx.next = nullptr;
    nx.dead = nullptr;
    v.n_total = nx.n;
    v.sh.push_back(nx);
    hipError_t e = v.refresh(st);
    Temps tmp(st);
    void* q = nullptr;
    void* dist = nullptr;
    if (e == hipSuccess) e = tmp.get(&q, (size_t)h.n * ix->d * ein);
    if (e == hipSuccess) e = tmp.get(&dist, (size_t)h.n * 4);
    if (e == hipSuccess) e = unpad_rows(h.orig, h.n, ix->d_pad_in, ein, q, ix->d, st);
    if (e == hipSuccess) e = ix->alloc(&nexts[s], (size_t)h.n * 4);
    if (e != hipSuccess) { rc = fail(MIANN_EDEVICE, "miann_build_next_map: %s", hipGetErrorString(e)); break; }
    // every node of shard s is a query keyed by its local id; the top-1 is its entry in the table
    rc = miann_search_impl(&v, q, h.n, 1, itopk, max_iters, &sp, nexts[s], dist, nullptr, st, nullptr, 0);
    if (rc == MIANN_OK) {
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) rc = fail(MIANN_EDEVICE, "miann_build_next_map: %s", hipGetErrorString(e));
    }
    v.sh.clear();  // the view borrows the shard's arrays
  }
  if (rc != MIANN_OK) {
    hipStreamSynchronize(st);
    for (uint32_t* p : nexts) ix->release(p);
    return rc;
  }
  for (int s = 0; s < ix->S; s++) {
    ix->release(ix->sh[s].next);
    ix->sh[s].next = nexts[s];
  }
  HIP_TRY(ix->refresh(st));
  return MIANN_OK;
}

}  // extern "C"
