// Host-callable launchers of the MFMA distance-tile kernels (knn.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace miann {

// f32(scale * decode(code)) rows of a store, padded to d_pad_f32.
hipError_t dequant_rows(const void* store, const float* scale, int store_dt, int64_t n, int d_pad, int d_pad_f32,
                        float* out, hipStream_t st);

// Queries-by-ghosts entry (Sec. 3.2.2, dense form): for every query whose start
// shard is `shard` (every query when !ppe), the exact top-t ghosts of that
// shard by (dist, id). Writes keys (dist bits << 32 | local id) to
// out[(q * S + shard) * t + i].
hipError_t dense_entry(int store_dt, const void* queries, int64_t nq, int d, const uint64_t* qkeys, int S, int shard,
                       int ppe, const float* g_f32, const void* g_store, const float* g_scale, const uint32_t* g_map,
                       int64_t R, int d_pad, int d_pad_f32, int t, uint64_t* out, hipStream_t st);

// Ghosts of all shards concatenated for the split-bf16 dense entry. Shard s
// owns columns [off[s], off[s+1]) (a multiple of 64 wide; its R[s] real
// ghosts first, then padding with norm +inf).
struct DenseShardDev {
  const void* g_store;  // [R][d_pad] ghost codes in the store type
  const float* g_scale; // [R] or null
  const uint32_t* g_map;// [R] ghost -> local node id
};
struct DenseGhosts {
  int64_t cols = 0;
  int dk = 0;                   // row length (elements), a multiple of 32
  uint16_t* hi = nullptr;       // [cols][dk] bf16
  uint16_t* lo = nullptr;       // [cols][dk] bf16, x - hi
  float* norm = nullptr;        // [cols]
  float* gmax_dev = nullptr;    // [S] largest ghost norm of each shard (the dense entry's error bound)
  int64_t* off_dev = nullptr;   // [S + 1]
  int64_t* R_dev = nullptr;     // [S]
  DenseShardDev* shards_dev = nullptr;  // [S]
  std::vector<int64_t> off, R;  // host copies
};
// hi / lo bf16 split and f32 norms of n rows ([n][dk] f32); rows n..n_pad padded (norm +inf).
hipError_t split_rows(const float* x, int64_t n, int64_t n_pad, int dk, uint16_t* hi, uint16_t* lo, float* norm,
                      hipStream_t st);
// Dense entry of every query on every shard (start_only = 0) or on its start shard (q_key mod S) only:
// the exact top-t ghosts of the shard by (dist, id), as keys (dist bits << 32 | local node id) in
// out[(q * S + s) * t + i].
// Scratch comes from the stream's kept blocks, or from `ext` (ext_bytes >= dense_entry_min_scratch, else
// hipErrorInvalidValue) when the caller must not allocate: rows are then processed in chunks that fit it.
hipError_t dense_entry_split(int store_dt, const void* queries, int64_t nq, int d, int d_pad, int dk,
                             const uint64_t* qkeys, int S, int start_only, const DenseGhosts& G, int t, uint64_t* out,
                             hipStream_t st, void* ext = nullptr, size_t ext_bytes = 0);
// Smallest caller buffer dense_entry_split accepts for these sizes (one chunk of block rows).
size_t dense_entry_min_scratch(int store_dt, int64_t nq, int d_pad, int dk, int S, int start_only,
                               const DenseGhosts& G);

// Exact k-NN of A rows against B rows by MFMA tiles + direct-form rescoring.
//   A_f32 [na][dpf], B_f32 [nb][dpf]: f32 copies for the GEMM-form selection.
//   A_raw / B_raw: the exact representation ([n][d_pad_raw], raw_dt) for rescoring;
//   A_raw == nullptr means the queries are unpadded f32/u8 rows of length d.
//   out: [na][k] keys (dist bits << 32 | base row index), sorted.
hipError_t knn_exact(const float* A_f32, int64_t na, const float* B_f32, int64_t nb, int dpf, int d,
                     int raw_dt, const void* A_raw, int a_raw_pad, const void* B_raw, const float* B_scale,
                     int b_raw_pad, int k, int exclude_self, const uint32_t* qlist, uint64_t* out, hipStream_t st);

// Candidate selection of the exact k-NN on the matrix cores (knn_split.hip): the kp smallest GEMM-form keys
// (dist bits << 32 | B row) of each A row, ascending, in out[na][kp]. Float rows go through split bf16
// operands (dpf a multiple of 32 up to 256); uint8 rows (u8 != 0: the f32 copies hold integers 0..255) through
// exact int8 products (dpf up to 256). kp up to 192.
bool knn_split_supported(int dpf, int kp, int u8);
hipError_t knn_split_select(const float* A_f32, int64_t na, const float* B_f32, int64_t nb, int dpf, int kp,
                            int exclude_self, int u8, uint64_t* out, hipStream_t st);

// Prepares padded f32 copies of queries (f32 or u8 rows of length d).
hipError_t queries_to_f32(const void* q, int q_dt, int64_t nq, int d, int dpf, float* out, hipStream_t st);

// Graph pruning (reverse-merge rule) from sorted K0-NN keys [n][K0].
hipError_t prune_graph(const uint64_t* knn, int64_t n, int K0, int deg, uint32_t* graph, hipStream_t st);

// Seeded random order: ids sorted by (splitmix(seed, i + 1), i).
hipError_t keyed_order(uint64_t seed, int64_t n, uint32_t* out, hipStream_t st);
// Sorts u32 values ascending (in place).
hipError_t sort_u32(uint32_t* v, int64_t n, hipStream_t st);

// Converts final keys to (ids, dists) outputs with a local -> global map.
hipError_t keys_to_output(const uint64_t* keys, int64_t nq, int k, const uint32_t* gmap, int is_u8, uint32_t* ids,
                          void* dists, hipStream_t st);
hipError_t keys_to_ids(const uint64_t* keys, int64_t n, int k, int col, uint32_t* out, int out_stride,
                       hipStream_t st);

hipError_t keys_to_stage(const uint64_t* keys, int64_t nq, int k, const uint32_t* gmap, int S, int s, uint64_t* so,
                         hipStream_t st);

// Sorts each of `rows` rows of k keys ascending (k <= 256).
hipError_t sort_rows(uint64_t* keys, int64_t rows, int k, hipStream_t st);

}  // namespace miann
