/*
 * miann — MI355X-native graph beam search (PathWeaver, arXiv 2507.17094).
 *
 * C-ABI of the native library libmiann.so. All entry points take plain
 * pointers and sizes. "device" pointers are HIP device (HBM) addresses on the
 * current device; "host" pointers are ordinary process memory. Streams are
 * hipStream_t passed as void* (NULL = the default stream).
 *
 * Conventions for every entry point
 *   - Returns a miann_status; never aborts. On failure, miann_last_error()
 *     returns a thread-local message naming the entry point and the cause.
 *   - Arguments are validated before anything is launched; a failed call
 *     enqueues no work and changes no output.
 *   - Asynchronous: miann_search only enqueues work on `stream` and returns.
 *     A device fault surfaces as MIANN_EDEVICE from a later call.
 *   - Ownership: the caller owns queries and output buffers; an index owns
 *     every array it holds (copied or built), and frees them in
 *     miann_index_free.
 *
 * Distances are SQUARED L2, sum_i (q_i - x_i)^2 (Sec. 2.2 Eq. 2 without the
 * square root; the order is the same). Float data: each difference q_i - x_i
 * is a float32 (x the stored value times its scale), its square is exact in
 * double, the squares are summed in double and the sum is rounded once to
 * float. uint8 data: exact int32. Every ordering is by the key (distance, id)
 * ascending.
 */
#ifndef MIANN_H
#define MIANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MIANN_OK = 0,
  MIANN_EINVAL = 1,      /* an argument is out of range or inconsistent */
  MIANN_ENOMEM = 2,      /* device or host allocation failed */
  MIANN_EDEVICE = 3,     /* a HIP call or an earlier kernel failed */
  MIANN_ESTATE = 4,      /* the object is not in a state that allows the call */
  MIANN_EUNSUPPORTED = 5 /* a valid combination that this build does not implement */
} miann_status;

/* Element types. F32 and U8 are input (original) types; F16 and FP8E4M3
 * (OCP E4M3 "fn": bias 7, max 448, no infinities) are storage types for the
 * traversal, with one float scale per vector. */
typedef enum { MIANN_F32 = 0, MIANN_F16 = 1, MIANN_FP8E4M3 = 2, MIANN_U8 = 3 } miann_dtype;

/* How the first stage of a search is seeded. */
typedef enum {
  MIANN_ENTRY_RANDOM = 0,      /* n_init random nodes (Sec. 2.2 Step 2) */
  MIANN_ENTRY_GHOST_GRAPH = 1, /* beam search on the ghost graph (Sec. 3.2.2) */
  MIANN_ENTRY_GHOST_DENSE = 2, /* exact top-t over all ghost nodes, MFMA distances */
  MIANN_ENTRY_SEEDS = 3,       /* caller-provided seed ids (e.g. a learned predictor) */
  MIANN_ENTRY_PREDICTED = 4    /* seeds per query; a row whose first seed is 0xFFFFFFFF (low predictor
                                  confidence) falls back to the ghost-graph entry */
} miann_entry;

typedef struct miann_index miann_index; /* opaque, library-owned */

/* Counter slots written per query when a counters buffer is given. */
enum {
  MIANN_CTR_NDIST = 0,       /* distance evaluations on the main graphs */
  MIANN_CTR_NEXP = 1,        /* parent expansions */
  MIANN_CTR_ITERS = 2,       /* search iterations, summed over stages */
  MIANN_CTR_DGS_SKIPPED = 3, /* neighbour slots skipped by the direction filter */
  MIANN_CTR_NDIST_GHOST = 4, /* distance evaluations in the ghost stage */
  MIANN_CTR_NEXP_GHOST = 5,  /* expansions in the ghost stage */
  MIANN_CTR_NRERANK = 6,     /* FP32 rerank evaluations (low-precision stores) */
  MIANN_CTR_LAST_TOPK = 7,   /* last iteration (1-based, 0 = none) in which the first k entries of p
                                changed, summed over stages: the iteration-budget trace */
  MIANN_NCTR = 8
};

/* ------------------------------------------------------------------------ */
/* Index construction                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t degree;      /* out-degree of every graph row, 2..64 */
  int32_t knn_k0;      /* neighbours kept by the exact k-NN before pruning; 0 = 2*degree */
  int32_t num_shards;  /* S >= 1 resident shards (Sec. 3.1.2); S = 1 keeps the input order */
  int32_t store_dtype; /* traversal storage: MIANN_F32/F16/FP8E4M3 for float input, MIANN_U8 for u8 */
  int32_t dgs_table;   /* nonzero: build the direction sign table (Sec. 3.3.2 (a)) */
  int32_t reserved;
  uint64_t seed;       /* partition seed */
} miann_build_params;

/* Builds an index from `n` base vectors of dimension `d` on the device:
 * random partition into S shards, exact K0-NN per shard by MFMA distance tiles
 * with fused top-K selection, pruning to `degree` (nearest half of the K0
 * list, then reverse neighbours, then the rest of the K0 list; each row sorted
 * by (distance, id)), the direction sign table, the inter-shard map
 * I(u) = argmin over shard (s+1) mod S of dist(u, w) (Sec. 3.1.2), and the
 * low-precision store if requested.
 *   base_dev : device, [n][d] row-major, in_dtype MIANN_F32 or MIANN_U8; read only,
 *              not retained (the index keeps its own permuted copy).
 *   Requires n >= S * (degree + 1), n < 2^30, 1 <= d <= 4096.
 * Synchronises `stream` before returning. *out receives a new index. */
miann_status miann_build_graph(const void* base_dev, int64_t n, int32_t d, int32_t in_dtype,
                               const miann_build_params* bp, void* stream, miann_index** out);

/* Builds the ghost shard of every shard (Sec. 3.2.2): samples `num_ghost` nodes
 * per shard (or round(ratio * n_s) when num_ghost == 0) uniformly without
 * replacement, copies their vectors, builds their own exact-k-NN graph of
 * `ghost_degree`, and maps each ghost to the node it copies. Replaces any
 * earlier ghost shard. Synchronises `stream`. */
miann_status miann_build_ghost(miann_index* idx, double ratio, int64_t num_ghost, int32_t ghost_degree,
                               uint64_t seed, void* stream);

/* One shard handed to miann_index_import. All pointers are device pointers,
 * copied by the call (the caller keeps ownership). */
typedef struct {
  int64_t n;                  /* nodes in this shard */
  const void* vectors;        /* [n][d] originals, in_dtype */
  const uint32_t* graph;      /* [n][degree] local neighbour ids, 0xFFFFFFFF = no edge */
  const uint32_t* global_ids; /* [n] local -> global id; NULL = identity */
  const uint32_t* next_map;   /* [n] I_s(u): local id in shard (s+1) mod S; NULL allowed when S = 1 */
  int64_t n_ghost;            /* ghost nodes R (0 = none) */
  const uint32_t* ghost_ids;  /* [R] local ids of the ghost nodes (sorted) */
  const uint32_t* ghost_graph;/* [R][ghost_degree] ghost-local neighbour ids */
} miann_shard_desc;

/* Creates an index from caller-built graphs (for example the output of an
 * external builder). The library quantises the store and builds the sign
 * table itself. Synchronises `stream`. */
miann_status miann_index_import(const miann_shard_desc* shards, int32_t num_shards, int32_t d, int32_t in_dtype,
                                int32_t store_dtype, int32_t degree, int32_t ghost_degree, int32_t dgs_table,
                                void* stream, miann_index** out);

/* Read-only views of an index's device arrays (owned by the index; valid
 * until miann_index_free or miann_build_ghost). */
typedef struct {
  int64_t n, n_ghost;
  int32_t d, d_pad;       /* d_pad = stored row length in elements (rows padded with zeros) */
  int32_t degree, ghost_degree, W; /* W = ceil(d / 32) sign words per edge */
  int32_t store_dtype, in_dtype;
  const void* store;      /* [n][d_pad] traversal codes */
  const float* scale;     /* [n] per-vector scales (F16/FP8) or NULL */
  const void* originals;  /* [n][row] F32/U8 originals, rows padded to 128 bytes (the store itself when not
                             quantised) */
  const uint32_t* graph;  /* [n][degree] */
  const uint32_t* sign;   /* [n][W][degree] (word-major per node) or NULL */
  const uint32_t* global_ids; /* [n] */
  const uint32_t* next_map;   /* [n] or NULL */
  const uint32_t* ghost_ids;  /* [R] local ids */
  const uint32_t* ghost_graph;/* [R][ghost_degree] */
} miann_shard_view;

miann_status miann_index_shard(const miann_index* idx, int32_t shard, miann_shard_view* out);
miann_status miann_index_info(const miann_index* idx, int32_t* num_shards, int64_t* n_total, int32_t* d,
                              int32_t* degree, int32_t* store_dtype);
/* Host seconds of the index's build steps (Sec. 5.7's breakdown): [0] the
 * graphs (exact K0-NN and pruning), [1] the direction tables, [2] the
 * inter-shard map, [3] the ghost shards (last miann_build_ghost). Steps the
 * index did not run read 0. */
miann_status miann_index_build_times(const miann_index* idx, double* seconds4);
void miann_index_free(miann_index* idx);

/* Dynamic updates (Sec. 6.2). */
/* Deletion flags: the m nodes with these global ids (device [m], unknown ids
 * ignored) stay in their graphs and are still traversed and handed over
 * between shards, but no search returns them: each stage's result is taken
 * from the entries of its priority queue that are not deleted, in queue
 * order (for low-precision stores, the rerank takes the first min(m k,
 * itopk) live entries). Flags accumulate over calls. Synchronises `stream`. */
miann_status miann_index_delete(miann_index* idx, const uint32_t* global_ids_dev, int64_t m, void* stream);
/* Insertion into one shard: the n new rows (device [n][d], the index's input
 * type) get the next global ids and the next local ids of `shard`; the shard's
 * graph is rebuilt over all its rows by the same exact K0-NN and pruning as
 * miann_build_graph (K0 of the original build, else 2 * degree), its
 * direction table and store are extended, the inter-shard maps into and out
 * of the shard are recomputed (exact 1-NN, Sec. 3.1.2), and, when the index
 * has ghost shards, every shard's ghosts are re-sampled with the same counts
 * from `ghost_seed` (pass the seed of the earlier miann_build_ghost to keep
 * the other shards' samples) and the dense arrays rebuilt. The old arrays of
 * the shard are freed. Not safe while searches on the index are in flight.
 * Synchronises `stream`. */
miann_status miann_index_append(miann_index* idx, int32_t shard, const void* vectors_dev, int64_t n, uint64_t ghost_seed,
                                void* stream);

/* Writes an index to a file at `path` (host file I/O; synchronises the
 * device): per shard the originals, graph, global ids, inter-shard map, ghost
 * ids and ghost graph, with the index's dimensions and types. EINVAL if the
 * file cannot be opened, EDEVICE if a copy or a write fails. */
miann_status miann_index_save(const miann_index* idx, const char* path);
/* Reads a file written by miann_index_save and imports it as with
 * miann_index_import (the store, sign table and dense ghost arrays are
 * rebuilt on the device), so the loaded index searches exactly like the saved
 * one. EINVAL for a missing, foreign, truncated or inconsistent file (all
 * checked on the host before any device allocation), EDEVICE if a device
 * allocation or copy fails; on any error *out is left unchanged.
 * Synchronises `stream`. */
miann_status miann_index_load(const char* path, void* stream, miann_index** out);

/* ------------------------------------------------------------------------ */
/* Search                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t search_width;     /* r: parents expanded per iteration (Sec. 2.2 Step 4); r * degree <= 64 */
  int32_t n_init;           /* random initial candidates (Step 2); 0 = degree; <= 4096 */
  int32_t entry;            /* miann_entry for the first stage */
  int32_t ghost_itopk;      /* l_g, priority-queue length in the ghost stage (<= 64) */
  int32_t ghost_iters;      /* T_g, iterations of the ghost stage */
  int32_t t_seeds;          /* ghost results handed to the main graph; 0 = min(l_g, itopk); <= 64 */
  int32_t dgs;              /* direction-guided selection on (Sec. 3.3.2) */
  int32_t discard_permille; /* rho * 1000: floor(rho * degree) slots skipped per DGS expansion */
  int32_t cooldown_permille;/* c * 1000: the last ceil(c * T) iterations run without DGS */
  int32_t random_discard;   /* ablation: skip random slots instead of the direction ranking */
  int32_t ppe;              /* 1: path extension between shards; 0: independent (naive) shards */
  int32_t forward_f;        /* results handed to the next shard (<= 16) */
  int32_t rerank_mult;      /* low-precision stores: FP32 rerank of the first min(m * k, itopk) */
  int32_t stop_on_no_change;/* also stop when an iteration inserts nothing into p */
  int32_t hash_log2;        /* visited-hash slots per query = 2^hash_log2 (0 = automatic, 8..13) */
  int32_t n_seeds;          /* entries per query in seeds_dev (MIANN_ENTRY_SEEDS) */
  int32_t ghost_every_stage;/* with path extension and a ghost entry: stages t >= 1 also start from their
                               shard's ghost-entry seeds, besides I(z) (an extension; 0 = stage 0 only) */
  int32_t dgs_threshold_permille; /* theta * 1000 in 1..1000: the direction filter keeps every slot whose sign
                               mismatch is at most floor(theta * d) instead of the n_keep best (the
                               similarity-threshold variant of Sec. 6.3); a parent with a skipped slot is
                               re-expanded in the cool-down. 0 = top-n selection */
  int32_t stage_waves;      /* waves per SIMD the stage kernel is built for: 0 = automatic (5 where the
                               wave's LDS leaves room for 20 waves per CU, else 4; FP8 stores always 4);
                               4 = the uncapped kernel; 6 = the 80-VGPR build, which exists for float32
                               rows of at most 224 elements and is taken when the LDS leaves room for 24
                               waves per CU (else the automatic choice); 5 = automatic. Results do not
                               depend on it. 6 pays when another stream's work fills the launch's tail, as
                               with independent batches on two streams; one stream alone runs 5 faster.
                               Other values: MIANN_EINVAL */
  uint64_t seed;            /* random-stream seed */
  const uint64_t* qkeys;    /* device [nq] query keys (index within a request), NULL = row index */
  const uint32_t* seeds;    /* device [nq][n_seeds] local ids in each query's start shard */
  const int32_t* max_iters_per_query; /* device [nq] per-query T, NULL = max_iters */
  float* phase_ms;          /* host [2 + S] or NULL: when set, the call records HIP events around
                               its launches, synchronises `stream` and writes the milliseconds of
                               [dense ghost entry, stage 0 .. stage S-1, shard merge] */
  void* const* phase_events;/* host [4] hipEvent_t (each may be NULL) or NULL: recorded on `stream` before the
                               ghost entry, before stage 0, after the last stage and after the shard merge,
                               without synchronising, so that back-to-back calls stay pipelined; the caller
                               reads the intervals with hipEventElapsedTime once the events completed */
} miann_search_params;

/* Fills the documented defaults: r = 1, n_init = degree, random entry,
 * l_g = 32, T_g = 8, t = min(l_g, itopk), DGS off, rho = 0.5, c = 0.3,
 * path extension on, f = 1, rerank x4, automatic hash, seed 6. */
void miann_search_params_default(miann_search_params* sp);

/* Batched beam search (Sec. 2.2; Sec. 3.1.2 for S > 1 shards; Sec. 3.2.2 ghost
 * entry; Sec. 3.3.2 direction-guided selection).
 *   queries_dev : device [nq][d], F32 for float indices, U8 for u8 indices.
 *   k, itopk    : 1 <= k <= itopk <= 512; low-precision stores need itopk >= rerank_mult * k
 *                 unless rerank_mult * k is capped by itopk.
 *   max_iters   : T >= 0 iterations per stage. T = 0 is valid: each stage returns its entry candidates
 *                 (seeds, hand-off or random starts) ordered, without expanding any.
 *   ids_dev     : device [nq][k] global ids, 0xFFFFFFFF where fewer than k were found.
 *   dists_dev   : device [nq][k] float (or int32 for u8), +inf / INT32_MAX padding.
 *   counters_dev: device [nq][MIANN_NCTR] int64, or NULL.
 * nq = 0 is a no-op. Enqueues on `stream` and returns. Results depend only on
 * (index, query, its key, params), not on the batch it is in. */
miann_status miann_search(const miann_index* idx, const void* queries_dev, int64_t nq, int32_t k, int32_t itopk,
                          int32_t max_iters, const miann_search_params* sp, uint32_t* ids_dev, void* dists_dev,
                          int64_t* counters_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as miann_search, with the same arguments, results and errors, whose
 * temporary buffers (path-extension hand-off, per-stage results, the dense
 * entry's query split, minima, bounds and candidate masks) all come from one
 * static device array of MIANN_NOALLOC_SCRATCH_MB MiB per GPU, held from the
 * library's load until the process ends. The call allocates nothing: no
 * hipMalloc, hipFree or pool allocation. A batch whose buffers do not fit
 * (about 1 KB per query and stage result, plus the dense entry's per-query
 * rows; the dense entry processes its queries in chunks that fit what is
 * left) fails with EINVAL before anything is launched; phase_ms must be NULL
 * (phase_events may be used). Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two streams, or two host threads) race and
 * must be serialised by the caller. */
#define MIANN_NOALLOC_SCRATCH_MB 64
miann_status miann_search_noalloc(const miann_index* idx, const void* queries_dev, int64_t nq, int32_t k,
                                  int32_t itopk, int32_t max_iters, const miann_search_params* sp, uint32_t* ids_dev,
                                  void* dists_dev, int64_t* counters_dev, void* stream);
/* Bytes of the array miann_search_noalloc carves its buffers from. */
size_t miann_noalloc_scratch_bytes(void);

/* The shard-to-shard lookup table built by search, as the paper builds it
 * (Sec. 4): every node u of shard s is a query of a search on shard (s+1) mod
 * S alone (its graph, direction table, store and ghost shard; deletion flags
 * do not apply), keyed by its local id u, with k = 1, `itopk`, `max_iters` and
 * the parameters `sp` (entry MIANN_ENTRY_RANDOM or MIANN_ENTRY_GHOST_GRAPH;
 * qkeys, seeds, max_iters_per_query, phase_ms and phase_events must be NULL);
 * the top-1 local id replaces I_s(u). The exact 1-NN map of miann_build_graph
 * is the same table built by an exhaustive scan. EINVAL for S < 2,
 * EUNSUPPORTED for the dense or seeded entries. Synchronises `stream`. */
miann_status miann_build_next_map(miann_index* idx, int32_t itopk, int32_t max_iters, const miann_search_params* sp,
                                  void* stream);

/* Exact k nearest neighbours of each query over all shards (Sec. 2.1 Eq. 1),
 * by MFMA distance tiles with fused selection and direct-form rescoring.
 * Same layouts as miann_search. k <= 256. Enqueues on `stream`. */
miann_status miann_exact_knn(const miann_index* idx, const void* queries_dev, int64_t nq, int32_t k,
                             uint32_t* ids_dev, void* dists_dev, void* stream);

/* Ghost index (0..R-1) of the nearest ghost node of shard `shard` to each row of
 * `vectors_dev` ([n][d], the index's input type), by (dist, ghost index): the
 * entry-region label of a vector. Enqueues on `stream`. */
miann_status miann_nearest_ghost(const miann_index* idx, int32_t shard, const void* vectors_dev, int64_t n,
                                 uint32_t* ghost_idx_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Learned entry / iteration-budget predictor                                */
/* ------------------------------------------------------------------------ */
/* A BF16 MLP d_in -> hidden -> hidden -> (n_entry logits + 1 budget output),
 * ReLU hidden layers, FP32 master weights, trained with Adam by the library's
 * own GEMM / loss / backward kernels. Loss per row: softmax cross-entropy of
 * the entry label + lambda * (budget output - log(1 + budget label))^2, mean
 * over the batch. Inputs to the GEMMs, stored activations and the output
 * gradient are rounded to bf16; accumulation is FP32. Not a part of the paper:
 * it predicts the ghost-staging entry region and the iteration budget. */
typedef struct miann_predictor miann_predictor;

typedef struct {
  int32_t d_in, hidden, n_entry;
  float *W1, *b1, *W2, *b2, *W3, *b3;       /* device FP32 masters: W1 [d_in][hidden], W2 [hidden][hidden],
                                               W3 [hidden][n_entry + 1], row-major (x W) */
  float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3; /* device gradients of the last step, same layouts */
} miann_predictor_view;

/* Weights U(-a, a) with a = sqrt(6 / fan_in) from SplitMix64(seed), biases 0. */
miann_status miann_predictor_create(int32_t d_in, int32_t hidden, int32_t n_entry, uint64_t seed,
                                    miann_predictor** out);
void miann_predictor_free(miann_predictor* p);
miann_status miann_predictor_view_get(miann_predictor* p, miann_predictor_view* out);
/* Refreshes the bf16 weight copies after the FP32 masters were written through the view. */
miann_status miann_predictor_sync_weights(miann_predictor* p, void* stream);
/* One forward + loss + backward over n rows (x [n][d_in] f32, entry [n] int32 in [0, n_entry), clamped
 * into that range,
 * budget [n] f32 = log(1 + iterations)); leaves the gradients in the view; applies one Adam step
 * (lr, betas 0.9 / 0.999, eps 1e-8) when `update`. Writes the mean loss to *loss_host. Synchronises. */
miann_status miann_predictor_step(miann_predictor* p, const float* x_dev, const int32_t* entry_dev,
                                  const float* budget_dev, int32_t n, float lambda, float lr, int32_t update,
                                  float* loss_host, void* stream);
/* Mini-batch training: each epoch visits the rows in a SplitMix64-keyed random order. epoch_loss_host
 * ([epochs], nullable) receives the mean batch loss of each epoch. Synchronises. */
miann_status miann_predictor_train(miann_predictor* p, const float* x_dev, const int32_t* entry_dev,
                                   const float* budget_dev, int64_t n, int32_t epochs, int32_t batch, float lr,
                                   float lambda, uint64_t seed, float* epoch_loss_host, void* stream);
/* Inference: for each row, confidence = max softmax probability of the entry logits; seeds_dev [n][t] =
 * ghost_map[index] of the t largest logits (seeds[0] = 0xFFFFFFFF when confidence < tau);
 * iters_dev [n] = clamp(ceil(budget_scale (exp(budget) - 1)), t_min, t_max), or t_max when confidence
 * < tau (budget_scale > 0 is the margin over the predicted iteration count; 1.25 .. 3 are typical);
 * top_entry_dev [n][t] (nullable) receives the raw entry indices. Enqueues on `stream`. */
miann_status miann_predictor_predict(const miann_predictor* p, const float* x_dev, int64_t n, int32_t t, float tau,
                                     const uint32_t* ghost_map_dev, int32_t t_min, int32_t t_max, float budget_scale,
                                     uint32_t* seeds_dev, int32_t* iters_dev, float* conf_dev,
                                     uint32_t* top_entry_dev, void* stream);

/* Training labels of the predictor on a one-shard float index, all on the
 * device: iters_dev [n] = the last iteration in which the top-k of the search
 * (k, itopk, max_iters, sp: normally the ghost entry) changed, budget_dev [n]
 * = log(1 + iters), and entry_dev [n] = the ghost index nearest to the exact
 * nearest node of the query (exact 1-NN, then the nearest ghost). queries_dev
 * [n][d] float32. EINVAL for S != 1, ESTATE without ghosts. Enqueues on
 * `stream`. */
miann_status miann_predictor_labels(const miann_index* idx, const float* queries_dev, int64_t n, int32_t k,
                                    int32_t itopk, int32_t max_iters, const miann_search_params* sp, int32_t* entry_dev,
                                    float* budget_dev, int32_t* iters_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching over a resident index                       */
/* ------------------------------------------------------------------------ */
/* A scheduler thread coalesces pending requests of the same search shape (k,
 * itopk, max_iters, parameters) into one launch of up to max_batch_queries,
 * admits a batch only while the in-flight queries and device bytes stay within
 * max_inflight_queries and memory_budget_bytes, and runs batches concurrently
 * on num_streams HIP streams. Queries are searched with their index inside
 * their request as the query key, so results are the same alone and in any mix.
 * Each stream's host and device staging buffers are allocated by
 * miann_server_create for a full batch with k <= 128 (fewer queries if the
 * memory budget does not cover that); a batch beyond that grows them once, a
 * step that blocks the scheduler. */
typedef struct miann_server miann_server;

typedef struct {
  int32_t num_streams;          /* concurrent batches (1..32), default 4 */
  int32_t reserved;
  int64_t max_batch_queries;    /* queries coalesced into one launch, default 8192 */
  int64_t max_inflight_queries; /* admission limit on queries on the device, default 65536 */
  int64_t memory_budget_bytes;  /* admission limit on device bytes of in-flight batches (staging buffers plus
                                   each batch's search temporaries), default 1 GiB */
} miann_server_config;

typedef struct {
  int64_t requests_done, queries_done, batches;
  int64_t peak_inflight_queries, peak_inflight_bytes;
  double elapsed_s;             /* since miann_server_create */
} miann_server_stats;

void miann_server_config_default(miann_server_config* cfg);
/* The index must outlive the server. */
miann_status miann_server_create(const miann_index* idx, const miann_server_config* cfg, miann_server** out);
/* Queues one request: queries_host [nq][d] host rows of the index's input type (copied by the call),
 * k, itopk, max_iters and parameters as for miann_search (sp may be NULL; its qkeys, seeds,
 * max_iters_per_query, phase_ms and phase_events must be NULL). Validates like miann_search; a request larger than
 * the server's limits is EINVAL. Thread-safe. *ticket identifies the request. */
miann_status miann_server_submit(miann_server* srv, const void* queries_host, int64_t nq, int32_t k, int32_t itopk,
                                 int32_t max_iters, const miann_search_params* sp, uint64_t* ticket);
/* Blocks until the request is done; copies ids [nq][k] and dists [nq][k] to host buffers (nullable) and
 * the latency from submission to completion in milliseconds. Each ticket can be waited for once. */
miann_status miann_server_wait(miann_server* srv, uint64_t ticket, uint32_t* ids_host, void* dists_host,
                               double* latency_ms);
/* Runs one search of nq (zero) queries with this shape on every stream of an
 * idle server, so that each stream's staging buffers and kept search scratch
 * reach the shape's size before requests arrive (the first use of a stream
 * otherwise grows them while a request waits). Blocks until done. */
miann_status miann_server_warm(miann_server* srv, int64_t nq, int32_t k, int32_t itopk, int32_t max_iters,
                               const miann_search_params* sp);
/* Open-loop replay of a request trace: a native thread submits request j
 * (rows row_start[j] .. row_start[j] + nq[j] of queries_host, a pool of
 * pool_rows rows; k[j], itopk[j], max_iters[j]; parameters sp) at
 * arrival_s[j] seconds after the start, on the host's steady clock (sleeping
 * until 200 us before, then spinning), while the calling thread waits for the
 * requests in order; latency_ms[j] runs from the scheduled arrival (not the
 * submission) to the completion of the request's batch, -1 for a failed
 * request. *wall_s (nullable) receives the time from the start to the last
 * completion. arrival_s must not decrease. Results are not copied out.
 * Blocks until every request is done. */
miann_status miann_server_replay(miann_server* srv, const void* queries_host, int64_t pool_rows,
                                 const int64_t* row_start, const int64_t* nq, const int32_t* k, const int32_t* itopk,
                                 const int32_t* max_iters, const double* arrival_s, int64_t n_req,
                                 const miann_search_params* sp, double* latency_ms, double* wall_s);
miann_status miann_server_get_stats(miann_server* srv, miann_server_stats* out);
/* Completes every queued request, then frees the server. */
void miann_server_destroy(miann_server* srv);

/* A search keeps its temporary buffers with the stream it ran on, so that
 * back-to-back calls on one stream allocate nothing (each block grows in
 * powers of two to the largest batch seen on that stream). This returns the
 * blocks kept for `stream` on the current device to the library's pool, in
 * stream order; call it before destroying a stream that searched, or to trim
 * memory. miann_server_destroy does it for its own streams. */
miann_status miann_release_scratch(void* stream);

/* Measurement probe (no part of the search): gathers the n rows ids_dev[i]
 * of table_dev ([n_rows][row_bytes] in device memory, row_bytes in {128,
 * 256, 384, 512, 768, 1024}) with the stage kernel's access pattern (8-lane
 * teams, 16-byte chunks, two rows per team in flight), folds each row into
 * out_dev[i]. Ids >= n_rows read row 0. Its bytes per second over a table much
 * larger than the caches is the achievable HBM ceiling of random row gathers.
 * Enqueues on `stream`. */
miann_status miann_gather_probe(const void* table_dev, int64_t n_rows, int32_t row_bytes, const uint32_t* ids_dev,
                                int64_t n, uint32_t* out_dev, void* stream);

/* Thread-local text of the last error (empty string if none). */
const char* miann_last_error(void);

/* Library version string. */
const char* miann_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MIANN_H */
