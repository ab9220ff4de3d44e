// Kernel argument blocks and launch entry points shared by the C-ABI layer
// (capi.cpp) and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miann {

constexpr int kMaxShards = 16;
constexpr int kMaxR = 8;        // search width cap
constexpr int kMaxL = 512;      // itopk cap
constexpr int kMaxSeedsLane = 64;
constexpr int kNumCtr = 8;

// Device arrays of one resident shard.
struct ShardDev {
  const void* store;        // [n][d_pad] traversal codes
  const float* scale;       // [n] (F16/FP8) or nullptr
  const float* orig;        // [n][d_pad_f32] FP32 originals for the rerank (low-precision stores)
  const uint32_t* graph;    // [n][deg]
  const uint32_t* sign;     // [n][W][deg] or nullptr
  const uint32_t* gmap;     // [n] local -> global
  const uint32_t* next;     // [n] local -> local id in shard (s+1)%S, or nullptr
  const void* g_store;      // [R][d_pad] ghost codes
  const float* g_scale;     // [R]
  const uint32_t* g_graph;  // [R][deg_g]
  const uint32_t* g_map;    // [R] ghost -> local id
  const uint8_t* dead;      // [n] deletion flags (traversed, never returned), or nullptr
  uint32_t n, R;
};

// Per-launch arguments, passed by value; every field is a scalar or a pointer
// (no arrays) so the kernel keeps them in scalar registers.
struct StageArgs {
  const ShardDev* sh;       // [S] device array owned by the index
  uint64_t seed;            // random-stream seed
  const void* queries;      // [nq][d] f32 or u8 (unpadded)
  int64_t nq;
  int d, d_pad, d_pad_f32, W, deg, degp, deg_g, degp_g;
  int k, l, r, T, n_init, l_g, T_g, t_seeds;
  int entry, dgs, n_keep, cooldown_pm, random_discard, stop_on_no_change, ghost_every;
  int dgs_thr;              // similarity threshold on the sign mismatch (keep mm <= dgs_thr), -1 = top-n selection
  int stage_waves;          // requested waves per SIMD of the stage kernel (0 = automatic, 4, 5, 6)
  int S, stage, ppe, f, rerank_m, lowp;
  int hash_log2, lp_pow2, waves_per_block;
  int per_wave_lds;         // bytes
  const uint64_t* qkeys;    // [nq] or nullptr
  const uint32_t* seeds;    // [nq][n_seeds] or nullptr
  int n_seeds;
  const int32_t* Tq;        // [nq] or nullptr
  const uint64_t* dense;    // [nq][S][t_seeds] keys (dist bits << 32 | local id) or nullptr
  const uint32_t* hand_in;  // [nq][f]
  uint32_t* hand_out;       // [nq][f]
  uint64_t* stage_out;      // [nq][S][k] keys (dist bits << 32 | global id)
  uint32_t* out_ids;        // [nq][k]   (S == 1)
  void* out_d;              // [nq][k]
  int64_t* ctr;             // [nq][8] or nullptr
};

// Bytes of LDS one wave needs for these arguments.
int stage_lds_bytes(const StageArgs& a);
hipError_t launch_stage(int dtype, int cpl, const StageArgs& a, hipStream_t st);
// Random-row gather probe (rows of row_bytes in {128, 256, 384, 512, 768, 1024}).
hipError_t launch_gather_probe(const void* table, int64_t n_rows, int row_bytes, const uint32_t* ids, int64_t n,
                               uint32_t* out, hipStream_t st);
hipError_t launch_merge(const uint64_t* stage_out, int64_t nq, int S, int k, int is_u8, uint32_t* ids, void* dists,
                        hipStream_t st);

}  // namespace miann
