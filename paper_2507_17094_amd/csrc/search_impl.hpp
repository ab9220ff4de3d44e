// Batched beam search over fixed-degree proximity graphs on gfx950 (the stage
// kernel; search_<type>.hip instantiate it per vector type).
//
// One wave64 searches one query (Sec. 4 runs one query per 32-thread block;
// here the whole CDNA wavefront is the unit). Per wave, LDS holds
//   p     : the priority queue of l (dist, id, flag) keys, sorted (Sec. 2.2)
//   c     : up to 64 candidate keys/ids of the current iteration
//   hash  : an open-addressed visited set that may forget (reset from p when
//           half full); merges reject keys already in p, so the result does
//           not depend on what the hash forgets
//   q     : the query, plus the query sign bits of the current parents
// Neighbour vectors are gathered by 8-lane teams, each lane reading 16-byte
// chunks of the row (rows are padded to 128-byte multiples). Each difference
// q_i - x_i is a float; its square is exact in double and the squares are
// summed in double, so a distance is the sum of the squared float differences
// rounded once to float, whatever the order of summation.
//
// Stages follow path extension (Sec. 3.1.2): stage t of query q runs on shard
// (q_key + t) mod S, seeded by the inter-shard map of the previous stage's top
// results; stage 0 may start with the ghost graph (Sec. 3.2.2). During the
// first T - ceil(c T) iterations the direction filter of Sec. 3.3.2 keeps only
// the neighbours whose stored sign bits agree most with the query's.
#pragma once
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace miann {

struct GraphCtx {
  const void* store;
  const float* scale;
  const uint32_t* graph;
  const uint32_t* sign;
  uint32_t n;
  int deg, degp;
};

__device__ __forceinline__ int hibit(int x) { return x <= 0 ? 0 : (1 << (31 - __clz(x))); }

// Number of keys in a[0..n) (sorted) whose flag-less value is below x.
__device__ __forceinline__ int count_below(const uint64_t* a, int n, uint64_t x) {
  int pos = 0;
  for (int step = hibit(n); step > 0; step >>= 1)
    if (pos + step <= n && key_noflag(a[pos + step - 1]) < x) pos += step;
  return pos;
}

template <int DT, int CPL>
struct Searcher {
  static constexpr int P16 = Fmt<DT>::per16;
  static constexpr int ESZ = Fmt<DT>::esize;
  static constexpr bool kScaled = (DT == DT_F16 || DT == DT_FP8);
  // candidate rows gathered per batch: G rounds of 8 rows, at most 8 16-byte chunks in flight per lane
  static constexpr int G = (8 / CPL) < 1 ? 1 : ((8 / CPL) > 4 ? 4 : (8 / CPL));

  const StageArgs a;
  uint64_t* pk;      // the priority queue p
  uint64_t* pk_alt;  // second buffer for merges
  uint64_t* ck;
  uint32_t* cid;
  uint32_t* hash;
  float* qf;
  uint8_t* qb;
  uint32_t* qsign;
  int* ppos;       // positions in p of the current parents
  uint32_t* pids;  // their node ids
  int hlog, hmask, hfill;
  int lane, team, tl;
  uint64_t qkey;
  uint32_t qq8;  // sum of q^2 over this lane's u8 elements
  unsigned long long* ctr;  // per-query counters (LDS), see kernels.hpp
  int dist_ctr;             // the counter distance evaluations go to

  __device__ Searcher(const StageArgs& args) : a(args) {}

  // counters live in LDS so that they hold no scalar registers in the loops
  __device__ __forceinline__ void ctr_add(int i, long long v) {
    if (lane == 0) __hip_atomic_fetch_add(ctr + i, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }

  // ---------------------------------------------------------------- hash
  __device__ __forceinline__ void hash_clear() {
    for (int i = lane; i <= hmask; i += 64) hash[i] = kNone;
    hfill = 0;
    wsync();
  }
  // true if id was already present; inserts it otherwise (if a slot is free nearby)
  __device__ __forceinline__ bool hash_seen_insert(uint32_t id, bool& inserted) {
    uint32_t h = (id * 0x9E3779B1u) >> (32 - hlog);
    inserted = false;
#pragma unroll 1
    for (int t = 0; t < 16; t++) {
      uint32_t s = (h + t) & hmask;
      uint32_t old = atomicCAS(&hash[s], kNone, id);
      if (old == kNone) { inserted = true; return false; }
      if (old == id) return true;
    }
    return false;
  }
  // returns whether `id` passes the visited filter (not seen before)
  __device__ __forceinline__ bool visit(bool active, uint32_t id) {
    bool ins = false, seen = true;
    if (active) seen = hash_seen_insert(id, ins);
    hfill += __popcll(ballot(ins));
    return active && !seen;
  }
  __device__ __forceinline__ void hash_rebuild(int l) {
    hash_clear();
    for (int i = 0; i < l; i += 64) {
      uint64_t key = (i + lane < l) ? pk[i + lane] : kDummy;
      visit(key != kDummy, key_id(key));
    }
    wsync();
  }

  // ---------------------------------------------------------------- p
  __device__ __forceinline__ void p_reset(int l) {
    for (int i = lane; i < l; i += 64) pk[i] = kDummy;
    wsync();
  }

  // Merge this lane's candidate key (lanes sorted ascending, kDummy = none)
  // into p[0..l). Keys whose (dist, id) is already in p, or repeats within c,
  // are dropped (the existing entry keeps its flag). Returns bit 0 if any
  // candidate entered p, bit 1 if one entered the first k positions.
  __device__ __forceinline__ int merge_sorted(uint64_t c, int l) {
    const uint64_t prev = shfl_u64(c, lane == 0 ? 0 : lane - 1);
    const bool real = c != kDummy;
    const uint64_t cn = key_noflag(c);
    bool dup = real && lane > 0 && key_noflag(prev) == cn;
    int pos = real ? count_below(pk, l, cn) : l;
    if (real && !dup && pos < l && key_noflag(pk[pos]) == cn) dup = true;
    const bool valid = real && !dup;
    const uint64_t vm = ballot(valid);
    if (vm == 0) return 0;
    const int nv = __popcll(vm);
    const int rank = lanes_below(vm);
    const int newpos = pos + rank;
    if (valid) ck[rank] = c;
    wsync();
    // p entries move right by the number of new keys below them; write into the other buffer
    for (int i = lane; i < l; i += 64) {
      const uint64_t pv = pk[i];
      const int np = i + count_below(ck, nv, key_noflag(pv));
      if (np < l) pk_alt[np] = pv;
    }
    const bool in = valid && newpos < l;
    if (in) pk_alt[newpos] = c;
    wsync();
    uint64_t* t = pk;
    pk = pk_alt;
    pk_alt = t;
    return (ballot(in) != 0 ? 1 : 0) | (ballot(in && newpos < a.k) != 0 ? 2 : 0);
  }

  // The same merge for l <= 64 without LDS searches: p (one entry per lane)
  // and the reversed candidates form a bitonic sequence; the elementwise
  // minimum and maximum are its lower and upper 64 keys, each sorted by a
  // half-cleaner network. In the sorted 128 keys a key whose (dist, id)
  // equals the next one's is dropped (the later copy has the larger flag:
  // p's entry), and the first l survivors become the new p.
  __device__ __forceinline__ int merge_sorted_small(uint64_t c, int l) {
    const uint64_t pv = lane < l ? pk[lane] : kDummy;
    const uint64_t cr = reverse_lanes_u64(c);
    uint64_t lo = pv < cr ? pv : cr;
    uint64_t hi = pv < cr ? cr : pv;
    lo = bitonic_merge_u64(lo);
    const int nx = (lane + 1) & 63;
    const uint64_t lo_n = shfl_u64(lo, nx);
    // Usual case: no key of the lower 64 repeats its successor, and the last
    // one repeats no key of the upper 64 (hi[0], its successor, is one of
    // them). Then the new p is the lower 64 as they stand, in place.
    {
      const uint64_t last = ((uint64_t)__builtin_amdgcn_readlane((int)(lo >> 32), 63) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)lo, 63);
      const bool rep_lo = lane < 63 && lo != kDummy && key_noflag(lo) == key_noflag(lo_n);
      const bool rep_hi = last != kDummy && key_noflag(hi) == key_noflag(last);
      if (ballot(rep_lo || rep_hi) == 0) {
        if (lane < l) pk[lane] = lo;
        wsync();
        const bool diff = lane < l && lo != pv;
        return (ballot(diff) != 0 ? 1 : 0) | (ballot(diff && lane < a.k) != 0 ? 2 : 0);
      }
    }
    hi = bitonic_merge_u64(hi);
    // the next key of the sorted 128: lo[i+1], hi[0] after lo[63], hi[i+1]
    const uint64_t hi_n = shfl_u64(hi, nx);
    const uint64_t lo_next = lane == 63 ? hi_n : lo_n;  // hi_n at lane 63 is hi[0]
    const uint64_t hi_next = lane == 63 ? kDummy : hi_n;
    const bool keep_lo = lo == kDummy || key_noflag(lo) != key_noflag(lo_next);
    const bool keep_hi = hi == kDummy || key_noflag(hi) != key_noflag(hi_next);
    const uint64_t mlo = ballot(keep_lo), mhi = ballot(keep_hi);
    const int pos_lo = lanes_below(mlo);
    const int pos_hi = __popcll(mlo) + lanes_below(mhi);
    if (keep_lo && pos_lo < l) pk_alt[pos_lo] = lo;
    if (keep_hi && pos_hi < l) pk_alt[pos_hi] = hi;
    wsync();
    const uint64_t nv = lane < l ? pk_alt[lane] : kDummy;
    const bool diff = nv != pv;
    const int changed = (ballot(diff) != 0 ? 1 : 0) | (ballot(diff && lane < a.k) != 0 ? 2 : 0);
    uint64_t* t = pk;
    pk = pk_alt;
    pk_alt = t;
    return changed;
  }

  __device__ __forceinline__ int merge(uint64_t c, int l) {
    return l <= 64 ? merge_sorted_small(c, l) : merge_sorted(c, l);
  }

  // ---------------------------------------------------------------- distances
  __device__ __forceinline__ void load_query(const void* qptr) {
    const int d = a.d;
    if constexpr (DT == DT_U8) {
      const uint8_t* q = (const uint8_t*)qptr;
      for (int i = lane; i < a.d_pad; i += 64) qb[i] = i < d ? q[i] : 0;
    } else {
      const float* q = (const float*)qptr;
      for (int i = lane; i < a.d_pad; i += 64) qf[i] = i < d ? q[i] : 0.f;
    }
    wsync();
    if constexpr (DT == DT_U8) {
      qq8 = 0;
#pragma unroll
      for (int m = 0; m < CPL; m++) {
        const uint4 qv = ((const uint4*)qb)[tl + 8 * m];
        qq8 = __builtin_amdgcn_udot4(qv.x, qv.x, qq8, false);
        qq8 = __builtin_amdgcn_udot4(qv.y, qv.y, qq8, false);
        qq8 = __builtin_amdgcn_udot4(qv.z, qv.z, qq8, false);
        qq8 = __builtin_amdgcn_udot4(qv.w, qv.w, qq8, false);
      }
    }
  }

  // Sums of the 8 lanes of each team for G rows at once (G = 1, 2, 4): each
  // step halves the rows a lane carries, sending the half its partner keeps
  // (the 8-lane mirror pairs lane i with 7 - i, then xor 2, then xor 1). Row
  // ρ ends in lanes tl with tl / (8 / G) == ρ; every lane of those holds it.
  template <typename V>
  static __device__ __forceinline__ V mirror8(V v) {
    if constexpr (sizeof(V) == 8) {
      const uint64_t u = __builtin_bit_cast(uint64_t, v);
      const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x141, 0xF, 0xF, false);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x141, 0xF, 0xF, false);
      return __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);
    } else {
      return __builtin_bit_cast(V, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
    }
  }
  template <typename V>
  static __device__ __forceinline__ V xor_any(V v, int j) {
    if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, xor_lane_u64(__builtin_bit_cast(uint64_t, v), j));
    else return __builtin_bit_cast(V, xor_lane_u32(__builtin_bit_cast(uint32_t, v), j));
  }
  template <typename V>
  __device__ __forceinline__ V team_reduce(V (&acc)[G]) const {
    const bool b2 = (tl & 4) != 0, b1 = (tl & 2) != 0;
    if constexpr (G == 1) {
      V v = acc[0];
      v += mirror8(v);
      v += xor_any(v, 2);
      v += xor_any(v, 1);
      return v;
    } else if constexpr (G == 2) {
      V v = b2 ? acc[1] : acc[0];
      v += mirror8(b2 ? acc[0] : acc[1]);
      v += xor_any(v, 2);
      v += xor_any(v, 1);
      return v;
    } else {
      V k0 = b2 ? acc[2] : acc[0], k1 = b2 ? acc[3] : acc[1];
      k0 += mirror8(b2 ? acc[0] : acc[2]);
      k1 += mirror8(b2 ? acc[1] : acc[3]);
      V v = b1 ? k1 : k0;
      v += xor_any(b1 ? k0 : k1, 2);
      v += xor_any(v, 1);
      return v;
    }
  }

  // Keys (dist, id, fresh) of the candidate ids cid[0..nc) into ck[0..nc).
  __device__ __forceinline__ void compute_dists(const GraphCtx& g, int nc) {
    const uint32_t row_bytes = (uint32_t)a.d_pad * ESZ;  // at most 1 KB
    constexpr int LPR = 8 / G;  // lanes of a team that end with one row's sum
    for (int r0 = 0; r0 < nc; r0 += 8 * G) {
      uint4 buf[G][CPL];
      float sc[G];
#pragma unroll
      for (int gi = 0; gi < G; gi++) {
        // every lane loads (row 0 for the unused teams), so the gathers need no branches
        const int ci = r0 + gi * 8 + team;
        const uint32_t lid = ci < nc ? cid[ci] : 0u;
        const gptr<u32x4_t> row = as_global((const u32x4_t*)((const char*)g.store + (uint64_t)lid * row_bytes));
#pragma unroll
        for (int m = 0; m < CPL; m++) buf[gi][m] = load16(row, tl + 8 * m);
        if constexpr (kScaled) sc[gi] = as_global(g.scale)[lid];
      }
      uint32_t dbits;
      if constexpr (DT == DT_U8) {
        int part[G];
#pragma unroll
        for (int gi = 0; gi < G; gi++) {
          uint32_t xx = 0, qx = 0;
#pragma unroll
          for (int m = 0; m < CPL; m++) {
            xx = __builtin_amdgcn_udot4(buf[gi][m].x, buf[gi][m].x, xx, false);
            xx = __builtin_amdgcn_udot4(buf[gi][m].y, buf[gi][m].y, xx, false);
            xx = __builtin_amdgcn_udot4(buf[gi][m].z, buf[gi][m].z, xx, false);
            xx = __builtin_amdgcn_udot4(buf[gi][m].w, buf[gi][m].w, xx, false);
            const uint4 qv = ((const uint4*)qb)[tl + 8 * m];
            qx = __builtin_amdgcn_udot4(buf[gi][m].x, qv.x, qx, false);
            qx = __builtin_amdgcn_udot4(buf[gi][m].y, qv.y, qx, false);
            qx = __builtin_amdgcn_udot4(buf[gi][m].z, qv.z, qx, false);
            qx = __builtin_amdgcn_udot4(buf[gi][m].w, qv.w, qx, false);
          }
          part[gi] = (int)(qq8 + xx - 2u * qx);
        }
        dbits = (uint32_t)team_reduce(part);
      } else {
        double acc[G];
#pragma unroll
        for (int gi = 0; gi < G; gi++) acc[gi] = 0.0;
        // query chunk m once for the G rows
#pragma unroll
        for (int m = 0; m < CPL; m++) {
          asm volatile("" ::: "memory");  // read each query chunk where it is used, not all up front
          float qe[P16];
          const float4* qc = (const float4*)(qf + (tl + 8 * m) * P16);
#pragma unroll
          for (int e4 = 0; e4 < P16 / 4; e4++) {
            const float4 qv = qc[e4];
            qe[4 * e4] = qv.x;
            qe[4 * e4 + 1] = qv.y;
            qe[4 * e4 + 2] = qv.z;
            qe[4 * e4 + 3] = qv.w;
          }
#pragma unroll
          for (int gi = 0; gi < G; gi++) {
            float x[P16];
            decode16<DT>(buf[gi][m], x);
#pragma unroll
            for (int e = 0; e < P16; e++) {
              const float xe = kScaled ? sc[gi] * x[e] : x[e];
              const float t = qe[e] - xe;  // float difference; its square is exact in double
              acc[gi] = __builtin_fma((double)t, (double)t, acc[gi]);
            }
          }
        }
        dbits = __float_as_uint((float)team_reduce(acc));
      }
      // lane tl = rho * LPR writes row rho of its team
      const int rho = tl / LPR;
      const int ci = r0 + rho * 8 + team;
      if (tl % LPR == 0 && ci < nc) ck[ci] = make_key(dbits, cid[ci], kFresh);
    }
    wsync();
  }

  // Filter ids (one per lane, active lanes only) through the visited set,
  // evaluate the new ones, and merge them into p.
  __device__ __forceinline__ int add_ids(const GraphCtx& g, bool active, uint32_t id, int l) {
    const bool take = visit(active, id);
    const uint64_t tm = ballot(take);
    const int nc = __popcll(tm);
    if (nc == 0) return 0;
    if (take) cid[lanes_below(tm)] = id;
    wsync();
    compute_dists(g, nc);
    ctr_add(dist_ctr, nc);
    uint64_t key = lane < nc ? ck[lane] : kDummy;
    wsync();
    key = nc > 32 ? bitonic_sort_u64<64>(key) : (nc > 16 ? bitonic_sort_u64<32>(key) : bitonic_sort_u64<16>(key));
    return merge(key, l);
  }

  // Seeds whose distance is already known (one key per lane, kDummy = none).
  __device__ __forceinline__ void add_keys(uint64_t key, int l) {
    const bool take = visit(key != kDummy, key_id(key));
    key = take ? key : kDummy;
    key = bitonic_sort_u64<64>(key);
    merge(key, l);
  }

  __device__ __forceinline__ void random_init(const GraphCtx& g, uint64_t stream, int n_init, int l) {
    for (int b = 0; b < n_init; b += 64) {
      if (hfill > ((hmask + 1) >> 1)) hash_rebuild(l);
      const int j = b + lane;
      uint32_t id = 0;
      if (j < n_init) id = (uint32_t)(sm_at(stream, qkey * (uint64_t)n_init + (uint64_t)j + 1) % (uint64_t)g.n);
      add_ids(g, j < n_init, id, l);
    }
  }

  // Query sign bits against each parent: bit i of word w is [q_j > x_j] for
  // element j = 32 w + i of the parent's (decoded, scaled) row, 0 for j >= d;
  // written to qsign[t * W + w]. Team t reads parent t's row in 16-byte chunks
  // like the distance gathers, so every parent arrives in one round trip; the
  // 32 / P16 chunks of a word sit in adjacent lanes and are OR-ed together.
  __device__ __forceinline__ void parent_signs(const GraphCtx& g, int npar) {
    const int W = a.W;
    const size_t row_bytes = (size_t)a.d_pad * ESZ;
    const bool mine = team < npar;
    const uint32_t pt = pids[mine ? team : 0];
    const gptr<u32x4_t> row = as_global((const u32x4_t*)((const char*)g.store + (size_t)pt * row_bytes));
    uint4 buf[CPL];
#pragma unroll
    for (int m = 0; m < CPL; m++) buf[m] = load16(row, tl + 8 * m);
    float su = 1.f;
    if constexpr (kScaled) su = as_global(g.scale)[pt];
    constexpr int LPW = 32 / P16;  // lanes (chunks) per 32-bit word
#pragma unroll
    for (int m = 0; m < CPL; m++) {
      const int c = tl + 8 * m;
      uint32_t bits = 0;
      if constexpr (DT == DT_U8) {
        const uint4 qv = ((const uint4*)qb)[c];
        const uint32_t xw[4] = {buf[m].x, buf[m].y, buf[m].z, buf[m].w};
        const uint32_t qw[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
        for (int e = 0; e < 16; e++) {
          const uint32_t qe = (qw[e >> 2] >> (8 * (e & 3))) & 0xFFu, xe = (xw[e >> 2] >> (8 * (e & 3))) & 0xFFu;
          bits |= (uint32_t)(qe > xe) << e;
        }
      } else {
        float x[P16];
        decode16<DT>(buf[m], x);
        const float* qc = qf + c * P16;
#pragma unroll
        for (int e = 0; e < P16; e++) bits |= (uint32_t)(qc[e] > (kScaled ? su * x[e] : x[e])) << e;
      }
      const int valid = a.d - c * P16;
      if (valid < P16) bits &= valid <= 0 ? 0u : ((1u << valid) - 1u);
      uint32_t wv = bits << (P16 * (tl % LPW));
      if constexpr (LPW >= 2) wv |= xor_lane<1>(wv);
      if constexpr (LPW >= 4) wv |= xor_lane<2>(wv);
      if constexpr (LPW >= 8) wv |= xor_lane<4>(wv);
      const int w = c / LPW;
      if (mine && tl % LPW == 0 && w < W) qsign[team * W + w] = wv;
    }
  }

  // ---------------------------------------------------------------- the loop
  // Steps 3-4 of Sec. 2.2 until no parent is eligible or T iterations ran.
  __device__ __forceinline__ void beam_loop(const GraphCtx& g, int l, int T, bool dgs_on, bool stop_nc, uint64_t stream,
                            int& n_exp, int& n_iter, int& last_topk) {
    const int r = a.r;
    const int n_cool = (a.cooldown_pm * T + 999) / 1000;
    const int t_dgs = T - n_cool;
    const int W = a.W;
    bool forced = false;
    int it = 0;
    while (it < T) {
      const bool dgs_phase = dgs_on && !forced && it < t_dgs;
      // parents: the first r eligible entries of p, in p order
      int npar = 0;
      for (int b = 0; b < l && npar < r; b += 64) {
        const int i = b + lane;
        const uint64_t key = i < l ? pk[i] : kDummy;
        const uint32_t fl = key_flag(key);
        const bool el = key != kDummy && (dgs_phase ? fl == kFresh : fl != kDone);
        const uint64_t m = ballot(el);
        const int below = lanes_below(m);
        if (el && npar + below < r) {
          ppos[npar + below] = i;
          pids[npar + below] = key_id(key);
        }
        npar += __popcll(m);
      }
      npar = npar < r ? npar : r;
      wsync();
      if (npar == 0) {
        if (dgs_phase) { forced = true; continue; }
        break;
      }
      if (hfill > ((hmask + 1) >> 1)) hash_rebuild(l);
      const int keep = dgs_phase ? a.n_keep : g.deg;
      // similarity-threshold selection (Sec. 6.3): the parents' flags follow from their kept counts below
      const bool thr_mode = dgs_phase && a.dgs_thr >= 0;
      const uint32_t newflag = (dgs_phase && keep < g.deg) ? kPartial : kDone;
      if (!thr_mode && lane < npar) pk[ppos[lane]] = (pk[ppos[lane]] & ~3ull) | newflag;
      // lane -> (parent, slot)
      const int pa = lane / g.degp, slot = lane % g.degp;
      const bool act = pa < npar && slot < g.deg;
      const uint32_t u = pa < npar ? pids[pa] : 0u;
      uint32_t nb = as_global(g.graph)[(size_t)u * g.deg + (act ? slot : 0)];
      nb = act ? nb : kNone;
      if (dgs_phase) {
        // this lane's direction-table words, loaded in the same round trip as the adjacency row
        constexpr int kSW = 8;
        // inactive lanes read slot 0 of a valid row (slots beyond deg would run past the table)
        const uint32_t* srow = g.sign + (size_t)u * W * g.deg + (act ? slot : 0);
        uint32_t sw[kSW];
#pragma unroll
        for (int w = 0; w < kSW; w++)
          sw[w] = (!a.random_discard && w < W) ? as_global(srow)[(size_t)w * g.deg] : 0u;
        if (!a.random_discard) parent_signs(g, npar);
        wsync();
        uint32_t rk = 0xFFFFFFFFu;
        int mm = 0;
        if (act) {
          if (a.random_discard) {
            const uint64_t h1 = sm_at(stream, qkey + 1);
            rk = ((uint32_t)(sm_mix(h1 ^ (((uint64_t)u << 8) | (uint64_t)slot)) >> 40) << 8) | (uint32_t)slot;
          } else {
#pragma unroll
            for (int w = 0; w < kSW; w++)
              if (w < W) mm += __popc(qsign[pa * W + w] ^ sw[w]);
            for (int w = kSW; w < W; w++) mm += __popc(qsign[pa * W + w] ^ srow[(size_t)w * g.deg]);
            rk = ((uint32_t)mm << 8) | (uint32_t)slot;
          }
        }
        if (thr_mode) {
          // keep every slot whose mismatch is at most the threshold; a parent with a skipped slot is partial
          const bool kept = act && mm <= a.dgs_thr;
          const uint64_t km = ballot(kept);
          if (lane < npar) {
            const uint64_t seg = g.deg >= 64 ? ~0ull : ((1ull << g.deg) - 1ull);
            const int nk = __popcll((km >> (lane * g.degp)) & seg);
            pk[ppos[lane]] = (pk[ppos[lane]] & ~3ull) | (nk < g.deg ? kPartial : kDone);
          }
          nb = kept ? nb : kNone;
          ctr_add(3, npar * g.deg - __popcll(km));
        } else {
          // the kept slots: the keep smallest (mismatch, slot) keys of each parent's segment, first in it
          rk = 2 * keep == g.degp ? bitonic_lower_half_u32_seg(rk, g.degp) : bitonic_sort_u32_seg(rk, g.degp);
          const bool kept = act && slot < keep && rk != 0xFFFFFFFFu;
          const int src = pa * g.degp + (int)(rk & 0xFFu);
          const uint32_t nb_sel = shfl_u32(nb, kept ? src : lane);
          nb = kept ? nb_sel : kNone;
          ctr_add(3, (g.deg - keep) * npar);
        }
      }
      const int changed = add_ids(g, nb != kNone, nb, l);
      n_exp += npar;
      it++;
      if (changed & 2) last_topk = it;
      if (stop_nc && !(changed & 1)) break;
    }
    n_iter += it;
  }

  // FP32 rerank of p[0..m) (low-precision stores): exact distances against the
  // FP32 originals, then sort.
  __device__ __forceinline__ void rerank(const float* orig, int m) {
    const int dpf = a.d_pad_f32;
    for (int r0 = 0; r0 < m; r0 += 8) {
      const int ci = r0 + team;
      const bool ok = ci < m && pk[ci] != kDummy;
      const uint32_t id = ok ? key_id(pk[ci]) : 0u;
      const float4* row = (const float4*)(orig + (size_t)id * dpf);
      double acc = 0.0;
      if (ok)
        for (int c = tl; c < dpf / 4; c += 8) {
          const float4 x = row[c];
          const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
          for (int e = 0; e < 4; e++) {
            const float t = qf[4 * c + e] - xs[e];
            acc = __builtin_fma((double)t, (double)t, acc);
          }
        }
      acc += xor_lane_f64(acc, 1);
      acc += xor_lane_f64(acc, 2);
      acc += xor_lane_f64(acc, 4);
      wsync();
      if (tl == 0 && ci < m && ok) pk[ci] = make_key(__float_as_uint((float)acc), id, kDone);
    }
    wsync();
    sort_p(m);
  }

  // Sorts pk[0..m) ascending (entries m..pow2(m) are padded with dummies).
  __device__ __forceinline__ void sort_p(int m) {
    int n = 1;
    while (n < m) n <<= 1;
    for (int i = m + lane; i < n; i += 64) pk[i] = kDummy;
    wsync();
    for (int kk = 2; kk <= n; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < n; i += 64) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const uint64_t x = pk[i], y = pk[ixj];
            const bool up = (i & kk) == 0;
            if ((x > y) == up) { pk[i] = y; pk[ixj] = x; }
          }
        }
        wsync();
      }
  }
};

// Each stage kernel exists in several register budgets. OCC = 0 leaves the
// VGPR count to the compiler (about 120 for f32 rows: 4 waves per SIMD).
// OCC = 5 caps it at 96 VGPRs for 5 waves per SIMD, at the price of a few
// spilled loop invariants; the launch takes it when the wave's LDS also
// leaves room for 5 waves (small itopk), where the extra wave hides more
// gather latency than the spills cost (f32, d = 96, itopk 64: 0.35 -> 0.32 ms
// per stage launch). OCC = 6 (80 VGPRs) exists for f32 rows of up to 7
// chunks per lane (d <= 224), which fit it without spills; the caller asks
// for it (stage_waves = 6). A launch of 10,000 queries fills 1.95 rounds of
// the 5-wave slots but 1.63 of the 6-wave ones, so on one stream the longer
// tail makes it slower; with independent batches on two streams the other
// batch fills the tail and the extra wave hides more gather latency (itopk
// 32, d = 96: 0.14-0.15 -> 0.12-0.14 ms per stage launch). With large itopk
// the LDS caps occupancy anyway and the uncapped kernel is faster.
template <int DT, int CPL, int OCC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1)))
void stage_kernel(StageArgs a) {
  extern __shared__ __align__(16) char smem[];
  // the wave index is the same on every lane: held in a scalar register, so that what follows from it (the
  // query, its shard and the shard's arrays) is scalar too and leaves the vector registers to the search
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * a.waves_per_block + wave;
  if (q >= a.nq) return;

  Searcher<DT, CPL> S(a);
  S.lane = lane_id();
  S.team = S.lane >> 3;
  S.tl = S.lane & 7;
  char* base = smem + (size_t)wave * a.per_wave_lds;
  S.pk = (uint64_t*)base;
  base += (size_t)a.lp_pow2 * 8;
  S.pk_alt = (uint64_t*)base;
  base += (size_t)a.lp_pow2 * 8;
  S.ck = (uint64_t*)base;
  base += 64 * 8;
  S.ctr = (unsigned long long*)base;
  base += kNumCtr * 8;
  S.cid = (uint32_t*)base;
  base += 64 * 4;
  S.hlog = a.hash_log2;
  S.hmask = (1 << a.hash_log2) - 1;
  S.hash = (uint32_t*)base;
  base += (size_t)4 << a.hash_log2;
  S.qf = (float*)base;
  S.qb = (uint8_t*)base;
  base += (size_t)a.d_pad * 4;
  S.qsign = (uint32_t*)base;
  base += (size_t)kMaxR * a.W * 4;
  S.ppos = (int*)base;
  base += kMaxR * 4;
  S.pids = (uint32_t*)base;
  if (S.lane < kNumCtr) S.ctr[S.lane] = 0;
  S.dist_ctr = 0;

  S.qkey = a.qkeys ? a.qkeys[q] : (uint64_t)q;
  const int Sh = a.S;
  const int s0 = (int)(S.qkey % (uint64_t)Sh);
  const int t = a.stage;
  const int s = (s0 + t) % Sh;
  const ShardDev sh = a.sh[s];
  const uint64_t stream_main = sm_at(a.seed, (uint64_t)(2 * s + 1));
  const uint64_t stream_ghost = sm_at(a.seed, (uint64_t)(2 * s + 2));
  const int T = a.Tq ? a.Tq[q] : a.T;
  const size_t qbytes = (size_t)a.d * (DT == DT_U8 ? 1 : 4);
  S.load_query((const char*)a.queries + (size_t)q * qbytes);

  GraphCtx gm{sh.store, sh.scale, sh.graph, sh.sign, sh.n, a.deg, a.degp};
  S.hash_clear();
  S.p_reset(a.l);
  const bool use_entry = (t == 0) || !a.ppe;
  int n_exp = 0, n_iter = 0;
  // predicted entry: the row's seeds, or the ghost graph when the predictor was not confident
  int entry = a.entry;
  if (entry == 4) entry = (t == 0 && a.seeds[(size_t)q * a.n_seeds] != kNone) ? 3 : 1;
  const bool ghost = entry == 1 || entry == 2;
  if (ghost && (use_entry || a.ghost_every)) {
    uint64_t seed = kDummy;
    if (entry == 1) {
      // ghost staging: a short search on the ghost graph (p and the hash serve as scratch)
      GraphCtx gg{sh.g_store, sh.g_scale, sh.g_graph, nullptr, sh.R, a.deg_g, a.degp_g};
      S.p_reset(a.l_g);
      int ge = 0, gi = 0, gl = 0;
      S.dist_ctr = 4;
      S.random_init(gg, stream_ghost, a.deg_g, a.l_g);
      S.beam_loop(gg, a.l_g, a.T_g, false, false, stream_ghost, ge, gi, gl);
      S.dist_ctr = 0;
      S.ctr_add(5, ge);
      const uint64_t gk = S.lane < a.t_seeds ? S.pk[S.lane] : kDummy;
      if (gk != kDummy) seed = make_key(key_dist(gk), sh.g_map[key_id(gk)], kFresh);
      wsync();
      S.hash_clear();
      S.p_reset(a.l);
    } else {
      const uint64_t dk = S.lane < a.t_seeds ? a.dense[((size_t)q * Sh + s) * a.t_seeds + S.lane] : kDummy;
      if (dk != kDummy) seed = make_key((uint32_t)(dk >> 32), (uint32_t)dk, kFresh);
      S.ctr_add(4, sh.R);
    }
    // the ghost seeds' distances are those of the nodes they copy
    S.add_keys(seed, a.l);
  }
  if (!use_entry) {
    // path extension: continue from I(z) of the previous stage's first f results
    const uint32_t id = S.lane < a.f ? a.hand_in[(size_t)q * a.f + S.lane] : kNone;
    S.add_ids(gm, id != kNone, id, a.l);
  } else if (!ghost) {
    if (entry == 3 && t == 0 && a.seeds) {
      for (int b = 0; b < a.n_seeds; b += 64) {
        const int j = b + S.lane;
        const uint32_t id = j < a.n_seeds ? a.seeds[(size_t)q * a.n_seeds + j] : kNone;
        S.add_ids(gm, id != kNone && id < sh.n, id, a.l);
      }
    } else {
      S.random_init(gm, stream_main, a.n_init, a.l);
    }
  }
  int last_topk = 0;
  S.beam_loop(gm, a.l, T, a.dgs != 0, a.stop_on_no_change != 0, stream_main, n_exp, n_iter, last_topk);
  S.ctr_add(1, n_exp);
  S.ctr_add(2, n_iter);
  S.ctr_add(7, last_topk);

  // hand-off to the next shard: I(z) for the first f entries
  if (Sh > 1 && a.ppe && t + 1 < Sh && S.lane < a.f) {
    const uint64_t key = S.pk[S.lane];
    a.hand_out[(size_t)q * a.f + S.lane] = key != kDummy ? sh.next[key_id(key)] : kNone;
  }
  wsync();
  if (sh.dead) {
    // deletion flags (Sec. 6.2): deleted nodes served the traversal and the hand-off above; the stage result
    // is taken from the live entries of p, in p order
    int nl = 0;
    for (int i0 = 0; i0 < a.l; i0 += 64) {
      const int i = i0 + S.lane;
      const uint64_t key = i < a.l ? S.pk[i] : kDummy;
      const bool live = key != kDummy && !as_global(sh.dead)[key_id(key)];
      const uint64_t m = ballot(live);
      if (live) S.pk_alt[nl + lanes_below(m)] = key;
      nl += __popcll(m);
    }
    for (int i = nl + S.lane; i < a.l; i += 64) S.pk_alt[i] = kDummy;
    wsync();
    uint64_t* tp = S.pk;
    S.pk = S.pk_alt;
    S.pk_alt = tp;
  }
  if (a.lowp) {
    int m = a.rerank_m * a.k;
    if (m > a.l) m = a.l;
    int real = 0;
    for (int i = 0; i < m; i += 64) real += __popcll(ballot(i + S.lane < m && S.pk[i + S.lane] != kDummy));
    S.ctr_add(6, real);
    S.rerank(sh.orig, m);
  }
  // the stage's k results, ordered by (dist, global id) for the reduction over shards
  for (int i = S.lane; i < a.k; i += 64) {
    const uint64_t key = S.pk[i];
    const uint32_t lid = key_id(key);
    S.pk[i] = key != kDummy ? (((uint64_t)key_dist(key) << 32) | (sh.gmap ? sh.gmap[lid] : lid)) : kDummy;
  }
  wsync();
  S.sort_p(a.k);
  for (int i = S.lane; i < a.k; i += 64) {
    const uint64_t key = S.pk[i];
    const bool ok = key != kDummy;
    if (Sh == 1) {
      a.out_ids[(size_t)q * a.k + i] = ok ? (uint32_t)key : kNone;
      if (DT == DT_U8)
        ((int32_t*)a.out_d)[(size_t)q * a.k + i] = ok ? (int32_t)(key >> 32) : 0x7FFFFFFF;
      else
        ((uint32_t*)a.out_d)[(size_t)q * a.k + i] = ok ? (uint32_t)(key >> 32) : 0x7F800000u;
    } else {
      a.stage_out[((size_t)q * Sh + t) * a.k + i] = key;
    }
  }
  wsync();
  if (a.ctr && S.lane < kNumCtr) {
    long long* c = (long long*)a.ctr + (size_t)q * kNumCtr + S.lane;
    *c = (t == 0 ? 0 : *c) + (long long)S.ctr[S.lane];
  }
}

template <int DT, int CPL, int OCC>
static hipError_t launch_occ(const StageArgs& a, hipStream_t st) {
  const int wpb = a.waves_per_block;
  const int64_t blocks = (a.nq + wpb - 1) / wpb;
  const size_t lds = (size_t)a.per_wave_lds * wpb;
  // once per kernel instance, also when host threads search concurrently
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    (void)hipFuncSetAttribute((const void*)stage_kernel<DT, CPL, OCC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
  });
  hipLaunchKernelGGL((stage_kernel<DT, CPL, OCC>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
  return hipGetLastError();
}

template <int DT, int CPL>
static hipError_t launch_t(const StageArgs& a, hipStream_t st) {
  // FP8 rows decode into 16 floats per chunk: at 96 VGPRs that kernel spills inside its loops (88 to 236 bytes
  // per lane) and is slower than at 4 waves, so it keeps the compiler's budget
  if constexpr (DT == DT_FP8) {
    return launch_occ<DT, CPL, 0>(a, st);
  } else {
    // 6 (5) waves per SIMD = 24 (20) per CU must fit the CU's 160 KB of LDS
    if constexpr (DT == DT_F32 && CPL <= 7)
      if (a.stage_waves == 6 && (int64_t)a.per_wave_lds * 24 <= 160 * 1024) return launch_occ<DT, CPL, 6>(a, st);
    if (a.stage_waves == 4) return launch_occ<DT, CPL, 0>(a, st);
    if ((int64_t)a.per_wave_lds * 20 <= 160 * 1024) return launch_occ<DT, CPL, 5>(a, st);
    return launch_occ<DT, CPL, 0>(a, st);
  }
}

template <int DT>
hipError_t launch_dt(int cpl, const StageArgs& a, hipStream_t st) {
  switch (cpl) {
    case 1: return launch_t<DT, 1>(a, st);
    case 2: return launch_t<DT, 2>(a, st);
    case 3: return launch_t<DT, 3>(a, st);
    case 4: return launch_t<DT, 4>(a, st);
    case 5: return launch_t<DT, 5>(a, st);
    case 6: return launch_t<DT, 6>(a, st);
    case 7: return launch_t<DT, 7>(a, st);
    case 8: return launch_t<DT, 8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace miann
