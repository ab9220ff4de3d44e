// Device-side building blocks shared by the miann kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miann {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kIdMask = 0x3FFFFFFFu;  // ids fit in 30 bits; 2 bits hold the entry flag
constexpr uint64_t kDummy = ~0ull;         // sorts after every real key

// Entry flags of the priority queue p.
constexpr uint32_t kFresh = 0;    // not expanded yet
constexpr uint32_t kPartial = 1;  // expanded with some neighbour slots skipped (direction filter)
constexpr uint32_t kDone = 2;     // fully expanded

enum : int { DT_F32 = 0, DT_F16 = 1, DT_FP8 = 2, DT_U8 = 3 };

// Keys order entries by (distance, id). Distances are non-negative, so the
// IEEE bit pattern of a float (or the value of a non-negative int32) orders
// like the number. Layout: dist bits << 32 | id << 2 | flag.
__device__ __forceinline__ uint64_t make_key(uint32_t dist_bits, uint32_t id, uint32_t flag) {
  return ((uint64_t)dist_bits << 32) | ((uint64_t)((id & kIdMask) << 2)) | flag;
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return ((uint32_t)k) >> 2; }
__device__ __forceinline__ uint32_t key_flag(uint64_t k) { return ((uint32_t)k) & 3u; }
__device__ __forceinline__ uint32_t key_dist(uint64_t k) { return (uint32_t)(k >> 32); }
__device__ __forceinline__ uint64_t key_noflag(uint64_t k) { return k >> 2; }

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) as a counter-based generator:
// output(ctr) = mix(seed + ctr * 0x9E3779B97F4A7C15).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t sm_at(uint64_t seed, uint64_t ctr) {
  return sm_mix(seed + ctr * 0x9E3779B97F4A7C15ull);
}

// ---------------------------------------------------------------------------
// Wave64 helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders this wave's LDS accesses: the LDS executes one wave's operations in
// issue order, so only compiler reordering must be prevented.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src, 64); }
__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m, 64); }
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = shfl_u32((uint32_t)v, src), hi = shfl_u32((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = shfl_xor_u32((uint32_t)v, m), hi = shfl_xor_u32((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double shfl_xor_f64(double v, int m) {
  return __longlong_as_double((long long)shfl_xor_u64((uint64_t)__double_as_longlong(v), m));
}
__device__ __forceinline__ int shfl_xor_i32(int v, int m) { return __shfl_xor(v, m, 64); }

// Lane i receives v from lane i ^ J (J = 1, 2, 4, ..., 32) without the LDS
// crossbar: DPP permutes inside 16-lane rows (quad permutes, the 8-lane
// mirror, rotation by 8) and gfx950's row-swap permutes across rows. Every
// mapping used is an involution, so none depends on a shift direction.
// v_permlane16_swap(v, v) exchanges the odd rows of its first result with the
// even rows of its second, v_permlane32_swap(v, v) the upper half of the first
// with the lower half of the second; so the second result holds the partner's
// value in even rows (lower half) and the first result in odd rows (upper half).
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  static_assert(J == 1 || J == 2 || J == 4 || J == 8 || J == 16 || J == 32, "J");
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (J == 4) {
    const int m = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);    // row_half_mirror: i -> 7 - i
    return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);        // quad_perm [3,2,1,0]
  } else if constexpr (J == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (J == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return __builtin_amdgcn_inverse_ballot_w64(0x0000FFFF0000FFFFull) ? r[1] : r[0];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __builtin_amdgcn_inverse_ballot_w64(0x00000000FFFFFFFFull) ? r[1] : r[0];
  }
}
// Both values of each lane pair (i, i ^ J) for J = 16 or 32, in an order that
// differs between the two lanes: {a, b} = {own value, partner's value}. A
// compare-exchange needs only the pair, so this skips the final select.
template <int J>
__device__ __forceinline__ void swap_pair_u64(uint64_t v, uint64_t& a, uint64_t& b) {
  static_assert(J == 16 || J == 32, "J");
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  if constexpr (J == 16) {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a = ((uint64_t)rh[0] << 32) | rl[0];
    b = ((uint64_t)rh[1] << 32) | rl[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = ((uint64_t)rh[0] << 32) | rl[0];
    b = ((uint64_t)rh[1] << 32) | rl[1];
  }
}
template <int J>
__device__ __forceinline__ void swap_pair_u32(uint32_t v, uint32_t& a, uint32_t& b) {
  static_assert(J == 16 || J == 32, "J");
  if constexpr (J == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = r[0];
    b = r[1];
  }
}
// Lane i receives v from lane 63 - i: the row mirror (i -> 15 - i inside each
// 16-lane row) followed by swapping rows 0 <-> 3 and 1 <-> 2.
__device__ __forceinline__ uint32_t reverse_lanes_u32(uint32_t v) {
  const uint32_t m = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  return xor_lane<32>(xor_lane<16>(m));
}
__device__ __forceinline__ uint64_t reverse_lanes_u64(uint64_t v) {
  return ((uint64_t)reverse_lanes_u32((uint32_t)(v >> 32)) << 32) | reverse_lanes_u32((uint32_t)v);
}
// Runtime j; inside fully unrolled loops the switch folds to one case.
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v, int j) {
  switch (j) {
    case 1: return xor_lane<1>(v);
    case 2: return xor_lane<2>(v);
    case 4: return xor_lane<4>(v);
    case 8: return xor_lane<8>(v);
    case 16: return xor_lane<16>(v);
    default: return xor_lane<32>(v);
  }
}
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v, int j) {
  const uint32_t lo = xor_lane_u32((uint32_t)v, j), hi = xor_lane_u32((uint32_t)(v >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double xor_lane_f64(double v, int j) {
  return __longlong_as_double((long long)xor_lane_u64((uint64_t)__double_as_longlong(v), j));
}
__device__ __forceinline__ int xor_lane_i32(int v, int j) { return (int)xor_lane_u32((uint32_t)v, j); }

// Global-memory views of generic pointers: loads through them compile to
// global_load (vector memory only) instead of flat_load, which would also
// count against the LDS wait counter.
template <typename T>
using gptr = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}
// 16-byte global load (a builtin vector type, so it can be read through gptr)
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 load16(gptr<u32x4_t> p, int i) {
  const u32x4_t v = p[i];
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Number of set lanes of `mask` below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Bitonic networks. Stage (K, J) of a sort over N keys (key index i = r * 64 +
// lane, r the register) exchanges keys i and i ^ J; key i keeps the smaller one
// iff (i & J) == 0 equals the pair's direction (ascending iff K == N or
// (i & K) == 0). Every stage is a template instance, so the lanes that keep the
// smaller key form a compile-time mask: one compare, a scalar XOR with the mask
// (take the partner where "partner < key" agrees with "keep the smaller") and
// two selects per 64-bit exchange.
constexpr uint64_t keep_min_mask(int K, int J, int N, int R) {
  uint64_t m = 0;
  for (int l = 0; l < 64; l++) {
    const int i = (R << 6) | l;
    const bool lower = (i & J) == 0;
    const bool up = (K >= N) || ((i & K) == 0);
    if (lower == up) m |= 1ull << l;
  }
  return m;
}

template <uint64_t WM, typename T>
__device__ __forceinline__ T exchange(T key, T other) {
  const bool take = __builtin_amdgcn_inverse_ballot_w64(~(__ballot(other < key) ^ WM));
  return take ? other : key;
}

// Compare-exchange of key with lane ^ J's key under the keep-min mask WM.
// Across rows (J >= 16) the pair comes from one row swap, and the result is
// the pair's minimum or maximum whatever the order of the pair.
template <uint64_t WM, int J>
__device__ __forceinline__ uint64_t xchg_u64(uint64_t key) {
  if constexpr (J >= 16) {
    uint64_t a, b;
    swap_pair_u64<J>(key, a, b);
    return exchange<WM>(a, b);
  } else {
    return exchange<WM>(key, xor_lane_u64(key, J));
  }
}
template <uint64_t WM, int J>
__device__ __forceinline__ uint32_t xchg_u32(uint32_t key) {
  if constexpr (J >= 16) {
    uint32_t a, b;
    swap_pair_u32<J>(key, a, b);
    return exchange<WM>(a, b);
  } else {
    return exchange<WM>(key, xor_lane_u32(key, J));
  }
}

template <int SEG, int K, int J>
__device__ __forceinline__ void bsort_stage_u64(uint64_t& key) {
  key = xchg_u64<keep_min_mask(K, J, SEG, 0), J>(key);
  if constexpr (J > 1) bsort_stage_u64<SEG, K, J / 2>(key);
  else if constexpr (K < SEG) bsort_stage_u64<SEG, K * 2, K>(key);
}
template <int SEG, int K, int J>
__device__ __forceinline__ void bsort_stage_u32(uint32_t& key) {
  key = xchg_u32<keep_min_mask(K, J, SEG, 0), J>(key);
  if constexpr (J > 1) bsort_stage_u32<SEG, K, J / 2>(key);
  else if constexpr (K < SEG) bsort_stage_u32<SEG, K * 2, K>(key);
}

// Bitonic sort of one u64 key per lane, ascending in segments of SEG lanes
// (SEG a power of two, 2..64).
template <int SEG>
__device__ __forceinline__ uint64_t bitonic_sort_u64(uint64_t key) {
  bsort_stage_u64<SEG, 2, 1>(key);
  return key;
}

template <int SEG>
__device__ __forceinline__ uint32_t bitonic_sort_u32(uint32_t key) {
  bsort_stage_u32<SEG, 2, 1>(key);
  return key;
}

// One stage (K, J) over NR registers, registers R.. (recursion over R).
template <int NR, int K, int J, int R>
__device__ __forceinline__ void bregs_stage(uint64_t (&v)[NR]) {
  if constexpr (R < NR) {
    if constexpr (J >= 64) {
      constexpr int jr = J >> 6;
      if constexpr ((R & jr) == 0) {
        // partner in register R | jr of the same lane; the direction depends on R only
        constexpr bool up = (K >= 64 * NR) || (((R << 6) & K) == 0);
        const uint64_t a = v[R], b = v[R | jr];
        const bool sw = (a > b) == up;
        v[R] = sw ? b : a;
        v[R | jr] = sw ? a : b;
      }
    } else {
      v[R] = xchg_u64<keep_min_mask(K, J, 64 * NR, R), J>(v[R]);
    }
    bregs_stage<NR, K, J, R + 1>(v);
  }
}
template <int NR, int K, int J>
__device__ __forceinline__ void bregs_sort(uint64_t (&v)[NR]) {
  bregs_stage<NR, K, J, 0>(v);
  if constexpr (J > 1) bregs_sort<NR, K, J / 2>(v);
  else if constexpr (K < 64 * NR) bregs_sort<NR, K * 2, K>(v);
}

// Bitonic sort of 64 * NR u64 keys held NR per lane (key index r * 64 + lane),
// ascending over the whole wave.
template <int NR>
__device__ __forceinline__ void bitonic_sort_regs(uint64_t (&v)[NR]) {
  bregs_sort<NR, 2, 1>(v);
}

template <int J>
__device__ __forceinline__ void bmerge_stage(uint64_t& key) {
  key = xchg_u64<keep_min_mask(64, J, 64, 0), J>(key);
  if constexpr (J > 1) bmerge_stage<J / 2>(key);
}
// Sorts a bitonic sequence of 64 keys (one per lane) ascending.
__device__ __forceinline__ uint64_t bitonic_merge_u64(uint64_t key) {
  bmerge_stage<32>(key);
  return key;
}

// The smaller half of each segment of SEG keys, unordered, in the segment's
// lower SEG/2 lanes: the halves are sorted in opposite directions and one
// compare-exchange across them keeps the minima below (the first step of the
// final bitonic merge; the remaining log2(SEG) - 1 steps would only order them).
template <int SEG, int K, int J>
__device__ __forceinline__ void bsel_stage_u32(uint32_t& key) {
  key = xchg_u32<keep_min_mask(K, J, SEG, 0), J>(key);
  if constexpr (J > 1) bsel_stage_u32<SEG, K, J / 2>(key);
  else if constexpr (K < SEG / 2) bsel_stage_u32<SEG, K * 2, K>(key);
}
template <int SEG>
__device__ __forceinline__ uint32_t bitonic_lower_half_u32(uint32_t key) {
  if constexpr (SEG > 2) bsel_stage_u32<SEG, 2, 1>(key);
  return xchg_u32<keep_min_mask(SEG, SEG / 2, SEG, 0), SEG / 2>(key);
}
__device__ __forceinline__ uint32_t bitonic_lower_half_u32_seg(uint32_t key, int seg) {
  switch (seg) {
    case 2: return bitonic_lower_half_u32<2>(key);
    case 4: return bitonic_lower_half_u32<4>(key);
    case 8: return bitonic_lower_half_u32<8>(key);
    case 16: return bitonic_lower_half_u32<16>(key);
    case 32: return bitonic_lower_half_u32<32>(key);
    default: return bitonic_lower_half_u32<64>(key);
  }
}

// Runtime-segment dispatch (seg in {2,4,...,64}).
__device__ __forceinline__ uint32_t bitonic_sort_u32_seg(uint32_t key, int seg) {
  switch (seg) {
    case 2: return bitonic_sort_u32<2>(key);
    case 4: return bitonic_sort_u32<4>(key);
    case 8: return bitonic_sort_u32<8>(key);
    case 16: return bitonic_sort_u32<16>(key);
    case 32: return bitonic_sort_u32<32>(key);
    default: return bitonic_sort_u32<64>(key);
  }
}

// ---------------------------------------------------------------------------
// Storage formats.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float f16_bits_to_f32(uint32_t h) {
  _Float16 v = __builtin_bit_cast(_Float16, (uint16_t)h);
  return (float)v;
}

// OCP FP8 E4M3 ("fn") -> float. gfx950's conversion instruction implements the
// OCP encoding; the search's distance parity with the CPU oracle checks it.
__device__ __forceinline__ void fp8x4_to_f32(uint32_t w, float* out) {
  auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  out[0] = lo[0];
  out[1] = lo[1];
  out[2] = hi[0];
  out[3] = hi[1];
}

template <int DT>
struct Fmt;
template <>
struct Fmt<DT_F32> { static constexpr int esize = 4; static constexpr int per16 = 4; };
template <>
struct Fmt<DT_F16> { static constexpr int esize = 2; static constexpr int per16 = 8; };
template <>
struct Fmt<DT_FP8> { static constexpr int esize = 1; static constexpr int per16 = 16; };
template <>
struct Fmt<DT_U8> { static constexpr int esize = 1; static constexpr int per16 = 16; };

// Decode one 16-byte chunk into floats (traversal values before the scale).
template <int DT>
__device__ __forceinline__ void decode16(const uint4& c, float* out) {
  if constexpr (DT == DT_F32) {
    out[0] = __uint_as_float(c.x); out[1] = __uint_as_float(c.y);
    out[2] = __uint_as_float(c.z); out[3] = __uint_as_float(c.w);
  } else if constexpr (DT == DT_F16) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
      out[2 * i] = f16_bits_to_f32(w[i] & 0xFFFFu);
      out[2 * i + 1] = f16_bits_to_f32(w[i] >> 16);
    }
  } else if constexpr (DT == DT_FP8) {
    fp8x4_to_f32(c.x, out); fp8x4_to_f32(c.y, out + 4);
    fp8x4_to_f32(c.z, out + 8); fp8x4_to_f32(c.w, out + 12);
  } else {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 16; i++) out[i] = (float)((w[i >> 2] >> (8 * (i & 3))) & 0xFFu);
  }
}

// Element i of a stored row (used for scalar, per-element access).
template <int DT>
__device__ __forceinline__ float load_elem(const void* row, int i) {
  if constexpr (DT == DT_F32) return ((const float*)row)[i];
  else if constexpr (DT == DT_F16) return f16_bits_to_f32(((const uint16_t*)row)[i]);
  else if constexpr (DT == DT_FP8) {
    uint32_t b = ((const uint8_t*)row)[i];
    float o[4];
    fp8x4_to_f32(b, o);
    return o[0];
  } else return (float)((const uint8_t*)row)[i];
}

}  // namespace miann
