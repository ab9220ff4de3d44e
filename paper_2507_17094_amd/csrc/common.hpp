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
// mapping used is an involution, so none depends on a shift direction; the
// row swaps return the lane's own value in one output and its partner's in
// the other, and the partner's is the one that differs (or both are equal).
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
    return r[0] == v ? r[1] : r[0];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return r[0] == v ? r[1] : r[0];
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

// Number of set lanes of `mask` below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Bitonic sort of one u64 key per lane, ascending in segments of SEG lanes
// (SEG a power of two, 2..64).
template <int SEG>
__device__ __forceinline__ uint64_t bitonic_sort_u64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= SEG; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      // the lane keeps the smaller key iff it is the lower lane of an ascending pair or the upper
      // of a descending one; one compare decides, the lane pattern is a scalar mask
      const uint64_t other = xor_lane_u64(key, j);
      const bool want_min = ((lane & j) == 0) == ((k == SEG) || ((lane & k) == 0));
      key = ((other < key) == want_min) ? other : key;
    }
  }
  return key;
}

template <int SEG>
__device__ __forceinline__ uint32_t bitonic_sort_u32(uint32_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= SEG; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t other = xor_lane_u32(key, j);
      const bool want_min = ((lane & j) == 0) == ((k == SEG) || ((lane & k) == 0));
      key = ((other < key) == want_min) ? other : key;
    }
  }
  return key;
}

// Bitonic sort of 64 * NR u64 keys held NR per lane (key index r * 64 + lane),
// ascending over the whole wave.
template <int NR>
__device__ __forceinline__ void bitonic_sort_regs(uint64_t (&v)[NR]) {
  const int lane = lane_id();
  constexpr int N = 64 * NR;
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int jr = j >> 6;
#pragma unroll
        for (int r = 0; r < NR; r++) {
          if ((r & jr) == 0) {
            const int p = r | jr;
            const bool up = (((r << 6) | lane) & k) == 0;
            const uint64_t a = v[r], b = v[p];
            const bool sw = (a > b) == up;
            v[r] = sw ? b : a;
            v[p] = sw ? a : b;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; r++) {
          const uint64_t other = xor_lane_u64(v[r], j);
          const bool want_min = ((lane & j) == 0) == ((((r << 6) | lane) & k) == 0);
          v[r] = ((other < v[r]) == want_min) ? other : v[r];
        }
      }
    }
  }
}

// Sorts a bitonic sequence of 64 keys (one per lane) ascending.
__device__ __forceinline__ uint64_t bitonic_merge_u64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int j = 32; j > 0; j >>= 1) {
    const uint64_t other = xor_lane_u64(key, j);
    key = ((other < key) == ((lane & j) == 0)) ? other : key;
  }
  return key;
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
