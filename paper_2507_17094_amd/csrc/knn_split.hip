// Candidate selection of the exact k-NN (graph build and ground truth) on the
// bf16 matrix cores. The build starts from exact neighbour lists (the graph
// construction the search runs on, Sec. 5); the GEMM form
// |a|^2 + |b|^2 - 2 a.b, with every operand split into two bf16 halves
// (x = hi + lo, three products hi.hi + hi.lo + lo.hi accumulated in f32,
// relative error about 2^-16 of |a||b|), only picks the kp best columns of
// each row, which the direct-form rescoring then orders exactly.
//
// A block of four waves owns 128 A rows; every wave keeps its 32 rows' hi and
// lo fragments in registers and streams all of B through LDS in tiles of 64
// columns (the next tile is read into registers while the current one is
// multiplied). Each row keeps a list of candidate keys (G bits << 32 | column)
// in global memory with its length in LDS: a column joins when its G is below
// the row's threshold, the kp-th smallest G kept so far. A list within 64 of
// its capacity is sorted and cut to its kp best by its wave, which tightens
// the threshold; after the last tile every list is cut and written out.
//
// uint8 rows take the integer matrix cores instead: shifted to int8 (x - 128,
// which leaves every difference and so every distance unchanged), products on
// v_mfma_i32_32x32x32_i8 are exact, and so is the GEMM form itself (integers
// below 2^24 held in f32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "knn.hpp"
#include "pool.hpp"

namespace miann {
namespace {

typedef __bf16 kbf16x8_t __attribute__((ext_vector_type(8)));
typedef float kf32x16_t __attribute__((ext_vector_type(16)));
typedef int ki32x4_t __attribute__((ext_vector_type(4)));
typedef int ki32x16_t __attribute__((ext_vector_type(16)));

constexpr int KR = 128;    // A rows per block (4 waves x 32)
constexpr int KT = 64;     // B columns per tile
constexpr int KCAP = 256;  // candidate keys a row holds before it is cut

__host__ __device__ constexpr int kstride(int dk) { return dk + 8; }  // LDS row stride (elements)
__host__ __device__ constexpr int kstride8(int dk) { return dk + 16; }  // int8 tiles: LDS row stride (bytes)

// 64 B rows x DK bf16 (hi and lo) staged by 256 threads: thread t owns tile row t / 4 and its 16-byte chunks
// c = t % 4 + 4 m (DK / 32 chunks per array).
template <int DK>
struct TileRegs {
  static constexpr int NCH = DK / 32;
  u32x4_t h[NCH], l[NCH];
  __device__ __forceinline__ void load(const uint16_t* __restrict__ H, const uint16_t* __restrict__ L, int64_t row,
                                       int c0) {
    const u32x4_t* hp = (const u32x4_t*)(H + row * DK) + c0;
    const u32x4_t* lp = (const u32x4_t*)(L + row * DK) + c0;
#pragma unroll
    for (int m = 0; m < NCH; m++) {
      h[m] = hp[4 * m];
      l[m] = lp[4 * m];
    }
  }
  __device__ __forceinline__ void store(uint16_t* Sh, uint16_t* Sl, int r, int c0) const {
    constexpr int P = kstride(DK);
#pragma unroll
    for (int m = 0; m < NCH; m++) {
      *(u32x4_t*)&Sh[r * P + (c0 + 4 * m) * 8] = h[m];
      *(u32x4_t*)&Sl[r * P + (c0 + 4 * m) * 8] = l[m];
    }
  }
};

// The same for int8 rows of DK bytes (DK / 64 chunks per thread).
template <int DK>
struct TileRegs8 {
  static constexpr int NCH = DK / 64;
  u32x4_t v[NCH];
  __device__ __forceinline__ void load(const int8_t* __restrict__ B, int64_t row, int c0) {
    const u32x4_t* p = (const u32x4_t*)(B + row * DK) + c0;
#pragma unroll
    for (int m = 0; m < NCH; m++) v[m] = p[4 * m];
  }
  __device__ __forceinline__ void store(int8_t* S, int r, int c0) const {
    constexpr int P = kstride8(DK);
#pragma unroll
    for (int m = 0; m < NCH; m++) *(u32x4_t*)&S[r * P + (c0 + 4 * m) * 16] = v[m];
  }
};

// Sorts row `row`'s list (n <= KCAP keys at L) and keeps its kp smallest; returns the kp-th smallest key (or
// kDummy when fewer than kp are held). One wave; the list was written by this wave.
__device__ __forceinline__ uint64_t cut_list(uint64_t* __restrict__ L, int n, int kp, int lane, uint64_t* dst) {
  // the wave's own global writes of the list are complete and visible before it is read back
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  uint64_t v[4];
#pragma unroll
  for (int r = 0; r < 4; r++) v[r] = r * 64 + lane < n ? L[r * 64 + lane] : kDummy;
  bitonic_sort_regs<4>(v);
#pragma unroll
  for (int r = 0; r < 4; r++)
    if (r * 64 + lane < kp) dst[r * 64 + lane] = v[r];
  const int i = kp - 1;
  uint64_t kth = kDummy;
#pragma unroll
  for (int r = 0; r < 4; r++)
    if ((i >> 6) == r) {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v[r], i & 63);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v[r] >> 32), i & 63);
      kth = ((uint64_t)hi << 32) | lo;
    }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  return kth;
}

// One block: rows [r0, r0 + 128) of A against all columns of B. A (na_pad rows) and B (nb_tiles * 64 rows)
// are hi / lo bf16 splits (I8: int8 rows, lo unused) with f32 norms; padding rows and columns carry norm +inf
// and never qualify. lists: [rows of this launch][KCAP] scratch; out: [rows][kp] keys, ascending.
template <int DK, bool I8>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DK <= 128 || I8 ? 2 : 1))) void knn_split_kernel(const void* __restrict__ Ah_, const void* __restrict__ Al_,
                                                        const float* __restrict__ an, int64_t na, int64_t row0,
                                                        const void* __restrict__ Bh_, const void* __restrict__ Bl_,
                                                        const float* __restrict__ bn, int64_t nb_tiles, int kp,
                                                        int exclude_self, uint64_t* __restrict__ lists,
                                                        uint64_t* __restrict__ out) {
  constexpr int P = kstride(DK);
  constexpr int KB = I8 ? DK / 32 : DK / 16;
  constexpr size_t kTileBytes = I8 ? (size_t)KT * kstride8(DK) : (size_t)2 * KT * P * 2;
  extern __shared__ __align__(16) char ksm[];
  uint16_t* Sh = (uint16_t*)ksm;
  uint16_t* Sl = Sh + KT * P;
  int8_t* S8 = (int8_t*)ksm;
  float* thr_s = (float*)(ksm + kTileBytes);
  int* cnt_s = (int*)(thr_s + KR);
  float* an_s = (float*)(cnt_s + KR);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int h = lane >> 5, col = lane & 31, wr = wave * 32;
  const int64_t rb0 = row0 + (int64_t)blockIdx.x * KR;  // first A row of the block
  uint64_t* blk_lists = lists + (int64_t)blockIdx.x * KR * KCAP;
  // this lane's A fragments: row wr + col, elements kb * 16 + h * 8 .. + 8 (I8: bytes kb * 32 + h * 16 .. + 16)
  kbf16x8_t ah[I8 ? 1 : KB], al[I8 ? 1 : KB];
  ki32x4_t a8[I8 ? KB : 1];
  if constexpr (I8) {
    const ki32x4_t* p8 = (const ki32x4_t*)((const int8_t*)Ah_ + (rb0 + wr + col) * DK + h * 16);
#pragma unroll
    for (int kb = 0; kb < KB; kb++) a8[kb] = p8[2 * kb];
  } else {
    const kbf16x8_t* hp = (const kbf16x8_t*)((const uint16_t*)Ah_ + (rb0 + wr + col) * DK + h * 8);
    const kbf16x8_t* lp = (const kbf16x8_t*)((const uint16_t*)Al_ + (rb0 + wr + col) * DK + h * 8);
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
      ah[kb] = hp[2 * kb];
      al[kb] = lp[2 * kb];
    }
  }
  if (tid < KR) {
    thr_s[tid] = INFINITY;
    cnt_s[tid] = 0;
    an_s[tid] = an[rb0 + tid];
  }
  // the candidate test's row term for the lane's 16 output rows wr + 8 (j / 4) + 4 h + j % 4:
  // tq = (qn - thr) / 2 (a column qualifies when G = qn + gn - 2 a.b < thr, i.e. a.b > tq + gn / 2; with
  // thr = +inf every column does, padding columns (gn = +inf) and rows (qn = +inf) never: NaN compares false).
  // The row norms stay in LDS: they are needed only to form a candidate's key and after a cut.
  float tq[16];
#pragma unroll
  for (int j = 0; j < 16; j++) tq[j] = -INFINITY;
  const int sr = tid >> 2, sc0 = tid & 3;
  TileRegs<I8 ? 32 : DK> nb;
  TileRegs8<I8 ? DK : 64> nb8;
  if constexpr (I8) nb8.load((const int8_t*)Bh_, sr, sc0);
  else nb.load((const uint16_t*)Bh_, (const uint16_t*)Bl_, sr, sc0);
  // the column norms of this lane's two columns, read one tile ahead like the tile itself
  float gnx[2] = {bn[col], bn[32 + col]};
  for (int64_t tt = 0; tt < nb_tiles; tt++) {
    const int64_t nxt = (tt + 1 < nb_tiles ? tt + 1 : tt) * KT + sr;  // (the last tile reloads itself)
    const float gcols[2] = {gnx[0], gnx[1]};
    {
      const int64_t nt = (tt + 1 < nb_tiles ? tt + 1 : tt) * KT;
      gnx[0] = bn[nt + col];
      gnx[1] = bn[nt + 32 + col];
    }
    __syncthreads();  // the previous tile is consumed
    if constexpr (I8) {
      nb8.store(S8, sr, sc0);
      nb8.load((const int8_t*)Bh_, nxt, sc0);
    } else {
      nb.store(Sh, Sl, sr, sc0);
      nb.load((const uint16_t*)Bh_, (const uint16_t*)Bl_, nxt, sc0);
    }
    __syncthreads();
    kf32x16_t acc[2];
    if constexpr (I8) {
      ki32x16_t acc8[2];
#pragma unroll
      for (int c = 0; c < 2; c++)
#pragma unroll
        for (int j = 0; j < 16; j++) acc8[c][j] = 0;
#pragma unroll
      for (int kb = 0; kb < KB; kb++) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
          const ki32x4_t b8 = *(const ki32x4_t*)&S8[(32 * c + col) * kstride8(DK) + kb * 32 + h * 16];
          acc8[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a8[kb], b8, acc8[c], 0, 0, 0);
        }
      }
#pragma unroll
      for (int c = 0; c < 2; c++)
#pragma unroll
        for (int j = 0; j < 16; j++) acc[c][j] = (float)acc8[c][j];
    } else {
#pragma unroll
      for (int c = 0; c < 2; c++)
#pragma unroll
        for (int j = 0; j < 16; j++) acc[c][j] = 0.f;
#pragma unroll
      for (int kb = 0; kb < KB; kb++) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
          const int rb = (32 * c + col) * P + kb * 16 + h * 8;
          const kbf16x8_t bh = *(const kbf16x8_t*)&Sh[rb], bl = *(const kbf16x8_t*)&Sl[rb];
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kb], bh, acc[c], 0, 0, 0);
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kb], bl, acc[c], 0, 0, 0);
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[kb], bh, acc[c], 0, 0, 0);
        }
      }
    }
    // candidates: G below the row's threshold, appended to the row's list (the key holds G itself, clamped
    // at 0); the two tiles that meet the block's own rows also skip the row's own column in a self join (a
    // separate copy of the scan, so that the common one is a compare and a branch per row and column half)
    auto scan = [&](auto self_tag) {
      constexpr bool kSelf = decltype(self_tag)::value;
#pragma unroll
      for (int c = 0; c < 2; c++) {
        const int64_t gc = tt * KT + 32 * c + col;
        const float gcol = gcols[c];
        const float gh = 0.5f * gcol;
#pragma unroll
        for (int j = 0; j < 16; j++) {
          const int row = wr + 8 * (j >> 2) + 4 * h + (j & 3);
          bool cand = acc[c][j] > tq[j] + gh;
          if constexpr (kSelf) cand = cand && gc != rb0 + row;
          const uint64_t bm = __ballot(cand);
          if (bm) {
            const uint32_t hm = h ? (uint32_t)(bm >> 32) : (uint32_t)bm;
            const int base = cnt_s[row];
            float v = an_s[row] + gcol - 2.f * acc[c][j];
            v = v < 0.f ? 0.f : v;
            if (cand)
              blk_lists[(int64_t)row * KCAP + base + __popc(hm & ((1u << col) - 1u))] =
                  ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)gc;
            if (col == 0) cnt_s[row] = base + __popc(hm);
          }
        }
      }
    };
    if (exclude_self && tt * KT < rb0 + KR && tt * KT + KT > rb0) scan(std::true_type{});
    else scan(std::false_type{});
    // lists that could overflow in the next tile (64 more keys at most) are cut to their kp best
    const int cr = cnt_s[wr + (lane & 31)];
    uint64_t need = __ballot(lane < 32 && cr > KCAP - KT);
    if (need) {
      while (need) {
        const int rr = __builtin_ctzll(need);
        need &= need - 1;
        const int row = wr + rr;
        uint64_t* L = blk_lists + (int64_t)row * KCAP;
        const int n = cnt_s[row];
        const uint64_t kth = cut_list(L, n, kp, lane, L);
        if (lane == 0) {
          cnt_s[row] = n < kp ? n : kp;
          thr_s[row] = kth == kDummy ? INFINITY : __uint_as_float((uint32_t)(kth >> 32));
        }
      }
#pragma unroll
      for (int j = 0; j < 16; j++) {
        const int row = wr + 8 * (j >> 2) + 4 * h + (j & 3);
        tq[j] = 0.5f * (an_s[row] - thr_s[row]);
      }
    }
  }
  // every row's kp best, ascending (kDummy past the columns it has)
  for (int rr = 0; rr < 32; rr++) {
    const int row = wr + rr;
    if (rb0 + row >= na) break;
    (void)cut_list(blk_lists + (int64_t)row * KCAP, cnt_s[row], kp, lane, out + (rb0 + row - row0) * kp);
  }
}

size_t knn_split_lds(int dk, bool i8) {
  return (i8 ? (size_t)KT * kstride8(dk) : (size_t)2 * KT * kstride(dk) * 2) + KR * 12;
}

template <int DK, bool I8>
hipError_t launch_knn_split(dim3 grid, hipStream_t st, const void* Ah, const void* Al, const float* an, int64_t na,
                            int64_t row0, const void* Bh, const void* Bl, const float* bn, int64_t nb_tiles, int kp,
                            int exclude_self, uint64_t* lists, uint64_t* out) {
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute((const void*)knn_split_kernel<DK, I8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
  });
  hipLaunchKernelGGL((knn_split_kernel<DK, I8>), grid, dim3(256), knn_split_lds(DK, I8), st, Ah, Al, an, na, row0,
                     Bh, Bl, bn, nb_tiles, kp, exclude_self, lists, out);
  return hipGetLastError();
}

// int8 rows (x - 128) of dk8 bytes and their f32 norms from f32 copies of uint8 rows ([n][dpf], integral values);
// elements past dpf are 0, rows n..n_pad are zeros with norm +inf. One wave per row.
__global__ __launch_bounds__(256) void shift_rows_i8_kernel(const float* __restrict__ x, int64_t n, int64_t n_pad,
                                                            int dpf, int dk8, int8_t* __restrict__ out,
                                                            float* __restrict__ norm) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n_pad) return;
  const int lane = threadIdx.x & 63;
  int s = 0;
  for (int c = lane; c < dk8; c += 64) {
    const int v = (r < n && c < dpf) ? (int)x[r * dpf + c] - 128 : 0;
    out[r * dk8 + c] = (int8_t)v;
    s += v * v;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o);
  if (lane == 0) norm[r] = r < n ? (float)s : INFINITY;
}

}  // namespace

static int dk8_of(int dpf) { return (dpf + 63) / 64 * 64; }

bool knn_split_supported(int dpf, int kp, int u8) {
  if (kp < 1 || kp > KCAP - KT || dpf < 1) return false;
  return u8 ? dk8_of(dpf) <= 256 : (dpf % 32 == 0 && dpf <= 256);
}

hipError_t knn_split_select(const float* A_f32, int64_t na, const float* B_f32, int64_t nb, int dpf, int kp,
                            int exclude_self, int u8, uint64_t* out, hipStream_t st) {
  if (na == 0) return hipSuccess;
  if (!knn_split_supported(dpf, kp, u8)) return hipErrorInvalidValue;
  const int dk = u8 ? dk8_of(dpf) : dpf;
  const size_t ebytes = u8 ? 1 : 4;  // bytes per element of the prepared rows (int8, or hi and lo bf16)
  // a self join (A is B) prepares the rows once, padded for both roles
  const bool same = A_f32 == B_f32 && na == nb;
  const int64_t na_pad = (na + KR - 1) / KR * KR, nb_pad = same ? na_pad : (nb + KT - 1) / KT * KT;
  // rows per launch: the candidate lists of at most 2^21 rows (4 GiB)
  const int64_t rows_per = std::min<int64_t>(na_pad, (int64_t)1 << 21);
  char *ab = nullptr, *bb = nullptr;
  float *an = nullptr, *bnrm = nullptr;
  uint64_t* lists = nullptr;
  hipError_t e = pool_malloc_async(&bb, (size_t)nb_pad * dk * ebytes, st);
  if (e == hipSuccess) e = pool_malloc_async(&bnrm, (size_t)nb_pad * 4, st);
  if (e == hipSuccess && !same) e = pool_malloc_async(&ab, (size_t)na_pad * dk * ebytes, st);
  if (e == hipSuccess && !same) e = pool_malloc_async(&an, (size_t)na_pad * 4, st);
  if (e == hipSuccess) e = pool_malloc_async(&lists, (size_t)rows_per * KCAP * 8, st);
  auto prep = [&](const float* x, int64_t n, int64_t n_pad, char* buf, float* nrm) -> hipError_t {
    if (u8) {
      hipLaunchKernelGGL(shift_rows_i8_kernel, dim3((unsigned)((n_pad + 3) / 4)), dim3(256), 0, st, x, n, n_pad, dpf,
                         dk, (int8_t*)buf, nrm);
      return hipGetLastError();
    }
    return split_rows(x, n, n_pad, dk, (uint16_t*)buf, (uint16_t*)buf + (size_t)n_pad * dk, nrm, st);
  };
  if (e == hipSuccess) e = prep(B_f32, nb, nb_pad, bb, bnrm);
  if (e == hipSuccess && !same) e = prep(A_f32, na, na_pad, ab, an);
  const char* Ab = same ? bb : ab;
  const float* An = same ? bnrm : an;
  const void* Al = u8 || !Ab ? nullptr : (const void*)((const uint16_t*)Ab + (size_t)(same ? nb_pad : na_pad) * dk);
  const void* Bl = u8 || !bb ? nullptr : (const void*)((const uint16_t*)bb + (size_t)nb_pad * dk);
  // MIANN_PROGRESS set: a line on stderr after each launch of a selection that takes several (the stream is
  // waited on for it)
  static const bool progress = std::getenv("MIANN_PROGRESS") != nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  for (int64_t row0 = 0; row0 < na_pad && e == hipSuccess; row0 += rows_per) {
    if (progress && row0 > 0 && hipStreamSynchronize(st) == hipSuccess)
      std::fprintf(stderr, "k-NN selection: %lld of %lld rows against %lld in %.1f s\n", (long long)row0,
                   (long long)na, (long long)nb,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
    const int64_t rows = std::min<int64_t>(rows_per, na_pad - row0);
    const dim3 grid((unsigned)(rows / KR));
    const int key = dk * 2 + (u8 ? 1 : 0);
    switch (key) {
#define MIANN_KNN(D, I)                                                                                              \
  case D * 2 + (I ? 1 : 0):                                                                                          \
    e = launch_knn_split<D, I>(grid, st, Ab, Al, An, na, row0, bb, Bl, bnrm, nb_pad / KT, kp, exclude_self, lists,   \
                               out + row0 * kp);                                                                     \
    break;
      MIANN_KNN(32, false)
      MIANN_KNN(64, false)
      MIANN_KNN(96, false)
      MIANN_KNN(128, false)
      MIANN_KNN(160, false)
      MIANN_KNN(192, false)
      MIANN_KNN(224, false)
      MIANN_KNN(256, false)
      MIANN_KNN(64, true)
      MIANN_KNN(128, true)
      MIANN_KNN(192, true)
      MIANN_KNN(256, true)
#undef MIANN_KNN
      default: e = hipErrorInvalidValue;
    }
  }
  if (lists) (void)hipFreeAsync(lists, st);
  if (an) (void)hipFreeAsync(an, st);
  if (ab) (void)hipFreeAsync(ab, st);
  if (bnrm) (void)hipFreeAsync(bnrm, st);
  if (bb) (void)hipFreeAsync(bb, st);
  return e;
}

}  // namespace miann
