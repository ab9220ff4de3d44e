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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "knn.hpp"
#include "pool.hpp"

namespace miann {
namespace {

typedef __bf16 kbf16x8_t __attribute__((ext_vector_type(8)));
typedef float kf32x16_t __attribute__((ext_vector_type(16)));

constexpr int KR = 128;    // A rows per block (4 waves x 32)
constexpr int KT = 64;     // B columns per tile
constexpr int KCAP = 256;  // candidate keys a row holds before it is cut

__host__ __device__ constexpr int kstride(int dk) { return dk + 8; }  // LDS row stride (elements)

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
// are hi / lo bf16 splits with f32 norms; padding rows and columns carry norm +inf and never qualify.
// lists: [rows of this launch][KCAP] scratch; out: [rows][kp] keys, ascending.
template <int DK>
__global__ __launch_bounds__(256) void knn_split_kernel(const uint16_t* __restrict__ Ah,
                                                        const uint16_t* __restrict__ Al, const float* __restrict__ an,
                                                        int64_t na, int64_t row0, const uint16_t* __restrict__ Bh,
                                                        const uint16_t* __restrict__ Bl,
                                                        const float* __restrict__ bn, int64_t nb_tiles, int kp,
                                                        int exclude_self, uint64_t* __restrict__ lists,
                                                        uint64_t* __restrict__ out) {
  constexpr int P = kstride(DK);
  constexpr int KB = DK / 16;
  extern __shared__ __align__(16) char ksm[];
  uint16_t* Sh = (uint16_t*)ksm;
  uint16_t* Sl = Sh + KT * P;
  float* thr_s = (float*)(Sl + KT * P);
  int* cnt_s = (int*)(thr_s + KR);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int h = lane >> 5, col = lane & 31, wr = wave * 32;
  const int64_t rb0 = row0 + (int64_t)blockIdx.x * KR;  // first A row of the block
  uint64_t* blk_lists = lists + (int64_t)blockIdx.x * KR * KCAP;
  // this lane's A fragments: row wr + col, elements kb * 16 + h * 8 .. + 8
  kbf16x8_t ah[KB], al[KB];
  {
    const kbf16x8_t* hp = (const kbf16x8_t*)(Ah + (rb0 + wr + col) * DK + h * 8);
    const kbf16x8_t* lp = (const kbf16x8_t*)(Al + (rb0 + wr + col) * DK + h * 8);
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
      ah[kb] = hp[2 * kb];
      al[kb] = lp[2 * kb];
    }
  }
  if (tid < KR) {
    thr_s[tid] = INFINITY;
    cnt_s[tid] = 0;
  }
  // the lane's 16 output rows wr + 8 (j / 4) + 4 h + j % 4: norms and thresholds
  float qr[16], tr[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    qr[j] = an[rb0 + wr + 8 * (j >> 2) + 4 * h + (j & 3)];
    tr[j] = INFINITY;
  }
  const int sr = tid >> 2, sc0 = tid & 3;
  TileRegs<DK> nb;
  nb.load(Bh, Bl, sr, sc0);
  for (int64_t tt = 0; tt < nb_tiles; tt++) {
    __syncthreads();  // the previous tile is consumed
    nb.store(Sh, Sl, sr, sc0);
    nb.load(Bh, Bl, (tt + 1 < nb_tiles ? tt + 1 : tt) * KT + sr, sc0);  // (the last tile reloads itself)
    __syncthreads();
    kf32x16_t acc[2];
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
    // candidates: G below the row's threshold (a NaN or +inf G never is); appended to the row's list
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const int64_t gc = tt * KT + 32 * c + col;
      const float gcol = bn[gc];
#pragma unroll
      for (int j = 0; j < 16; j++) {
        const int row = wr + 8 * (j >> 2) + 4 * h + (j & 3);
        float v = qr[j] + gcol - 2.f * acc[c][j];
        v = v < 0.f ? 0.f : v;
        const bool cand = v < tr[j] && !(exclude_self && gc == rb0 + row);
        const uint64_t bm = __ballot(cand);
        if (bm) {
          const uint32_t hm = h ? (uint32_t)(bm >> 32) : (uint32_t)bm;
          const int base = cnt_s[row];
          if (cand)
            blk_lists[(int64_t)row * KCAP + base + __popc(hm & ((1u << col) - 1u))] =
                ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)gc;
          if (col == 0) cnt_s[row] = base + __popc(hm);
        }
      }
    }
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
      for (int j = 0; j < 16; j++) tr[j] = thr_s[wr + 8 * (j >> 2) + 4 * h + (j & 3)];
    }
  }
  // every row's kp best, ascending (kDummy past the columns it has)
  for (int rr = 0; rr < 32; rr++) {
    const int row = wr + rr;
    if (rb0 + row >= na) break;
    (void)cut_list(blk_lists + (int64_t)row * KCAP, cnt_s[row], kp, lane, out + (rb0 + row - row0) * kp);
  }
}

size_t knn_split_lds(int dk) { return (size_t)2 * KT * kstride(dk) * 2 + KR * 8; }

template <int DK>
hipError_t launch_knn_split(dim3 grid, hipStream_t st, const uint16_t* Ah, const uint16_t* Al, const float* an,
                            int64_t na, int64_t row0, const uint16_t* Bh, const uint16_t* Bl, const float* bn,
                            int64_t nb_tiles, int kp, int exclude_self, uint64_t* lists, uint64_t* out) {
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute((const void*)knn_split_kernel<DK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
  });
  hipLaunchKernelGGL(knn_split_kernel<DK>, grid, dim3(256), knn_split_lds(DK), st, Ah, Al, an, na, row0, Bh, Bl, bn,
                     nb_tiles, kp, exclude_self, lists, out);
  return hipGetLastError();
}

}  // namespace

bool knn_split_supported(int dk, int kp) { return dk % 32 == 0 && dk >= 32 && dk <= 256 && kp >= 1 && kp <= KCAP - KT; }

hipError_t knn_split_select(const float* A_f32, int64_t na, const float* B_f32, int64_t nb, int dpf, int kp,
                            int exclude_self, uint64_t* out, hipStream_t st) {
  if (na == 0) return hipSuccess;
  if (!knn_split_supported(dpf, kp)) return hipErrorInvalidValue;
  const int dk = dpf;
  // a self join (A is B) splits the rows once, padded for both roles
  const bool same = A_f32 == B_f32 && na == nb;
  const int64_t na_pad = (na + KR - 1) / KR * KR, nb_pad = same ? na_pad : (nb + KT - 1) / KT * KT;
  // rows per launch: the candidate lists of at most 2^21 rows (4 GiB)
  const int64_t rows_per = std::min<int64_t>(na_pad, (int64_t)1 << 21);
  uint16_t *ah = nullptr, *bh = nullptr;
  float *an = nullptr, *bnrm = nullptr;
  uint64_t* lists = nullptr;
  hipError_t e = pool_malloc_async(&bh, (size_t)nb_pad * dk * 4, st);
  if (e == hipSuccess) e = pool_malloc_async(&bnrm, (size_t)nb_pad * 4, st);
  if (e == hipSuccess && !same) e = pool_malloc_async(&ah, (size_t)na_pad * dk * 4, st);
  if (e == hipSuccess && !same) e = pool_malloc_async(&an, (size_t)na_pad * 4, st);
  if (e == hipSuccess) e = pool_malloc_async(&lists, (size_t)rows_per * KCAP * 8, st);
  uint16_t* bl = bh ? bh + (size_t)nb_pad * dk : nullptr;
  if (e == hipSuccess) e = split_rows(B_f32, nb, nb_pad, dk, bh, bl, bnrm, st);
  if (e == hipSuccess && !same) e = split_rows(A_f32, na, na_pad, dk, ah, ah + (size_t)na_pad * dk, an, st);
  const uint16_t* Ah = same ? bh : ah;
  const uint16_t* Al = same ? bl : (ah ? ah + (size_t)na_pad * dk : nullptr);
  const float* An = same ? bnrm : an;
  for (int64_t row0 = 0; row0 < na_pad && e == hipSuccess; row0 += rows_per) {
    const int64_t rows = std::min<int64_t>(rows_per, na_pad - row0);
    const dim3 grid((unsigned)(rows / KR));
    switch (dk) {
#define MIANN_KNN(D)                                                                                           \
  case D:                                                                                                      \
    e = launch_knn_split<D>(grid, st, Ah, Al, An, na, row0, bh, bl, bnrm, nb_pad / KT, kp, exclude_self, lists, \
                            out + row0 * kp);                                                                  \
    break;
      MIANN_KNN(32)
      MIANN_KNN(64)
      MIANN_KNN(96)
      MIANN_KNN(128)
      MIANN_KNN(160)
      MIANN_KNN(192)
      MIANN_KNN(224)
      MIANN_KNN(256)
#undef MIANN_KNN
      default: e = hipErrorInvalidValue;
    }
  }
  if (lists) hipFreeAsync(lists, st);
  if (bnrm) hipFreeAsync(bnrm, st);
  if (an) hipFreeAsync(an, st);
  if (bh) hipFreeAsync(bh, st);
  if (ah) hipFreeAsync(ah, st);
  return e;
}

}  // namespace miann
