/*
 * CPU oracle for the graph beam search of PathWeaver (arXiv 2507.17094).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * HIP path is checked against. It shares no code, header, table or constant
 * generator with the HIP library, and nothing in the product links it.
 *
 * Everything here is scalar C, one query per thread, with the steps written in
 * the order the paper gives them:
 *   - k-NN problem and L2 distance           : Sec. 2.1 (Eq. 1), Sec. 2.2 (Eq. 2)
 *   - beam search with priority queue p and
 *     candidate list c, Steps 1-4            : Sec. 2.2
 *   - path extension (inter-shard edge map I,
 *     staged search, reduction)              : Sec. 3.1.2 (the I(u) equation)
 *   - ghost staging (sampled auxiliary shard): Sec. 3.2.2
 *   - direction-guided selection (sign table,
 *     XOR + popcount, top-n, cool-down)      : Sec. 3.3.2 and Sec. 4
 *
 * Readings of points the paper leaves open (all documented in the design notes):
 *   - distances are SQUARED L2 (monotone in Eq. 2, so ranks are unchanged);
 *     float inputs: each difference q_i - x_i is rounded to float, its square
 *     (exact in double) is summed in double in index order, and the sum is
 *     rounded once to float; uint8 inputs use exact integer arithmetic.
 *   - every ordering is by the key (dist, id), ascending, id unsigned.
 *   - parents are the first r *unexpanded* entries of p; the search stops when
 *     no entry is eligible or after T iterations.
 *   - DGS ranks all slots by (mismatch, slot), keeps n_keep, then applies the
 *     visited filter; skipped neighbours are not marked visited; a parent
 *     expanded under DGS with slots skipped becomes "partial" and is eligible
 *     again in the cool-down.
 *   - random numbers come from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014),
 *     used as a counter-based generator: out(ctr) = mix(seed + ctr * gamma).
 *
 * Parity pins are in tests/test_oracle_*.py.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define DT_F32 0
#define DT_F16 1
#define DT_FP8 2
#define DT_U8 3

#define FLAG_FRESH 0
#define FLAG_PARTIAL 1
#define FLAG_DONE 2

#define NONE_ID 0xFFFFFFFFu
#define ORC_MAXS 16
#define ORC_MAX_GIVEN 4096 /* seeds per query accepted by orc_search */
#define NCTR 8

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014): the state advances by gamma and  */
/* each output is the state passed through the published mixing function. */
/* ------------------------------------------------------------------ */
static const uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ctr-th output (ctr >= 1) of a SplitMix64 generator seeded with `seed`. */
uint64_t orc_splitmix(uint64_t seed, uint64_t ctr) { return orc_mix64(seed + ctr * GAMMA); }

/* Stream seeds: one per (role, shard). */
uint64_t orc_stream_main(uint64_t seed, int shard) { return orc_splitmix(seed, (uint64_t)(2 * shard + 1)); }
uint64_t orc_stream_ghost(uint64_t seed, int shard) { return orc_splitmix(seed, (uint64_t)(2 * shard + 2)); }
uint64_t orc_stream_sample(uint64_t seed, int shard) { return orc_splitmix(seed, (uint64_t)(0x100 + shard)); }

/* ------------------------------------------------------------------ */
/* Number formats, decoded from their definitions.                     */
/* ------------------------------------------------------------------ */

/* IEEE binary16: 1 sign, 5 exponent (bias 15), 10 mantissa bits. */
float orc_f16_decode(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 0) v = ldexp((double)m, -24);
  else if (e == 31) v = m ? NAN : INFINITY;
  else v = ldexp((double)(1024 + m), e - 25);
  return (float)(s ? -v : v);
}

/* OCP FP8 E4M3 ("fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits,
 * no infinities, S.1111.111 is NaN, largest finite magnitude 448. */
float orc_fp8_decode(uint8_t b) {
  int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
  double v;
  if (e == 15 && m == 7) return NAN;
  if (e == 0) v = ldexp((double)m, -9);
  else v = ldexp((double)(8 + m), e - 10);
  return (float)(s ? -v : v);
}

/* Round-to-nearest-even onto a sorted table of the non-negative finite
 * values of a format; `codes` gives the bit pattern of each table entry.
 * Plain search over the table keeps the rounding rule visible. */
static int rne_pick(double a, const double* vals, int n) {
  /* vals ascending, a >= 0, a <= vals[n-1] */
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (vals[mid] <= a) lo = mid; else hi = mid;
  }
  if (vals[lo] == a) return lo;
  if (vals[hi] == a) return hi;
  double dl = a - vals[lo], dh = vals[hi] - a;
  if (dl < dh) return lo;
  if (dh < dl) return hi;
  return (lo % 2 == 0) ? lo : hi; /* tie: even code (mantissa LSB 0) */
}

static double fp8_vals[127];
static double f16_vals[31 * 1024]; /* non-negative finite codes 0..0x7BFF */
static pthread_once_t fmt_once = PTHREAD_ONCE_INIT;
static void fmt_init(void) {
  for (int c = 0; c < 127; c++) fp8_vals[c] = orc_fp8_decode((uint8_t)c);
  for (int c = 0; c < 31 * 1024; c++) f16_vals[c] = orc_f16_decode((uint16_t)c);
}

/* FP8 E4M3fn encode, round-to-nearest-even, saturating at +-448. */
uint8_t orc_fp8_encode(float x) {
  pthread_once(&fmt_once, fmt_init);
  if (isnan(x)) return 0x7F;
  uint8_t sign = signbit(x) ? 0x80 : 0;
  double a = fabs((double)x);
  if (a >= 448.0) return sign | 126; /* 126 = 0.1111.110 = 448 */
  return sign | (uint8_t)rne_pick(a, fp8_vals, 127);
}

/* IEEE binary16 encode, round-to-nearest-even (overflow -> inf). */
uint16_t orc_f16_encode(float x) {
  pthread_once(&fmt_once, fmt_init);
  if (isnan(x)) return 0x7E00;
  uint16_t sign = signbit(x) ? 0x8000 : 0;
  double a = fabs((double)x);
  /* halfway between 65504 and the next (virtual) step 65536 rounds to inf */
  if (a >= 65520.0) return sign | 0x7C00;
  if (a > 65504.0) return sign | 0x7BFF;
  return sign | (uint16_t)rne_pick(a, f16_vals, 31 * 1024);
}

/* Per-vector quantisation: FP8 scale s = max|x| / 448 (s = 1 for x = 0),
 * code = RNE_fp8(x / s); FP16 stores s = 1 and code = RNE_fp16(x). */
void orc_quantize(const float* x, int64_t n, int d, int dtype, void* codes, float* scale) {
  for (int64_t v = 0; v < n; v++) {
    const float* row = x + v * d;
    if (dtype == DT_FP8) {
      float mx = 0.f;
      for (int i = 0; i < d; i++) { float a = fabsf(row[i]); if (a > mx) mx = a; }
      float s = (mx == 0.f) ? 1.f : mx / 448.f;
      scale[v] = s;
      uint8_t* c = (uint8_t*)codes + v * d;
      for (int i = 0; i < d; i++) c[i] = orc_fp8_encode(row[i] / s);
    } else { /* DT_F16 */
      scale[v] = 1.f;
      uint16_t* c = (uint16_t*)codes + v * d;
      for (int i = 0; i < d; i++) c[i] = orc_f16_encode(row[i]);
    }
  }
}

/* ------------------------------------------------------------------ */
/* Vector store and the distance of Eq. 2 (squared).                   */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t dtype;
  int32_t d;
  int64_t n;
  const void* codes;  /* n x d elements of dtype, row-major */
  const float* scale; /* n per-vector scales (F16/FP8), else NULL */
} orc_store;

/* Traversal value of element i of vector v: f32(s_v * decode(code)). */
static inline float elem(const orc_store* st, int64_t v, int i) {
  int64_t o = v * st->d + i;
  switch (st->dtype) {
    case DT_F32: return ((const float*)st->codes)[o];
    case DT_F16: return st->scale[v] * orc_f16_decode(((const uint16_t*)st->codes)[o]);
    case DT_FP8: return st->scale[v] * orc_fp8_decode(((const uint8_t*)st->codes)[o]);
    default: return (float)((const uint8_t*)st->codes)[o];
  }
}

/* dist(q, x_v) = sum_i (q_i - x_v,i)^2. Float: the float differences, squared
 * exactly and summed in double in index order, rounded once to float. uint8:
 * exact integer. Returned as double, which holds either result exactly. */
static double dist_qv(const orc_store* st, const void* q, int64_t v) {
  const int d = st->d;
  if (st->dtype == DT_U8) {
    const uint8_t* a = (const uint8_t*)q;
    const uint8_t* b = (const uint8_t*)st->codes + v * d;
    int64_t acc = 0;
    for (int i = 0; i < d; i++) { int64_t t = (int64_t)a[i] - (int64_t)b[i]; acc += t * t; }
    return (double)acc;
  }
  const float* a = (const float*)q;
  double acc = 0.0;
  for (int i = 0; i < d; i++) {
    float t = a[i] - elem(st, v, i); /* the float difference */
    acc += (double)t * (double)t;    /* its square is exact in double */
  }
  return (double)(float)acc;
}

/* Pointer to the raw row of vector v (used when a stored vector is a query). */
static const void* row_ptr(const orc_store* st, int64_t v) {
  size_t b = st->dtype == DT_F32 ? 4 : st->dtype == DT_F16 ? 2 : 1;
  return (const char*)st->codes + (size_t)v * st->d * b;
}

double orc_dist(const orc_store* st, const void* q, int64_t v) { return dist_qv(st, q, v); }

/* ------------------------------------------------------------------ */
/* Keys: (dist, id) ascending.                                         */
/* ------------------------------------------------------------------ */
typedef struct {
  double d;
  uint32_t id;
  uint8_t flag;
  uint8_t from_c; /* 0 = already in p, 1 = new candidate (merge tie-break) */
} entry;

static inline int key_less(double da, uint32_t ia, double db, uint32_t ib) {
  return da < db || (da == db && ia < ib);
}

static int entry_cmp(const void* a, const void* b) {
  const entry* x = (const entry*)a;
  const entry* y = (const entry*)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  if (x->id < y->id) return -1;
  if (x->id > y->id) return 1;
  return (int)x->from_c - (int)y->from_c;
}

/* ------------------------------------------------------------------ */
/* Thread pool over independent rows.                                  */
/* ------------------------------------------------------------------ */
typedef void (*row_fn)(void* ctx, int64_t row, void* scratch);
typedef struct {
  row_fn fn;
  void* ctx;
  int64_t n;
  int64_t next;
  pthread_mutex_t mu;
  size_t scratch_bytes;
  void (*fini)(void* scratch);
} pool_job;

static int g_threads = 0;
void orc_set_threads(int t) { g_threads = t; }
int orc_get_threads(void) {
  if (g_threads > 0) return g_threads;
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

static void* pool_worker(void* arg) {
  pool_job* j = (pool_job*)arg;
  void* scratch = j->scratch_bytes ? calloc(1, j->scratch_bytes) : NULL;
  for (;;) {
    pthread_mutex_lock(&j->mu);
    int64_t r = j->next;
    j->next += 16;
    pthread_mutex_unlock(&j->mu);
    if (r >= j->n) break;
    int64_t e = r + 16 < j->n ? r + 16 : j->n;
    for (int64_t i = r; i < e; i++) j->fn(j->ctx, i, scratch);
  }
  if (j->fini && scratch) j->fini(scratch);
  free(scratch);
  return NULL;
}

static void run_rows(row_fn fn, void* ctx, int64_t n, size_t scratch_bytes) {
  pool_job j = {fn, ctx, n, 0, PTHREAD_MUTEX_INITIALIZER, scratch_bytes, NULL};
  int t = orc_get_threads();
  if (t > 64) t = 64;
  pthread_t th[64];
  for (int i = 0; i < t; i++) pthread_create(&th[i], NULL, pool_worker, &j);
  for (int i = 0; i < t; i++) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------ */
/* Exact k-NN (Eq. 1): the k smallest (dist, id) over all points.      */
/* ------------------------------------------------------------------ */
typedef struct {
  const orc_store* base;
  const orc_store* qs; /* queries as a store (so stored vectors can be queries) */
  int k;
  int exclude_self;    /* skip id == row (graph build on the base itself) */
  uint32_t* out_id;
  double* out_d;
} knn_ctx;

static void knn_row(void* vctx, int64_t row, void* scratch) {
  (void)scratch;
  knn_ctx* c = (knn_ctx*)vctx;
  const void* q = row_ptr(c->qs, row);
  int k = c->k, cnt = 0;
  uint32_t* ids = c->out_id + row * k;
  double* ds = c->out_d + row * k;
  for (int64_t v = 0; v < c->base->n; v++) {
    if (c->exclude_self && v == row) continue;
    double dv = dist_qv(c->base, q, v);
    if (cnt == k && !key_less(dv, (uint32_t)v, ds[k - 1], ids[k - 1])) continue;
    int pos = cnt < k ? cnt : k - 1;
    while (pos > 0 && key_less(dv, (uint32_t)v, ds[pos - 1], ids[pos - 1])) {
      ds[pos] = ds[pos - 1];
      ids[pos] = ids[pos - 1];
      pos--;
    }
    ds[pos] = dv;
    ids[pos] = (uint32_t)v;
    if (cnt < k) cnt++;
  }
  for (int i = cnt; i < k; i++) { ids[i] = NONE_ID; ds[i] = INFINITY; }
}

void orc_knn(const orc_store* base, const orc_store* queries, int k, int exclude_self,
             uint32_t* out_id, double* out_d) {
  knn_ctx c = {base, queries, k, exclude_self, out_id, out_d};
  run_rows(knn_row, &c, queries->n, 0);
}

/* ------------------------------------------------------------------ */
/* Fixed-degree graph: K0-NN lists reduced to `deg` by reverse-merge    */
/* pruning, each row sorted by (dist, id).                              */
/* ------------------------------------------------------------------ */
typedef struct {
  const orc_store* st;
  const uint32_t* knn; /* n x K0 */
  const double* knnd;
  int K0, deg, half;
  const int64_t* rev_off; /* CSR of reverse lists, each sorted by (dist, id) */
  const uint32_t* rev_id;
  uint32_t* out;
} prune_ctx;

static void prune_row(void* vctx, int64_t u, void* scratch) {
  (void)scratch;
  prune_ctx* c = (prune_ctx*)vctx;
  int deg = c->deg, cnt = 0;
  uint32_t row[1024];
  double rowd[1024];
  const uint32_t* L = c->knn + u * c->K0;
  const double* Ld = c->knnd + u * c->K0;
  /* (1) the first ceil(deg/2) nearest neighbours */
  for (int j = 0; j < c->half; j++) { row[cnt] = L[j]; rowd[cnt] = Ld[j]; cnt++; }
  /* (2) reverse neighbours, nearest first */
  for (int64_t t = c->rev_off[u]; t < c->rev_off[u + 1] && cnt < deg; t++) {
    uint32_t v = c->rev_id[t];
    int dup = 0;
    for (int j = 0; j < cnt; j++) if (row[j] == v) { dup = 1; break; }
    if (dup) continue;
    row[cnt] = v;
    rowd[cnt] = dist_qv(c->st, row_ptr(c->st, u), v);
    cnt++;
  }
  /* (3) the remaining k-NN entries */
  for (int j = c->half; j < c->K0 && cnt < deg; j++) {
    uint32_t v = L[j];
    int dup = 0;
    for (int i = 0; i < cnt; i++) if (row[i] == v) { dup = 1; break; }
    if (dup) continue;
    row[cnt] = v;
    rowd[cnt] = Ld[j];
    cnt++;
  }
  /* (4) sort the row by (dist, id) (insertion sort) */
  for (int i = 1; i < cnt; i++) {
    uint32_t v = row[i];
    double dv = rowd[i];
    int j = i;
    while (j > 0 && key_less(dv, v, rowd[j - 1], row[j - 1])) { row[j] = row[j - 1]; rowd[j] = rowd[j - 1]; j--; }
    row[j] = v;
    rowd[j] = dv;
  }
  for (int j = 0; j < deg; j++) c->out[u * deg + j] = j < cnt ? row[j] : NONE_ID;
}

typedef struct { double d; uint32_t v; } dv_pair;
static int dv_cmp(const void* a, const void* b) {
  const dv_pair* x = (const dv_pair*)a;
  const dv_pair* y = (const dv_pair*)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return x->v < y->v ? -1 : x->v > y->v ? 1 : 0;
}

/* Prune given K0-NN lists (rows sorted by (dist, id), no self) to `deg`. */
int orc_prune(const orc_store* st, const uint32_t* knn, const double* knnd, int K0, int deg, uint32_t* out) {
  int64_t n = st->n;
  if (deg > 1024 || K0 < deg) return 1;
  int half = (deg + 1) / 2;
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t v = 0; v < n; v++)
    for (int j = 0; j < half; j++) cnt[knn[v * K0 + j] + 1]++;
  for (int64_t u = 0; u < n; u++) cnt[u + 1] += cnt[u];
  int64_t total = cnt[n];
  dv_pair* rev = (dv_pair*)malloc(sizeof(dv_pair) * (size_t)(total ? total : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t v = 0; v < n; v++)
    for (int j = 0; j < half; j++) {
      uint32_t u = knn[v * K0 + j];
      rev[fill[u]].v = (uint32_t)v;
      rev[fill[u]].d = knnd[v * K0 + j]; /* dist(u, v) == dist(v, u) */
      fill[u]++;
    }
  for (int64_t u = 0; u < n; u++) qsort(rev + cnt[u], (size_t)(cnt[u + 1] - cnt[u]), sizeof(dv_pair), dv_cmp);
  uint32_t* rid = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(total ? total : 1));
  for (int64_t t = 0; t < total; t++) rid[t] = rev[t].v;
  prune_ctx c = {st, knn, knnd, K0, deg, half, cnt, rid, out};
  run_rows(prune_row, &c, n, 0);
  free(rid);
  free(fill);
  free(rev);
  free(cnt);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Direction table (Sec. 3.3.2 (a), Sec. 4): per edge (u, slot j, v),  */
/* bit i of word i/32 (LSB first) = [x_v[i] > x_u[i]]; pad bits 0.      */
/* Layout here: S[u][j][w].                                             */
/* ------------------------------------------------------------------ */
void orc_sign_table(const orc_store* st, const uint32_t* graph, int deg, uint32_t* out) {
  int d = st->d, W = (d + 31) / 32;
  for (int64_t u = 0; u < st->n; u++)
    for (int j = 0; j < deg; j++) {
      uint32_t v = graph[u * deg + j];
      uint32_t* o = out + ((size_t)u * deg + j) * W;
      for (int w = 0; w < W; w++) o[w] = 0;
      if (v == NONE_ID) continue;
      for (int i = 0; i < d; i++)
        if (elem(st, v, i) > elem(st, u, i)) o[i / 32] |= 1u << (i % 32);
    }
}

/* ------------------------------------------------------------------ */
/* Random partition and ghost sample, from SplitMix64 sort keys.       */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t key; uint32_t id; } key_id;
static int key_id_cmp(const void* a, const void* b) {
  const key_id* x = (const key_id*)a;
  const key_id* y = (const key_id*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->id < y->id ? -1 : x->id > y->id ? 1 : 0;
}

/* perm = ids ordered by (mix(seed + (i+1) gamma), i). */
void orc_keyed_order(uint64_t seed, int64_t n, uint32_t* perm) {
  key_id* a = (key_id*)malloc(sizeof(key_id) * (size_t)n);
  for (int64_t i = 0; i < n; i++) { a[i].key = orc_splitmix(seed, (uint64_t)i + 1); a[i].id = (uint32_t)i; }
  qsort(a, (size_t)n, sizeof(key_id), key_id_cmp);
  for (int64_t i = 0; i < n; i++) perm[i] = a[i].id;
  free(a);
}

/* ------------------------------------------------------------------ */
/* Visited set V (exact), plus two forgetful policies used to check    */
/* that the result does not depend on the policy.                      */
/* ------------------------------------------------------------------ */
#define VP_EXACT 0
#define VP_FORGET_EACH_ITER 1
#define VP_SMALL_HASH 2
#define SMALL_HASH 128

typedef struct {
  int policy;
  uint8_t* bits;     /* exact: one byte per node (graph size) */
  uint32_t* touched; /* ids set in bits, to clear them */
  int64_t ntouched, cap_touched;
  uint32_t hash[SMALL_HASH];
  int hfill;
} visited;

static void vis_clear(visited* V) {
  for (int64_t i = 0; i < V->ntouched; i++) V->bits[V->touched[i]] = 0;
  V->ntouched = 0;
  for (int i = 0; i < SMALL_HASH; i++) V->hash[i] = NONE_ID;
  V->hfill = 0;
}

/* returns 1 if id was already in V; otherwise inserts it (when it can) and returns 0 */
static int vis_test_insert(visited* V, uint32_t id) {
  if (V->policy == VP_SMALL_HASH) {
    uint32_t h = (id * 0x9E3779B1u) >> 25; /* 7 bits */
    for (int t = 0; t < 8; t++) {
      uint32_t s = (h + t) & (SMALL_HASH - 1);
      if (V->hash[s] == id) return 1;
      if (V->hash[s] == NONE_ID) {
        if (V->hfill >= SMALL_HASH / 2) return 0; /* full enough: forget (do not insert) */
        V->hash[s] = id;
        V->hfill++;
        return 0;
      }
    }
    return 0;
  }
  if (V->bits[id]) return 1;
  V->bits[id] = 1;
  if (V->ntouched == V->cap_touched) {
    V->cap_touched = V->cap_touched ? 2 * V->cap_touched : 1024;
    V->touched = (uint32_t*)realloc(V->touched, sizeof(uint32_t) * (size_t)V->cap_touched);
  }
  V->touched[V->ntouched++] = id;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Beam search on one graph (Sec. 2.2 Steps 1-4, with Sec. 3.3.2).     */
/* ------------------------------------------------------------------ */
typedef struct {
  const orc_store* st; /* traversal representation */
  const uint32_t* graph;
  int deg;
  const uint32_t* sign; /* S[u][j][W] or NULL */
  int W;
} graph_view;

typedef struct {
  int l, r, T, n_init, k;
  int dgs_on, n_keep, cooldown_pm, random_discard;
  int visited_policy, stop_on_no_change;
  int dgs_thr; /* < 0: keep the n_keep best-ranked slots; >= 0: keep every slot whose mismatch is <= dgs_thr */
} beam_cfg;

typedef struct {
  entry* p;      /* l */
  entry* c;      /* r * deg + seeds */
  entry* merged; /* l + cap_c */
  int cap_c;
  visited V;
} beam_scratch;

static void merge_into_p(entry* p, int l, entry* c, int nc, entry* tmp, int* changed, int k, int* topk_changed) {
  /* p <- first l of sort(p U c); an id present twice keeps its p entry. */
  int n = 0;
  for (int i = 0; i < l; i++) { tmp[n] = p[i]; tmp[n].from_c = 0; n++; }
  for (int i = 0; i < nc; i++) { tmp[n] = c[i]; tmp[n].from_c = 1; n++; }
  qsort(tmp, (size_t)n, sizeof(entry), entry_cmp);
  int m = 0, ch = 0;
  for (int i = 0; i < n && m < l; i++) {
    if (m > 0 && tmp[i].id != NONE_ID && tmp[i].id == p[m - 1].id) continue; /* duplicate id */
    if (tmp[i].from_c && tmp[i].id != NONE_ID) {
      ch = 1;
      if (topk_changed && m < k) *topk_changed = 1;
    }
    p[m] = tmp[i];
    p[m].from_c = 0;
    m++;
  }
  if (changed) *changed = ch;
}

static inline int popc32(uint32_t x) {
  int c = 0;
  while (x) { x &= x - 1; c++; }
  return c;
}

/* One search. seeds (may be NULL) are node ids of this graph, in order.
 * On return p[0..l) holds the final priority queue. ctr[0..3] accumulate
 * n_dist, n_exp, iters, n_dgs_skipped; ctr[4] is set to the last iteration
 * (1-based, 0 = none) in which the first k entries of p changed. */
static void beam_search(const graph_view* g, const void* q, uint64_t qkey, uint64_t stream,
                        const uint32_t* seeds, int n_seeds, const beam_cfg* cfg, int T,
                        beam_scratch* sc, int64_t* ctr) {
  const int l = cfg->l, deg = g->deg;
  entry* p = sc->p;
  entry* c = sc->c;
  visited* V = &sc->V;
  V->policy = cfg->visited_policy;
  vis_clear(V);

  /* Step 1: p holds l dummies at infinite distance. */
  for (int i = 0; i < l; i++) { p[i].d = INFINITY; p[i].id = NONE_ID; p[i].flag = FLAG_DONE; p[i].from_c = 0; }

  /* Step 2: the initial candidates: the given seeds, else n_init random nodes. */
  int nc = 0;
  int n0 = seeds ? n_seeds : cfg->n_init;
  for (int j = 0; j < n0; j++) {
    uint32_t id;
    if (seeds) {
      id = seeds[j];
      if (id == NONE_ID) continue;
    } else {
      uint64_t h = orc_splitmix(stream, qkey * (uint64_t)cfg->n_init + (uint64_t)j + 1);
      id = (uint32_t)(h % (uint64_t)g->st->n);
    }
    if (vis_test_insert(V, id)) continue;
    /* Step 3: distances of the candidates. */
    c[nc].d = dist_qv(g->st, q, id);
    c[nc].id = id;
    c[nc].flag = FLAG_FRESH;
    nc++;
    ctr[0]++;
  }
  merge_into_p(p, l, c, nc, sc->merged, NULL, 0, NULL);

  /* Steps 3-4 repeated. */
  const int n_cool = (cfg->cooldown_pm * T + 999) / 1000; /* ceil(c * T) */
  const int t_dgs = T - n_cool;
  int forced = 0;
  int it = 0;
  for (;;) {
    if (it >= T) break;
    int dgs_phase = cfg->dgs_on && !forced && it < t_dgs;
    /* parents: first r eligible entries of p */
    int par[64], npar = 0;
    for (int i = 0; i < l && npar < cfg->r; i++) {
      if (p[i].id == NONE_ID) break;
      int el = dgs_phase ? (p[i].flag == FLAG_FRESH) : (p[i].flag != FLAG_DONE);
      if (el) par[npar++] = i;
    }
    if (npar == 0) {
      if (dgs_phase) { forced = 1; continue; }
      break;
    }
    if (cfg->visited_policy == VP_FORGET_EACH_ITER) {
      vis_clear(V);
      for (int i = 0; i < l; i++) if (p[i].id != NONE_ID) vis_test_insert(V, p[i].id);
    } else if (cfg->visited_policy == VP_SMALL_HASH && V->hfill >= SMALL_HASH / 2) {
      vis_clear(V);
      for (int i = 0; i < l; i++) if (p[i].id != NONE_ID) vis_test_insert(V, p[i].id);
    }
    int keep = dgs_phase ? cfg->n_keep : deg;
    const int thr_mode = dgs_phase && cfg->dgs_thr >= 0;
    for (int a = 0; a < npar; a++) p[par[a]].flag = (dgs_phase && keep < deg) ? FLAG_PARTIAL : FLAG_DONE;
    nc = 0;
    for (int a = 0; a < npar; a++) {
      uint32_t u = p[par[a]].id;
      const uint32_t* nb = g->graph + (size_t)u * deg;
      int order[1024];
      for (int j = 0; j < deg; j++) order[j] = j;
      if (thr_mode) {
        /* similarity-threshold pruning (Sec. 6.3): keep each slot whose mismatch is at most the threshold,
         * in slot order; the parent is partly expanded only if some slot was skipped */
        uint32_t qs[64];
        for (int w = 0; w < g->W; w++) qs[w] = 0;
        for (int i = 0; i < g->st->d; i++) {
          int gt;
          if (g->st->dtype == DT_U8) gt = ((const uint8_t*)q)[i] > ((const uint8_t*)g->st->codes)[(size_t)u * g->st->d + i];
          else gt = ((const float*)q)[i] > elem(g->st, u, i);
          if (gt) qs[i / 32] |= 1u << (i % 32);
        }
        int nk = 0;
        for (int j = 0; j < deg; j++) {
          int mm = 0;
          const uint32_t* sj = g->sign + ((size_t)u * deg + j) * g->W;
          for (int w = 0; w < g->W; w++) mm += popc32(qs[w] ^ sj[w]);
          if (mm <= cfg->dgs_thr) order[nk++] = j;
        }
        keep = nk;
        p[par[a]].flag = nk < deg ? FLAG_PARTIAL : FLAG_DONE;
        ctr[3] += deg - nk;
      } else if (dgs_phase) {
        /* rank slots by (mismatch, slot); mismatch = popcount(qsign XOR S[u][j]) */
        uint64_t rk[1024];
        if (cfg->random_discard) {
          uint64_t h1 = orc_splitmix(stream, qkey + 1);
          /* random rank key: the top 24 bits of a SplitMix64 output per (query, parent, slot) */
          for (int j = 0; j < deg; j++) rk[j] = orc_mix64(h1 ^ (((uint64_t)u << 8) | (uint64_t)j)) >> 40;
        } else {
          uint32_t qs[64];
          for (int w = 0; w < g->W; w++) qs[w] = 0;
          for (int i = 0; i < g->st->d; i++) {
            int gt;
            if (g->st->dtype == DT_U8) gt = ((const uint8_t*)q)[i] > ((const uint8_t*)g->st->codes)[(size_t)u * g->st->d + i];
            else gt = ((const float*)q)[i] > elem(g->st, u, i);
            if (gt) qs[i / 32] |= 1u << (i % 32);
          }
          for (int j = 0; j < deg; j++) {
            int mm = 0;
            const uint32_t* sj = g->sign + ((size_t)u * deg + j) * g->W;
            for (int w = 0; w < g->W; w++) mm += popc32(qs[w] ^ sj[w]);
            rk[j] = (uint64_t)mm;
          }
        }
        /* stable insertion sort of slots by rk then slot */
        for (int i = 1; i < deg; i++) {
          int s = order[i];
          int j = i;
          while (j > 0 && (rk[order[j - 1]] > rk[s] || (rk[order[j - 1]] == rk[s] && order[j - 1] > s))) {
            order[j] = order[j - 1];
            j--;
          }
          order[j] = s;
        }
        ctr[3] += deg - keep;
      }
      for (int t = 0; t < keep; t++) {
        uint32_t v = nb[order[t]];
        if (v == NONE_ID) continue;
        if (vis_test_insert(V, v)) continue;
        c[nc].d = dist_qv(g->st, q, v);
        c[nc].id = v;
        c[nc].flag = FLAG_FRESH;
        nc++;
        ctr[0]++;
      }
      ctr[1]++;
    }
    int changed = 0, topk = 0;
    merge_into_p(p, l, c, nc, sc->merged, &changed, cfg->k, &topk);
    it++;
    if (topk) ctr[4] = it; /* last iteration in which the first k entries of p changed */
    if (cfg->stop_on_no_change && !changed) break;
  }
  ctr[2] += it;
}

static void scratch_init(beam_scratch* sc, int l, int cap_c, int64_t nmax) {
  sc->p = (entry*)malloc(sizeof(entry) * (size_t)l);
  sc->c = (entry*)malloc(sizeof(entry) * (size_t)cap_c);
  sc->merged = (entry*)malloc(sizeof(entry) * (size_t)(l + cap_c));
  sc->cap_c = cap_c;
  memset(&sc->V, 0, sizeof(visited));
  sc->V.bits = (uint8_t*)calloc((size_t)nmax, 1);
}
static void scratch_free(beam_scratch* sc) {
  free(sc->p);
  free(sc->c);
  free(sc->merged);
  free(sc->V.bits);
  free(sc->V.touched);
}

/* ------------------------------------------------------------------ */
/* The search over an index: ghost staging, per-shard stages with path */
/* extension (or naive sharding), optional FP32 rerank, final merge.    */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t S, dtype, d, deg, W, deg_g;
  int64_t n_total;
  int64_t n[ORC_MAXS];
  const void* codes[ORC_MAXS];
  const float* scale[ORC_MAXS];
  const float* orig[ORC_MAXS];      /* FP32 originals for the rerank (low-precision stores) */
  const uint32_t* graph[ORC_MAXS];
  const uint32_t* sign[ORC_MAXS];   /* S[u][j][W] */
  const uint32_t* gmap[ORC_MAXS];   /* local -> global id */
  const uint32_t* next[ORC_MAXS];   /* I_s: local id in shard s -> local id in shard (s+1) % S */
  int64_t R[ORC_MAXS];
  const void* g_codes[ORC_MAXS];
  const float* g_scale[ORC_MAXS];
  const uint32_t* g_graph[ORC_MAXS];
  const uint32_t* g_map[ORC_MAXS];  /* ghost id -> local id in its shard */
  const uint8_t* dead[ORC_MAXS];    /* nonzero: the node is deleted (still traversed, never returned), or NULL */
} orc_index;

#define ENTRY_RANDOM 0
#define ENTRY_GHOST_GRAPH 1
#define ENTRY_GHOST_DENSE 2
#define ENTRY_SEEDS 3
#define ENTRY_PREDICTED 4 /* given seeds; a row whose first seed is NONE uses the ghost graph */

typedef struct {
  int32_t k, l, r, T, n_init;
  int32_t entry;
  int32_t l_g, T_g, t_seeds;
  int32_t dgs_on, discard_pm, cooldown_pm, random_discard;
  int32_t ppe_on, forward_f, rerank_mult;
  int32_t visited_policy, stop_on_no_change;
  int32_t ghost_every_stage, dgs_threshold_pm; /* 0: top-n selection; 1..1000: similarity threshold */
  uint64_t seed;
} orc_params;

typedef struct {
  const orc_index* ix;
  const orc_params* pr;
  const void* queries;
  const uint64_t* qkeys;        /* NULL: qkey = row */
  const uint32_t* given_seeds;  /* [nq][n_given] local ids of the start shard, or NULL */
  int n_given;
  const int32_t* given_T;       /* [nq] or NULL */
  uint32_t* out_id;
  void* out_d;
  int64_t* ctr;                 /* [nq][NCTR] or NULL */
  uint32_t* out_ghost;          /* [nq][t] ghost ids picked in stage 0 or NULL */
} search_ctx;

typedef struct { double d; uint32_t id; } res;
static int res_cmp(const void* a, const void* b) {
  const res* x = (const res*)a;
  const res* y = (const res*)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return x->id < y->id ? -1 : x->id > y->id ? 1 : 0;
}

static size_t qbytes(const orc_index* ix) { return (size_t)ix->d * (ix->dtype == DT_U8 ? 1 : 4); }

static void search_row(void* vctx, int64_t row, void* vscratch) {
  search_ctx* C = (search_ctx*)vctx;
  const orc_index* ix = C->ix;
  const orc_params* P = C->pr;
  beam_scratch* sc = (beam_scratch*)vscratch;
  const void* q = (const char*)C->queries + (size_t)row * qbytes(ix);
  uint64_t qkey = C->qkeys ? C->qkeys[row] : (uint64_t)row;
  int S = ix->S, k = P->k, l = P->l;
  int64_t ctr[NCTR] = {0};
  int T = C->given_T ? C->given_T[row] : P->T;
  int s0 = (int)(qkey % (uint64_t)S);
  int lowp = ix->dtype == DT_F16 || ix->dtype == DT_FP8;

  res* all = (res*)malloc(sizeof(res) * (size_t)S * (size_t)k);
  int nall = 0;
  uint32_t seeds[ORC_MAX_GIVEN + 1024 + 64]; /* given seeds, or the hand-off plus ghost seeds */
  int nseeds = 0;
  uint32_t handoff[64];
  int nhand = 0;

  beam_cfg cfg;
  cfg.l = l; cfg.r = P->r; cfg.T = T; cfg.n_init = P->n_init; cfg.k = k;
  cfg.dgs_on = P->dgs_on;
  cfg.n_keep = ix->deg - (P->discard_pm * ix->deg) / 1000;
  cfg.cooldown_pm = P->cooldown_pm;
  cfg.random_discard = P->random_discard;
  cfg.visited_policy = P->visited_policy;
  cfg.stop_on_no_change = P->stop_on_no_change;
  /* threshold mode: keep a slot when mismatch * 1000 <= theta_pm * d, i.e. mismatch <= floor(theta_pm d / 1000) */
  cfg.dgs_thr = P->dgs_threshold_pm > 0 ? (int)(((int64_t)P->dgs_threshold_pm * ix->d) / 1000) : -1;

  for (int t = 0; t < S; t++) {
    int s = (s0 + t) % S;
    orc_store st = {ix->dtype, ix->d, ix->n[s], ix->codes[s], ix->scale[s]};
    graph_view g = {&st, ix->graph[s], ix->deg, ix->sign[s], ix->W};
    const uint32_t* sd = NULL;
    nseeds = 0;
    int use_entry = (t == 0 || !P->ppe_on);
    int ent = P->entry;
    if (ent == ENTRY_PREDICTED)
      ent = (t == 0 && C->given_seeds && C->given_seeds[(size_t)row * C->n_given] != NONE_ID) ? ENTRY_SEEDS
                                                                                             : ENTRY_GHOST_GRAPH;
    const int ghost = ent == ENTRY_GHOST_GRAPH || ent == ENTRY_GHOST_DENSE;
    if (!use_entry) {
      /* path extension: continue from I(z) for the first f results of the previous stage */
      for (int i = 0; i < nhand; i++) seeds[nseeds++] = handoff[i];
      sd = seeds;
    }
    if (ghost && (use_entry || P->ghost_every_stage)) {
      /* ghost staging on this shard (also on later stages when ghost_every_stage is set) */
      orc_store gs = {ix->dtype, ix->d, ix->R[s], ix->g_codes[s], ix->g_scale[s]};
      int tt = P->t_seeds;
      res top[1024];
      int ntop = 0;
      if (ent == ENTRY_GHOST_GRAPH) {
        /* ghost stage: the same search on the ghost graph, DGS off */
        graph_view gg = {&gs, ix->g_graph[s], ix->deg_g, NULL, ix->W};
        beam_cfg gc = cfg;
        gc.l = P->l_g; gc.T = P->T_g; gc.n_init = ix->deg_g; gc.dgs_on = 0; gc.stop_on_no_change = 0;
        beam_scratch* gsc = sc + 1;
        int64_t gctr[5] = {0, 0, 0, 0, 0};
        beam_search(&gg, q, qkey, orc_stream_ghost(P->seed, s), NULL, 0, &gc, P->T_g, gsc, gctr);
        ctr[4] += gctr[0];
        ctr[5] += gctr[1];
        for (int i = 0; i < tt && i < P->l_g; i++) {
          if (gsc->p[i].id == NONE_ID) break;
          top[ntop].d = gsc->p[i].d;
          top[ntop].id = gsc->p[i].id;
          ntop++;
        }
      } else {
        /* dense: exact top-t over all ghost nodes */
        for (int64_t gi = 0; gi < gs.n; gi++) {
          double dv = dist_qv(&gs, q, gi);
          if (ntop == tt && !key_less(dv, (uint32_t)gi, top[tt - 1].d, top[tt - 1].id)) continue;
          int pos = ntop < tt ? ntop : tt - 1;
          while (pos > 0 && key_less(dv, (uint32_t)gi, top[pos - 1].d, top[pos - 1].id)) { top[pos] = top[pos - 1]; pos--; }
          top[pos].d = dv;
          top[pos].id = (uint32_t)gi;
          if (ntop < tt) ntop++;
        }
        ctr[4] += gs.n;
      }
      for (int i = 0; i < ntop; i++) {
        if (C->out_ghost && t == 0) C->out_ghost[(size_t)row * P->t_seeds + i] = top[i].id;
        seeds[nseeds++] = ix->g_map[s][top[i].id];
      }
      if (C->out_ghost && t == 0)
        for (int i = ntop; i < tt; i++) C->out_ghost[(size_t)row * P->t_seeds + i] = NONE_ID;
      sd = seeds;
    } else if (use_entry && ent == ENTRY_SEEDS && C->given_seeds && t == 0) {
      for (int i = 0; i < C->n_given; i++) seeds[nseeds++] = C->given_seeds[(size_t)row * C->n_given + i];
      sd = seeds;
    }
    int64_t bctr[5] = {0, 0, 0, 0, 0};
    beam_search(&g, q, qkey, orc_stream_main(P->seed, s), sd, nseeds, &cfg, T, sc, bctr);
    ctr[0] += bctr[0]; ctr[1] += bctr[1]; ctr[2] += bctr[2]; ctr[3] += bctr[3]; ctr[7] += bctr[4];

    /* hand-off for the next stage: I_s(z) for the first f entries of p */
    nhand = 0;
    if (P->ppe_on && S > 1)
      for (int i = 0; i < P->forward_f && i < l; i++) {
        if (sc->p[i].id == NONE_ID) break;
        handoff[nhand++] = ix->next[s][sc->p[i].id];
      }

    /* deleted nodes (Sec. 6.2, a deletion flag) served the traversal and the hand-off above; the stage
     * result is taken from the entries of p that are not deleted, in p order */
    entry live[1024];
    int nlive = 0;
    for (int i = 0; i < l; i++) {
      if (sc->p[i].id == NONE_ID) break;
      if (ix->dead[s] && ix->dead[s][sc->p[i].id]) continue;
      live[nlive++] = sc->p[i];
    }
    /* stage result: first k (after an FP32 rerank of the first min(m k, l) for low precision) */
    res loc[1024];
    int nloc = 0;
    if (lowp) {
      orc_store o = {DT_F32, ix->d, ix->n[s], ix->orig[s], NULL};
      int m = P->rerank_mult * k;
      if (m > l) m = l;
      for (int i = 0; i < m && i < nlive; i++) {
        loc[nloc].d = dist_qv(&o, q, live[i].id);
        loc[nloc].id = live[i].id;
        nloc++;
        ctr[6]++;
      }
      qsort(loc, (size_t)nloc, sizeof(res), res_cmp);
    } else {
      for (int i = 0; i < nlive; i++) {
        loc[nloc].d = live[i].d;
        loc[nloc].id = live[i].id;
        nloc++;
      }
    }
    for (int i = 0; i < k && i < nloc; i++) {
      all[nall].d = loc[i].d;
      all[nall].id = ix->gmap[s][loc[i].id];
      nall++;
    }
  }
  /* reduction over shards: first k of the union by (dist, global id) */
  qsort(all, (size_t)nall, sizeof(res), res_cmp);
  uint32_t* oid = C->out_id + (size_t)row * k;
  for (int i = 0; i < k; i++) {
    int ok = i < nall;
    oid[i] = ok ? all[i].id : NONE_ID;
    if (ix->dtype == DT_U8) ((int32_t*)C->out_d)[(size_t)row * k + i] = ok ? (int32_t)all[i].d : 2147483647;
    else ((float*)C->out_d)[(size_t)row * k + i] = ok ? (float)all[i].d : INFINITY;
  }
  if (C->ctr) for (int i = 0; i < NCTR; i++) C->ctr[(size_t)row * NCTR + i] = ctr[i];
  free(all);
}

typedef struct {
  search_ctx* C;
  int cap_c;
  int64_t nmax, gmax;
} search_pool;

static void search_scratch_fini(void* scratch) {
  beam_scratch** slot = (beam_scratch**)scratch;
  if (*slot) {
    scratch_free(&(*slot)[0]);
    scratch_free(&(*slot)[1]);
    free(*slot);
  }
}

static void search_row_pooled(void* vctx, int64_t row, void* scratch) {
  search_pool* sp = (search_pool*)vctx;
  beam_scratch** slot = (beam_scratch**)scratch;
  if (!*slot) {
    beam_scratch* sc = (beam_scratch*)calloc(2, sizeof(beam_scratch));
    int lmax = sp->C->pr->l > sp->C->pr->l_g ? sp->C->pr->l : sp->C->pr->l_g;
    scratch_init(&sc[0], lmax, sp->cap_c, sp->nmax);
    scratch_init(&sc[1], lmax, sp->cap_c, sp->gmax > 0 ? sp->gmax : 1);
    *slot = sc;
  }
  search_row(sp->C, row, *slot);
}

/* Validates the parameters the same way the library does; returns 0 on success. */
int orc_search(const orc_index* ix, const orc_params* P, const void* queries, int64_t nq,
               const uint64_t* qkeys, const uint32_t* given_seeds, int n_given, const int32_t* given_T,
               uint32_t* out_id, void* out_d, int64_t* ctr, uint32_t* out_ghost) {
  if (P->k < 1 || P->l < P->k || P->l > 1024 || P->r < 1 || P->r > 64 || P->T < 0) return 1;
  if (ix->S < 1 || ix->S > ORC_MAXS) return 1;
  if (P->forward_f > 64 || P->t_seeds > 1024 || P->n_init > 1024 || ix->deg > 1024) return 1;
  if (P->dgs_threshold_pm < 0 || P->dgs_threshold_pm > 1000 || (P->dgs_threshold_pm > 0 && P->random_discard)) return 1;
  if (n_given < 0 || n_given > ORC_MAX_GIVEN) return 1;
  search_ctx C = {ix, P, queries, qkeys, given_seeds, n_given, given_T, out_id, out_d, ctr, out_ghost};
  int64_t nmax = 1, gmax = 1;
  for (int s = 0; s < ix->S; s++) {
    if (ix->n[s] > nmax) nmax = ix->n[s];
    if (ix->R[s] > gmax) gmax = ix->R[s];
  }
  int cap = P->r * ix->deg;
  int cap2 = P->r * (ix->deg_g > 0 ? ix->deg_g : 1);
  if (cap2 > cap) cap = cap2;
  if (P->n_init > cap) cap = P->n_init;
  if (P->t_seeds > cap) cap = P->t_seeds;
  if (n_given > cap) cap = n_given;
  /* a later stage may take the hand-off and the ghost seeds together */
  if (P->t_seeds + P->forward_f > cap) cap = P->t_seeds + P->forward_f;
  search_pool sp = {&C, cap, nmax, gmax};

  /* per-thread scratch is a pointer slot filled lazily, freed below */
  int t = orc_get_threads();
  if (t > 64) t = 64;
  pool_job j = {search_row_pooled, &sp, nq, 0, PTHREAD_MUTEX_INITIALIZER, sizeof(void*), search_scratch_fini};
  pthread_t th[64];
  for (int i = 0; i < t; i++) pthread_create(&th[i], NULL, pool_worker, &j);
  for (int i = 0; i < t; i++) pthread_join(th[i], NULL);
  return 0;
}
