"""CPU oracle for PathWeaver's graph beam search (arXiv 2507.17094).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
CPU-baseline leg use this package. It never imports the HIP library, and the
HIP library never loads it. The arithmetic lives in ``oracle.c`` (plain C,
scalar, one query per thread); this module marshals numpy arrays and holds a
few plain numpy helpers (recall, brute force on tiny inputs).

Section references are to the paper:
  Sec. 2.1 Eq. 1 (k-NN), Sec. 2.2 Eq. 2 and Steps 1-4 (beam search),
  Sec. 3.1.2 (path extension and the inter-shard map I),
  Sec. 3.2.2 (ghost staging), Sec. 3.3.2 and Sec. 4 (direction-guided selection),
  Sec. 5.1 (Recall@k).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

DT_F32, DT_F16, DT_FP8, DT_U8 = 0, 1, 2, 3
DTYPES = {"f32": DT_F32, "f16": DT_F16, "fp8": DT_FP8, "u8": DT_U8}
NONE_ID = 0xFFFFFFFF
MAXS = 16
NCTR = 8
ENTRY = {"random": 0, "ghost_graph": 1, "ghost_dense": 2, "seeds": 3, "predicted": 4}
VISITED = {"exact": 0, "forget_each_iter": 1, "small_hash": 2}
# counter slots
CTR_NAMES = ["n_dist", "n_exp", "iters", "n_dgs_skipped", "n_dist_ghost", "n_exp_ghost", "n_rerank", "last_topk_change"]


def compile_lib(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain C, no GPU code)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp,
                               SRC_PATH, "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Store(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("d", C.c_int32), ("n", C.c_int64),
                ("codes", C.c_void_p), ("scale", C.c_void_p)]


class Index(C.Structure):
    _fields_ = [("S", C.c_int32), ("dtype", C.c_int32), ("d", C.c_int32), ("deg", C.c_int32),
                ("W", C.c_int32), ("deg_g", C.c_int32), ("n_total", C.c_int64),
                ("n", C.c_int64 * MAXS), ("codes", C.c_void_p * MAXS), ("scale", C.c_void_p * MAXS),
                ("orig", C.c_void_p * MAXS), ("graph", C.c_void_p * MAXS), ("sign", C.c_void_p * MAXS),
                ("gmap", C.c_void_p * MAXS), ("next", C.c_void_p * MAXS), ("R", C.c_int64 * MAXS),
                ("g_codes", C.c_void_p * MAXS), ("g_scale", C.c_void_p * MAXS),
                ("g_graph", C.c_void_p * MAXS), ("g_map", C.c_void_p * MAXS), ("dead", C.c_void_p * MAXS)]


class Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("l", C.c_int32), ("r", C.c_int32), ("T", C.c_int32), ("n_init", C.c_int32),
                ("entry", C.c_int32), ("l_g", C.c_int32), ("T_g", C.c_int32), ("t_seeds", C.c_int32),
                ("dgs_on", C.c_int32), ("discard_pm", C.c_int32), ("cooldown_pm", C.c_int32),
                ("random_discard", C.c_int32), ("ppe_on", C.c_int32), ("forward_f", C.c_int32),
                ("rerank_mult", C.c_int32), ("visited_policy", C.c_int32), ("stop_on_no_change", C.c_int32),
                ("ghost_every_stage", C.c_int32), ("dgs_threshold_pm", C.c_int32), ("seed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(compile_lib())
        u64, i64, i32, vp = C.c_uint64, C.c_int64, C.c_int32, C.c_void_p
        L.orc_mix64.restype = u64
        L.orc_mix64.argtypes = [u64]
        L.orc_splitmix.restype = u64
        L.orc_splitmix.argtypes = [u64, u64]
        for f in ("orc_stream_main", "orc_stream_ghost", "orc_stream_sample"):
            getattr(L, f).restype = u64
            getattr(L, f).argtypes = [u64, C.c_int]
        L.orc_f16_decode.restype = C.c_float
        L.orc_f16_decode.argtypes = [C.c_uint16]
        L.orc_fp8_decode.restype = C.c_float
        L.orc_fp8_decode.argtypes = [C.c_uint8]
        L.orc_fp8_encode.restype = C.c_uint8
        L.orc_fp8_encode.argtypes = [C.c_float]
        L.orc_f16_encode.restype = C.c_uint16
        L.orc_f16_encode.argtypes = [C.c_float]
        L.orc_quantize.argtypes = [vp, i64, C.c_int, C.c_int, vp, vp]
        L.orc_dist.restype = C.c_double
        L.orc_dist.argtypes = [C.POINTER(Store), vp, i64]
        L.orc_knn.argtypes = [C.POINTER(Store), C.POINTER(Store), C.c_int, C.c_int, vp, vp]
        L.orc_prune.restype = C.c_int
        L.orc_prune.argtypes = [C.POINTER(Store), vp, vp, C.c_int, C.c_int, vp]
        L.orc_sign_table.argtypes = [C.POINTER(Store), vp, C.c_int, vp]
        L.orc_keyed_order.argtypes = [u64, i64, vp]
        L.orc_search.restype = C.c_int
        L.orc_search.argtypes = [C.POINTER(Index), C.POINTER(Params), vp, i64, vp, vp, C.c_int, vp, vp, vp, vp, vp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def threads() -> int:
    return int(lib().orc_get_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data


def _store(x: np.ndarray, dtype: int, scale: np.ndarray | None = None) -> Store:
    assert x.flags.c_contiguous
    return Store(dtype, x.shape[1], x.shape[0], x.ctypes.data, _ptr(scale))


def _dt_of(x: np.ndarray) -> int:
    return DT_U8 if x.dtype == np.uint8 else DT_F32


# ---------------------------------------------------------------------------
# Random streams (SplitMix64 used as a counter-based generator)
# ---------------------------------------------------------------------------
def splitmix(seed: int, ctr: int) -> int:
    return int(lib().orc_splitmix(seed & (2**64 - 1), ctr & (2**64 - 1)))


def mix64(z: int) -> int:
    return int(lib().orc_mix64(z & (2**64 - 1)))


def keyed_order(seed: int, n: int) -> np.ndarray:
    """ids ordered by (splitmix(seed, i + 1), i): a seeded random permutation."""
    out = np.empty(n, dtype=np.uint32)
    lib().orc_keyed_order(seed, n, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Number formats
# ---------------------------------------------------------------------------
def fp8_decode(codes: np.ndarray) -> np.ndarray:
    L = lib()
    return np.array([L.orc_fp8_decode(int(c)) for c in np.asarray(codes).ravel()], dtype=np.float32).reshape(np.shape(codes))


def f16_decode(codes: np.ndarray) -> np.ndarray:
    L = lib()
    return np.array([L.orc_f16_decode(int(c)) for c in np.asarray(codes).ravel()], dtype=np.float32).reshape(np.shape(codes))


def fp8_encode(x: np.ndarray) -> np.ndarray:
    L = lib()
    return np.array([L.orc_fp8_encode(float(v)) for v in np.asarray(x, np.float32).ravel()], dtype=np.uint8).reshape(np.shape(x))


def f16_encode(x: np.ndarray) -> np.ndarray:
    L = lib()
    return np.array([L.orc_f16_encode(float(v)) for v in np.asarray(x, np.float32).ravel()], dtype=np.uint16).reshape(np.shape(x))


def quantize(x: np.ndarray, dtype: str):
    """Per-vector quantisation. Returns (codes, scale)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, d = x.shape
    if dtype == "fp8":
        codes = np.empty((n, d), np.uint8)
    elif dtype == "f16":
        codes = np.empty((n, d), np.uint16)
    else:
        raise ValueError(dtype)
    scale = np.empty(n, np.float32)
    lib().orc_quantize(x.ctypes.data, n, d, DTYPES[dtype], codes.ctypes.data, scale.ctypes.data)
    return codes, scale


def dequantize(codes: np.ndarray, scale: np.ndarray, dtype: str) -> np.ndarray:
    """Traversal values f32(s * decode(c))."""
    dec = fp8_decode(codes) if dtype == "fp8" else f16_decode(codes)
    return (scale[:, None].astype(np.float32) * dec).astype(np.float32)


# ---------------------------------------------------------------------------
# Distances, exact k-NN, graph, sign table
# ---------------------------------------------------------------------------
def dist(x: np.ndarray, q: np.ndarray, v: int, dtype: str = None, scale=None) -> float:
    dt = DTYPES[dtype] if dtype else _dt_of(x)
    st = _store(np.ascontiguousarray(x), dt, scale)
    q = np.ascontiguousarray(q)
    return float(lib().orc_dist(C.byref(st), q.ctypes.data, v))


def knn(base: np.ndarray, queries: np.ndarray, k: int, exclude_self: bool = False):
    """Exact k-NN (Eq. 1) under (dist, id). Returns (ids u32 [nq,k], dists f64 [nq,k])."""
    base = np.ascontiguousarray(base)
    queries = np.ascontiguousarray(queries)
    dt = _dt_of(base)
    sb, sq = _store(base, dt), _store(queries, dt)
    ids = np.empty((queries.shape[0], k), np.uint32)
    ds = np.empty((queries.shape[0], k), np.float64)
    lib().orc_knn(C.byref(sb), C.byref(sq), k, 1 if exclude_self else 0, ids.ctypes.data, ds.ctypes.data)
    return ids, ds


def prune(base: np.ndarray, knn_ids: np.ndarray, knn_d: np.ndarray, deg: int) -> np.ndarray:
    base = np.ascontiguousarray(base)
    st = _store(base, _dt_of(base))
    K0 = knn_ids.shape[1]
    out = np.empty((base.shape[0], deg), np.uint32)
    knn_ids = np.ascontiguousarray(knn_ids, np.uint32)
    knn_d = np.ascontiguousarray(knn_d, np.float64)
    rc = lib().orc_prune(C.byref(st), knn_ids.ctypes.data, knn_d.ctypes.data, K0, deg, out.ctypes.data)
    if rc:
        raise ValueError("prune: bad arguments")
    return out


def build_graph(base: np.ndarray, deg: int, K0: int | None = None) -> np.ndarray:
    """Exact K0-NN (K0 = 2 deg) then reverse-merge pruning to `deg`, rows by (dist, id)."""
    K0 = K0 or 2 * deg
    ids, ds = knn(base, base, K0, exclude_self=True)
    return prune(base, ids, ds, deg)


def sign_table(base: np.ndarray, graph: np.ndarray) -> np.ndarray:
    """S[u][j][w]: bit i of word i/32 = [x_v[i] > x_u[i]] for edge (u, j, v)."""
    base = np.ascontiguousarray(base)
    n, d = base.shape
    deg = graph.shape[1]
    W = (d + 31) // 32
    out = np.empty((n, deg, W), np.uint32)
    st = _store(base, _dt_of(base))
    g = np.ascontiguousarray(graph, np.uint32)
    lib().orc_sign_table(C.byref(st), g.ctypes.data, deg, out.ctypes.data)
    return out


def recall(gt: np.ndarray, ann: np.ndarray, k: int) -> float:
    """Recall@k (Sec. 5.1): mean |GT_k intersect ANN_k| / k."""
    tot = 0
    for a, b in zip(gt[:, :k], ann[:, :k]):
        tot += len(set(a.tolist()) & set(b.tolist()))
    return tot / (k * gt.shape[0])


# ---------------------------------------------------------------------------
# Index: shards, graphs, sign tables, inter-shard map, ghost shards
# ---------------------------------------------------------------------------
def stream_sample(seed: int, shard: int) -> int:
    return int(lib().orc_stream_sample(seed & (2**64 - 1), shard))


@dataclass
class OracleIndex:
    dtype: str
    d: int
    deg: int
    S: int
    n_total: int
    shards: list = field(default_factory=list)  # per shard dict
    deg_g: int = 0
    _keep: list = field(default_factory=list)

    def cstruct(self) -> Index:
        ix = Index()
        ix.S, ix.dtype, ix.d, ix.deg = self.S, DTYPES[self.dtype], self.d, self.deg
        ix.W, ix.deg_g, ix.n_total = (self.d + 31) // 32, self.deg_g, self.n_total
        for s, sh in enumerate(self.shards):
            ix.n[s] = sh["n"]
            ix.codes[s] = _ptr(sh["codes"])
            ix.scale[s] = _ptr(sh.get("scale"))
            ix.orig[s] = _ptr(sh.get("orig"))
            ix.graph[s] = _ptr(sh["graph"])
            ix.sign[s] = _ptr(sh.get("sign"))
            ix.gmap[s] = _ptr(sh["gmap"])
            ix.next[s] = _ptr(sh.get("next"))
            ix.R[s] = sh.get("R", 0)
            ix.g_codes[s] = _ptr(sh.get("g_codes"))
            ix.g_scale[s] = _ptr(sh.get("g_scale"))
            ix.g_graph[s] = _ptr(sh.get("g_graph"))
            ix.g_map[s] = _ptr(sh.get("g_map"))
            ix.dead[s] = _ptr(sh.get("dead"))
        return ix


def partition(n: int, S: int, seed: int) -> list:
    """Random partition into S shards (Sec. 3.1.2). S = 1 keeps the identity order.
    Shard s holds pi[floor(sN/S) : floor((s+1)N/S)], pi = ids by SplitMix64 key."""
    if S == 1:
        return [np.arange(n, dtype=np.uint32)]
    pi = keyed_order(seed, n)
    return [pi[(s * n) // S: ((s + 1) * n) // S].copy() for s in range(S)]


def ghost_sample(n_s: int, R: int, seed: int, shard: int) -> np.ndarray:
    """The R local ids with the smallest SplitMix64 keys, sorted by id (Sec. 3.2.2 step 1)."""
    order = keyed_order(stream_sample(seed, shard), n_s)
    return np.sort(order[:R]).astype(np.uint32)


def build_index(X: np.ndarray, deg: int, S: int = 1, seed: int = 5, store: str | None = None,
                graph: np.ndarray | None = None, dgs: bool = True, ghost_R: int | None = None,
                ghost_ratio: float | None = None, deg_g: int = 32, K0: int | None = None) -> OracleIndex:
    """Builds everything the search needs, from the FP32 (or uint8) originals X.

    store: traversal representation ("f32", "u8", "f16", "fp8"); default from X.
    graph: optional prebuilt graph (only for S == 1), else built here.
    """
    X = np.ascontiguousarray(X)
    n, d = X.shape
    base_dt = "u8" if X.dtype == np.uint8 else "f32"
    store = store or base_dt
    ix = OracleIndex(dtype=store, d=d, deg=deg, S=S, n_total=n, deg_g=deg_g)
    parts = partition(n, S, seed)
    for s in range(S):
        gm = parts[s]
        Xs = np.ascontiguousarray(X[gm])
        sh = {"n": len(gm), "gmap": gm, "orig_base": Xs}
        if graph is not None:
            assert S == 1
            sh["graph"] = np.ascontiguousarray(graph, np.uint32)
        else:
            sh["graph"] = build_graph(Xs, deg, K0)
        if dgs:
            sh["sign"] = sign_table(Xs, sh["graph"])
        if store in ("f16", "fp8"):
            codes, scale = quantize(Xs, store)
            sh["codes"], sh["scale"], sh["orig"] = codes, scale, Xs
        else:
            sh["codes"] = Xs
        ix.shards.append(sh)
    if S > 1:
        for s in range(S):
            nxt = ix.shards[(s + 1) % S]["orig_base"]
            ids, _ = knn(nxt, ix.shards[s]["orig_base"], 1)
            ix.shards[s]["next"] = np.ascontiguousarray(ids[:, 0])
    if ghost_R or ghost_ratio:
        for s in range(S):
            sh = ix.shards[s]
            R = ghost_R if ghost_R else int(np.floor(ghost_ratio * sh["n"] + 0.5))
            _ghost_shard(sh, R, seed, s, deg_g)
    return ix


def _ghost_shard(sh: dict, R: int, seed: int, s: int, deg_g: int) -> None:
    """Ghost shard of one shard (Sec. 3.2.2): R sampled nodes, their copies and their own graph."""
    gam = ghost_sample(sh["n"], R, seed, s)
    Xg = np.ascontiguousarray(sh["orig_base"][gam])
    sh["R"] = R
    sh["g_map"] = gam
    sh["g_graph"] = build_graph(Xg, deg_g)
    sh["g_codes"] = np.ascontiguousarray(sh["codes"][gam])
    if "scale" in sh:
        sh["g_scale"] = np.ascontiguousarray(sh["scale"][gam])


def delete(ix: OracleIndex, global_ids) -> None:
    """Deletion flags (Sec. 6.2): the nodes stay in the graphs and are traversed, but no result returns them."""
    gl = set(int(g) for g in np.asarray(global_ids).ravel())
    for sh in ix.shards:
        dead = sh.get("dead")
        if dead is None:
            dead = np.zeros(sh["n"], np.uint8)
        dead = dead | np.array([int(g) in gl for g in sh["gmap"]], np.uint8)
        sh["dead"] = np.ascontiguousarray(dead)


def append(ix: OracleIndex, s: int, Xnew: np.ndarray, ghost_seed: int = 5, K0: int | None = None) -> None:
    """Insertion into an existing shard (Sec. 6.2): the new rows get the next global ids and the next local ids
    of shard s; the shard's graph and direction table are rebuilt over all its rows, its store re-made, its
    ghost shard re-sampled with the same count, and the inter-shard maps into and out of the shard refreshed
    (I(u) of Sec. 3.1.2, exact)."""
    sh = ix.shards[s]
    Xnew = np.ascontiguousarray(Xnew)
    n_old = sh["n"]
    Xs = np.ascontiguousarray(np.concatenate([sh["orig_base"], Xnew]))
    sh["orig_base"] = Xs
    sh["n"] = len(Xs)
    sh["gmap"] = np.ascontiguousarray(np.concatenate([sh["gmap"], np.arange(ix.n_total, ix.n_total + len(Xnew),
                                                                            dtype=np.uint32)]))
    ix.n_total += len(Xnew)
    sh["graph"] = build_graph(Xs, ix.deg, K0)
    if "sign" in sh:
        sh["sign"] = sign_table(Xs, sh["graph"])
    if ix.dtype in ("f16", "fp8"):
        sh["codes"], sh["scale"] = quantize(Xs, ix.dtype)
        sh["orig"] = Xs
    else:
        sh["codes"] = Xs
    if "dead" in sh:
        sh["dead"] = np.ascontiguousarray(np.concatenate([sh["dead"], np.zeros(len(Xnew), np.uint8)]))
    S = ix.S
    if S > 1:
        nxt = ix.shards[(s + 1) % S]["orig_base"]
        sh["next"] = np.ascontiguousarray(knn(nxt, Xs, 1)[0][:, 0])
        prev = ix.shards[(s - 1) % S]
        prev["next"] = np.ascontiguousarray(knn(Xs, prev["orig_base"], 1)[0][:, 0])
    if sh.get("R"):
        _ghost_shard(sh, sh["R"], ghost_seed, s, ix.deg_g)
    del n_old


def next_map_by_search(ix: OracleIndex, s: int, **kw) -> np.ndarray:
    """The shard-to-shard lookup table built by search (Sec. 4, implementation of path extension): every node
    of shard s is a query of a search on shard (s+1) mod S alone (that shard's graph, direction table, store
    and ghost shard; no deletion flags), keyed by its local id, and the top-1 local id is the entry I_s(u).
    kw are the search parameters of `search` (k is 1; path extension does not apply to one shard)."""
    nx = ix.shards[(s + 1) % ix.S]
    view = OracleIndex(dtype=ix.dtype, d=ix.d, deg=ix.deg, S=1, n_total=nx["n"], deg_g=ix.deg_g)
    sh = {k: v for k, v in nx.items() if k not in ("next", "dead")}
    sh["gmap"] = np.arange(nx["n"], dtype=np.uint32)
    view.shards.append(sh)
    src = ix.shards[s]["orig_base"]
    kw = dict(kw)
    kw["k"] = 1
    ids, _, _ = search(view, src, qkeys=np.arange(len(src), dtype=np.uint64), **kw)
    return np.ascontiguousarray(ids[:, 0])


DEFAULTS = dict(k=10, l=64, r=1, T=64, n_init=None, entry="random", l_g=32, T_g=8, t_seeds=None,
                dgs_on=False, discard=0.5, cooldown=0.3, random_discard=False, ppe_on=True, forward_f=1,
                rerank_mult=4, visited="exact", stop_on_no_change=False, ghost_every_stage=False, seed=6,
                dgs_threshold=0.0)


def make_params(ix: OracleIndex, **kw) -> Params:
    o = dict(DEFAULTS)
    o.update(kw)
    p = Params()
    p.k, p.l, p.r, p.T = o["k"], o["l"], o["r"], o["T"]
    p.n_init = o["n_init"] if o["n_init"] is not None else ix.deg
    p.entry = ENTRY[o["entry"]]
    p.l_g, p.T_g = o["l_g"], o["T_g"]
    p.t_seeds = o["t_seeds"] if o["t_seeds"] is not None else min(o["l_g"], o["l"])
    p.dgs_on = int(bool(o["dgs_on"]))
    p.discard_pm = int(round(o["discard"] * 1000))
    p.cooldown_pm = int(round(o["cooldown"] * 1000))
    p.random_discard = int(bool(o["random_discard"]))
    p.ppe_on, p.forward_f, p.rerank_mult = int(bool(o["ppe_on"])), o["forward_f"], o["rerank_mult"]
    p.visited_policy = VISITED[o["visited"]]
    p.stop_on_no_change = int(bool(o["stop_on_no_change"]))
    p.ghost_every_stage = int(bool(o["ghost_every_stage"]))
    p.dgs_threshold_pm = int(round(o["dgs_threshold"] * 1000))
    p.seed = o["seed"] & (2**64 - 1)
    return p


def search(ix: OracleIndex, Q: np.ndarray, qkeys: np.ndarray | None = None, seeds: np.ndarray | None = None,
           T_per_query: np.ndarray | None = None, want_ghost: bool = False, **kw):
    """The oracle search. Returns (ids [nq,k] u32, dists [nq,k] f32|i32, counters [nq,8] i64[, ghost ids])."""
    p = make_params(ix, **kw)
    Q = np.ascontiguousarray(Q, np.uint8 if ix.dtype == "u8" else np.float32)
    nq = Q.shape[0]
    cix = ix.cstruct()
    ids = np.empty((nq, p.k), np.uint32)
    ds = np.empty((nq, p.k), np.int32 if ix.dtype == "u8" else np.float32)
    ctr = np.zeros((nq, NCTR), np.int64)
    qk = None if qkeys is None else np.ascontiguousarray(qkeys, np.uint64)
    sd = None if seeds is None else np.ascontiguousarray(seeds, np.uint32)
    ng = 0 if sd is None else sd.shape[1]
    Tq = None if T_per_query is None else np.ascontiguousarray(T_per_query, np.int32)
    gh = np.empty((nq, p.t_seeds), np.uint32) if want_ghost else None
    rc = lib().orc_search(C.byref(cix), C.byref(p), Q.ctypes.data, nq, _ptr(qk), _ptr(sd), ng, _ptr(Tq),
                          ids.ctypes.data, ds.ctypes.data, ctr.ctypes.data, _ptr(gh))
    if rc:
        raise ValueError("oracle search: invalid parameters")
    if want_ghost:
        return ids, ds, ctr, gh
    return ids, ds, ctr


def brute_force_numpy(base: np.ndarray, Q: np.ndarray, k: int):
    """Textbook brute force with numpy (independent of oracle.c): squared L2 of the float
    differences (squares summed in float64; exact integers for uint8), ordered by (dist, id).
    Only for tiny inputs."""
    if base.dtype == np.uint8:
        D = ((Q[:, None, :].astype(np.int64) - base[None, :, :].astype(np.int64)) ** 2).sum(-1).astype(np.float64)
    else:
        diff = Q[:, None, :].astype(np.float32) - base[None, :, :].astype(np.float32)
        D = (diff.astype(np.float64) ** 2).sum(-1)
    out = np.empty((Q.shape[0], k), np.int64)
    for i in range(Q.shape[0]):
        out[i] = np.lexsort((np.arange(base.shape[0]), D[i]))[:k]
    return out, D
