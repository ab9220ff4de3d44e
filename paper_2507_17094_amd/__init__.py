"""miann: MI355X-native graph beam search (PathWeaver, arXiv 2507.17094).

Thin Python binding over the C-ABI of ``libmiann.so`` (``include/miann.h``).
It only marshals arguments: torch tensors provide device memory and the HIP
stream, and every step of the search runs in the library's HIP kernels. There
is no CPU fallback: without the built library on a GPU machine, every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmiann.so")

F32, F16, FP8E4M3, U8 = 0, 1, 2, 3
DTYPE_CODES = {"f32": F32, "f16": F16, "fp8": FP8E4M3, "u8": U8}
ENTRY_RANDOM, ENTRY_GHOST_GRAPH, ENTRY_GHOST_DENSE, ENTRY_SEEDS = 0, 1, 2, 3
ENTRY_CODES = {"random": 0, "ghost_graph": 1, "ghost_dense": 2, "seeds": 3, "predicted": 4}
NCTR = 8
NONE_ID = 0xFFFFFFFF
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EUNSUPPORTED"}

EXPORTS = [
    "miann_build_graph", "miann_build_ghost", "miann_index_import", "miann_index_shard", "miann_index_info",
    "miann_index_free", "miann_search_params_default", "miann_search", "miann_search_noalloc",
    "miann_noalloc_scratch_bytes", "miann_exact_knn", "miann_last_error",
    "miann_version", "miann_nearest_ghost", "miann_predictor_create", "miann_predictor_free",
    "miann_predictor_view_get", "miann_predictor_sync_weights", "miann_predictor_step", "miann_predictor_train",
    "miann_predictor_predict", "miann_server_config_default", "miann_server_create", "miann_server_submit",
    "miann_server_wait", "miann_server_get_stats", "miann_server_destroy", "miann_index_save", "miann_index_load",
]


class MiannError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class BuildParams(C.Structure):
    _fields_ = [("degree", C.c_int32), ("knn_k0", C.c_int32), ("num_shards", C.c_int32),
                ("store_dtype", C.c_int32), ("dgs_table", C.c_int32), ("reserved", C.c_int32),
                ("seed", C.c_uint64)]


class ShardDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("vectors", C.c_void_p), ("graph", C.c_void_p), ("global_ids", C.c_void_p),
                ("next_map", C.c_void_p), ("n_ghost", C.c_int64), ("ghost_ids", C.c_void_p),
                ("ghost_graph", C.c_void_p)]


class ShardView(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_ghost", C.c_int64), ("d", C.c_int32), ("d_pad", C.c_int32),
                ("degree", C.c_int32), ("ghost_degree", C.c_int32), ("W", C.c_int32),
                ("store_dtype", C.c_int32), ("in_dtype", C.c_int32),
                ("store", C.c_void_p), ("scale", C.c_void_p), ("originals", C.c_void_p), ("graph", C.c_void_p),
                ("sign", C.c_void_p), ("global_ids", C.c_void_p), ("next_map", C.c_void_p),
                ("ghost_ids", C.c_void_p), ("ghost_graph", C.c_void_p)]


class SearchParams(C.Structure):
    _fields_ = [("search_width", C.c_int32), ("n_init", C.c_int32), ("entry", C.c_int32),
                ("ghost_itopk", C.c_int32), ("ghost_iters", C.c_int32), ("t_seeds", C.c_int32),
                ("dgs", C.c_int32), ("discard_permille", C.c_int32), ("cooldown_permille", C.c_int32),
                ("random_discard", C.c_int32), ("ppe", C.c_int32), ("forward_f", C.c_int32),
                ("rerank_mult", C.c_int32), ("stop_on_no_change", C.c_int32), ("hash_log2", C.c_int32),
                ("n_seeds", C.c_int32), ("ghost_every_stage", C.c_int32), ("dgs_threshold_permille", C.c_int32),
                ("stage_waves", C.c_int32), ("seed", C.c_uint64), ("qkeys", C.c_void_p), ("seeds", C.c_void_p),
                ("max_iters_per_query", C.c_void_p), ("phase_ms", C.c_void_p),
                ("phase_events", C.c_void_p)]


class ServerConfig(C.Structure):
    _fields_ = [("num_streams", C.c_int32), ("reserved", C.c_int32), ("max_batch_queries", C.c_int64),
                ("max_inflight_queries", C.c_int64), ("memory_budget_bytes", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("requests_done", C.c_int64), ("queries_done", C.c_int64), ("batches", C.c_int64),
                ("peak_inflight_queries", C.c_int64), ("peak_inflight_bytes", C.c_int64), ("elapsed_s", C.c_double)]


class PredictorView(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("hidden", C.c_int32), ("n_entry", C.c_int32)] + \
               [(n, C.c_void_p) for n in ("W1", "b1", "W2", "b2", "W3", "b3", "gW1", "gb1", "gW2", "gb2", "gW3", "gb3")]


_lib = None


def lib_path() -> str:
    return LIB_PATH


def load():
    """Loads libmiann.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MiannError(3, f"{LIB_PATH} is missing: build it with paper_2507_17094_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    i32, i64, u64, vp = C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
    L.miann_build_graph.argtypes = [vp, i64, i32, i32, C.POINTER(BuildParams), vp, C.POINTER(vp)]
    L.miann_build_ghost.argtypes = [vp, C.c_double, i64, i32, u64, vp]
    L.miann_index_import.argtypes = [C.POINTER(ShardDesc), i32, i32, i32, i32, i32, i32, i32, vp, C.POINTER(vp)]
    L.miann_index_shard.argtypes = [vp, i32, C.POINTER(ShardView)]
    L.miann_index_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.miann_index_save.argtypes = [vp, C.c_char_p]
    L.miann_index_load.argtypes = [C.c_char_p, vp, C.POINTER(vp)]
    L.miann_index_free.argtypes = [vp]
    L.miann_index_free.restype = None
    L.miann_search_params_default.argtypes = [C.POINTER(SearchParams)]
    L.miann_search_params_default.restype = None
    L.miann_search.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(SearchParams), vp, vp, vp, vp]
    L.miann_search_noalloc.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(SearchParams), vp, vp, vp, vp]
    L.miann_noalloc_scratch_bytes.argtypes = []
    L.miann_noalloc_scratch_bytes.restype = C.c_size_t
    L.miann_exact_knn.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    L.miann_index_delete.argtypes = [vp, vp, i64, vp]
    L.miann_index_append.argtypes = [vp, i32, vp, i64, u64, vp]
    L.miann_build_next_map.argtypes = [vp, i32, i32, C.POINTER(SearchParams), vp]
    L.miann_release_scratch.argtypes = [vp]
    L.miann_gather_probe.argtypes = [vp, i64, i32, vp, i64, vp, vp]
    L.miann_index_build_times.argtypes = [vp, C.POINTER(C.c_double)]
    L.miann_predictor_labels.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(SearchParams), vp, vp, vp, vp]
    L.miann_last_error.restype = C.c_char_p
    L.miann_version.restype = C.c_char_p
    L.miann_nearest_ghost.argtypes = [vp, i32, vp, i64, vp, vp]
    L.miann_predictor_create.argtypes = [i32, i32, i32, u64, C.POINTER(vp)]
    L.miann_predictor_free.argtypes = [vp]
    L.miann_predictor_free.restype = None
    L.miann_predictor_view_get.argtypes = [vp, C.POINTER(PredictorView)]
    L.miann_predictor_sync_weights.argtypes = [vp, vp]
    L.miann_predictor_step.argtypes = [vp, vp, vp, vp, i32, C.c_float, C.c_float, i32, C.POINTER(C.c_float), vp]
    L.miann_predictor_train.argtypes = [vp, vp, vp, vp, i64, i32, i32, C.c_float, C.c_float, u64,
                                        C.POINTER(C.c_float), vp]
    L.miann_predictor_predict.argtypes = [vp, vp, i64, i32, C.c_float, vp, i32, i32, C.c_float, vp, vp, vp, vp, vp]
    L.miann_server_config_default.argtypes = [C.POINTER(ServerConfig)]
    L.miann_server_config_default.restype = None
    L.miann_server_create.argtypes = [vp, C.POINTER(ServerConfig), C.POINTER(vp)]
    L.miann_server_submit.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(SearchParams), C.POINTER(u64)]
    L.miann_server_wait.argtypes = [vp, u64, vp, vp, C.POINTER(C.c_double)]
    L.miann_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    L.miann_server_warm.argtypes = [vp, i64, i32, i32, i32, C.POINTER(SearchParams)]
    L.miann_server_replay.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, i64, C.POINTER(SearchParams), vp,
                                      C.POINTER(C.c_double)]
    L.miann_server_destroy.argtypes = [vp]
    L.miann_server_destroy.restype = None
    for f in ("miann_server_create", "miann_server_submit", "miann_server_wait", "miann_server_get_stats",
              "miann_server_warm", "miann_server_replay"):
        getattr(L, f).restype = C.c_int
    for f in ("miann_build_graph", "miann_build_ghost", "miann_index_import", "miann_index_shard",
              "miann_index_info", "miann_search", "miann_search_noalloc", "miann_exact_knn", "miann_index_delete",
              "miann_index_append", "miann_build_next_map", "miann_release_scratch", "miann_predictor_labels",
              "miann_gather_probe", "miann_index_build_times", "miann_nearest_ghost", "miann_predictor_create",
              "miann_predictor_view_get", "miann_predictor_sync_weights", "miann_predictor_step",
              "miann_predictor_train", "miann_predictor_predict"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != 0:
        raise MiannError(rc, load().miann_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _require_cuda(t, name):
    if t is not None and not t.is_cuda:
        raise MiannError(1, f"{name} must be a device tensor")


def _require(t, name, dtypes, shape):
    """Checks a device tensor's dtype (one of `dtypes`), shape (None = any size in that axis) and layout."""
    if t is None:
        return None
    _require_cuda(t, name)
    if t.dtype not in dtypes:
        raise MiannError(1, f"{name}: dtype {t.dtype} not in {list(dtypes)}")
    if t.dim() != len(shape) or any(w is not None and w != n for w, n in zip(shape, t.shape)):
        raise MiannError(1, f"{name}: shape {tuple(t.shape)} does not match {shape}")
    if not t.is_contiguous():
        raise MiannError(1, f"{name} must be contiguous")
    return t


@dataclass
class SearchOptions:
    """Python mirror of miann_search_params (see include/miann.h)."""
    search_width: int = 1
    n_init: int = 0
    entry: str = "random"
    ghost_itopk: int = 32
    ghost_iters: int = 8
    t_seeds: int = 0
    dgs: bool = False
    discard: float = 0.5
    cooldown: float = 0.3
    random_discard: bool = False
    ppe: bool = True
    forward_f: int = 1
    rerank_mult: int = 4
    stop_on_no_change: bool = False
    hash_log2: int = 0
    ghost_every_stage: bool = False
    dgs_threshold: float = 0.0  # theta of the similarity-threshold direction filter (0 = top-n selection)
    stage_waves: int = 0  # stage kernel's waves per SIMD (0 automatic, 4, 5, 6); 6 pays with batches on two streams
    seed: int = 6

    def cstruct(self, qkeys=None, seeds=None, max_iters_per_query=None) -> SearchParams:
        p = SearchParams()
        load().miann_search_params_default(C.byref(p))
        p.search_width = self.search_width
        p.n_init = self.n_init
        p.entry = ENTRY_CODES[self.entry] if isinstance(self.entry, str) else int(self.entry)
        p.ghost_itopk = self.ghost_itopk
        p.ghost_iters = self.ghost_iters
        p.t_seeds = self.t_seeds
        p.dgs = int(bool(self.dgs))
        p.discard_permille = int(round(self.discard * 1000))
        p.cooldown_permille = int(round(self.cooldown * 1000))
        p.random_discard = int(bool(self.random_discard))
        p.ppe = int(bool(self.ppe))
        p.forward_f = self.forward_f
        p.rerank_mult = self.rerank_mult
        p.stop_on_no_change = int(bool(self.stop_on_no_change))
        p.hash_log2 = self.hash_log2
        p.ghost_every_stage = int(bool(self.ghost_every_stage))
        p.dgs_threshold_permille = int(round(self.dgs_threshold * 1000))
        p.stage_waves = self.stage_waves
        p.seed = self.seed & (2**64 - 1)
        p.qkeys = _ptr(qkeys)
        if seeds is not None:
            p.seeds = _ptr(seeds)
            p.n_seeds = seeds.shape[1]
        p.max_iters_per_query = _ptr(max_iters_per_query)
        return p


class Index:
    """An index owned by the native library (freed with the object)."""

    def __init__(self, handle: int, in_dtype: int):
        self._h = C.c_void_p(handle)
        self.in_dtype = in_dtype

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.miann_index_free(self._h)
            self._h = C.c_void_p(0)

    @property
    def handle(self):
        return self._h

    def info(self):
        S, n, d, deg, st = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().miann_index_info(self._h, C.byref(S), C.byref(n), C.byref(d), C.byref(deg), C.byref(st)))
        return dict(num_shards=S.value, n=n.value, d=d.value, degree=deg.value, store_dtype=st.value)

    def build_times(self) -> dict:
        """Host seconds of the build steps (graph, direction table, inter-shard map, ghost shards)."""
        t = (C.c_double * 4)()
        _check(load().miann_index_build_times(self._h, t))
        return dict(graph_s=t[0], direction_table_s=t[1], inter_shard_map_s=t[2], ghost_s=t[3])

    def save(self, path: str) -> None:
        """Writes the index to a file (originals, graphs, maps and ghost shards)."""
        _check(load().miann_index_save(self._h, os.fsencode(path)))

    @staticmethod
    def load(path: str, stream=None) -> "Index":
        """Reads a file written by save(); the store, sign table and dense ghost arrays are rebuilt."""
        h = C.c_void_p()
        _check(load().miann_index_load(os.fsencode(path), _stream_ptr(stream), C.byref(h)))
        v = ShardView()
        _check(load().miann_index_shard(h, 0, C.byref(v)))
        return Index(h.value, v.in_dtype)

    def shard(self, s: int) -> ShardView:
        v = ShardView()
        _check(load().miann_index_shard(self._h, s, C.byref(v)))
        return v

    # -- build ------------------------------------------------------------
    @staticmethod
    def build(base, degree: int, num_shards: int = 1, store: str | None = None, dgs_table: bool = True,
              knn_k0: int = 0, seed: int = 5, stream=None) -> "Index":
        torch = _torch()
        _require_cuda(base, "base")
        base = base.contiguous()
        if base.dtype not in (torch.float32, torch.uint8) or base.dim() != 2:
            raise MiannError(1, f"base: need a 2-D float32 or uint8 tensor, got {base.dtype} {tuple(base.shape)}")
        in_dt = U8 if base.dtype == torch.uint8 else F32
        st = DTYPE_CODES[store] if store else in_dt
        bp = BuildParams(degree, knn_k0, num_shards, st, int(bool(dgs_table)), 0, seed & (2**64 - 1))
        h = C.c_void_p()
        _check(load().miann_build_graph(base.data_ptr(), base.shape[0], base.shape[1], in_dt, C.byref(bp),
                                        _stream_ptr(stream), C.byref(h)))
        return Index(h.value, in_dt)

    @staticmethod
    def import_shards(shards: list, d: int, in_dtype: str = "f32", store: str | None = None, degree: int = 32,
                      ghost_degree: int = 0, dgs_table: bool = True, stream=None) -> "Index":
        """shards: list of dicts with device tensors vectors, graph, [global_ids, next_map, ghost_ids, ghost_graph]."""
        arr = (ShardDesc * len(shards))()
        for i, sh in enumerate(shards):
            for k_, v in sh.items():
                if hasattr(v, "is_cuda"):
                    _require_cuda(v, k_)
            arr[i].n = sh["vectors"].shape[0]
            arr[i].vectors = sh["vectors"].data_ptr()
            arr[i].graph = sh["graph"].data_ptr()
            arr[i].global_ids = _ptr(sh.get("global_ids"))
            arr[i].next_map = _ptr(sh.get("next_map"))
            gi = sh.get("ghost_ids")
            arr[i].n_ghost = 0 if gi is None else gi.shape[0]
            arr[i].ghost_ids = _ptr(gi)
            arr[i].ghost_graph = _ptr(sh.get("ghost_graph"))
        in_dt = DTYPE_CODES[in_dtype]
        st = DTYPE_CODES[store] if store else in_dt
        h = C.c_void_p()
        _check(load().miann_index_import(arr, len(shards), d, in_dt, st, degree, ghost_degree, int(bool(dgs_table)),
                                         _stream_ptr(stream), C.byref(h)))
        return Index(h.value, in_dt)

    def build_ghost(self, ratio: float = 0.0, num_ghost: int = 0, ghost_degree: int = 32, seed: int = 5,
                    stream=None) -> None:
        _check(load().miann_build_ghost(self._h, float(ratio), int(num_ghost), ghost_degree, seed & (2**64 - 1),
                                        _stream_ptr(stream)))

    def build_next_map(self, itopk: int, max_iters: int, opts: SearchOptions | None = None, stream=None) -> None:
        """Replaces every shard's inter-shard map by the lookup table built by search (top-1 of a search of each
        node on the next shard)."""
        p = (opts or SearchOptions()).cstruct()
        _check(load().miann_build_next_map(self._h, itopk, max_iters, C.byref(p), _stream_ptr(stream)))

    # -- dynamic updates (Sec. 6.2) ------------------------------------------
    def delete(self, global_ids, stream=None) -> None:
        """Deletion flags for these global ids (device int32/uint32 tensor): traversed, never returned."""
        torch = _torch()
        _require(global_ids, "global_ids", (torch.int32, torch.uint32), (None,))
        _check(load().miann_index_delete(self._h, global_ids.data_ptr(), global_ids.shape[0], _stream_ptr(stream)))

    def append(self, shard: int, vectors, ghost_seed: int = 5, stream=None) -> None:
        """Inserts rows into one shard (the next global ids) and rebuilds that shard's graph, direction table,
        inter-shard maps and the ghost shards (re-sampled from ghost_seed)."""
        torch = _torch()
        info = self.info()
        _require(vectors, "vectors", (torch.uint8,) if self.in_dtype == U8 else (torch.float32,), (None, info["d"]))
        _check(load().miann_index_append(self._h, shard, vectors.data_ptr(), vectors.shape[0],
                                         ghost_seed & (2**64 - 1), _stream_ptr(stream)))

    # -- search -----------------------------------------------------------
    def search(self, queries, k: int, itopk: int, max_iters: int, opts: SearchOptions | None = None,
               qkeys=None, seeds=None, max_iters_per_query=None, counters: bool = False, out=None, stream=None,
               phase_ms=None, phase_events=None, noalloc: bool = False):
        """Returns (ids [nq,k] int32 view of uint32, dists [nq,k] float32|int32[, counters [nq,8] int64]).
        phase_ms: optional list that receives per-launch milliseconds [dense, stage 0..S-1, merge]
        (the call then synchronises the stream).
        phase_events: optional 4 raw hipEvent_t handles (ints or None), recorded before the ghost entry,
        before stage 0, after the last stage and after the merge; the call does not wait for them.
        noalloc: call miann_search_noalloc (temporary buffers from the library's static device array; pass
        `out` as well to keep the whole call free of allocations)."""
        torch = _torch()
        d = self.info()["d"]
        qdt = torch.uint8 if self.in_dtype == U8 else torch.float32
        _require_cuda(queries, "queries")
        if queries.dtype != qdt or queries.dim() != 2 or queries.shape[1] != d:
            raise MiannError(1, f"queries: need [nq, {d}] {qdt}, got {queries.dtype} {tuple(queries.shape)}")
        queries = queries.contiguous()
        nq = queries.shape[0]
        _require(qkeys, "qkeys", (torch.int64, torch.uint64), (nq,))
        if seeds is not None:
            _require(seeds, "seeds", (torch.int32, torch.uint32), (nq, None))
        _require(max_iters_per_query, "max_iters_per_query", (torch.int32,), (nq,))
        opts = opts or SearchOptions()
        ddt = torch.int32 if self.in_dtype == U8 else torch.float32
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
            dists = torch.empty((nq, k), dtype=ddt, device=queries.device)
        else:
            ids, dists = out
            _require(ids, "out ids", (torch.int32, torch.uint32), (nq, k))
            _require(dists, "out dists", (ddt,), (nq, k))
        ctr = torch.empty((nq, NCTR), dtype=torch.int64, device=queries.device) if counters else None
        p = opts.cstruct(qkeys, seeds, max_iters_per_query)
        tbuf = None
        if phase_ms is not None:
            tbuf = (C.c_float * (2 + self.info()["num_shards"]))()
            p.phase_ms = C.cast(tbuf, C.c_void_p)
        evbuf = None
        if phase_events is not None:
            if len(phase_events) != 4:
                raise ValueError("phase_events needs 4 event handles")
            evbuf = (C.c_void_p * 4)(*[e or None for e in phase_events])
            p.phase_events = C.cast(evbuf, C.c_void_p)
        fn = load().miann_search_noalloc if noalloc else load().miann_search
        _check(fn(self._h, queries.data_ptr(), nq, k, itopk, max_iters, C.byref(p), ids.data_ptr(), dists.data_ptr(),
                  _ptr(ctr), _stream_ptr(stream)))
        if tbuf is not None:
            phase_ms[:] = list(tbuf)
        return (ids, dists, ctr) if counters else (ids, dists)

    def exact_knn(self, queries, k: int, stream=None):
        torch = _torch()
        _require_cuda(queries, "queries")
        nq = queries.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
        dists = torch.empty((nq, k), dtype=torch.int32 if self.in_dtype == U8 else torch.float32, device=queries.device)
        _check(load().miann_exact_knn(self._h, queries.data_ptr(), nq, k, ids.data_ptr(), dists.data_ptr(),
                                      _stream_ptr(stream)))
        return ids, dists


class Predictor:
    """Learned entry / iteration-budget predictor (BF16 MLP trained by the library's kernels)."""

    def __init__(self, d_in: int, hidden: int, n_entry: int, seed: int = 1):
        h = C.c_void_p()
        _check(load().miann_predictor_create(d_in, hidden, n_entry, seed & (2**64 - 1), C.byref(h)))
        self._h = h
        self.d_in, self.hidden, self.n_entry = d_in, hidden, n_entry

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.miann_predictor_free(self._h)
            self._h = C.c_void_p(0)

    def view(self) -> PredictorView:
        v = PredictorView()
        _check(load().miann_predictor_view_get(self._h, C.byref(v)))
        return v

    def tensors(self, grads: bool = False) -> dict:
        """Device tensors aliasing the FP32 masters (or the gradients)."""
        torch = _torch()
        v = self.view()
        shapes = {"W1": (self.d_in, self.hidden), "b1": (self.hidden,), "W2": (self.hidden, self.hidden),
                  "b2": (self.hidden,), "W3": (self.hidden, self.n_entry + 1), "b3": (self.n_entry + 1,)}
        out = {}
        for k, shp in shapes.items():
            ptr = getattr(v, ("g" + k) if grads else k)
            n = 1
            for s_ in shp:
                n *= s_
            t = torch.empty(shp, dtype=torch.float32, device="cuda")
            _hip_copy(t.data_ptr(), ptr, n * 4)
            out[k] = t
        return out

    def set_weights(self, w: dict, stream=None) -> None:
        v = self.view()
        for k, t in w.items():
            t = t.contiguous().float().cuda()
            _hip_copy(getattr(v, k), t.data_ptr(), t.numel() * 4)
        _check(load().miann_predictor_sync_weights(self._h, _stream_ptr(stream)))

    def step(self, x, entry, budget, lam: float = 1.0, lr: float = 1e-3, update: bool = False, stream=None) -> float:
        loss = C.c_float()
        _check(load().miann_predictor_step(self._h, x.data_ptr(), entry.data_ptr(), budget.data_ptr(), x.shape[0],
                                           lam, lr, int(update), C.byref(loss), _stream_ptr(stream)))
        return loss.value

    def train(self, x, entry, budget, epochs: int, batch: int = 4096, lr: float = 1e-3, lam: float = 1.0,
              seed: int = 3, stream=None) -> list:
        losses = (C.c_float * epochs)()
        _check(load().miann_predictor_train(self._h, x.data_ptr(), entry.data_ptr(), budget.data_ptr(), x.shape[0],
                                            epochs, batch, lr, lam, seed & (2**64 - 1), losses, _stream_ptr(stream)))
        return list(losses)

    def predict(self, x, t: int, tau: float, ghost_map, t_min: int, t_max: int, budget_scale: float = 1.25,
                stream=None):
        """Returns (seeds [n,t] int32 view of uint32, iters [n] int32, conf [n] f32, top entries [n,t])."""
        torch = _torch()
        if ghost_map.shape[0] < self.n_entry:
            raise MiannError(1, f"ghost_map has {ghost_map.shape[0]} entries, the predictor has {self.n_entry}")
        n = x.shape[0]
        seeds = torch.empty((n, t), dtype=torch.int32, device=x.device)
        iters = torch.empty(n, dtype=torch.int32, device=x.device)
        conf = torch.empty(n, dtype=torch.float32, device=x.device)
        top = torch.empty((n, t), dtype=torch.int32, device=x.device)
        _check(load().miann_predictor_predict(self._h, x.data_ptr(), n, t, tau, ghost_map.data_ptr(), t_min, t_max,
                                              budget_scale, seeds.data_ptr(), iters.data_ptr(), conf.data_ptr(), top.data_ptr(),
                                              _stream_ptr(stream)))
        return seeds, iters, conf, top


_hip = None


def _hip_copy(dst: int, src: int, nbytes: int) -> None:
    """Device-to-device copy between raw pointers (hipMemcpy, kind = default)."""
    global _hip
    torch = _torch()
    torch.cuda.synchronize()
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    rc = _hip.hipMemcpy(dst, src, nbytes, 4)
    if rc != 0:
        raise MiannError(3, f"hipMemcpy failed ({rc})")


def nearest_ghost(index: "Index", vectors, shard: int = 0, stream=None):
    """Ghost index of the nearest ghost node of `shard` for each row of `vectors` (device tensor)."""
    torch = _torch()
    out = torch.empty(vectors.shape[0], dtype=torch.int32, device=vectors.device)
    _check(load().miann_nearest_ghost(index.handle, shard, vectors.data_ptr(), vectors.shape[0], out.data_ptr(),
                                      _stream_ptr(stream)))
    return out


class Server:
    """Continuous-batching serving loop over a resident index (host query rows in, host results out)."""

    def __init__(self, index: "Index", num_streams: int = 4, max_batch_queries: int = 8192,
                 max_inflight_queries: int = 65536, memory_budget_bytes: int = 1 << 30):
        cfg = ServerConfig()
        load().miann_server_config_default(C.byref(cfg))
        cfg.num_streams, cfg.max_batch_queries = num_streams, max_batch_queries
        cfg.max_inflight_queries, cfg.memory_budget_bytes = max_inflight_queries, memory_budget_bytes
        h = C.c_void_p()
        _check(load().miann_server_create(index.handle, C.byref(cfg), C.byref(h)))
        self._h, self._index = h, index
        self._d = index.info()["d"]
        self._shapes = {}  # ticket -> (nq, k) of its request

    def submit(self, queries, k: int, itopk: int, max_iters: int, opts: SearchOptions | None = None) -> int:
        """queries: numpy array [nq][d] (float32, or uint8 for u8 indices). Returns a ticket."""
        import numpy as np
        qdt = np.uint8 if self._index.in_dtype == U8 else np.float32
        q = np.asarray(queries)
        if q.dtype != qdt or q.ndim != 2 or q.shape[1] != self._d:
            raise MiannError(1, f"queries: need [nq, {self._d}] {np.dtype(qdt)}, got {q.dtype} {q.shape}")
        q = np.ascontiguousarray(q)
        p = (opts or SearchOptions()).cstruct()
        t = C.c_uint64()
        _check(load().miann_server_submit(self._h, q.ctypes.data, q.shape[0], k, itopk, max_iters, C.byref(p),
                                          C.byref(t)))
        self._shapes[t.value] = (q.shape[0], k)
        return t.value

    def wait(self, ticket: int, nq: int | None = None, k: int | None = None):
        """Returns (ids uint32 [nq,k], dists [nq,k], latency_ms); the sizes are the request's own (nq and k, if
        given, must match them)."""
        import numpy as np
        if ticket not in self._shapes:
            raise MiannError(1, f"unknown or already waited ticket {ticket}")
        rq, rk = self._shapes[ticket]
        if (nq is not None and nq != rq) or (k is not None and k != rk):
            raise MiannError(1, f"ticket {ticket} is a request of {rq} queries with k = {rk}")
        nq, k = rq, rk
        del self._shapes[ticket]
        ids = np.empty((nq, k), np.uint32)
        dists = np.empty((nq, k), np.int32 if self._index.in_dtype == U8 else np.float32)
        lat = C.c_double()
        _check(load().miann_server_wait(self._h, ticket, ids.ctypes.data, dists.ctypes.data, C.byref(lat)))
        return ids, dists, lat.value

    def warm(self, nq: int, k: int, itopk: int, max_iters: int, opts: SearchOptions | None = None) -> None:
        """Sizes every stream's buffers for this shape with one search of nq zero queries per stream."""
        p = (opts or SearchOptions()).cstruct()
        _check(load().miann_server_warm(self._h, nq, k, itopk, max_iters, C.byref(p)))

    def replay(self, pool, row_start, nq, ks, itopks, max_iters, arrival_s, opts: SearchOptions | None = None):
        """Open-loop replay of a request trace (numpy arrays; request j = pool rows row_start[j] : row_start[j] +
        nq[j] arriving at arrival_s[j] seconds). Returns (latency_ms from the scheduled arrival [n_req], wall s)."""
        import numpy as np
        qdt = np.uint8 if self._index.in_dtype == U8 else np.float32
        pool = np.ascontiguousarray(pool)
        if pool.dtype != qdt or pool.ndim != 2 or pool.shape[1] != self._d:
            raise MiannError(1, f"pool: need [n, {self._d}] {np.dtype(qdt)}")
        n = len(arrival_s)
        rs = np.ascontiguousarray(row_start, np.int64)
        nn = np.ascontiguousarray(nq, np.int64)
        k = np.ascontiguousarray(ks, np.int32)
        it = np.ascontiguousarray(itopks, np.int32)
        T = np.ascontiguousarray(max_iters, np.int32)
        arr = np.ascontiguousarray(arrival_s, np.float64)
        if any(a.shape != (n,) for a in (rs, nn, k, it, T)):
            raise MiannError(1, "replay: trace arrays of different lengths")
        lat = np.empty(n, np.float64)
        wall = C.c_double()
        p = (opts or SearchOptions()).cstruct()
        _check(load().miann_server_replay(self._h, pool.ctypes.data, len(pool), rs.ctypes.data, nn.ctypes.data,
                                          k.ctypes.data, it.ctypes.data, T.ctypes.data, arr.ctypes.data, n,
                                          C.byref(p), lat.ctypes.data, C.byref(wall)))
        return lat, wall.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().miann_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            load().miann_server_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        if _lib is not None:
            self.close()


def as_u32(t):
    """int32 tensor holding uint32 ids -> numpy uint32."""
    return t.cpu().numpy().view("uint32")


def version() -> str:
    return load().miann_version().decode()
