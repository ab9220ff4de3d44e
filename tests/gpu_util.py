"""Helpers for the GPU parity tests: moving oracle-built indices to the device
library, reading device arrays back, and comparing results element by element."""
from __future__ import annotations

import ctypes
import sys

import numpy as np

import oracle
import paper_2507_17094_amd as miann

_hip = None


def hip():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip


def d2h(ptr: int, count: int, dtype) -> np.ndarray:
    """Copies `count` elements of `dtype` from a device pointer."""
    import torch
    torch.cuda.synchronize()
    out = np.empty(count, dtype=dtype)
    if count:
        rc = hip().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)
        assert rc == 0, rc
    return out


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray):
    import torch
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_device_index(ox: oracle.OracleIndex, dgs: bool = True) -> miann.Index:
    """Imports an oracle-built index (graphs, maps, ghost shards) into the library."""
    shards = []
    for sh in ox.shards:
        d = dict(vectors=dev(sh["orig_base"]), graph=dev(sh["graph"]), global_ids=dev(sh["gmap"]))
        if "next" in sh:
            d["next_map"] = dev(sh["next"])
        if "g_map" in sh:
            d["ghost_ids"] = dev(sh["g_map"])
            d["ghost_graph"] = dev(sh["g_graph"])
        shards.append(d)
    in_dt = "u8" if ox.shards[0]["orig_base"].dtype == np.uint8 else "f32"
    return miann.Index.import_shards(shards, d=ox.d, in_dtype=in_dt, store=ox.dtype, degree=ox.deg,
                                     ghost_degree=ox.deg_g if "g_map" in ox.shards[0] else 0, dgs_table=dgs)


def oracle_kwargs(k, itopk, T, o: miann.SearchOptions) -> dict:
    return dict(k=k, l=itopk, r=o.search_width, T=T, n_init=o.n_init or None, entry=o.entry, l_g=o.ghost_itopk,
                T_g=o.ghost_iters, t_seeds=o.t_seeds or None, dgs_on=o.dgs, discard=o.discard, cooldown=o.cooldown,
                random_discard=o.random_discard, ppe_on=o.ppe, forward_f=o.forward_f, rerank_mult=o.rerank_mult,
                stop_on_no_change=o.stop_on_no_change, ghost_every_stage=o.ghost_every_stage, seed=o.seed,
                dgs_threshold=o.dgs_threshold)


def run_both(ox, gx, Q: np.ndarray, k, itopk, T, opts: miann.SearchOptions, qkeys=None, seeds=None, Tq=None):
    import torch
    qd = dev(Q)
    gi, gd, gc = gx.search(qd, k, itopk, T, opts, counters=True,
                           qkeys=None if qkeys is None else torch.from_numpy(qkeys.astype(np.int64)).cuda(),
                           seeds=None if seeds is None else dev(seeds.astype(np.uint32)),
                           max_iters_per_query=None if Tq is None else dev(Tq.astype(np.int32)))
    torch.cuda.synchronize()
    g = (gi.cpu().numpy().view(np.uint32), gd.cpu().numpy(), gc.cpu().numpy())
    o = oracle.search(ox, Q, qkeys=qkeys, seeds=seeds, T_per_query=Tq, **oracle_kwargs(k, itopk, T, opts))
    return g, o


def ghost_entry(opts) -> bool:
    return opts.entry in ("ghost_graph", "ghost_dense", "predicted")


def compare(g, o, min_frac=0.999, check_counters=True, label="", ndist_check=True):
    """Element-wise parity. Returns the fraction of queries whose id lists match."""
    gi, gd, gc = g
    oi, od, oc = o
    same = np.all(gi == oi, axis=1)
    frac = float(same.mean()) if len(same) else 1.0
    say(f"  [{label}] id lists identical on {same.sum()}/{len(same)} queries")
    assert frac >= min_frac, f"{label}: only {frac:.4f} of id lists match"
    if od.dtype == np.int32:
        assert np.array_equal(gd[same], od[same]), f"{label}: u8 distances differ"
    else:
        a, b = gd[same].astype(np.float64), od[same].astype(np.float64)
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin)
        rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-30)
        assert rel.max(initial=0) <= 1e-5, f"{label}: max relative distance error {rel.max()}"
    if check_counters:
        # expansions, iterations, skipped slots, ghost expansions and rerank counts are
        # determined by the search path alone; distance counts depend on the visited hash
        for c in (1, 2, 3, 5, 6, 7):
            assert np.array_equal(gc[same, c], oc[same, c]), f"{label}: counter {c} differs"
        if ndist_check:
            # the device reuses the distances of ghost seeds; otherwise it evaluates at least
            # what the exact visited set evaluates
            assert np.all(gc[same, 0] >= oc[same, 0])
    return frac


def oracle_from_device(gx, X):
    """CPU copy of a device-built index (graph, sign table, shard maps, ghost shards) for the oracle."""
    info = gx.info()
    ox = oracle.OracleIndex(dtype="u8" if X.dtype == np.uint8 else "f32", d=info["d"], deg=info["degree"],
                            S=info["num_shards"], n_total=info["n"])
    for s in range(info["num_shards"]):
        v = gx.shard(s)
        n, deg, W = v.n, v.degree, v.W
        gmap = d2h(v.global_ids, n, np.uint32)
        Xs = np.ascontiguousarray(X[gmap])
        sh = dict(n=n, gmap=gmap, orig_base=Xs, codes=Xs, graph=d2h(v.graph, n * deg, np.uint32).reshape(n, deg))
        if v.sign:
            sh["sign"] = np.ascontiguousarray(d2h(v.sign, n * W * deg, np.uint32).reshape(n, W, deg).transpose(0, 2, 1))
        if v.next_map:
            sh["next"] = d2h(v.next_map, n, np.uint32)
        if v.n_ghost:
            sh["R"] = v.n_ghost
            sh["g_map"] = d2h(v.ghost_ids, v.n_ghost, np.uint32)
            sh["g_graph"] = d2h(v.ghost_graph, v.n_ghost * v.ghost_degree, np.uint32).reshape(v.n_ghost,
                                                                                                v.ghost_degree)
            sh["g_codes"] = np.ascontiguousarray(Xs[sh["g_map"]])
            ox.deg_g = v.ghost_degree
        ox.shards.append(sh)
    return ox
