#!/usr/bin/env python
"""Throughput of the batched graph beam search on one MI355X.

Workload (the paper-shaped sharded configuration): N = 1,000,000 base vectors,
d = 96 float32 from a 1,000-component Gaussian mixture (std 0.25), 4 shards
resident on the GPU with path extension between them, a degree-32 graph per
shard built on the GPU (MFMA exact k-NN + pruning), ghost staging over a 1%
sample per shard with its own degree-32 graph, the direction-guided filter,
10,000 queries, k = 10. The search width is swept over itopk in
{32, 64, 128, 256} (and the iteration budget), and the fastest setting whose
recall@10 against exact ground truth is >= 0.95 is timed.

One step = one batched search of all queries through the whole hot path
(ghost entry, per-shard stages with path extension, cross-shard merge).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QPS at recall@10≥0.95, 1 MI355X, tuned vs plain FP32 search; p99 latency"
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "sharded1m": dict(N=1_000_000, d=96, C=1000, sigma=0.25, nq=10_000, k=10, deg=32, S=4, ghost_ratio=0.01,
                      deg_g=32, itopks=(32, 64, 128, 256)),
    "tiny": dict(N=10_000, d=128, C=32, sigma=0.3, nq=1_000, k=10, deg=32, S=1, ghost_ratio=0.01, deg_g=32,
                 itopks=(32, 64, 128)),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recall(gt, ann, k):
    hit = 0
    for a, b in zip(gt[:, :k], ann[:, :k]):
        hit += len(np.intersect1d(a, b))
    return hit / (k * len(gt))


def d2h(ptr, count, dtype):
    import ctypes
    import torch
    torch.cuda.synchronize()
    out = np.empty(count, dtype=dtype)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    if count:
        assert hip.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) == 0
    return out


def oracle_from_device(gx, X):
    """CPU copy of a device-built index (graph, sign table, shard maps, ghost shards) for the oracle."""
    import oracle
    info = gx.info()
    ox = oracle.OracleIndex(dtype="f32", d=info["d"], deg=info["degree"], S=info["num_shards"], n_total=info["n"])
    for s in range(info["num_shards"]):
        v = gx.shard(s)
        n, deg, W = v.n, v.degree, v.W
        gmap = d2h(v.global_ids, n, np.uint32)
        Xs = np.ascontiguousarray(X[gmap])
        sh = dict(n=n, gmap=gmap, orig_base=Xs, codes=Xs,
                  graph=d2h(v.graph, n * deg, np.uint32).reshape(n, deg),
                  sign=np.ascontiguousarray(d2h(v.sign, n * W * deg, np.uint32).reshape(n, W, deg).transpose(0, 2, 1)))
        if v.next_map:
            sh["next"] = d2h(v.next_map, n, np.uint32)
        if v.n_ghost:
            sh["R"] = v.n_ghost
            sh["g_map"] = d2h(v.ghost_ids, v.n_ghost, np.uint32)
            sh["g_graph"] = d2h(v.ghost_graph, v.n_ghost * v.ghost_degree, np.uint32).reshape(v.n_ghost, v.ghost_degree)
            sh["g_codes"] = np.ascontiguousarray(Xs[sh["g_map"]])
            ox.deg_g = v.ghost_degree
        ox.shards.append(sh)
    return ox


def algorithmic_bytes(ctr, d, deg, deg_g, W, n_keep, S, k, row_bytes, ghost_in_stage):
    """Bytes the stage kernel must move per batch, from the per-query counters:
    gathered vectors (n_dist rows), adjacency rows (n_exp), direction-table rows
    and parent vectors of the expansions made under the filter, ghost-graph
    vectors and rows (graph-mode entry, which runs inside the stage kernel),
    the query per stage and the results per stage. The dense entry runs in its
    own kernel and is not counted here."""
    n_dist, n_exp, skipped = ctr[:, 0].sum(), ctr[:, 1].sum(), ctr[:, 3].sum()
    n_dist_g, n_exp_g = (ctr[:, 4].sum(), ctr[:, 5].sum()) if ghost_in_stage else (0, 0)
    n_exp_dgs = skipped / max(1, deg - n_keep) if deg > n_keep else 0
    nq = ctr.shape[0]
    vec = n_dist * row_bytes
    b = (vec + n_exp * deg * 4 + n_exp_dgs * (deg * W * 4 + row_bytes) + n_dist_g * row_bytes + n_exp_g * deg_g * 4
         + nq * S * (d * 4 + k * 8))
    return float(b), float(vec)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sharded1m", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=0, help="queries for the oracle leg (0 = all)")
    ap.add_argument("--plain", type=int, default=1, help="also sweep the plain (unsharded, random-entry) search")
    ap.add_argument("--fixed", default="", help="skip the sweep: itopk,T,entry,search_width,ghost_every_stage")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the path-extension ring is "
                                   "exercised with shards resident on one GPU)"}))
        sys.exit(2)

    import torch

    import paper_2507_17094_amd as miann
    import synth

    W = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    t0 = time.time()
    if W["N"] > 100_000:
        X = synth.mixture(W["N"], W["d"], W["C"], W["sigma"], synth.SEED_BASE)
        Q = synth.mixture(W["nq"], W["d"], W["C"], W["sigma"], synth.SEED_QUERIES)
    else:
        X = synth.mixture_small(W["N"], W["d"], W["C"], W["sigma"], synth.SEED_BASE)
        Q = synth.mixture_small(W["nq"], W["d"], W["C"], W["sigma"], synth.SEED_QUERIES)
    log(f"data {X.shape} {Q.shape} in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    k, nq = W["k"], W["nq"]

    torch.cuda.synchronize()
    t0 = time.time()
    gx = miann.Index.build(Xd, degree=W["deg"], num_shards=W["S"], dgs_table=True, seed=5)
    t_graph = time.time() - t0
    t0 = time.time()
    gx.build_ghost(ratio=W["ghost_ratio"], ghost_degree=W["deg_g"], seed=5)
    t_ghost = time.time() - t0
    log(f"build: graph {t_graph:.2f}s ghost {t_ghost:.2f}s")
    t0 = time.time()
    gt_i, gt_d = gx.exact_knn(Qd, k)
    torch.cuda.synchronize()
    t_gt = time.time() - t0
    gt = gt_i.cpu().numpy().view(np.uint32)
    log(f"ground truth (MFMA exact k-NN) {t_gt:.2f}s")

    def run(ix, itopk, T, opts, counters=False):
        return ix.search(Qd, k, itopk, T, opts, counters=counters)

    def timed(ix, itopk, T, opts, reps=2):
        run(ix, itopk, T, opts)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            run(ix, itopk, T, opts)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    def sweep(ix, form, opts_list, itopks, Ts):
        rows = []
        for itopk in itopks:
            for T in Ts:
                if T > 2 * itopk:
                    continue
                for name, opts in opts_list:
                    ids, _ = run(ix, itopk, T, opts)
                    torch.cuda.synchronize()
                    rc = recall(gt, ids.cpu().numpy().view(np.uint32), k)
                    sec = timed(ix, itopk, T, opts)
                    rows.append(dict(form=form, variant=name, itopk=itopk, T=T, recall=rc, qps=nq / sec, opts=opts))
                    log(f"  {form:6s} {name:14s} itopk={itopk:3d} T={T:4d} recall={rc:.4f} qps={nq / sec:,.0f}")
        ok = [r for r in rows if r["recall"] >= 0.95]
        best = max(ok, key=lambda r: r["qps"]) if ok else max(rows, key=lambda r: r["recall"])
        return best, rows

    tuned_opts = []
    for r in (1, 2):
        tuned_opts += [(f"gs+dgs r{r}", miann.SearchOptions(entry="ghost_graph", dgs=True, search_width=r)),
                       (f"gsdense+dgs r{r}", miann.SearchOptions(entry="ghost_dense", dgs=True, search_width=r)),
                       (f"gsdense-all+dgs r{r}", miann.SearchOptions(entry="ghost_dense", dgs=True, search_width=r,
                                                                     ghost_every_stage=True))]
    if args.fixed:
        f = args.fixed.split(",")
        fo = miann.SearchOptions(entry=f[2], dgs=True, search_width=int(f[3]), ghost_every_stage=bool(int(f[4])))
        ids, _ = run(gx, int(f[0]), int(f[1]), fo)
        torch.cuda.synchronize()
        best = dict(form="tuned", variant="fixed", itopk=int(f[0]), T=int(f[1]), opts=fo,
                    recall=recall(gt, ids.cpu().numpy().view(np.uint32), k), qps=0.0)
        tuned_rows = [best]
    else:
        log("sweep: tuned (ghost staging + direction filter + path extension)")
        best, tuned_rows = sweep(gx, "tuned", tuned_opts, W["itopks"], (16, 32, 64, 128))

    plain = None
    if args.plain:
        log("building the plain unsharded index")
        gp = miann.Index.build(Xd, degree=W["deg"], num_shards=1, dgs_table=False, seed=5)
        plain_opts = [(f"n_init={n}", miann.SearchOptions(n_init=n)) for n in (2048, 4096)]
        pbest, _ = sweep(gp, "plain", plain_opts, W["itopks"], (32, 64, 128))
        plain = {k_: pbest[k_] for k_ in ("variant", "itopk", "T", "recall", "qps")}
        del gp

    itopk, T, opts = best["itopk"], best["T"], best["opts"]
    # counters and live per-launch timing of the chosen setting
    ids, dists, ctr = run(gx, itopk, T, opts, counters=True)
    ctr = ctr.cpu().numpy()
    phases = []
    for _ in range(3):
        ph = []
        gx.search(Qd, k, itopk, T, opts, phase_ms=ph)
        phases.append(ph)
    phases = np.array(phases).mean(0)
    S = W["S"]
    stage_ms = phases[1:1 + S]
    v0 = gx.shard(0)
    row_bytes = v0.d_pad * 4
    n_keep = W["deg"] - (int(round(opts.discard * 1000)) * W["deg"]) // 1000 if opts.dgs else W["deg"]
    bytes_total, vec_bytes = algorithmic_bytes(ctr, W["d"], W["deg"], W["deg_g"], v0.W, n_keep, S, k, row_bytes,
                                               opts.entry == "ghost_graph")
    stage_total_ms = float(stage_ms.sum())
    achieved = bytes_total / (stage_total_ms * 1e-3) / 1e9

    # timed steps
    for _ in range(args.warmup):
        run(gx, itopk, T, opts)
    torch.cuda.synchronize()
    starts, ends = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run(gx, itopk, T, opts)
        e1.record()
        starts.append(e0)
        ends.append(e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([s_.elapsed_time(e_) for s_, e_ in zip(starts, ends)])
    ms_per_step = wall / args.steps * 1e3
    qps = nq * args.steps / wall

    out = {
        "metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={W['N']} d={W['d']} f32 vectors, {W['C']}-component mixture "
                               f"std {W['sigma']}, degree {W['deg']}, {S} resident shards with path extension, "
                               f"ghost ratio {W['ghost_ratio']}, direction filter", "nq": nq, "k": k,
                   "itopk": itopk, "max_iters": T, "entry": opts.entry, "dgs": bool(opts.dgs),
                   "search_width": opts.search_width, "ghost_every_stage": bool(opts.ghost_every_stage),
                   "recall@10": best["recall"], "distance_accumulation": "f64 of f32 inputs"},
        "latency_ms": {"batch_p50": float(np.percentile(step_ms, 50)), "batch_p99": float(np.percentile(step_ms, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "stage_kernel", "stage_ms": [float(x) for x in stage_ms],
                     "bytes_per_launch": bytes_total / S,
                     "gathered_vector_GBps": vec_bytes / (stage_total_ms * 1e-3) / 1e9},
        "counters_per_query": {"n_dist": float(ctr[:, 0].mean()), "n_exp": float(ctr[:, 1].mean()),
                               "iters": float(ctr[:, 2].mean()), "dgs_skipped": float(ctr[:, 3].mean()),
                               "n_dist_ghost": float(ctr[:, 4].mean())},
        "build_s": {"graph": t_graph, "ghost": t_ghost, "ground_truth": t_gt},
        "plain": plain,
        "sweep": [{k_: r[k_] for k_ in ("form", "variant", "itopk", "T", "recall", "qps")} for r in tuned_rows],
    }
    if args.cpu_baseline:
        import oracle
        ox = oracle_from_device(gx, X)
        m = args.cpu_sample or nq
        okw = dict(k=k, l=itopk, T=T, entry=opts.entry, dgs_on=opts.dgs, l_g=opts.ghost_itopk, T_g=opts.ghost_iters,
                   r=opts.search_width, ghost_every_stage=opts.ghost_every_stage)
        t0 = time.perf_counter()
        oi, od, _ = oracle.search(ox, Q[:m], **okw)
        t_cpu = time.perf_counter() - t0
        gi = ids.cpu().numpy().view(np.uint32)[:m]
        out["cpu_baseline"] = {"value": m / t_cpu, "unit": "queries/s", "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"first {m} of the {nq} queries, same index and parameters"}
        out["parity_full_size"] = {"queries": m, "id_lists_identical": float(np.all(gi == oi, axis=1).mean())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
