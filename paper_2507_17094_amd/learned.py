"""Learned entry / iteration-budget predictor around the search (host orchestration).

Every step runs in the library's kernels; this module only sequences C-ABI
calls:

1. traces: the search without the predictor (ghost entry) runs on training
   queries with counters; the iteration in which its top-k last changed is the
   budget label y = log(1 + iterations). The entry label is the ghost node
   nearest to the query's exact nearest neighbour (MFMA exact k-NN, then the
   nearest-ghost kernel), i.e. the region a converged plain search ends in.
2. training: the BF16 MLP (d -> hidden -> hidden -> R + 1) with the library's
   forward/backward/Adam kernels.
3. use: seeds = ghost map of the top-t entry logits, per-query budget
   T_q = clamp(ceil(s (exp(y) - 1)), t_min, T_max) with a margin s (default 2); queries whose
   confidence (max softmax probability) is below tau fall back to the ghost
   entry inside the same search launch.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import Index, Predictor, SearchOptions


@dataclass
class Labels:
    entry: object   # torch int32 [n] ghost index
    budget: object  # torch float32 [n] log(1 + iterations)
    iters: object   # torch int32 [n]


def make_labels(index: Index, queries, k: int, itopk: int, t_max: int, opts: SearchOptions) -> Labels:
    """Entry and budget labels for `queries` (device float32 [n][d]) on a one-shard index
    (miann_predictor_labels: the search's trace, the exact nearest node and its nearest ghost, all on the device)."""
    import torch
    from . import _check, _require, _stream_ptr, load
    _require(queries, "queries", (torch.float32,), (None, index.info()["d"]))
    n = queries.shape[0]
    entry = torch.empty(n, dtype=torch.int32, device=queries.device)
    budget = torch.empty(n, dtype=torch.float32, device=queries.device)
    iters = torch.empty(n, dtype=torch.int32, device=queries.device)
    p = opts.cstruct()
    _check(load().miann_predictor_labels(index.handle, queries.data_ptr(), n, k, itopk, t_max, C.byref(p),
                                         entry.data_ptr(), budget.data_ptr(), iters.data_ptr(), _stream_ptr()))
    return Labels(entry=entry, budget=budget, iters=iters)


def train(index: Index, queries, labels: Labels, hidden: int = 256, epochs: int = 10, batch: int = 4096,
          lr: float = 1e-3, lam: float = 1.0, seed: int = 1) -> tuple:
    v = index.shard(0)
    P = Predictor(queries.shape[1], hidden, int(v.n_ghost), seed=seed)
    losses = P.train(queries, labels.entry, labels.budget, epochs=epochs, batch=batch, lr=lr, lam=lam, seed=seed + 1)
    return P, losses


def ghost_map(index: Index):
    """Device copy of shard 0's ghost map (ghost index -> node id), int32 view of uint32."""
    import torch
    from . import _hip_copy
    v = index.shard(0)
    gmap = torch.empty(int(v.n_ghost), dtype=torch.int32, device="cuda")
    _hip_copy(gmap.data_ptr(), v.ghost_ids, int(v.n_ghost) * 4)
    return gmap


def predicted_search(index: Index, P: Predictor, queries, k: int, itopk: int, t: int, tau: float, t_min: int,
                     t_max: int, opts: SearchOptions, counters: bool = False, gmap=None, budget_scale: float = 2.0):
    """Seeds and per-query budgets from the predictor; low-confidence queries use the ghost entry.
    `gmap` (from ghost_map) may be passed to avoid copying the ghost map on every call."""
    if gmap is None:
        gmap = ghost_map(index)
    seeds, iters, conf, _ = P.predict(queries, t, tau, gmap, t_min, t_max, budget_scale)
    o = SearchOptions(**{**opts.__dict__, "entry": "predicted"})
    out = index.search(queries, k, itopk, t_max, o, seeds=seeds, max_iters_per_query=iters, counters=counters)
    return out, seeds, iters, conf
