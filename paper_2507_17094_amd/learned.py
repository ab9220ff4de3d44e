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

from dataclasses import dataclass

from . import Index, Predictor, SearchOptions, nearest_ghost


@dataclass
class Labels:
    entry: object   # torch int32 [n] ghost index
    budget: object  # torch float32 [n] log(1 + iterations)
    iters: object   # torch int32 [n]


def make_labels(index: Index, queries, k: int, itopk: int, t_max: int, opts: SearchOptions) -> Labels:
    """Entry and budget labels for `queries` (device float32 [n][d]) on a one-shard index."""
    import torch
    assert index.info()["num_shards"] == 1, "the learned entry is defined for one shard"
    _, _, ctr = index.search(queries, k, itopk, t_max, opts, counters=True)
    last = ctr[:, 7].to(torch.int32)
    nn_ids, _ = index.exact_knn(queries, 1)
    # vectors of the exact nearest neighbours (global id == local id for one shard)
    nn_vec = _gather_rows(index, nn_ids[:, 0])
    entry = nearest_ghost(index, nn_vec)
    return Labels(entry=entry, budget=torch.log1p(last.float()), iters=last)


def _gather_rows(index: Index, ids):
    """Original vectors of `ids` from shard 0 (device gather through torch indexing of a view)."""
    import torch
    v = index.shard(0)
    d, n = v.d, v.n
    esz = 1 if index.in_dtype == 3 else 4
    dp = (d * esz + 127) // 128 * 128 // esz  # originals rows are padded to 128 bytes
    flat = torch.empty(n * dp * esz, dtype=torch.uint8, device="cuda")
    from . import _hip_copy
    _hip_copy(flat.data_ptr(), v.originals, n * dp * esz)
    rows = flat.view(n, dp * esz)[ids.long()]
    if esz == 4:
        return rows.view(torch.float32)[:, :d].contiguous()
    return rows[:, :d].contiguous()


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
