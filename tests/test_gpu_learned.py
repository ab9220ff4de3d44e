"""The learned entry / budget predictor end to end: labels from traces of the
search itself, training by the library's kernels, and the predicted-entry search
on held-out queries. Checks (1) parity of the predicted-entry search with the
oracle given the same seeds and budgets, and (2) what the network gains over
ghost staging: at the same iteration cap the predicted entry reaches at least
ghost staging's recall with fewer distance evaluations, and with per-query
budgets it stays within 0.005 of ghost staging's full-budget recall at a
fifth fewer distance evaluations."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import oracle_from_device, oracle_kwargs, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")
from paper_2507_17094_amd import learned  # noqa: E402


def cost(c):
    """distance evaluations per query, main graph plus ghost stage"""
    c = c.cpu().numpy()
    return float((c[:, 0] + c[:, 4]).mean())


def test_predictor_gain_over_ghost_staging():
    d, C = 48, 40
    X = synth.mixture_small(40_000, d, C, 0.3, 401)
    Qtr = synth.mixture_small(20_000, d, C, 0.3, 402)
    Qte = synth.mixture_small(2_000, d, C, 0.3, 403)
    Xd = torch.from_numpy(X).cuda()
    gx = miann.Index.build(Xd, degree=32, num_shards=1, dgs_table=True, seed=5)
    gx.build_ghost(ratio=0.01, ghost_degree=32, seed=5)
    opts = miann.SearchOptions(entry="ghost_graph", dgs=True)
    k, itopk, T = 10, 64, 96
    tr = torch.from_numpy(Qtr).cuda()
    te = torch.from_numpy(Qte).cuda()
    labels = learned.make_labels(gx, tr, k, itopk, T, opts)
    # the labels against the oracle on a sample: the trace counter of the same search, and the ghost nearest to
    # the exact nearest node (brute force over nodes, then over ghosts)
    ox = oracle_from_device(gx, X)
    m = 400
    _, _, oc = oracle.search(ox, Qtr[:m], **oracle_kwargs(k, itopk, T, opts))
    it = labels.iters.cpu().numpy()[:m]
    assert np.mean(it == oc[:, 7]) >= 0.995  # (a near tie may change one query's path, as in the search parity)
    assert np.allclose(labels.budget.cpu().numpy()[:m], np.log1p(it.astype(np.float64)), rtol=1e-6, atol=0)
    nn, _ = oracle.knn(X, Qtr[:m], 1)
    gids = ox.shards[0]["g_map"]
    ge, _ = oracle.knn(X[gids], X[nn[:, 0]], 1)
    assert np.mean(labels.entry.cpu().numpy()[:m] == ge[:, 0]) >= 0.999
    P, losses = learned.train(gx, tr, labels, hidden=128, epochs=12, batch=2048, lr=2e-3)
    say(f"  losses {[round(x, 3) for x in losses]}")
    assert losses[-1] < 0.5 * losses[0]
    gt, _ = gx.exact_knn(te, k)
    gt = gt.cpu().numpy().view(np.uint32)

    def rec(ids):
        return oracle.recall(gt, ids.cpu().numpy().view(np.uint32), k)

    gmap = learned.ghost_map(gx)
    po = miann.SearchOptions(entry="predicted", dgs=True)
    # (a) entry only: the same iteration cap for both
    seeds, _, conf, _ = P.predict(te, 32, 0.0, gmap, 4, T)
    for Tc in (32, 64):
        b = gx.search(te, k, itopk, Tc, opts, counters=True)
        p = gx.search(te, k, itopk, Tc, po, seeds=seeds, counters=True)
        say(f"  cap {Tc}: ghost staging recall {rec(b[0]):.4f} dists {cost(b[2]):.0f} | "
            f"predicted entry recall {rec(p[0]):.4f} dists {cost(p[2]):.0f}")
        assert rec(p[0]) >= rec(b[0]) - 0.002
        assert cost(p[2]) < cost(b[2])
    # (b) entry and per-query budget against ghost staging at the full budget
    base = gx.search(te, k, itopk, T, opts, counters=True)
    (pi, pd, pc), seeds2, iters, conf2 = learned.predicted_search(gx, P, te, k, itopk, 32, 0.05, 4, T, opts,
                                                                  counters=True, gmap=gmap, budget_scale=3.0)
    rb, rp = rec(base[0]), rec(pi)
    fb = float((conf2.cpu().numpy() < 0.05).mean())
    say(f"  full budget: ghost staging recall {rb:.4f} dists {cost(base[2]):.0f}; predictor recall {rp:.4f} "
        f"dists {cost(pc):.0f} mean budget {iters.float().mean().item():.1f} fallback {fb:.3f}")
    assert rp >= rb - 0.005
    assert cost(pc) < 0.8 * cost(base[2])
    # parity of the predicted-entry search with the oracle on the same seeds and budgets
    ox = oracle_from_device(gx, X)
    oi, od, oc = oracle.search(ox, Qte, seeds=seeds2.cpu().numpy().view(np.uint32),
                               T_per_query=iters.cpu().numpy(), **oracle_kwargs(k, itopk, T, po))
    same = np.all(pi.cpu().numpy().view(np.uint32) == oi, axis=1).mean()
    say(f"  parity with the oracle: {same:.4f}")
    assert same >= 0.999
