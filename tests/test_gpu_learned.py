"""The learned entry / budget predictor end to end: labels from traces of the
search itself, training by the library's kernels, and the predicted-entry search
on held-out queries. Checks (1) parity of the predicted-entry search with the
oracle given the same seeds and budgets, and (2) the gain over ghost staging:
fewer distance evaluations at no loss of recall."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import oracle_from_device, oracle_kwargs, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
miann = pytest.importorskip("paper_2507_17094_amd")
from paper_2507_17094_amd import learned  # noqa: E402


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
    P, losses = learned.train(gx, tr, labels, hidden=128, epochs=12, batch=2048, lr=2e-3)
    say(f"  losses {[round(x, 3) for x in losses]}")
    assert losses[-1] < losses[0]
    gt, _ = gx.exact_knn(te, k)
    gt = gt.cpu().numpy().view(np.uint32)
    base = gx.search(te, k, itopk, T, opts, counters=True)
    (pi, pd, pc), seeds, iters, conf = learned.predicted_search(gx, P, te, k, itopk, 32, 0.05, 4, T, opts,
                                                                counters=True)
    torch.cuda.synchronize()
    rb = oracle.recall(gt, base[0].cpu().numpy().view(np.uint32), k)
    rp = oracle.recall(gt, pi.cpu().numpy().view(np.uint32), k)
    cb = base[2].cpu().numpy()
    cp = pc.cpu().numpy()
    cost_b = (cb[:, 0] + cb[:, 4]).mean()
    cost_p = (cp[:, 0] + cp[:, 4]).mean()
    fb = float((conf.cpu().numpy() < 0.05).mean())
    say(f"  ghost staging: recall {rb:.4f}, distances/query {cost_b:.1f}, iterations {cb[:, 2].mean():.1f}")
    say(f"  predictor:     recall {rp:.4f}, distances/query {cost_p:.1f}, iterations {cp[:, 2].mean():.1f}, "
        f"fallback {fb:.3f}")
    assert rp >= rb - 0.01
    assert cost_p < cost_b
    # parity of the predicted-entry search with the oracle on the same seeds and budgets
    ox = oracle_from_device(gx, X)
    po = miann.SearchOptions(**{**opts.__dict__, "entry": "predicted"})
    oi, od, oc = oracle.search(ox, Qte, seeds=seeds.cpu().numpy().view(np.uint32),
                               T_per_query=iters.cpu().numpy(), **oracle_kwargs(k, itopk, T, po))
    same = np.all(pi.cpu().numpy().view(np.uint32) == oi, axis=1).mean()
    say(f"  parity with the oracle: {same:.4f}")
    assert same >= 0.999
