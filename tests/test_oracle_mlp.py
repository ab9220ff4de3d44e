"""Pins for the predictor's CPU reference (oracle/mlp.py): its backward pass
against central finite differences of its own float64 loss, the closed-form
output gradient of softmax cross-entropy, and the bf16 rounding helper against
torch's bfloat16 conversion."""
import numpy as np
import pytest

from oracle import mlp


def small_model(d=7, h=9, R=5, seed=0):
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((d, h)) * 0.5, "b1": rng.standard_normal(h) * 0.1,
            "W2": rng.standard_normal((h, h)) * 0.4, "b2": rng.standard_normal(h) * 0.1,
            "W3": rng.standard_normal((h, R + 1)) * 0.4, "b3": rng.standard_normal(R + 1) * 0.1}


def test_backward_matches_finite_differences():
    P = small_model()
    rng = np.random.default_rng(1)
    x = rng.standard_normal((6, 7))
    lab = rng.integers(0, 5, 6)
    y = rng.standard_normal(6)
    lam = 0.7
    _, g, _ = mlp.forward_backward(P, x, lab, y, lam, bf16_mode=False)
    eps = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = mlp.loss_only(P, x, lab, y, lam)
            flat[idx] = old - eps
            lm = mlp.loss_only(P, x, lab, y, lam)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_output_gradient_is_softmax_minus_onehot():
    P = small_model(R=4)
    x = np.random.default_rng(2).standard_normal((3, 7))
    lab = np.array([0, 3, 1])
    _, g, cache = mlp.forward_backward(P, x, lab, np.zeros(3), 0.0, bf16_mode=False)
    Z = cache["Z"][:, :4]
    p = np.exp(Z - Z.max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    p[np.arange(3), lab] -= 1.0
    # dL/db3 over the entry logits is the column sum of (softmax - onehot) / B
    assert np.allclose(g["b3"][:4], p.sum(0) / 3, atol=1e-12)
    assert abs(g["b3"][4]) < 1e-15  # lambda = 0: no budget gradient


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(5000) * 10, rng.standard_normal(1000) * 1e-3,
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(mlp.bf16(x), ref)


def test_readout_budget_and_fallback():
    Z = np.array([[0.0, 5.0, 5.0, 1.0, np.log(1 + 7.5 / 1.25)], [1.0, 1.0, 1.0, 1.0, 0.0]])
    seeds, T, conf, order = mlp.readout(Z, 2, 0.3, np.array([10, 11, 12, 13]), 4, 100)
    assert order[0].tolist() == [1, 2]  # tie -> smaller index first
    assert seeds[0].tolist() == [11, 12] and T[0] == 8
    assert conf[1] == pytest.approx(0.25) and seeds[1, 0] == 0xFFFFFFFF and T[1] == 100
    # the margin scales the budget: ceil(3 * 6) = 18
    _, T3, _, _ = mlp.readout(Z, 2, 0.3, np.array([10, 11, 12, 13]), 4, 100, budget_scale=3.0)
    assert T3[0] == 18 and T3[1] == 100
