"""CPU checks of the predictor parity tolerances (tests/mlp_bounds.py): a
float32-accumulating implementation with the device's bf16 rounding points,
summing in shuffled orders, stays inside the element-wise bounds around the
float64 reference, most bf16 values agree exactly, and planted mistakes of the
kind the bounds must catch (a dropped bias-gradient slice, the budget head's
lambda dropped, a wrong-sign term) fall outside them."""
import numpy as np
import pytest

import mlp_bounds as mb
from oracle import mlp


def model(d, h, R, seed):
    rng = np.random.default_rng(seed)
    a1, a2 = np.sqrt(6 / d), np.sqrt(6 / h)
    return {"W1": rng.uniform(-a1, a1, (d, h)), "b1": rng.standard_normal(h) * 0.05,
            "W2": rng.uniform(-a2, a2, (h, h)), "b2": rng.standard_normal(h) * 0.05,
            "W3": rng.uniform(-a2, a2, (h, R + 1)), "b3": rng.standard_normal(R + 1) * 0.05}


@pytest.mark.parametrize("d,h,R,B,lam", [(16, 32, 20, 40, 0.5), (48, 96, 120, 64, 3.0), (96, 256, 300, 48, 1.0)])
def test_bounds_cover_float32_accumulation(d, h, R, B, lam):
    P = model(d, h, R, 1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((B, d)).astype(np.float32)
    lab = rng.integers(0, R, B)
    y = rng.uniform(0, 4, B)
    loss, lb, g, E = mb.grad_bounds(P, x, lab, y, lam)
    ref_loss, ref_g, _ = mlp.forward_backward(P, x, lab, y, lam, bf16_mode=True)
    assert loss == pytest.approx(ref_loss, rel=1e-12)
    for k in ref_g:
        assert np.allclose(g[k], ref_g[k], rtol=1e-12, atol=1e-15), k
    tight = mb.tight_grad_tolerances(P, x, lab, y, lam)
    assert abs(E["b3"][R]) < 0.05 * abs(g["b3"][R])  # the budget head's check is meaningful
    for seed in range(3):
        eloss, eg, _ = mb.emulate_f32_device(P, x, lab, y, lam, order_seed=seed)
        assert abs(eloss - loss) <= lb
        for k in g:
            err = np.abs(eg[k] - g[k])
            assert np.all(err <= E[k]), (k, float((err - E[k]).max()))
            assert (err <= tight[k]).mean() >= 0.99, k
    # the bounds are tight: most entries carry less than 1% of the sum of the terms' magnitudes
    F = mb.forward_bounds(P, x)
    H1, E1 = F["H1"]
    assert (E1 == 0).mean() > 0.9  # bf16 activations are required to match exactly almost everywhere


def test_bounds_catch_planted_mistakes():
    d, h, R, B, lam = 24, 48, 30, 50, 0.5
    P = model(d, h, R, 3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((B, d)).astype(np.float32)
    lab = rng.integers(0, R, B)
    y = rng.uniform(0, 4, B)
    _, _, g, E = mb.grad_bounds(P, x, lab, y, lam)
    _, eg, _ = mb.emulate_f32_device(P, x, lab, y, lam)
    # (1) the budget head's gradient computed with lambda = 1 instead of lambda
    _, eg1, _ = mb.emulate_f32_device(P, x, lab, y, 1.0)
    assert np.any(np.abs(eg1["W3"][:, R] - g["W3"][:, R]) > E["W3"][:, R])
    assert np.abs(eg1["b3"][R] - g["b3"][R]) > E["b3"][R]
    # (2) a slice of a bias gradient left at zero
    bad = eg["b2"].copy()
    bad[:8] = 0.0
    assert np.any(np.abs(bad - g["b2"]) > E["b2"])
    # (3) one wrong-sign row of the first layer's gradient
    badw = eg["W1"].copy()
    badw[3] = -badw[3]
    assert np.any(np.abs(badw - g["W1"]) > E["W1"])


def test_tight_logit_tolerance_covers_float32_accumulation():
    d, h, R, n = 96, 256, 1000, 200
    P = model(d, h, R, 5)
    x = np.random.default_rng(4).standard_normal((n, d)).astype(np.float32)
    Z, EZ = mb.forward_bounds(P, x)["Z"]
    T = mb.tight_logit_tolerance(P, x)
    for seed in range(2):
        _, _, Ze = mb.emulate_f32_device(P, x, np.zeros(n, np.int64), np.zeros(n), 1.0, order_seed=seed)
        err = np.abs(Ze - Z)
        assert np.all(err <= EZ)
        assert (err <= T).mean() >= 0.99
