"""Element-wise tolerances for the predictor's GPU parity tests (test infrastructure).

The device and the CPU reference (oracle/mlp.py) round to bfloat16 at the same
points: the inputs, the weight copies used by the products, the hidden
activations after bias and ReLU, and the gradients fed to the backward
products. They differ only in how products are accumulated: float32 on the
device (in an order the matrix cores choose), float64 in the reference. This
module carries, next to every reference value r, a bound E with |device - r| <= E:

* A float32 dot product of K exact products (bf16 x bf16 is exact in float32)
  plus a bias differs from the exact sum by at most (K + 2) 2^-24 times the sum
  of the terms' magnitudes (doubled here, in case the matrix cores' accumulator
  truncates instead of rounding to nearest). Errors of the operands add sum(E_a |b| + |a| E_b +
  E_a E_b).
* Rounding to bfloat16 is monotone: if the device's value lies in [r - E, r + E]
  its rounded value lies in [f(r - E), f(r + E)]. Where both ends round to the
  same bfloat16 value (no rounding boundary within the interval) the device's
  rounded value equals the reference's exactly, so E becomes 0; otherwise it is
  the width of that interval.
* ReLU masks in the backward pass are uncertain only where the activation's
  interval reaches zero; there the device value may be 0 or the unmasked one.
* Softmax: |d log p_j| <= |dz_j| + max_k |dz_k|, plus a few float32 roundings
  per term (exp, the R-term sum, the division).

So most bf16 values are required to be bit-identical, and only values whose
float32 accumulation could land on the other side of a bf16 rounding boundary
get one bf16 step of slack, which the later products then carry forward.

These worst-case bounds hold for every element, but they compound through the
layers (each possible bf16 step is assumed to happen, all in one direction), so
at hidden size 256 they are loose. The tight tolerance (`tight_*`) is the
probabilistic bound of Higham and Mary (SIAM J. Sci. Comput. 41(5), 2019): a
float32 sum of K terms is within lambda sqrt(K) u times the sum of their
magnitudes except with probability below 2 K exp(-lambda^2 / 2), taken here
with lambda = 16, for each product computed from the reference's own bf16
operands (no upstream bf16 step). The tests require every element within the
worst-case bound and nearly every element within the tight one.
"""
from __future__ import annotations

import numpy as np

from oracle.mlp import bf16

U = 2.0 ** -24  # float32 unit roundoff


def _round_bound(a, e, fn=bf16):
    """Reference value fn(a) and the bound on |fn(a') - fn(a)| for |a' - a| <= e (fn monotone)."""
    r = fn(a)
    lo, hi = fn(a - e), fn(a + e)
    return r, np.maximum(hi - r, r - lo)


def _relu_bf16(x):
    return bf16(np.maximum(x, 0.0))


def _matmul_bound(A, EA, B, EB, bias=None, K=None):
    """Bound on |float32 (A' B' + bias) - (A B + bias)|, |A' - A| <= EA, |B' - B| <= EB."""
    K = A.shape[1] if K is None else K
    absA, absB = np.abs(A), np.abs(B)
    mag = absA @ absB
    if bias is not None:
        mag = mag + np.abs(bias)
    prop = EA @ absB + absA @ EB + EA @ EB
    # 2 (K + 2) u: each of the K + 1 additions rounds once, with slack for an accumulator that
    # rounds toward zero instead of to nearest
    return prop + 2 * (K + 2) * U * (mag + prop)


def _masked_round_bound(a, e, h_ref, h_err):
    """bf16(a * [h > 0]) where h is an activation with bound h_err: the mask is certain unless the
    activation's interval reaches zero."""
    sure_on = h_ref - h_err > 0
    sure_off = (h_ref == 0) & (h_err == 0)
    r = bf16(a * (h_ref > 0))
    lo, hi = bf16(a - e), bf16(a + e)
    on_err = np.maximum(hi - r, r - lo)
    off_err = np.abs(r)
    amb_err = np.maximum(np.maximum(on_err, off_err), np.maximum(np.abs(lo - r), np.abs(hi - r)))
    E = np.where(sure_on, on_err, np.where(sure_off, off_err * 0.0, amb_err))
    return r, E


def forward_bounds(params: dict, x):
    """Reference forward (bf16 rounding points, float64 sums) with bounds. Returns dict of (value, bound)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    X = bf16(x)
    W1b, W2b, W3b = bf16(W1), bf16(W2), bf16(W3)
    zX, zW1, zW2, zW3 = (np.zeros_like(a) for a in (X, W1b, W2b, W3b))
    pre1 = X @ W1b + b1
    e1 = _matmul_bound(X, zX, W1b, zW1, b1)
    H1, E1 = _round_bound(pre1, e1, _relu_bf16)
    pre2 = H1 @ W2b + b2
    e2 = _matmul_bound(H1, E1, W2b, zW2, b2)
    H2, E2 = _round_bound(pre2, e2, _relu_bf16)
    Z = H2 @ W3b + b3
    EZ = _matmul_bound(H2, E2, W3b, zW3, b3)
    return dict(X=(X, zX), W1b=W1b, W2b=W2b, W3b=W3b, H1=(H1, E1), H2=(H2, E2), Z=(Z, EZ))


def softmax_bounds(Z, EZ, R):
    """Softmax over the first R columns with the bound of |p' - p| (float32 device arithmetic)."""
    logits = Z[:, :R]
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    s = e.sum(axis=1, keepdims=True)
    p = e / s
    Erow = EZ[:, :R].max(axis=1, keepdims=True)
    rel = EZ[:, :R] + Erow + (R + 8) * U
    return p, p * np.expm1(rel) * 1.01, s[:, 0], m[:, 0], Erow[:, 0]


def grad_bounds(params: dict, x, lab, y, lam: float):
    """Reference loss and gradients (oracle/mlp.py's rounding points) with element-wise bounds.
    Returns (loss, loss_bound, grads, bounds)."""
    F = forward_bounds(params, x)
    X, EX = F["X"]
    H1, E1 = F["H1"]
    H2, E2 = F["H2"]
    Z, EZ = F["Z"]
    W2b, W3b = F["W2b"], F["W3b"]
    B = X.shape[0]
    R = Z.shape[1] - 1
    lab = np.clip(np.asarray(lab, np.int64), 0, R - 1)
    y = np.asarray(y, np.float64)
    p, Ep, s, m, Erow = softmax_bounds(Z, EZ, R)
    onehot = np.zeros_like(p)
    onehot[np.arange(B), lab] = 1.0
    a = np.empty_like(Z)
    ea = np.empty_like(Z)
    a[:, :R] = (p - onehot) / B
    ea[:, :R] = (Ep + 4 * U * (np.abs(p - onehot) + 1.0)) / B
    diff = Z[:, R] - y
    a[:, R] = 2.0 * lam * diff / B
    ea[:, R] = 2.0 * abs(lam) * (EZ[:, R] + 4 * U * (np.abs(diff) + np.abs(y))) / B
    dZ, EdZ = _round_bound(a, ea)
    g, Eg = {}, {}
    g["W3"] = H2.T @ dZ
    Eg["W3"] = _matmul_bound(H2.T, E2.T, dZ, EdZ, K=B)
    g["b3"] = dZ.sum(axis=0)
    Eg["b3"] = EdZ.sum(axis=0) + (B + 2) * U * np.abs(dZ).sum(axis=0)
    a2 = dZ @ W3b.T
    e2 = _matmul_bound(dZ, EdZ, W3b.T, np.zeros_like(W3b.T))
    dH2, EdH2 = _masked_round_bound(a2, e2, H2, E2)
    g["W2"] = H1.T @ dH2
    Eg["W2"] = _matmul_bound(H1.T, E1.T, dH2, EdH2, K=B)
    g["b2"] = dH2.sum(axis=0)
    Eg["b2"] = EdH2.sum(axis=0) + (B + 2) * U * np.abs(dH2).sum(axis=0)
    a1 = dH2 @ W2b.T
    e1 = _matmul_bound(dH2, EdH2, W2b.T, np.zeros_like(W2b.T))
    dH1, EdH1 = _masked_round_bound(a1, e1, H1, E1)
    g["W1"] = X.T @ dH1
    Eg["W1"] = _matmul_bound(X.T, EX.T, dH1, EdH1, K=B)
    g["b1"] = dH1.sum(axis=0)
    Eg["b1"] = EdH1.sum(axis=0) + (B + 2) * U * np.abs(dH1).sum(axis=0)
    ce = np.log(s) + m - Z[np.arange(B), lab]
    loss = float(np.mean(ce + lam * diff * diff))
    e_ce = 2 * Erow + EZ[np.arange(B), lab] + (R + 16) * U * (np.abs(ce) + np.abs(m) + 1.0)
    e_bud = abs(lam) * (2 * np.abs(diff) * EZ[:, R] + EZ[:, R] ** 2 + 4 * U * diff * diff)
    loss_bound = float(np.mean(e_ce + e_bud) + (B + 4) * U * np.mean(np.abs(ce) + abs(lam) * diff * diff))
    return loss, loss_bound, g, Eg


def emulate_f32_device(params: dict, x, lab, y, lam: float, order_seed: int = 0):
    """A float32-accumulating implementation with the device's rounding points, summing every product
    in a shuffled order: a stand-in for a device whose accumulation order is unknown. Used on the CPU to
    check that the bounds above cover such an implementation."""
    rng = np.random.default_rng(order_seed)
    f32 = np.float32

    def mm(A, Bm, bias=None):
        A = np.asarray(A, f32)
        Bm = np.asarray(Bm, f32)
        K = A.shape[1]
        perm = rng.permutation(K)
        acc = np.zeros((A.shape[0], Bm.shape[1]), f32)
        for k in perm:
            acc = (acc + np.outer(A[:, k], Bm[k, :]).astype(f32)).astype(f32)
        if bias is not None:
            acc = (acc + np.asarray(bias, f32)).astype(f32)
        return acc

    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    X = bf16(x)
    W1b, W2b, W3b = bf16(W1), bf16(W2), bf16(W3)
    H1 = bf16(np.maximum(mm(X, W1b, b1), 0))
    H2 = bf16(np.maximum(mm(H1, W2b, b2), 0))
    Z = mm(H2, W3b, b3).astype(np.float64)
    B = X.shape[0]
    R = Z.shape[1] - 1
    lab = np.clip(np.asarray(lab, np.int64), 0, R - 1)
    Zf = Z.astype(f32)
    m = Zf[:, :R].max(axis=1, keepdims=True)
    e = np.exp((Zf[:, :R] - m).astype(f32)).astype(f32)
    s = e.sum(axis=1, dtype=f32, keepdims=True)
    p = (e / s).astype(f32)
    onehot = np.zeros_like(p)
    onehot[np.arange(B), lab] = 1
    invB = f32(1.0 / B)
    dZ = np.empty(Z.shape, np.float64)
    dZ[:, :R] = bf16(((p - onehot).astype(f32) * invB).astype(f32))
    dZ[:, R] = bf16((f32(2.0 * lam) * (Zf[:, R] - np.asarray(y, f32)).astype(f32) * invB).astype(f32))
    g = {"W3": mm(H2.T, dZ), "b3": dZ.astype(f32).sum(axis=0, dtype=f32)}
    dH2 = bf16(mm(dZ, W3b.T) * (H2 > 0))
    g["W2"], g["b2"] = mm(H1.T, dH2), dH2.astype(f32).sum(axis=0, dtype=f32)
    dH1 = bf16(mm(dH2, W2b.T) * (H1 > 0))
    g["W1"], g["b1"] = mm(X.T, dH1), dH1.astype(f32).sum(axis=0, dtype=f32)
    ce = np.log(s[:, 0]) + m[:, 0] - Zf[np.arange(B), lab]
    diff = Zf[:, R] - np.asarray(y, f32)
    loss = float(np.mean(ce + lam * diff * diff))
    return loss, {k: np.asarray(v, np.float64) for k, v in g.items()}, Z


LAMBDA = 16.0


def tight_matmul(A, B, bias=None):
    """Higham-Mary tolerance of a float32 product A B (+ bias) with exact operands."""
    K = A.shape[1]
    mag = np.abs(A) @ np.abs(B)
    if bias is not None:
        mag = mag + np.abs(bias)
    return LAMBDA * np.sqrt(K + 1) * U * mag + U * np.abs(A @ B if bias is None else A @ B + bias)


def tight_grad_tolerances(params: dict, x, lab, y, lam: float):
    """Tight tolerances of the gradients, from the reference's own bf16 operands (no bf16 step upstream)."""
    from oracle import mlp
    _, g, cache = mlp.forward_backward(params, x, lab, y, lam, bf16_mode=True)
    W2b, W3b = bf16(params["W2"]), bf16(params["W3"])
    X, H1, H2, Z = bf16(x), cache["H1"], cache["H2"], cache["Z"]
    B, R = X.shape[0], Z.shape[1] - 1
    p = cache["p"]
    onehot = np.zeros_like(p)
    onehot[np.arange(B), np.clip(np.asarray(lab, np.int64), 0, R - 1)] = 1
    dZ = np.empty_like(Z)
    dZ[:, :R] = bf16((p - onehot) / B)
    dZ[:, R] = bf16(2.0 * lam * (Z[:, R] - np.asarray(y, np.float64)) / B)
    dH2 = bf16((dZ @ W3b.T) * (H2 > 0))
    dH1 = bf16((dH2 @ W2b.T) * (H1 > 0))
    t = {"W3": tight_matmul(H2.T, dZ), "W2": tight_matmul(H1.T, dH2), "W1": tight_matmul(X.T, dH1)}
    for k, G in (("b3", dZ), ("b2", dH2), ("b1", dH1)):
        t[k] = LAMBDA * np.sqrt(B + 1) * U * np.abs(G).sum(axis=0)
    return t


def tight_logit_tolerance(params: dict, x):
    """Tight tolerance of the output layer's float32 logits from the reference's own bf16 H2."""
    from oracle import mlp
    _, _, cache = mlp.forward_backward(params, x, np.zeros(len(x), np.int64), np.zeros(len(x)), 0.0,
                                       bf16_mode=True)
    return tight_matmul(cache["H2"], bf16(params["W3"]), params["b3"])


def readout_bounds(params: dict, x):
    """Reference logits of inference and their bounds."""
    F = forward_bounds(params, x)
    return F["Z"]
