"""CPU reference of the entry / budget predictor MLP (TEST INFRASTRUCTURE).

Plain numpy in float64. The network is x -> relu(x W1 + b1) -> relu(. W2 + b2)
-> z = . W3 + b3, with z[:, :R] the entry logits and z[:, R] the log-budget
output. Loss per row: softmax cross-entropy of the entry label plus
lambda * (z_R - y)^2; the batch loss is the mean over rows.

With bf16=True the values are rounded to bfloat16 (round to nearest even, via
float32) at exactly the points where the device path rounds: the inputs, the
weight copies used by the products, the stored hidden activations, and the
gradients fed to the backward products. With bf16=False it is the exact
float64 model, which the finite-difference pins check.

The predictor is not part of the paper (it is an addition on top of ghost
staging); parity of its kernels is against this reference.
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (RNE) through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(f), f, out)
    return out.astype(np.float64)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def forward_backward(params: dict, x, lab, y, lam: float, bf16_mode: bool = True):
    """Returns (loss, grads dict, cache). params: W1 [d,h], b1 [h], W2 [h,h], b2 [h], W3 [h,R+1], b3 [R+1]."""
    rb = bf16 if bf16_mode else _id
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    X = rb(x)
    W1b, W2b, W3b = rb(W1), rb(W2), rb(W3)
    B = X.shape[0]
    R = W3.shape[1] - 1
    H1 = rb(np.maximum(X @ W1b + b1, 0.0))
    H2 = rb(np.maximum(H1 @ W2b + b2, 0.0))
    Z = H2 @ W3b + b3
    logits = Z[:, :R]
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    s = e.sum(axis=1, keepdims=True)
    p = e / s
    lab = np.asarray(lab, np.int64)
    y = np.asarray(y, np.float64)
    ce = np.log(s[:, 0]) + m[:, 0] - logits[np.arange(B), lab]
    diff = Z[:, R] - y
    loss = float(np.mean(ce + lam * diff * diff))
    onehot = np.zeros_like(p)
    onehot[np.arange(B), lab] = 1.0
    dZ = np.empty_like(Z)
    dZ[:, :R] = (p - onehot) / B
    dZ[:, R] = 2.0 * lam * diff / B
    dZ = rb(dZ)
    g = {}
    g["W3"] = H2.T @ dZ
    g["b3"] = dZ.sum(axis=0)
    dH2 = rb((dZ @ W3b.T) * (H2 > 0))
    g["W2"] = H1.T @ dH2
    g["b2"] = dH2.sum(axis=0)
    dH1 = rb((dH2 @ W2b.T) * (H1 > 0))
    g["W1"] = X.T @ dH1
    g["b1"] = dH1.sum(axis=0)
    return loss, g, dict(Z=Z, H1=H1, H2=H2, p=p)


def loss_only(params, x, lab, y, lam, bf16_mode=False) -> float:
    return forward_backward(params, x, lab, y, lam, bf16_mode)[0]


def adam_step(params: dict, grads: dict, state: dict, lr: float, step: int, b1=0.9, b2=0.999, eps=1e-8) -> dict:
    """One Adam update (Kingma and Ba, 2015); state holds m and v per tensor."""
    out = {}
    for k, w in params.items():
        gk = np.asarray(grads[k], np.float64)
        m = b1 * state.get("m_" + k, 0.0) + (1 - b1) * gk
        v = b2 * state.get("v_" + k, 0.0) + (1 - b2) * gk * gk
        state["m_" + k], state["v_" + k] = m, v
        mh = m / (1 - b1 ** step)
        vh = v / (1 - b2 ** step)
        out[k] = np.asarray(w, np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return out


def readout(Z, t: int, tau: float, gmap, t_min: int, t_max: int, budget_scale: float = 1.25):
    """Seeds = gmap of the t largest entry logits (ties: smaller index), budget = clamp(ceil(s (e^z_R - 1))),
    confidence = max softmax probability; seeds[:, 0] = NONE and budget = t_max when confidence < tau."""
    Z = np.asarray(Z, np.float64)
    R = Z.shape[1] - 1
    logits = Z[:, :R]
    order = np.stack([np.lexsort((np.arange(R), -row))[:t] for row in logits])
    m = logits.max(axis=1, keepdims=True)
    conf = 1.0 / np.exp(logits - m).sum(axis=1)
    seeds = np.asarray(gmap, np.uint32)[order]
    seeds[conf < tau, 0] = 0xFFFFFFFF
    T = np.clip(np.ceil(budget_scale * (np.exp(Z[:, R]) - 1.0)), t_min, t_max).astype(np.int32)
    T[conf < tau] = t_max  # fallback queries keep the full budget
    return seeds, T, conf, order
