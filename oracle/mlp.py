"""Small fully connected ReLU network in float64 (test infrastructure).

The learned cost model is a multilayer perceptron: ``len(widths)-2`` hidden
layers with ReLU, a linear output, mean-squared-error loss and the Adam update
(Kingma & Ba). Nothing of it is in the paper, whose chain rule is the greedy
heuristic of Sec. II; the network is a planner variant. Written from the
definitions:

  h_0 = x,  z_l = W_l h_{l-1} + b_l,  h_l = max(z_l, 0) (l < last),  y = z_last
  L = (1/N) sum_n (y_n - t_n)^2
  dL/dy_n = 2 (y_n - t_n) / N
  dL/dW_l = sum_n delta_l,n h_{l-1,n}^T,   dL/db_l = sum_n delta_l,n
  delta_{l-1} = (W_l^T delta_l) * [z_{l-1} > 0]

Parameters are lists ``[(W_1, b_1), ...]`` with W_l of shape (out, in).
Batches are row-major: x has shape (N, in).
"""
from __future__ import annotations

import numpy as np


def init(widths, seed_gen) -> list:
    """He-normal weights, zero biases, drawn from ``seed_gen`` (a numpy
    Generator passed in by the caller)."""
    params = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        w = seed_gen.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)
        params.append((w, np.zeros(fan_out)))
    return params


def forward(params, x):
    """Returns (y, cache); y has shape (N,)."""
    h = np.asarray(x, dtype=np.float64)
    zs, hs = [], [h]
    for l, (w, b) in enumerate(params):
        z = h @ np.asarray(w, np.float64).T + np.asarray(b, np.float64)
        zs.append(z)
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
        hs.append(h)
    return h[:, 0], (zs, hs)


def mse(y, t) -> float:
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(params, cache, y, t) -> list:
    """Gradients [(dW_l, db_l)] of the MSE loss."""
    zs, hs = cache
    n = y.shape[0]
    delta = (2.0 / n) * (np.asarray(y, np.float64) - np.asarray(t, np.float64))[:, None]
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w = np.asarray(params[l][0], np.float64)
        grads[l] = (delta.T @ hs[l], delta.sum(axis=0))
        if l > 0:
            delta = (delta @ w) * (zs[l - 1] > 0)
    return grads


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; ``state`` is a dict carrying t, m and v across calls."""
    t = state.get("t", 0) + 1
    m = state.get("m") or [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    v = state.get("v") or [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    out, new_m, new_v = [], [], []
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
        pair = []
        mm, vv = [], []
        for p, g, mp, vp in ((w, gw, mw, vw), (b, gb, mb, vb)):
            mp = beta1 * mp + (1 - beta1) * g
            vp = beta2 * vp + (1 - beta2) * g * g
            mhat = mp / (1 - beta1 ** t)
            vhat = vp / (1 - beta2 ** t)
            pair.append(p - lr * mhat / (np.sqrt(vhat) + eps))
            mm.append(mp)
            vv.append(vp)
        out.append(tuple(pair))
        new_m.append(tuple(mm))
        new_v.append(tuple(vv))
    state.update(t=t, m=new_m, v=new_v)
    return out
