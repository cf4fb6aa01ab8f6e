"""CPU oracle -- the surrogate network in FP64, with optional BF16 rounding.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``.

Multi-layer perceptron  x -> SiLU(W1 x + b1) -> ... -> W_L h + b_L  (linear
output), SiLU(z) = z sigma(z).  Forward, backward (weight gradients and the
input gradient d yhat / d x) and the Adam update (Kingma & Ba 2015) written
out plainly.  With ``bf16=True`` the weights and the layer inputs are
rounded to bfloat16 (round to nearest even) before each product, and so
are the back-propagated gradients entering a product, as the GPU kernels
feed the matrix cores; sums stay in the working precision.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round float values to the nearest bfloat16 (ties to even), returned
    as float64 (via the float32 bit pattern)."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, bf16: bool = False):
    """params: list of (W (out x in), b (out,)).  X: (n, in).  Returns yhat
    (n,) and the cache of pre-activations and layer inputs."""
    h = np.asarray(X, np.float64)
    cache = []
    L = len(params)
    for k, (W, b) in enumerate(params):
        hin = bf16_round(h) if bf16 else h
        Wk = bf16_round(W) if bf16 else W
        z = hin @ Wk.T + b
        cache.append((hin, z))
        h = silu(z) if k + 1 < L else z
    return h[:, 0], cache


def backward(params, cache, dy, bf16: bool = False):
    """dy: d loss / d yhat (n,).  Returns weight gradients [(dW, db)] and
    d loss / d X."""
    L = len(params)
    grads = [None] * L
    g = np.asarray(dy, np.float64)[:, None]
    for k in range(L - 1, -1, -1):
        W, _ = params[k]
        hin, z = cache[k]
        if k + 1 < L:
            g = g * silu_grad(z)
        gb = bf16_round(g) if bf16 else g
        grads[k] = (gb.T @ hin, g.sum(axis=0))
        Wk = bf16_round(W) if bf16 else W
        g = gb @ Wk
    return grads, g


def mse_loss(params, X, y, bf16: bool = False):
    yhat, cache = forward(params, X, bf16)
    r = yhat - y
    n = X.shape[0]
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    grads, dX = backward(params, cache, dy, bf16)
    return loss, grads


def input_gradient(params, X, bf16: bool = False):
    """d yhat / d X for every row (the surrogate's gradient in theta)."""
    yhat, cache = forward(params, X, bf16)
    _, dX = backward(params, cache, np.ones(X.shape[0]), bf16)
    return yhat, dX


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place; state = dict(t, m, v) (created when empty)."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    new = []
    for k, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        mW, mb = state["m"][k]
        vW, vb = state["v"][k]
        mW = b1 * mW + (1 - b1) * gW
        mb = b1 * mb + (1 - b1) * gb
        vW = b2 * vW + (1 - b2) * gW * gW
        vb = b2 * vb + (1 - b2) * gb * gb
        state["m"][k] = (mW, mb)
        state["v"][k] = (vW, vb)
        c1 = 1 - b1 ** t
        c2 = 1 - b2 ** t
        W = W - lr * (mW / c1) / (np.sqrt(vW / c2) + eps)
        b = b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps)
        new.append((W, b))
    params[:] = new
    return params
