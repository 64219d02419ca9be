"""FP64 CPU oracle of the warm-start multilayer perceptron.

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU BF16 kernels'
forward pass and gradients; shares no code with the HIP library.

Network: x [B, n_in] -> (Linear, SiLU) x depth -> Linear -> y [B, n_out],
Linear(h) = h W + b with W [fan_in, fan_out]; SiLU(z) = z sigmoid(z).
Loss: mean over samples and outputs of (y - y_ref)^2.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(n_in: int, width: int, depth: int, n_out: int, seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (the
    common default for linear layers)."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [width] * depth + [n_out]
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = 1.0 / np.sqrt(a)
        params.append((rng.uniform(-lim, lim, (a, b)), rng.uniform(-lim, lim, b)))
    return params


def forward(params, x):
    """Returns the output and the pre-activations of every hidden layer."""
    h = np.asarray(x, np.float64)
    zs, hs = [], [h]
    for li, (W, b) in enumerate(params):
        z = h @ W + b
        if li < len(params) - 1:
            zs.append(z)
            h = silu(z)
            hs.append(h)
        else:
            return z, zs, hs
    raise AssertionError


def loss_and_grads(params, x, y_ref):
    """MSE loss and its gradient with respect to every W and b (backward
    pass written out layer by layer)."""
    y, zs, hs = forward(params, x)
    B, n_out = y.shape
    loss = float(np.mean((y - y_ref) ** 2))
    g = 2.0 * (y - y_ref) / (B * n_out)  # dL/dy
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_in = hs[li]
        grads[li] = (h_in.T @ g, g.sum(axis=0))
        if li > 0:
            g = (g @ W.T) * dsilu(zs[li - 1])
    return loss, grads


def adam_step(params, grads, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new
    (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        nm, nv, np_ = [], [], []
        for p, gp, mp, vp in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mp = b1 * mp + (1 - b1) * gp
            vp = b2 * vp + (1 - b2) * gp * gp
            mh = mp / (1 - b1 ** t)
            vh = vp / (1 - b2 ** t)
            np_.append(p - lr * mh / (np.sqrt(vh) + eps))
            nm.append(mp)
            nv.append(vp)
        out_p.append(tuple(np_))
        out_m.append(tuple(nm))
        out_v.append(tuple(nv))
    return out_p, out_m, out_v


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(flat, n_in, width, depth, n_out):
    dims = [n_in] + [width] * depth + [n_out]
    out, o = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = flat[o:o + a * b].reshape(a, b)
        o += a * b
        bb = flat[o:o + b]
        o += b
        out.append((W.copy(), bb.copy()))
    return out
