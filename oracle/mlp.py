"""Oracle: per-area warm-start MLP (forward, backward, Adam) -- TEST INFRASTRUCTURE ONLY.

The learned warm start is not in the paper; it is the library's extension
that maps an area's measurements to a starting (|V|, theta) for Gauss-Newton.
Per area k the network is

    X  = (z_k - mu_k) / sigma_k                 (area k's measurements)
    H1 = relu(X W1 + b1),  H2 = relu(H1 W2 + b2),  Y = H2 W3 + b3

with W1 [m_k x H], W2 [H x H], W3 [H x O_k] (row-major, "in x out"), O_k = 2 x
(area k's own buses), outputs ordered bus by bus (ascending id) as
(|V|, theta), standardised by per-output mean and std.  The loss is the mean
squared error over the batch and every output of every area.

Precision recipe (the GPU kernels follow it, so this oracle can mirror them):
every matrix-product operand is rounded to bfloat16 (round to nearest even,
via float32), products accumulate in float32 on the GPU (float64 here), and
the bias, the pre-activation, the loss and all gradients are kept in float32
on the GPU (float64 here).  With recipe=False nothing is rounded: the exact
FP64 network, used for the finite-difference pin.

Pins (tests/test_oracle_mlp.py): finite differences of the exact loss; the
bf16 rounding against torch's bfloat16 conversion and hand-picked ties; the
first Adam step against its closed form lr * g / (|g| + eps).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to bfloat16 (via float32, round to nearest even), return float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def relu(x):
    return np.maximum(x, 0.0)


def area_forward(p, X, recipe=True):
    """p = dict(W1, b1, W2, b2, W3, b3) float64; X [B x m_k]."""
    r = bf16 if recipe else (lambda a: a)
    A0 = r(X)
    P1 = r(A0) @ r(p["W1"]) + p["b1"]
    H1 = relu(P1)
    A1 = r(H1)
    P2 = A1 @ r(p["W2"]) + p["b2"]
    H2 = relu(P2)
    A2 = r(H2)
    Y = A2 @ r(p["W3"]) + p["b3"]
    return {"A0": A0, "P1": P1, "A1": A1, "P2": P2, "A2": A2, "Y": Y}


def loss_and_grads(params, Xs, Ts, recipe=True):
    """MSE over all areas' outputs; returns (loss, grads per area)."""
    r = bf16 if recipe else (lambda a: a)
    B = Xs[0].shape[0]
    n_out = sum(T.shape[1] for T in Ts)
    loss = 0.0
    grads = []
    for p, X, T in zip(params, Xs, Ts):
        c = area_forward(p, X, recipe)
        E = c["Y"] - T
        loss += float(np.sum(E * E))
        dY = 2.0 * E / (B * n_out)
        g = {"W3": c["A2"].T @ r(dY), "b3": dY.sum(0)}
        dH2 = (r(dY) @ r(p["W3"]).T) * (c["P2"] > 0)
        g["W2"] = c["A1"].T @ r(dH2)
        g["b2"] = dH2.sum(0)
        dH1 = (r(dH2) @ r(p["W2"]).T) * (c["P1"] > 0)
        g["W1"] = c["A0"].T @ r(dH1)
        g["b1"] = dH1.sum(0)
        grads.append(g)
    return loss / (B * n_out), grads


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(params):
    """Per-area blocks W1 b1 W2 b2 W3 b3 (row-major), areas in order."""
    return np.concatenate([np.ravel(p[k]) for p in params for k in PARAM_ORDER])


def unflatten(vec, shapes):
    """shapes: list of (m_k, H, O_k)."""
    out, o = [], 0
    for m, H, O in shapes:
        p = {}
        for k, shp in (("W1", (m, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                       ("W3", (H, O)), ("b3", (O,))):
            n = int(np.prod(shp))
            p[k] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(shp)
            o += n
        out.append(p)
    return out
