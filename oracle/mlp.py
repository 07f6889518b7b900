"""Oracle for the learned surrogate: MLP forward/backward and Adam, in float64.

Test infrastructure only.  The network is not part of the paper; its shape is
30 -> 128 -> 128 -> 128 -> 15 with GELU activations, mapping the scaled offsets
of a 2D 15-node stencil to its scaled Laplacian weights.

Arithmetic is float64 except that values are rounded to bfloat16 (round to
nearest, ties to even) exactly where the GPU kernels round them before a matrix
product:
    forward : the input x, every weight matrix W_i, every hidden activation h_i;
    backward: the output gradient g, and every pre-activation gradient dz_i.
Bias gradients use the unrounded gradients.  With ``rounding=False`` the
function is the plain float64 network (used by the finite-difference check).

GELU is the exact erf form g(z) = z * Phi(z) = z/2 * (1 + erf(z / sqrt 2)),
with g'(z) = Phi(z) + z * phi(z).  Loss = mean over batch x 15 of (y - t)^2.
Adam: m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
      theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LAYERS = ((30, 128), (128, 128), (128, 128), (128, 15))


def bf16(x) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (8 significant bits), ties to even.

    Normal range only (the network's values are far from bfloat16 under/overflow).
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                     # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    Phi = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def forward(params, x, rounding: bool = True):
    """params: dict W1..W4 [out, in], b1..b4 [out].  x: [B, 30].  Returns (y, cache)."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    h = rnd(x)
    cache = {"a0": h}
    for L in range(1, 5):
        W = rnd(params[f"W{L}"])
        z = h @ W.T + params[f"b{L}"]
        cache[f"Wr{L}"] = W
        if L < 4:
            cache[f"z{L}"] = z
            h = rnd(gelu(z))
            cache[f"a{L}"] = h
        else:
            y = z
    return y, cache


def loss_and_grads(params, x, t, rounding: bool = True):
    """Mean-squared-error loss and its gradient w.r.t. every parameter."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(params, x, rounding)
    B = y.shape[0]
    diff = y - t
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / (B * y.shape[1])          # dL/dy
    grads = {}
    for L in range(4, 0, -1):
        grads[f"b{L}"] = g.sum(axis=0)
        gr = rnd(g)
        grads[f"W{L}"] = gr.T @ c[f"a{L - 1}"]
        if L > 1:
            dh = gr @ c[f"Wr{L}"]
            g = dh * gelu_prime(c[f"z{L - 1}"])
    return loss, grads, y


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v (dicts) and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, g in grads.items():
        m = state.setdefault("m", {}).setdefault(k, np.zeros_like(g))
        v = state.setdefault("v", {}).setdefault(k, np.zeros_like(g))
        m *= b1
        m += (1.0 - b1) * g
        v *= b2
        v += (1.0 - b2) * g * g
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def stencil_features(X, offsets, idx, nodes=None, canonical=False):
    """Inputs of the network: scaled offsets (x_j - x_i)/s in stencil order, flattened.

    s = max_j ||x_j - x_i|| (the scaling of the weight computation).  With
    ``canonical`` the offsets are first expressed in the stencil's canonical
    frame: rotated so that node 1 (the nearest neighbour) lies on +x, then
    reflected in x so that node 2 has y >= 0.  The Laplacian weights of a
    stencil do not change under rotations and reflections, so this loses
    nothing.  Each operation is a separately rounded float64 operation:
        c = o1x / |o1|, s_ = o1y / |o1|, f = -1 if c*o2y - s_*o2x < 0 else 1,
        x' = (c*ox + s_*oy) / s,  y' = (f * (c*oy - s_*ox)) / s.
    Returns (F [B, 2n] float64 interleaved x,y per node, s [B]).
    """
    X = np.asarray(X, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    N = offsets.shape[0] - 1
    nodes = np.arange(N) if nodes is None else np.asarray(nodes)
    n = int(offsets[nodes[0] + 1] - offsets[nodes[0]])
    pos = offsets[nodes][:, None] + np.arange(n)[None, :]
    P = X[np.asarray(idx)[pos]]
    O = P - P[:, :1, :]
    s = np.sqrt(O[:, :, 0] * O[:, :, 0] + O[:, :, 1] * O[:, :, 1]).max(axis=1)
    if not canonical:
        Xh = O / s[:, None, None]
        return Xh.reshape(len(nodes), -1), s
    o1x, o1y = O[:, 1, 0], O[:, 1, 1]
    r = np.sqrt(o1x * o1x + o1y * o1y)
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.where(r > 0, o1x / r, 1.0)
        sn = np.where(r > 0, o1y / r, 0.0)
    f = np.where(c * O[:, 2, 1] - sn * O[:, 2, 0] < 0, -1.0, 1.0)
    ox, oy = O[:, :, 0], O[:, :, 1]
    xr = (c[:, None] * ox + sn[:, None] * oy) / s[:, None]
    yr = (f[:, None] * (c[:, None] * oy - sn[:, None] * ox)) / s[:, None]
    return np.stack([xr, yr], axis=-1).reshape(len(nodes), -1), s
