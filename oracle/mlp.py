"""FP64 oracle of the Fourier-feature MLP velocity model (NumPy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). The paper's workflows include
neural-network velocity representations trained through the solver (Sec. 1);
the network is the stated workload: 2-D coordinates -> 64 random Fourier
frequencies (cos and sin: 128 features) -> 4 hidden layers of 256 ReLU -> 1,
v = vmin + vscale * sigmoid(y).

Precision model (mirrors where the GPU stores bfloat16): the features, every
weight matrix and every hidden activation (after bias + ReLU) and every
back-propagated pre-activation gradient are rounded to bfloat16 with
round-to-nearest-even; all sums are taken in float64 here (float32 on the GPU).
With emulate=False nothing is rounded (plain float64 network, for finite
differences).
"""
from __future__ import annotations

import numpy as np

NFREQ = 64
NFEAT = 2 * NFREQ
WIDTH = 256
DEPTH = 4

# parameter vector layout: W1 [256][128], b1, W2 [256][256], b2, W3, b3, W4, b4,
# w5 [256], b5 (weights stored out x in)
SHAPES = [(WIDTH, NFEAT), (WIDTH,)] + [(WIDTH, WIDTH), (WIDTH,)] * (DEPTH - 1) + [(WIDTH,), (1,)]


def n_params() -> int:
    return int(sum(np.prod(s) for s in SHAPES))


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even); returned as float64.
    Works on the float32 bit pattern: add 0x7FFF plus the lowest kept bit, then
    clear the 16 discarded bits."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def coords(nx: int, nz: int) -> np.ndarray:
    """Normalised coordinates of every model cell, [nz*nx][2] = (i/(nx-1), j/(nz-1))."""
    i = np.arange(nx) / max(nx - 1, 1)
    j = np.arange(nz) / max(nz - 1, 1)
    J, I = np.meshgrid(j, i, indexing="ij")
    return np.stack([I.ravel(), J.ravel()], 1)


def encode(B, nx: int, nz: int, emulate=True) -> np.ndarray:
    """gamma = [cos(2 pi B x), sin(2 pi B x)]; B [64][2]."""
    x = coords(nx, nz)
    ph = 2.0 * np.pi * (x @ np.asarray(B, dtype=np.float64).T)
    g = np.concatenate([np.cos(ph), np.sin(ph)], axis=1)
    return bf16(g) if emulate else g


def forward(theta, gamma, vmin=1500.0, vscale=3200.0, emulate=True):
    """Returns (v [M], cache)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta)
    h = gamma
    hs = [gamma]
    for l in range(DEPTH):
        W, b = r(p[2 * l]), p[2 * l + 1]
        h = r(np.maximum(h @ W.T + b, 0.0))
        hs.append(h)
    w5, b5 = r(p[2 * DEPTH]), p[2 * DEPTH + 1]
    y = h @ w5 + b5[0]
    s = 1.0 / (1.0 + np.exp(-y))
    return vmin + vscale * s, {"hs": hs, "y": y, "s": s}


def backward(theta, cache, dv, vscale=3200.0, emulate=True, return_dz=False):
    """Gradient of sum(dv * v) with respect to the parameter vector.

    With return_dz, also returns the four pre-activation gradients of hidden
    layers 1..4 (as stored: bf16-rounded when emulating)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta)
    hs, s = cache["hs"], cache["s"]
    grads = [None] * len(p)
    dzs = [None] * DEPTH
    dy = np.asarray(dv, dtype=np.float64) * vscale * s * (1.0 - s)
    w5 = r(p[2 * DEPTH])
    grads[2 * DEPTH] = hs[DEPTH].T @ dy
    grads[2 * DEPTH + 1] = np.array([dy.sum()])
    dz = r(np.outer(dy, w5) * (hs[DEPTH] > 0))
    for l in range(DEPTH - 1, -1, -1):
        dzs[l] = dz
        grads[2 * l] = dz.T @ hs[l]
        grads[2 * l + 1] = dz.sum(axis=0)
        if l > 0:
            dz = r((dz @ r(p[2 * l])) * (hs[l] > 0))
    g = np.concatenate([gr.ravel() for gr in grads])
    return (g, dzs) if return_dz else g


def adam(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """Weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for s in SHAPES:
        if len(s) == 2:
            out.append(rng.uniform(-1, 1, s) / np.sqrt(s[1]))
        elif s == (WIDTH,) and len(out) == 2 * DEPTH:  # w5 (fan_in 256)
            out.append(rng.uniform(-1, 1, s) / np.sqrt(WIDTH))
        else:
            out.append(np.zeros(s))
    return np.concatenate([o.ravel() for o in out])
