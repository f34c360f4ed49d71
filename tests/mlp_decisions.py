"""Gradient of the MLP velocity model on given rounding decisions (test code).

The full-size MLP test cannot expect the float32 kernels and the float64
oracle to take every bf16 rounding and ReLU decision alike. It first checks
that each of the kernel's stored pre-activation gradients dZ is a valid
rounding of a value within the float32 summation bound of the exact one, and
then compares the parameter gradient computed from those same stored values.
This module computes that last step, dW_l = dZ_l^T H_{l-1}, db_l = sum dZ_l and
the output layer's terms, from the stored activations and dZ; a CPU test
checks it against the oracle's own backward on the oracle's own decisions.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as omlp


def gradient_on_decisions(theta, hs, s, dzs, dv, vscale=3200.0):
    """hs: [features, H1..H4]; s: sigmoid output; dzs: [dZ1..dZ4] (as stored)."""
    p = omlp.unpack(theta)
    depth = omlp.DEPTH
    dy = np.asarray(dv, dtype=np.float64) * vscale * s * (1.0 - s)
    grads = [None] * len(p)
    grads[2 * depth] = hs[depth].T @ dy
    grads[2 * depth + 1] = np.array([dy.sum()])
    for l in range(depth):
        grads[2 * l] = dzs[l].T @ hs[l]
        grads[2 * l + 1] = dzs[l].sum(axis=0)
    return np.concatenate([g.ravel() for g in grads])
