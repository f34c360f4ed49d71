"""Fourier-feature MLP velocity model trained through the solver's adjoint.

The paper's workflows include neural-network velocity representations (Sec. 1):
the velocity of every model cell is the output of a small network of the cell's
coordinates, and the network is trained with the gradients the wave-equation
adjoint returns. Here: 64 random Fourier frequencies (128 features), 4 hidden
layers of 256 ReLU, v = vmin + vscale * sigmoid(y), bf16 MFMA matrix products
with float32 accumulation, float32 master weights updated by Adam. All
arithmetic runs in libsweep's kernels; this class holds the device buffers.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from ._lib import check, lib
from .propagator import _ptr, _stream

__all__ = ["MLPVelocity", "adam_step"]

_sigs = {
    "sweep_mlp_param_count": (ctypes.c_size_t, []),
    "sweep_mlp_pack_count": (ctypes.c_size_t, []),
    "sweep_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int]),
    "sweep_mlp_encode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "sweep_mlp_cast": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sweep_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p]),
    "sweep_mlp_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "sweep_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_int, ctypes.c_void_p]),
}


def _align(x: int) -> int:
    return (x + 255) // 256 * 256


def _lib():
    L = lib()
    for name, (res, args) in _sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def adam_step(theta: torch.Tensor, m: torch.Tensor, v: torch.Tensor, g: torch.Tensor, t: int,
              lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """In-place Adam update of float32 device tensors (step t >= 1)."""
    for x in (theta, m, v, g):
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
            raise TypeError("adam_step needs contiguous float32 CUDA tensors")
    n = theta.numel()
    if not (m.numel() == v.numel() == g.numel() == n):
        raise ValueError("adam_step: size mismatch")
    check(_lib().sweep_adam_step(_ptr(theta), _ptr(m), _ptr(v), _ptr(g), n, lr, b1, b2, eps, t,
                                 _stream()))


class MLPVelocity:
    """v[nz][nx] = vmin + vscale * sigmoid(MLP(gamma(i/(nx-1), j/(nz-1))))."""

    def __init__(self, nx: int, nz: int, B: np.ndarray, theta0: np.ndarray,
                 vmin: float = 1500.0, vscale: float = 3200.0,
                 device: Optional[torch.device] = None):
        L = _lib()
        self.nx, self.nz, self.M = nx, nz, nx * nz
        self.vmin, self.vscale = float(vmin), float(vscale)
        dev = torch.device(device) if device is not None else torch.device("cuda")
        self.P = int(L.sweep_mlp_param_count())
        theta0 = np.asarray(theta0, dtype=np.float32)
        if theta0.shape != (self.P,):
            raise ValueError(f"theta0 must have {self.P} entries")
        self.theta = torch.tensor(theta0, device=dev)
        self.m = torch.zeros_like(self.theta)
        self.v2 = torch.zeros_like(self.theta)
        self.t = 0
        self.B = torch.tensor(np.asarray(B, dtype=np.float32).reshape(64, 2), device=dev)
        self.feats = torch.empty(self.M * 128, dtype=torch.int16, device=dev)
        self.wpack = torch.empty(int(L.sweep_mlp_pack_count()), dtype=torch.int16, device=dev)
        self.work = torch.empty(int(L.sweep_mlp_workspace_bytes(self.M)), dtype=torch.uint8,
                                device=dev)
        self.grad = torch.zeros_like(self.theta)
        check(L.sweep_mlp_encode(_ptr(self.B), nx, nz, _ptr(self.feats), _stream()))
        self._cast()

    def _cast(self):
        check(_lib().sweep_mlp_cast(_ptr(self.theta), _ptr(self.wpack), _stream()))

    def forward(self) -> torch.Tensor:
        """Velocity [nz][nx] (float32); keeps the activations for backward()."""
        v = torch.empty((self.nz, self.nx), dtype=torch.float32, device=self.theta.device)
        check(_lib().sweep_mlp_forward(_ptr(self.wpack), _ptr(self.theta), _ptr(self.feats),
                                       self.M, self.vmin, self.vscale, _ptr(v), _ptr(self.work),
                                       self.work.numel(), _stream()))
        return v

    def backward(self, dv: torch.Tensor) -> torch.Tensor:
        """Gradient of sum(dv * v) with respect to theta (needs the last forward)."""
        dv = dv.contiguous()
        if dv.numel() != self.M or dv.dtype != torch.float32:
            raise ValueError("dv must be float32 with nx*nz entries")
        check(_lib().sweep_mlp_backward(_ptr(self.wpack), _ptr(self.feats), self.M, self.vscale,
                                        _ptr(dv), _ptr(self.grad), _ptr(self.work),
                                        self.work.numel(), _stream()))
        return self.grad

    def activations(self):
        """The four hidden activations kept by the last forward(), as float32
        [nz*nx][256] tensors (views of the bfloat16 stash, widened)."""
        return self._bf16_block(0)

    def pre_activation_grads(self):
        """dZ1..dZ4 kept by the last backward(): gradients with respect to the
        hidden pre-activations, as float32 [nz*nx][256] tensors."""
        y_end = _align(_align(4 * self.M * 512) + 4 * self.M)
        return self._bf16_block(y_end)

    def _bf16_block(self, off: int):
        n = self.M * 256
        raw = self.work[off: off + 4 * n * 2].view(torch.int16).view(4, self.M, 256)
        return [(raw[l].to(torch.int32) << 16).view(torch.float32) for l in range(4)]

    def reset_optimizer(self):
        """Zero the Adam moments and step count (start of a new optimisation)."""
        self.m.zero_()
        self.v2.zero_()
        self.t = 0

    def step(self, grad: torch.Tensor, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
             eps: float = 1e-8):
        """Adam on the float32 master weights, then refresh the bf16 copies."""
        self.t += 1
        adam_step(self.theta, self.m, self.v2, grad, self.t, lr, b1, b2, eps)
        self._cast()
