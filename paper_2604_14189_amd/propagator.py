"""Python face of libsweep: plans, forward / backward, autograd.

Mirrors the paper's Propagator / Source / Receiver split (Sec. 2.1): a Plan
fixes the grid, time axis, absorbing pad, sources and receivers; `forward`
returns shot gathers for every shot at once (batch modelling, Sec. 2.2) and
`backward` returns d(loss)/d(model) through the exact adjoint. PyTorch supplies
device memory and the stream; all arithmetic happens in libsweep's kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import ACOUSTIC, ACOUSTIC_VD, ELASTIC, VTI, Problem, Tuning, check, lib

__all__ = ["Plan", "Batch", "WaveFn", "l2_misfit", "ACOUSTIC", "ELASTIC", "ACOUSTIC_VD", "VTI"]


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, shape, name: str, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """A modelling problem on one GPU: all shots advance in the same launches.

    src_xz: int array [nshots, 2] of model-grid cells (x, z);
    rec_xz: int array [nshots, nrec, 2]. Model tensors are [nparam, nz, nx]
    (acoustic: vp only, so [nz, nx] is also accepted).
    """

    def __init__(self, *, nx: int, nz: int, h: float, dt: float, nt: int, pml: int,
                 src_xz, rec_xz, pml_vmax: float, pml_f0: float, pml_R: float = 1e-3,
                 ckpt_every: int = 50, physics: int = ACOUSTIC, free_surface: int = 0,
                 device: Optional[torch.device] = None):
        src = np.ascontiguousarray(src_xz, dtype=np.int32)
        rec = np.ascontiguousarray(rec_xz, dtype=np.int32)
        if src.ndim == 3 and src.shape[2] == 2:
            self.nsrc = src.shape[1]  # encoded shots: several sources per shot
        elif src.ndim == 2 and src.shape[1] == 2:
            self.nsrc = 1
        else:
            raise ValueError("src_xz must be [nshots, 2] or [nshots, nsrc, 2]")
        self._src3 = src.ndim == 3
        if rec.ndim != 3 or rec.shape[0] != src.shape[0] or rec.shape[2] != 2:
            raise ValueError("rec_xz must be [nshots, nrec, 2]")
        self.pb = Problem(physics, nx, nz, pml, free_surface, h, dt, nt, pml_vmax, pml_f0,
                          pml_R, ckpt_every, src.shape[0], rec.shape[1], self.nsrc)
        self.nshots, self.nrec, self.nt, self.nx, self.nz = (src.shape[0], rec.shape[1], nt,
                                                               nx, nz)
        self.physics = physics
        # acoustic: vp; elastic: vp, vs, rho; first-order variable density: vp, rho;
        # VTI: vv (vertical velocity), v (NMO velocity), eta
        self.nparam = {ACOUSTIC: 1, ELASTIC: 3, ACOUSTIC_VD: 2, VTI: 3}[physics]
        self.ncomp = 1 if physics in (ACOUSTIC, VTI) else 2
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self._src, self._rec = src, rec
        if torch.cuda.is_available():
            if self.device.index is None:
                self.device = torch.device("cuda", torch.cuda.current_device())
            self._ctx = _lib.context(self.device.index)
        else:
            # host-side use only (workspace sizes, tilings): the plan is bound
            # to no device, and its first GPU call fails in the library
            self._ctx = None
        h_ = ctypes.c_void_p()
        check(lib().sweep_plan_create(self._ctx, ctypes.byref(self.pb),
                                      src.ctypes.data_as(ctypes.c_void_p),
                                      rec.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h_)))
        self._h = h_
        self._work = None
        self._fwd_id = 0
        self._saved_id = -1

    @classmethod
    def from_workload(cls, w, **kw) -> "Plan":
        """Plan for a synth.Workload (its sources, receivers and constants)."""
        args = dict(nx=w.nx, nz=w.nz, h=w.h, dt=w.dt, nt=w.nt, pml=w.pml,
                    src_xz=w.sources(), rec_xz=w.receivers(), pml_vmax=w.pml_vmax(),
                    pml_f0=w.f0, pml_R=w.pml_R, ckpt_every=w.ckpt_every,
                    physics=ACOUSTIC if w.physics == "acoustic" else ELASTIC,
                    free_surface=w.free_surface)
        args.update(kw)
        return cls(**args)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().sweep_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ---------------------------------------------------------------- tuning
    @property
    def tuning(self) -> dict:
        t = Tuning()
        check(lib().sweep_plan_get_tuning(self._h, ctypes.byref(t)))
        return {"rz": t.rz, "pml_rz": t.pml_rz, "use_graph": t.use_graph, "tblock": t.tblock,
                "keep_b": t.keep_b}

    def set_tuning(self, rz: Optional[int] = None, pml_rz: Optional[int] = None,
                   use_graph: Optional[int] = None, tblock: Optional[int] = None,
                   keep_b: Optional[int] = None):
        """Change the given fields of the tuning and keep the others:
        rz: rows per thread of the interior kernel (tiles of 64 x 4 rz);
        pml_rz: rows per thread of the C-PML kernels (<= rz; when only rz is
        given, min(4, rz));
        tblock: time steps per pass over the deep interior tiles (1 or 2);
        keep_b: checkpoint segments (the last ones) whose backward inputs
        (acoustic: B'^n; elastic and variable density: the five trace planes)
        the saving forward stores, so that backward() does not recompute them
        (more workspace, the same bits; in a Batch each plan keeps its own
        count, and a batch refuses a backward after a member's tuning changed
        since its saving forward)."""
        cur = self.tuning
        if rz is not None and pml_rz is None:
            pml_rz = min(4, rz)
        t = Tuning(cur["rz"] if rz is None else rz, cur["pml_rz"] if pml_rz is None else pml_rz,
                   cur["use_graph"] if use_graph is None else int(use_graph),
                   cur["tblock"] if tblock is None else tblock,
                   cur["keep_b"] if keep_b is None else keep_b)
        check(lib().sweep_plan_set_tuning(self._h, ctypes.byref(t)))
        self._saved_id = -1

    def autotune(self, model: torch.Tensor, wavelet: torch.Tensor, steps: int = 20,
                 cache_path: Optional[str] = None) -> int:
        """Pick the fastest tiling (rz, pml_rz) and time-blocking depth (tblock)
        for this plan (cached); returns rz (all three are in .tuning afterwards)."""
        if self.nparam == 1 and model.dim() == 2:
            model = model.unsqueeze(0)
        _need(model, self._model_shape(), "model")
        _need(wavelet, self.wavelet_shape(), "wavelet")
        work = self._workspace(False)
        rz = ctypes.c_int()
        check(lib().sweep_plan_autotune(self._h, _ptr(model), _ptr(wavelet), _ptr(work),
                                        work.numel(), steps,
                                        cache_path.encode() if cache_path else None,
                                        _stream(), ctypes.byref(rz)))
        self._saved_id = -1
        return rz.value

    def padded(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        check(lib().sweep_plan_padded(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def tiles(self) -> dict:
        """The acoustic tiling: tiles are 64 columns x `rows` rows; the interior
        ones (no C-PML cell) form the rectangle of tile columns [x0, x1) and
        rows [z0, z1), `deep` of them advancing two steps per pass; the others
        are the frame."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rect = (ctypes.c_int * 5)()
        check(lib().sweep_plan_tiles(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                     rect))
        return {"interior": a.value, "frame": b.value, "rows": c.value,
                "x0": rect[0], "x1": rect[1], "z0": rect[2], "z1": rect[3], "deep": rect[4]}

    def workspace_bytes(self, for_backward: bool) -> int:
        return int(lib().sweep_plan_workspace_bytes(self._h, int(bool(for_backward))))

    def _workspace(self, for_backward: bool) -> torch.Tensor:
        need = self.workspace_bytes(for_backward)
        if self._work is None or self._work.numel() < need:
            self._work = None
            torch.cuda.synchronize(self.device)
            self._work = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._work

    def reserve_workspace(self, for_backward: bool = True) -> int:
        """Allocate the workspace now rather than at the first forward (before
        a timed or captured region, or to learn whether a tuning fits in
        memory: torch.OutOfMemoryError if it does not). Returns its bytes."""
        return self._workspace(for_backward).numel()

    def release_workspace(self):
        self._work = None
        self._saved_id = -1

    # ---------------------------------------------------------------- compute
    def _model_shape(self):
        return (self.nparam, self.nz, self.nx)

    def wavelet_shape(self):
        """[nshots, nt], or [nshots, nsrc, nt] when the sources were given as
        [nshots, nsrc, 2] (encoded shots)."""
        if not self._src3:
            return (self.nshots, self.nt)
        return (self.nshots, self.nsrc, self.nt)

    def gathers_shape(self):
        if self.ncomp == 1:
            return (self.nshots, self.nt, self.nrec)
        return (self.nshots, self.nt, self.nrec, self.ncomp)

    def forward(self, model: torch.Tensor, wavelet: torch.Tensor, save: bool = False,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Shot gathers [nshots, nt, nrec(, ncomp)] for every shot."""
        if self.nparam == 1 and model.dim() == 2:
            model = model.unsqueeze(0)
        _need(model, self._model_shape(), "model")
        _need(wavelet, self.wavelet_shape(), "wavelet")
        if out is None:
            out = torch.empty(self.gathers_shape(), dtype=torch.float32, device=model.device)
        _need(out, self.gathers_shape(), "out")
        work = self._workspace(save)
        check(lib().sweep_forward(self._h, _ptr(model), _ptr(wavelet), _ptr(out), _ptr(work),
                                  work.numel(), int(bool(save)), _stream()))
        self._fwd_id += 1
        self._saved_id = self._fwd_id if save else -1
        return out

    def forward_noalloc(self, model: torch.Tensor, wavelet: torch.Tensor,
                        out: torch.Tensor) -> torch.Tensor:
        """Shot gathers into `out` with the library's static per-GPU workspace
        instead of the plan's (nothing is allocated: small plans only, whose
        forward workspace fits in 32 MiB; no state for backward())."""
        if self.nparam == 1 and model.dim() == 2:
            model = model.unsqueeze(0)
        _need(model, self._model_shape(), "model")
        _need(wavelet, self.wavelet_shape(), "wavelet")
        _need(out, self.gathers_shape(), "out")
        check(lib().sweep_forward_noalloc(self._h, _ptr(model), _ptr(wavelet), _ptr(out),
                                          _stream()))
        self._fwd_id += 1
        self._saved_id = -1
        return out

    def born(self, model: torch.Tensor, dmodel: torch.Tensor, wavelet: torch.Tensor,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Born (tangent-linear) gathers [nshots, nt, nrec] = (d gathers / d vp)
        . dmodel (Eq. 16), acoustic plans only. The adjoint of this map is
        backward(). Uses the backward-sized workspace and leaves no saved
        forward state."""
        if self.nparam != 1:
            raise ValueError("born() is defined for acoustic plans")
        model = model.unsqueeze(0) if model.dim() == 2 else model
        dmodel = dmodel.unsqueeze(0) if dmodel.dim() == 2 else dmodel
        _need(model, self._model_shape(), "model")
        _need(dmodel, self._model_shape(), "dmodel")
        _need(wavelet, self.wavelet_shape(), "wavelet")
        if out is None:
            out = torch.empty(self.gathers_shape(), dtype=torch.float32, device=model.device)
        _need(out, self.gathers_shape(), "out")
        work = self._workspace(True)
        check(lib().sweep_born_forward(self._h, _ptr(model), _ptr(dmodel), _ptr(wavelet),
                                       _ptr(out), _ptr(work), work.numel(), _stream()))
        self._fwd_id += 1
        self._saved_id = -1
        return out

    def backward(self, resid: torch.Tensor, out: Optional[torch.Tensor] = None,
                 forward_id: Optional[int] = None) -> torch.Tensor:
        """d(loss)/d(model) [nparam, nz, nx] for d(loss)/d(gathers) = resid."""
        if self._saved_id < 0 or (forward_id is not None and forward_id != self._saved_id):
            raise RuntimeError("backward() needs the state saved by the matching "
                               "forward(save=True); a later forward overwrote it")
        _need(resid, self.gathers_shape(), "resid")
        if out is None:
            out = torch.empty(self._model_shape(), dtype=torch.float32, device=resid.device)
        _need(out, self._model_shape(), "out")
        work = self._work
        check(lib().sweep_backward(self._h, _ptr(resid), _ptr(out), _ptr(work), work.numel(),
                                   _stream()))
        return out

    # ---------------------------------------------------------------- timing
    # fwd = forward, adj = adjoint, rec = segment recomputation (stores B^n);
    # acoustic: *_int = interior-tile kernel (single steps), *_zpml / *_xpml =
    # z-frame / x-frame C-PML kernels, *_deep = two-step passes over the deep
    # interior tiles; elastic: the whole step in the *_int slot
    KERNEL_CLASSES = ("fwd_int", "fwd_zpml", "fwd_xpml", "adj_int", "adj_zpml", "adj_xpml",
                      "rec_int", "rec_zpml", "rec_xpml", "fwd_deep", "adj_deep", "rec_deep")

    def set_profiling(self, enable: bool, period: int = 1):
        """Time the step kernels with HIP events (every `period`-th step)."""
        check(lib().sweep_plan_set_profiling(self._h, max(1, int(period)) if enable else 0))

    def graph_nodes(self):
        """(forward, backward): kernel launches held by the captured graphs
        (tuning use_graph = 1)."""
        f, b = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().sweep_plan_graph_nodes(self._h, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value

    def kernel_times(self) -> dict:
        """{class: (launches, total_ms)} since the last set_profiling()."""
        out = {}
        for i, name in enumerate(self.KERNEL_CLASSES):
            n, ms = ctypes.c_int(), ctypes.c_double()
            check(lib().sweep_plan_kernel_time(self._h, i, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (n.value, ms.value)
        return out

    @property
    def last_forward_id(self) -> int:
        return self._fwd_id


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


class Batch:
    """Several acoustic plans (different grids, shot counts, step counts)
    advanced together: one launch per kernel kind and time step serves all of
    them (batch modelling of different models, Sec. 2.2). Results equal those
    of each plan run alone, bit for bit. With use_graph the whole forward /
    backward is captured once as a hipGraph and replayed."""

    def __init__(self, plans, use_graph: bool = False):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        self._ctx = self.plans[0]._ctx if self.plans else None
        check(lib().sweep_batch_create(self._ctx, arr, len(self.plans), ctypes.byref(h)))
        self._h = h
        self._work = None
        self._saved = False
        self.set_graph(use_graph)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().sweep_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def set_graph(self, use_graph: bool):
        check(lib().sweep_batch_set_graph(self._h, int(bool(use_graph))))

    def workspace_bytes(self, for_backward: bool) -> int:
        return int(lib().sweep_batch_workspace_bytes(self._h, int(bool(for_backward))))

    def graph_nodes(self):
        """(forward, backward): kernel launches held by the captured graphs."""
        f, b = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().sweep_batch_graph_nodes(self._h, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value

    def autotune(self, models, wavelets, steps: int = 10, gradient: bool = True,
                 cache_path: Optional[str] = None) -> dict:
        """Pick the fastest tiling (rz, pml_rz) and time-blocking depth (tblock)
        for the whole batch (cached) and set it on every plan; returns it. With
        `gradient` the timed steps are the mix of a gradient (forward,
        recomputation and reverse steps), else forward steps only."""
        ms, ws = [], []
        for p, m, w in zip(self.plans, models, wavelets):
            if p.nparam == 1 and m.dim() == 2:
                m = m.unsqueeze(0)
            _need(m, p._model_shape(), "model")
            _need(w, (p.nshots, p.nt), "wavelet")
            ms.append(m)
            ws.append(w)
        need = self.workspace_bytes(gradient)
        if self._work is None or self._work.numel() < need:
            self._work = None
            torch.cuda.synchronize()
            self._work = torch.empty(need, dtype=torch.uint8, device=ms[0].device)
        chosen = (ctypes.c_int * 3)()
        check(lib().sweep_batch_autotune(self._h, _ptr_array(ms), _ptr_array(ws), _ptr(self._work),
                                         self._work.numel(), steps, int(bool(gradient)),
                                         cache_path.encode() if cache_path else None,
                                         _stream(), chosen))
        self._saved = False
        for p in self.plans:
            p._saved_id = -1
        return {"rz": chosen[0], "pml_rz": chosen[1], "tblock": chosen[2]}

    def forward(self, models, wavelets, save: bool = False, out=None):
        """Gathers of every plan; `out` (optional): the gathers tensors to
        write (fixed buffers keep a captured graph valid across calls)."""
        outs = []
        ms, ws = [], []
        for q, (p, m, w) in enumerate(zip(self.plans, models, wavelets)):
            if p.nparam == 1 and m.dim() == 2:
                m = m.unsqueeze(0)
            _need(m, p._model_shape(), "model")
            _need(w, (p.nshots, p.nt), "wavelet")
            ms.append(m)
            ws.append(w)
            if out is None:
                outs.append(torch.empty(p.gathers_shape(), dtype=torch.float32, device=m.device))
            else:
                _need(out[q], p.gathers_shape(), "out")
                outs.append(out[q])
        need = self.workspace_bytes(save)
        if self._work is None or self._work.numel() < need:
            self._work = None
            torch.cuda.synchronize()
            self._work = torch.empty(need, dtype=torch.uint8, device=ms[0].device)
        check(lib().sweep_batch_forward(self._h, _ptr_array(ms), _ptr_array(ws),
                                        _ptr_array(outs), _ptr(self._work), self._work.numel(),
                                        int(bool(save)), _stream()))
        self._saved = bool(save)
        return outs

    def backward(self, resids, out=None):
        if not self._saved:
            raise RuntimeError("Batch.backward needs a preceding forward(save=True)")
        grads = []
        for q, (p, r) in enumerate(zip(self.plans, resids)):
            _need(r, p.gathers_shape(), "resid")
            if out is None:
                grads.append(torch.empty(p._model_shape(), dtype=torch.float32, device=r.device))
            else:
                _need(out[q], p._model_shape(), "out")
                grads.append(out[q])
        check(lib().sweep_batch_backward(self._h, _ptr_array(list(resids)), _ptr_array(grads),
                                         _ptr(self._work), self._work.numel(), _stream()))
        return grads


class WaveFn(torch.autograd.Function):
    """gathers = F(model); backward returns J^T grad_gathers via the adjoint."""

    @staticmethod
    def forward(ctx, model, wavelet, plan: Plan):
        squeeze = plan.nparam == 1 and model.dim() == 2
        g = plan.forward(model.contiguous(), wavelet.contiguous(), save=True)
        ctx.plan = plan
        ctx.fid = plan.last_forward_id
        ctx.squeeze = squeeze
        return g

    @staticmethod
    def backward(ctx, grad_g):
        grad = ctx.plan.backward(grad_g.contiguous(), forward_id=ctx.fid)
        if ctx.squeeze:
            grad = grad[0]
        return grad, None, None


def l2_misfit(pred: torch.Tensor, obs: torch.Tensor, resid: Optional[torch.Tensor] = None):
    """(resid, J): resid = pred - obs, J = 0.5 sum resid^2 (float64 tensor on
    device); `resid` (optional) is the buffer to write."""
    if pred.shape != obs.shape:
        raise ValueError("pred and obs shapes differ")
    _need(pred, pred.shape, "pred")
    _need(obs, obs.shape, "obs")
    n = pred.numel()
    if resid is None:
        resid = torch.empty_like(pred)
    _need(resid, pred.shape, "resid")
    J = torch.empty((), dtype=torch.float64, device=pred.device)
    scratch = torch.empty(int(lib().sweep_l2_misfit_scratch_bytes(n)), dtype=torch.uint8,
                          device=pred.device)
    check(lib().sweep_l2_misfit(_ptr(pred), _ptr(obs), _ptr(resid), _ptr(J), n, _ptr(scratch),
                                _stream()))
    return resid, J
