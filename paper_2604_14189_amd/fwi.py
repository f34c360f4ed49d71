"""Full-waveform inversion driven by the solver's adjoint gradients: plain
grid-parameterised FWI and FWI through a neural (Fourier-feature MLP)
velocity model (the paper's neural-network velocity representations, Sec. 1).

Both minimise J = 1/2 sum (d(v) - d_obs)^2 with Adam. The loss is normalised
by the first iteration's misfit J0 so that Adam's eps acts on a unit-scale
problem: Adam on g / J0 with eps gives the same iterates as Adam on g with
eps * J0, which is what is passed to the kernel (no extra scaling pass).

Every iteration is: (MLP forward) -> forward modelling of all shots with
checkpoints -> L2 misfit -> adjoint gradient dJ/dv -> (MLP backward) -> Adam.
All of it runs in libsweep's kernels; torch provides the buffers.

    python -m paper_2604_14189_amd.fwi [--iters 200] [--prefit 1000] [--workload NAME]

prints one JSON line per reported iteration and a final summary line.
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Optional

import numpy as np
import torch

from .mlp import MLPVelocity, adam_step
from .propagator import Plan, l2_misfit

__all__ = ["GridFWI", "NeuralFWI", "MultiScaleFWI", "LSRTM", "lowpass", "prefit", "rmse"]


def rmse(v: torch.Tensor, v_true: np.ndarray) -> float:
    return float(np.sqrt(np.mean((v.detach().double().cpu().numpy().reshape(v_true.shape)
                                  - v_true) ** 2)))


class GridFWI:
    """Adam directly on the velocity of every model cell (lr in m/s)."""

    def __init__(self, plan: Plan, v0: torch.Tensor, wavelet: torch.Tensor, d_obs: torch.Tensor,
                 lr: float = 10.0, eps: float = 1e-8):
        self.plan, self.wav, self.d_obs = plan, wavelet, d_obs
        self.v = v0.clone().contiguous()
        self.m = torch.zeros_like(self.v)
        self.s = torch.zeros_like(self.v)
        self.d = torch.empty(plan.gathers_shape(), dtype=torch.float32, device=v0.device)
        self.g = torch.empty((1,) + tuple(self.v.shape), dtype=torch.float32, device=v0.device)
        self.lr, self.eps, self.t, self.J0 = lr, eps, 0, None

    def step(self) -> float:
        d = self.plan.forward(self.v, self.wav, save=True, out=self.d)
        r, J = l2_misfit(d, self.d_obs)
        self.plan.backward(r, out=self.g)
        J = float(J.item())
        if self.J0 is None:
            self.J0 = J
        self.t += 1
        adam_step(self.v.view(-1), self.m.view(-1), self.s.view(-1), self.g.view(-1), self.t,
                  self.lr, eps=self.eps * self.J0)
        return J

    @property
    def velocity(self) -> torch.Tensor:
        return self.v


def lowpass(x: torch.Tensor, dt: float, fmax: float, dim: int = -1) -> torch.Tensor:
    """Zero-phase low-pass along `dim` (time): the spectrum is kept up to
    0.75 fmax and tapered to zero at fmax with a half cosine. Driver-level
    preparation of the data of one frequency band (not a step of the
    modelling), applied alike to the wavelets and the observed gathers."""
    n = x.shape[dim]
    X = torch.fft.rfft(x.double(), dim=dim)
    f = torch.fft.rfftfreq(n, d=dt).to(x.device)
    f0 = 0.75 * fmax
    w = torch.where(f <= f0, torch.ones_like(f),
                    torch.where(f >= fmax, torch.zeros_like(f),
                                0.5 * (1.0 + torch.cos(np.pi * (f - f0) / (fmax - f0)))))
    shape = [1] * x.dim()
    shape[dim] = -1
    y = torch.fft.irfft(X * w.view(shape), n=n, dim=dim)
    return y.to(x.dtype).contiguous()


class MultiScaleFWI:
    """Multi-scale (frequency-continuation) grid FWI: stages of increasing
    highest frequency; each stage low-passes the wavelets and the observed
    data to its band and runs grid FWI (Adam, fresh moments per stage) from
    the previous stage's model. Fitting the low frequencies first keeps the
    early model updates free of cycle skipping (the paper's workflows, Sec. 1).
    stages: [(fmax in Hz, iterations), ...]; fmax None is the full band."""

    def __init__(self, plan: Plan, v0: torch.Tensor, wavelet: torch.Tensor, d_obs: torch.Tensor,
                 stages, dt: float, lr: float = 10.0, eps: float = 1e-8):
        self.plan, self.wav, self.d_obs, self.dt = plan, wavelet, d_obs, dt
        self.stages = list(stages)
        self.v = v0.clone().contiguous()
        self.lr, self.eps = lr, eps
        self.history = []  # (stage, fmax, iteration, J of the stage's band)

    def run(self, callback=None) -> torch.Tensor:
        for k, (fmax, iters) in enumerate(self.stages):
            if fmax is None:
                wav, obs = self.wav, self.d_obs
            else:
                wav = lowpass(self.wav, self.dt, fmax, dim=-1)
                obs = lowpass(self.d_obs, self.dt, fmax, dim=1)
            opt = GridFWI(self.plan, self.v, wav, obs, lr=self.lr, eps=self.eps)
            for it in range(iters):
                J = opt.step()
                self.history.append((k, fmax, it, J))
                if callback:
                    callback(k, fmax, it, J, opt)
            self.v = opt.velocity
        return self.v

    @property
    def velocity(self) -> torch.Tensor:
        return self.v


class LSRTM:
    """Least-squares reverse-time migration: the model perturbation dv that
    fits data d with Born modelling about a fixed background v0 (Eq. 16),
    min 1/2 |L dv - d|^2 with L = plan.born(v0, ., wavelet), by conjugate
    gradients on the normal equations (CGLS). L^T r is the adjoint gradient
    plan.backward(r) after a saving forward on v0 (Born modelling leaves no
    saved state, so each application re-runs it). Each iteration applies L
    once and L^T once; the data residual |r| falls monotonically (up to the
    operators' float32 rounding). Sums are taken in float64."""

    def __init__(self, plan: Plan, v0: torch.Tensor, wavelet: torch.Tensor, d: torch.Tensor):
        self.plan, self.v0, self.wav = plan, v0.contiguous(), wavelet
        self.x = torch.zeros_like(self.v0)
        self.r = d.clone().contiguous()
        self.s = self._adjoint(self.r)
        self.p = self.s.clone()
        self.gamma = self._dot(self.s, self.s)
        self.history = [self._norm(self.r)]  # |r| after each iteration, |d| first

    @staticmethod
    def _dot(a: torch.Tensor, b: torch.Tensor) -> float:
        return float(torch.sum(a.double() * b.double()).item())

    def _norm(self, a: torch.Tensor) -> float:
        return self._dot(a, a) ** 0.5

    def _adjoint(self, r: torch.Tensor) -> torch.Tensor:
        self.plan.forward(self.v0, self.wav, save=True)
        return self.plan.backward(r).reshape(self.v0.shape).clone()

    def step(self) -> float:
        """One CGLS iteration; returns the data residual norm |L dv - d|."""
        q = self.plan.born(self.v0, self.p, self.wav)
        qq = self._dot(q, q)
        if qq == 0.0 or self.gamma == 0.0:
            return self.history[-1]
        alpha = self.gamma / qq
        self.x.add_(self.p, alpha=alpha)
        self.r.add_(q, alpha=-alpha)
        self.s = self._adjoint(self.r)
        gamma = self._dot(self.s, self.s)
        self.p = self.s + (gamma / self.gamma) * self.p
        self.gamma = gamma
        self.history.append(self._norm(self.r))
        return self.history[-1]

    @property
    def perturbation(self) -> torch.Tensor:
        return self.x


class NeuralFWI:
    """Adam on the MLP parameters; the velocity is the network's output. The
    network's Adam state starts from zero (moments left by a pre-fit belong to
    a different loss and would swamp the FWI gradients)."""

    def __init__(self, plan: Plan, net: MLPVelocity, wavelet: torch.Tensor, d_obs: torch.Tensor,
                 lr: float = 1e-3, eps: float = 1e-8):
        self.plan, self.net, self.wav, self.d_obs = plan, net, wavelet, d_obs
        net.reset_optimizer()
        dev = net.theta.device
        self.d = torch.empty(plan.gathers_shape(), dtype=torch.float32, device=dev)
        self.g = torch.empty((1, net.nz, net.nx), dtype=torch.float32, device=dev)
        self.lr, self.eps, self.J0 = lr, eps, None
        self.v = None

    def step(self) -> float:
        self.v = self.net.forward()
        d = self.plan.forward(self.v, self.wav, save=True, out=self.d)
        r, J = l2_misfit(d, self.d_obs)
        self.plan.backward(r, out=self.g)
        gt = self.net.backward(self.g.view(self.net.nz, self.net.nx))
        J = float(J.item())
        if self.J0 is None:
            self.J0 = J
        self.net.step(gt, lr=self.lr, eps=self.eps * self.J0)
        return J

    @property
    def velocity(self) -> torch.Tensor:
        return self.net.forward()


def prefit(net: MLPVelocity, target: torch.Tensor, steps: int, lr: float = 1e-3) -> float:
    """Fit the network to a velocity model by least squares (1/2 sum (v - target)^2),
    with the same kernels, from a fresh Adam state; returns the final RMS misfit in m/s."""
    target = target.contiguous()
    net.reset_optimizer()
    L = None
    for _ in range(steps):
        v = net.forward()
        r, L = l2_misfit(v, target)
        net.step(net.backward(r), lr=lr)
    return float(np.sqrt(2.0 * float(L.item()) / target.numel())) if L is not None else float("nan")


def _main(argv: Optional[list] = None):
    import synth
    from .propagator import Plan

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="layered1000x300")
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--prefit", type=int, default=1000)
    ap.add_argument("--report", type=int, default=10)
    ap.add_argument("--lr-grid", type=float, default=10.0)
    ap.add_argument("--lr-mlp", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--methods", default="grid,mlp",
                    help="comma-separated subset of grid, mlp, multiscale")
    ap.add_argument("--stages", default="0.5:0.25,0.75:0.25,1:0.5",
                    help="multi-scale stages, fmax/f0:fraction of the iterations, comma-separated")
    args = ap.parse_args(argv)
    methods = [m for m in args.methods.split(",") if m]

    w = synth.workload(args.workload)
    dev = torch.device("cuda:0")
    v_true = w.true_model()
    v_init = synth.smooth(v_true, 20.0)
    src, rec = w.sources().astype(np.int32), w.receivers().astype(np.int32)
    wav = torch.tensor(w.wavelets(), dtype=torch.float32, device=dev)
    plan = Plan(nx=w.nx, nz=w.nz, h=w.h, dt=w.dt, nt=w.nt, pml=w.pml, src_xz=src, rec_xz=rec,
                pml_vmax=w.pml_vmax(), pml_f0=w.f0, pml_R=w.pml_R, ckpt_every=w.ckpt_every)
    vt = torch.tensor(v_true, dtype=torch.float32, device=dev)
    d_obs = plan.forward(vt, wav).clone()
    v0 = torch.tensor(v_init, dtype=torch.float32, device=dev)

    B = synth.rff_frequencies(seed=args.seed)
    net = MLPVelocity(w.nx, w.nz, B, _init_theta(args.seed), vmin=1500.0, vscale=3200.0,
                      device=dev)
    t0 = time.perf_counter()
    fit = prefit(net, v0, args.prefit)
    torch.cuda.synchronize()
    print(json.dumps({"prefit_steps": args.prefit, "prefit_rms_ms": fit,
                      "prefit_s": round(time.perf_counter() - t0, 2),
                      "rmse_start_grid": rmse(v0, v_true),
                      "rmse_start_mlp": rmse(net.forward(), v_true)}), flush=True)

    runs = {}
    if "grid" in methods:
        runs["grid"] = GridFWI(plan, v0, wav, d_obs, lr=args.lr_grid)
    if "mlp" in methods:
        runs["mlp"] = NeuralFWI(plan, net, wav, d_obs, lr=args.lr_mlp)
    summary = {}
    if "multiscale" in methods:
        stages = []
        for tok in args.stages.split(","):
            fr, share = (float(x) for x in tok.split(":"))
            stages.append((None if fr >= 1.0 else fr * w.f0 * 2.5, int(round(share * args.iters))))
        ms = MultiScaleFWI(plan, v0, wav, d_obs, stages, dt=w.dt, lr=args.lr_grid)
        t0 = time.perf_counter()

        def report(k, fmax, it, J, opt):
            if it % args.report == 0:
                print(json.dumps({"method": "multiscale", "stage": k, "fmax": fmax, "iter": it,
                                  "J_rel_band": J / opt.J0, "rmse": rmse(opt.velocity, v_true),
                                  "s": round(time.perf_counter() - t0, 1)}), flush=True)

        vms = ms.run(report)
        torch.cuda.synchronize()
        g0 = GridFWI(plan, v0, wav, d_obs)
        J0 = g0.step()
        _, Jf = l2_misfit(plan.forward(vms, wav), d_obs)
        summary["multiscale"] = {"J_rel_final": float(Jf.item()) / J0,
                                 "rmse_final": rmse(vms, v_true),
                                 "stages": [(f, n) for f, n in stages],
                                 "s_per_iter": round((time.perf_counter() - t0) / args.iters, 3)}
    for name, opt in runs.items():
        t0 = time.perf_counter()
        J = None
        for it in range(1, args.iters + 1):
            J = opt.step()
            if it % args.report == 0 or it == 1:
                print(json.dumps({"method": name, "iter": it, "J_rel": J / opt.J0,
                                  "rmse": rmse(opt.velocity, v_true),
                                  "s": round(time.perf_counter() - t0, 1)}), flush=True)
        torch.cuda.synchronize()
        vfin = opt.velocity
        d = plan.forward(vfin, wav)
        _, Jf = l2_misfit(d, d_obs)
        summary[name] = {"J_rel_final": float(Jf.item()) / opt.J0, "rmse_final": rmse(vfin, v_true),
                         "s_per_iter": round((time.perf_counter() - t0) / args.iters, 3)}
    if "grid" in summary and "mlp" in summary:
        summary["mlp_gain"] = {
            "rmse_ratio_grid_over_mlp": summary["grid"]["rmse_final"] / summary["mlp"]["rmse_final"],
            "misfit_ratio_grid_over_mlp":
                summary["grid"]["J_rel_final"] / summary["mlp"]["J_rel_final"]}
    print(json.dumps({"summary": summary, "workload": args.workload, "iters": args.iters,
                      "lr_grid": args.lr_grid, "lr_mlp": args.lr_mlp}), flush=True)


def _init_theta(seed: int) -> np.ndarray:
    """Weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), zero biases, in the parameter
    order W1, b1, W2, b2, W3, b3, W4, b4, w5, b5."""
    rng = np.random.default_rng(seed + 1)
    shapes = [(256, 128), (256,), (256, 256), (256,), (256, 256), (256,), (256, 256), (256,),
              (256,), (1,)]
    fan = {0: 128, 2: 256, 4: 256, 6: 256, 8: 256}
    out = []
    for k, s in enumerate(shapes):
        if k in fan:
            out.append(rng.uniform(-1.0, 1.0, s) / np.sqrt(fan[k]))
        else:
            out.append(np.zeros(s))
    return np.concatenate([o.ravel() for o in out]).astype(np.float32)


if __name__ == "__main__":
    _main()
