"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module generates *inputs only*: velocity models, source wavelets, shot and
receiver geometry and the workload definitions. It holds none of the solver's
arithmetic (no stencil, no damping profile, no adjoint), so the GPU path and the
oracle remain independent implementations that meet only here.

The paper (arXiv 2604.14189) fixes none of these numerically; the recipes below
are the stated synthetic stand-ins:

* layered-plus-anomaly models: 8 layers of seeded random thickness with velocity
  increasing with depth, plus 20 Gaussian anomalies of +-10 % (radius 5-30 cells);
* Ricker wavelet with peak frequency f0 and a 1.5/f0 delay (the paper's examples
  drive every equation with a Ricker source, Sec. 3.1.3);
* shots evenly spaced along a shallow line, one receiver per column.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "ricker", "bandlimited_noise", "rff_frequencies", "layered_anomaly", "interface_model", "smooth", "elastic_model", "vti_model",
    "surface_shots", "line_receivers", "Workload", "workload", "batched_workloads",
    "WORKLOADS",
]


def ricker(f0: float, nt: int, dt: float, delay: Optional[float] = None,
           dtype=np.float64) -> np.ndarray:
    """Ricker wavelet s(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
    tau = n dt - delay, delay = 1.5 / f0 unless given; unit peak."""
    if delay is None:
        delay = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt - delay
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(dtype)


def layered_anomaly(nx: int, nz: int, vmin: float, vmax: float, seed: int,
                    nlayers: int = 8, nanom: int = 20) -> np.ndarray:
    """Velocity [nz][nx] (float64): layers increasing with depth plus Gaussian
    anomalies of +-10 %, clipped to [vmin, vmax]."""
    rng = np.random.default_rng(seed)
    thick = rng.uniform(0.5, 1.5, nlayers)
    edges = np.round(np.cumsum(thick) / thick.sum() * nz).astype(int)
    edges[-1] = nz
    layer_v = np.linspace(vmin, vmax, nlayers)
    v = np.empty((nz, nx), dtype=np.float64)
    top = 0
    for k in range(nlayers):
        v[top:edges[k], :] = layer_v[k]
        top = edges[k]
    zz, xx = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    pert = np.zeros_like(v)
    for _ in range(nanom):
        cx = rng.uniform(0, nx)
        cz = rng.uniform(0, nz)
        r = rng.uniform(5, 30)
        amp = 0.10 * (1.0 if rng.uniform() < 0.5 else -1.0)
        pert += amp * np.exp(-((xx - cx) ** 2 + (zz - cz) ** 2) / (2.0 * r * r))
    v = v * (1.0 + pert)
    return np.clip(v, vmin, vmax)


def interface_model(nx: int = 200, nz: int = 200, v0: float = 2000.0, v1: float = 2500.0,
                    depth: int = 100) -> np.ndarray:
    """Homogeneous v0 with a one-cell-sharp horizontal interface to v1 at row `depth`."""
    v = np.full((nz, nx), v0, dtype=np.float64)
    v[depth:, :] = v1
    return v


def smooth(v: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian smoothing (initial FWI model)."""
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(np.asarray(v, dtype=np.float64), sigma, mode="nearest")


def elastic_model(nx: int, nz: int, seed: int, vpmin: float = 1800.0, vpmax: float = 4500.0,
                  vp_vs: float = 1.73, noise: float = 0.05) -> np.ndarray:
    """[3][nz][nx] = (vp, vs, rho): layered vp, vs = vp/1.73 with +-5 % seeded
    uniform noise per cell, rho = 310 vp^0.25 (Gardner)."""
    vp = layered_anomaly(nx, nz, vpmin, vpmax, seed)
    rng = np.random.default_rng(seed + 7919)
    vs = vp / vp_vs * (1.0 + rng.uniform(-noise, noise, vp.shape))
    rho = 310.0 * vp ** 0.25
    return np.stack([vp, vs, rho])


def vti_model(nx: int, nz: int, seed: int, vmin: float = 1500.0, vmax: float = 4700.0,
              eta_max: float = 0.12, iso_rows: int = 20) -> np.ndarray:
    """VTI model [3][nz][nx] = (vv, v, eta): vv from the layered generator, the
    NMO velocity v up to 3 % above it (smooth seeded field), eta up to eta_max
    growing with depth below an isotropic top zone of iso_rows rows (where the
    sources and receivers of the workloads sit, as the pseudo-acoustic
    formulation asks)."""
    rng = np.random.default_rng(seed + 1000)
    vv = layered_anomaly(nx, nz, vmin, vmax, seed)
    vn = vv * (1.0 + 0.03 * smooth(rng.uniform(0.0, 1.0, (nz, nx)), 5.0) / 0.5)
    vn = np.minimum(vn, vv * 1.03)
    ramp = np.clip((np.arange(nz)[:, None] - iso_rows) / 40.0, 0.0, 1.0)
    eta = eta_max * ramp * np.clip(smooth(rng.uniform(0.5, 1.0, (nz, nx)), 5.0), 0.0, 1.0)
    return np.stack([vv, vn, eta])


def surface_shots(nx: int, nshots: int, depth: int) -> np.ndarray:
    """Shot cells [nshots][2] = (x, z), x = floor((i + 1/2) nx / nshots)."""
    xs = np.floor((np.arange(nshots) + 0.5) * nx / nshots).astype(np.int32)
    return np.stack([xs, np.full(nshots, depth, np.int32)], axis=1).astype(np.int32)


def line_receivers(nx: int, nshots: int, depth: int, nrec: Optional[int] = None) -> np.ndarray:
    """Receivers [nshots][nrec][2]: one per column at `depth` (or nrec evenly
    spaced columns), the same set for every shot."""
    if nrec is None or nrec == nx:
        xs = np.arange(nx, dtype=np.int32)
    else:
        xs = np.floor((np.arange(nrec) + 0.5) * nx / nrec).astype(np.int32)
    one = np.stack([xs, np.full(len(xs), depth, np.int32)], axis=1)
    return np.ascontiguousarray(np.broadcast_to(one, (nshots,) + one.shape)).astype(np.int32)


def bandlimited_noise(shape, f0: float, dt: float, seed: int) -> np.ndarray:
    """Seeded white noise along the last-but-one (time) axis of `shape`
    [..., nt, nrec], filtered by a Ricker of peak f0 so it lies in the band of
    the simulation; a stand-in residual for adjoint tests."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    w = ricker(f0, int(round(3.0 / f0 / dt)) + 1, dt, delay=1.5 / f0)
    from scipy.signal import fftconvolve
    k = w.reshape((1,) * (x.ndim - 2) + (-1, 1))
    y = fftconvolve(x, k, mode="full", axes=x.ndim - 2)
    n0 = (len(w) - 1) // 2
    sl = [slice(None)] * x.ndim
    sl[x.ndim - 2] = slice(n0, n0 + shape[-2])
    return np.ascontiguousarray(y[tuple(sl)])


def rff_frequencies(nfreq: int = 64, sigma: float = 10.0, seed: int = 0) -> np.ndarray:
    """Random Fourier frequencies B [nfreq][2] ~ N(0, sigma^2) for the MLP
    velocity model's coordinate encoding."""
    return np.random.default_rng(seed + 1234).normal(0.0, sigma, (nfreq, 2))


@dataclasses.dataclass
class Workload:
    """One modelling problem: grid, time axis, absorbing pad, sources, receivers."""
    name: str
    physics: str                 # "acoustic", "elastic" or "vti"
    nx: int
    nz: int
    h: float
    dt: float
    nt: int
    pml: int
    f0: float
    nshots: int
    nrec: int
    src_depth: int
    rec_depth: int
    free_surface: int = 0
    pml_R: float = 1e-3
    ckpt_every: int = 50
    seed: int = 0
    vmin: float = 1500.0
    vmax: float = 4700.0

    # ---- inputs ----
    def true_model(self) -> np.ndarray:
        if self.name.startswith("interface"):
            return interface_model(self.nx, self.nz)
        if self.physics == "vti":
            return vti_model(self.nx, self.nz, self.seed, self.vmin, self.vmax)
        if self.physics == "elastic":
            return elastic_model(self.nx, self.nz, self.seed, self.vmin, self.vmax)
        return layered_anomaly(self.nx, self.nz, self.vmin, self.vmax, self.seed)

    def initial_model(self, sigma: float = 20.0) -> np.ndarray:
        m = self.true_model()
        if m.ndim == 3:
            return np.stack([smooth(c, sigma) for c in m])
        return smooth(m, sigma)

    def pml_vmax(self) -> float:
        m = self.true_model()
        if self.physics == "vti":  # the fastest (horizontal) speed v sqrt(1 + 2 eta)
            return float((m[1] * np.sqrt(1.0 + 2.0 * m[2])).max())
        return float(m[0].max() if m.ndim == 3 else m.max())

    def sources(self) -> np.ndarray:
        if self.nshots == 1:
            return np.array([[self.nx // 2, self.src_depth]], np.int32)
        return surface_shots(self.nx, self.nshots, self.src_depth)

    def receivers(self) -> np.ndarray:
        return line_receivers(self.nx, self.nshots, self.rec_depth, self.nrec)

    def wavelets(self, dtype=np.float64) -> np.ndarray:
        w = ricker(self.f0, self.nt, self.dt, dtype=dtype)
        return np.ascontiguousarray(np.broadcast_to(w, (self.nshots, self.nt))).astype(dtype)

    # ---- sizes ----
    @property
    def NX(self) -> int:
        return self.nx + 2 * self.pml

    @property
    def NZ(self) -> int:
        return self.nz + (1 if self.free_surface else 2) * self.pml

    def cell_updates(self) -> int:
        return self.nshots * self.NX * self.NZ * self.nt

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The five workloads. The first is small enough for the oracle to finish in
# seconds; the rest are the full-size measurement problems.
WORKLOADS = {
    # 200x200 acoustic forward, interface at depth 100, source (100,5), 200 receivers.
    "interface200": Workload("interface200", "acoustic", 200, 200, 10.0, 1e-3, 1000, 20,
                             10.0, 1, 200, 5, 5, vmin=2000.0, vmax=2500.0),
    # 1000x300 acoustic FWI gradient, 64 shots, 1000 receivers, 3000 steps.
    "layered1000x300": Workload("layered1000x300", "acoustic", 1000, 300, 10.0, 1e-3, 3000,
                                40, 8.0, 64, 1000, 5, 5),
    # 1000x300 pseudo-acoustic VTI: the acoustic benchmark's grid, shots and
    # receivers with an anisotropic model (eta up to 0.12 below the top 20 rows).
    "vti1000x300": Workload("vti1000x300", "vti", 1000, 300, 10.0, 1e-3, 3000, 40, 8.0, 64,
                            1000, 5, 5),
    # 600x300 elastic, free surface, 32 explosive shots, 600 2-component receivers.
    "elastic600x300": Workload("elastic600x300", "elastic", 600, 300, 5.0, 0.5e-3, 4000, 30,
                               15.0, 32, 600, 5, 5, free_surface=1, vmin=1800.0,
                               vmax=4500.0),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_workloads() -> List[Workload]:
    """Eight uneven acoustic problems: grids 200x200 ... 1200x400, shots
    16 + round(32 m / 7), steps 2000 + round(2000 m / 7), 256 shots in total."""
    sizes = [(200, 200), (400, 200), (600, 300), (800, 300), (1000, 300), (1000, 400),
             (1200, 400), (1200, 400)]
    out = []
    for m, (nx, nz) in enumerate(sizes):
        out.append(Workload(f"batch{m}_{nx}x{nz}", "acoustic", nx, nz, 10.0, 1e-3,
                            2000 + int(round(2000 * m / 7)), 40, 8.0,
                            16 + int(round(32 * m / 7)), nx, 5, 5, seed=m))
    return out
