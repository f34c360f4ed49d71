"""Seeded problem cases: geometry, models and wavelets as float32-exact
inputs, handed alike to the HIP path and to the oracle (the GPU sees float32;
the oracle sees the same values widened to float64, so both start from
bit-identical inputs). Inputs only: no arithmetic of the method lives here.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import synth


def f32(a) -> np.ndarray:
    """Round to float32 and return as float64 (the values the GPU sees)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclasses.dataclass
class Case:
    """One acoustic problem with explicit geometry and float32-exact inputs."""
    nx: int
    nz: int
    pml: int
    h: float
    dt: float
    nt: int
    f0: float
    vmax: float
    v: np.ndarray          # [nz][nx] float64 holding float32 values
    src: np.ndarray        # [nshots][2] int32
    rec: np.ndarray        # [nshots][nrec][2] int32
    wav: np.ndarray        # [nshots][nt] float64 holding float32 values
    ckpt: int = 50
    R: float = 1e-3

    @property
    def nshots(self):
        return self.src.shape[0]

    @property
    def nrec(self):
        return self.rec.shape[1]

    def oracle_problem(self, orc, nthreads=0):
        return orc.problem(self.nx, self.nz, self.pml, self.h, self.dt, self.nt, self.vmax,
                           self.f0, self.R, nshots=self.nshots, nrec=self.nrec,
                           ckpt_every=self.ckpt, nthreads=nthreads)

    def plan(self, **kw):
        import paper_2604_14189_amd as sw
        return sw.Plan(nx=self.nx, nz=self.nz, h=self.h, dt=self.dt, nt=self.nt, pml=self.pml,
                       src_xz=self.src, rec_xz=self.rec, pml_vmax=self.vmax, pml_f0=self.f0,
                       pml_R=self.R, ckpt_every=self.ckpt, **kw)


def case_from_workload(w: synth.Workload, nshots=None, shots=None, nt=None) -> Case:
    src = w.sources()
    rec = w.receivers()
    wav = w.wavelets()
    if shots is not None:
        src, rec, wav = src[shots], rec[shots], wav[shots]
    if nt is not None:
        wav = wav[:, :nt]
    return Case(w.nx, w.nz, w.pml, w.h, w.dt, nt or w.nt, w.f0, w.pml_vmax(),
                f32(w.true_model()), src.astype(np.int32), rec.astype(np.int32), f32(wav),
                ckpt=w.ckpt_every, R=w.pml_R)


def random_case(seed: int, nx=150, nz=77, pml=10, nt=240, nshots=3, nrec=41, ckpt=17,
                dup=True) -> Case:
    """Ragged grid (not a multiple of the tile size), sources near edges, random
    receivers including coincident ones."""
    rng = np.random.default_rng(seed)
    v = f32(synth.layered_anomaly(nx, nz, 1500.0, 3500.0, seed + 100))
    src = np.stack([rng.integers(0, nx, nshots), rng.integers(0, nz, nshots)], 1)
    src[0] = [0, 0]                       # corner of the model, next to the pad
    if nshots > 1:
        src[1] = [nx - 1, nz // 2]
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))],
                   2)
    if dup and nrec > 3:
        rec[:, 1] = rec[:, 0]             # coincident receivers
        rec[:, 2] = rec[:, 0]
    rec[0, -1] = [nx - 1, nz - 1]
    wav = f32(np.stack([synth.ricker(15.0 + 3 * s, nt, 1e-3) for s in range(nshots)]))
    return Case(nx, nz, pml, 10.0, 1e-3, nt, 15.0, 3500.0, v, src.astype(np.int32),
                rec.astype(np.int32), wav, ckpt=ckpt)


@dataclasses.dataclass
class ElCase:
    """One elastic problem (model [3][nz][nx] = vp, vs, rho) with float32-exact inputs."""
    nx: int
    nz: int
    pml: int
    h: float
    dt: float
    nt: int
    f0: float
    vmax: float
    model: np.ndarray
    src: np.ndarray
    rec: np.ndarray
    wav: np.ndarray
    fs: int = 1
    ckpt: int = 50
    R: float = 1e-3

    @property
    def nshots(self):
        return self.src.shape[0]

    @property
    def nrec(self):
        return self.rec.shape[1]

    def oracle_problem(self, orc, nthreads=0):
        return orc.problem(self.nx, self.nz, self.pml, self.h, self.dt, self.nt, self.vmax,
                           self.f0, self.R, nshots=self.nshots, nrec=self.nrec,
                           free_surface=self.fs, ckpt_every=self.ckpt, nthreads=nthreads)

    def plan(self, **kw):
        import paper_2604_14189_amd as sw
        return sw.Plan(nx=self.nx, nz=self.nz, h=self.h, dt=self.dt, nt=self.nt, pml=self.pml,
                       src_xz=self.src, rec_xz=self.rec, pml_vmax=self.vmax, pml_f0=self.f0,
                       pml_R=self.R, ckpt_every=self.ckpt, physics=sw.ELASTIC,
                       free_surface=self.fs, **kw)


def random_el_case(seed: int, fs=1, nx=90, nz=70, pml=10, nt=300, nshots=3, nrec=23,
                   ckpt=23) -> ElCase:
    rng = np.random.default_rng(seed)
    m = f32(synth.elastic_model(nx, nz, seed + 50))
    src = np.stack([rng.integers(0, nx, nshots), rng.integers(0, nz, nshots)], 1)
    src[0] = [0, 0]
    if nshots > 1:
        src[1] = [nx - 1, nz - 1]
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))],
                   2)
    if nrec > 3:
        rec[:, 1] = rec[:, 0]
        rec[:, 2] = [0, 0]
    wav = f32(np.stack([synth.ricker(20.0 + 2 * s, nt, 0.4e-3) for s in range(nshots)]))
    return ElCase(nx, nz, pml, 5.0, 0.4e-3, nt, 20.0, 4500.0, m, src.astype(np.int32),
                  rec.astype(np.int32), wav, fs=fs, ckpt=ckpt)


def el_case_from_workload(w: synth.Workload, shots=None, nt=None) -> ElCase:
    src, rec, wav = w.sources(), w.receivers(), w.wavelets()
    if shots is not None:
        src, rec, wav = src[shots], rec[shots], wav[shots]
    if nt is not None:
        wav = wav[:, :nt]
    return ElCase(w.nx, w.nz, w.pml, w.h, w.dt, nt or w.nt, w.f0, w.pml_vmax(),
                  f32(w.true_model()), src.astype(np.int32), rec.astype(np.int32), f32(wav),
                  fs=w.free_surface, ckpt=w.ckpt_every, R=w.pml_R)
