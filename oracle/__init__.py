"""FP64 CPU oracle for the SWEEP hot path (arXiv 2604.14189).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The product path (the HIP library and
its Python binding) never imports, links or calls it, and it never imports the
product path: the two share only the seeded inputs of the `synth` module.

The C++ part (acoustic.cpp, elastic.cpp) is built with
``g++ -O3 -fopenmp -ffp-contract=off`` into ``liboracle.so`` next to this file.
The discretisation it follows is written out in ``oracle/README.md``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["acoustic.cpp", "elastic.cpp", "vti.cpp"]


def build(force: bool = True) -> str:
    """Compile liboracle.so (plain g++, no GPU code)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O3", "-fopenmp", "-ffp-contract=off", "-std=c++17", "-shared", "-fPIC",
           "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("nz", ctypes.c_int), ("pml", ctypes.c_int),
        ("free_surface", ctypes.c_int), ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("nt", ctypes.c_int), ("pml_vmax", ctypes.c_double), ("pml_f0", ctypes.c_double),
        ("pml_R", ctypes.c_double), ("nshots", ctypes.c_int), ("nrec", ctypes.c_int),
        ("ckpt_every", ctypes.c_int), ("nthreads", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def problem(nx, nz, pml, h, dt, nt, pml_vmax, pml_f0, pml_R=1e-3, nshots=1, nrec=0,
            free_surface=0, ckpt_every=0, nthreads=0) -> Problem:
    return Problem(nx, nz, pml, free_surface, h, dt, nt, pml_vmax, pml_f0, pml_R, nshots, nrec,
                   ckpt_every, nthreads)


def problem_from(w, nthreads: int = 0, ckpt_every: Optional[int] = None, pml_vmax=None,
                 nshots: Optional[int] = None) -> Problem:
    """Problem struct from a synth.Workload."""
    return problem(w.nx, w.nz, w.pml, w.h, w.dt, w.nt,
                   w.pml_vmax() if pml_vmax is None else pml_vmax, w.f0, w.pml_R,
                   w.nshots if nshots is None else nshots, w.nrec, w.free_surface,
                   w.ckpt_every if ckpt_every is None else ckpt_every, nthreads)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


# ---------------------------------------------------------------- building blocks
def pml_profile(n, lo_pad, hi_pad, h, dt, vmax, f0, R=1e-3, shift=0.0):
    a = np.zeros(n)
    b = np.zeros(n)
    _check(lib().orc_pml_profile(n, lo_pad, hi_pad, ctypes.c_double(shift), ctypes.c_double(h),
                                 ctypes.c_double(dt), ctypes.c_double(vmax),
                                 ctypes.c_double(f0), ctypes.c_double(R), _d(a), _d(b)),
           "pml_profile")
    return a, b


def d2_1d(f, h):
    f = _f64(f)
    out = np.zeros_like(f)
    _check(lib().orc_d2_1d(_d(f), len(f), ctypes.c_double(h), _d(out)), "d2_1d")
    return out


def d1_1d(f, h):
    f = _f64(f)
    out = np.zeros_like(f)
    _check(lib().orc_d1_1d(_d(f), len(f), ctypes.c_double(h), _d(out)), "d1_1d")
    return out


# ---------------------------------------------------------------- acoustic
def ac_forward(pb: Problem, v, src, wavelet, rec) -> np.ndarray:
    v, src, wavelet, rec = _f64(v), _i32(src), _f64(wavelet), _i32(rec)
    out = np.zeros((pb.nshots, pb.nt, pb.nrec))
    _check(lib().orc_ac_forward(ctypes.byref(pb), _d(v), _i(src), _d(wavelet), _i(rec),
                                _d(out)), "ac_forward")
    return out


def ac_wavefield(pb: Problem, v, src, wavelet) -> np.ndarray:
    v, src, wavelet = _f64(v), _i32(src), _f64(wavelet)
    NX, NZ = pb.nx + 2 * pb.pml, pb.nz + 2 * pb.pml
    out = np.zeros((pb.nt, NZ, NX))
    _check(lib().orc_ac_wavefield(ctypes.byref(pb), _d(v), _i(src), _d(wavelet), _d(out)),
           "ac_wavefield")
    return out


def ac_gradient(pb: Problem, v, src, wavelet, rec, resid, want_wavelet=False,
                want_gathers=False):
    """Returns (grad_v, grad_wavelet or None, gathers or None)."""
    v, src, wavelet, rec, resid = _f64(v), _i32(src), _f64(wavelet), _i32(rec), _f64(resid)
    g = np.zeros((pb.nz, pb.nx))
    gw = np.zeros((pb.nshots, pb.nt)) if want_wavelet else None
    ga = np.zeros((pb.nshots, pb.nt, pb.nrec)) if want_gathers else None
    _check(lib().orc_ac_gradient(ctypes.byref(pb), _d(v), _i(src), _d(wavelet), _i(rec),
                                 _d(resid), _d(g), _d(gw) if gw is not None else None,
                                 _d(ga) if ga is not None else None), "ac_gradient")
    return g, gw, ga


def ac_forward_encoded(pb: Problem, v, src, wavelet, rec) -> np.ndarray:
    """Encoded shots: src [nshots][nsrc][2], wavelet [nshots][nsrc][nt]."""
    v, src, wavelet, rec = _f64(v), _i32(src), _f64(wavelet), _i32(rec)
    nsrc = src.shape[1]
    assert src.shape == (pb.nshots, nsrc, 2) and wavelet.shape == (pb.nshots, nsrc, pb.nt)
    out = np.zeros((pb.nshots, pb.nt, pb.nrec))
    _check(lib().orc_ac_forward_encoded(ctypes.byref(pb), ctypes.c_int(nsrc), _d(v), _i(src),
                                        _d(wavelet), _i(rec), _d(out)), "ac_forward_encoded")
    return out


def ac_gradient_encoded(pb: Problem, v, src, wavelet, rec, resid) -> np.ndarray:
    v, src, wavelet, rec, resid = _f64(v), _i32(src), _f64(wavelet), _i32(rec), _f64(resid)
    nsrc = src.shape[1]
    assert src.shape == (pb.nshots, nsrc, 2) and wavelet.shape == (pb.nshots, nsrc, pb.nt)
    g = np.zeros((pb.nz, pb.nx))
    _check(lib().orc_ac_gradient_encoded(ctypes.byref(pb), ctypes.c_int(nsrc), _d(v), _i(src),
                                         _d(wavelet), _i(rec), _d(resid), _d(g)),
           "ac_gradient_encoded")
    return g


def ac_born(pb: Problem, v, dv, src, wavelet, rec) -> np.ndarray:
    v, dv, src, wavelet, rec = _f64(v), _f64(dv), _i32(src), _f64(wavelet), _i32(rec)
    out = np.zeros((pb.nshots, pb.nt, pb.nrec))
    _check(lib().orc_ac_born(ctypes.byref(pb), _d(v), _d(dv), _i(src), _d(wavelet), _i(rec),
                             _d(out)), "ac_born")
    return out


# ---------------------------------------------------------------- elastic
def _el_NZ(pb: Problem) -> int:
    return pb.nz + (1 if pb.free_surface else 2) * pb.pml


def el_forward(pb: Problem, model, src, wavelet, rec) -> np.ndarray:
    model, src, wavelet, rec = _f64(model), _i32(src), _f64(wavelet), _i32(rec)
    out = np.zeros((pb.nshots, pb.nt, pb.nrec, 2))
    _check(lib().orc_el_forward(ctypes.byref(pb), _d(model), _i(src), _d(wavelet), _i(rec),
                                _d(out)), "el_forward")
    return out


def el_wavefield(pb: Problem, model, src, wavelet) -> np.ndarray:
    model, src, wavelet = _f64(model), _i32(src), _f64(wavelet)
    out = np.zeros((pb.nt, 5, _el_NZ(pb), pb.nx + 2 * pb.pml))
    _check(lib().orc_el_wavefield(ctypes.byref(pb), _d(model), _i(src), _d(wavelet), _d(out)),
           "el_wavefield")
    return out


def el_gradient(pb: Problem, model, src, wavelet, rec, resid, want_wavelet=False,
                want_gathers=False):
    model, src, wavelet, rec, resid = (_f64(model), _i32(src), _f64(wavelet), _i32(rec),
                                       _f64(resid))
    g = np.zeros((3, pb.nz, pb.nx))
    gw = np.zeros((pb.nshots, pb.nt)) if want_wavelet else None
    ga = np.zeros((pb.nshots, pb.nt, pb.nrec, 2)) if want_gathers else None
    _check(lib().orc_el_gradient(ctypes.byref(pb), _d(model), _i(src), _d(wavelet), _i(rec),
                                 _d(resid), _d(g), _d(gw) if gw is not None else None,
                                 _d(ga) if ga is not None else None), "el_gradient")
    return g, gw, ga


def el_born(pb: Problem, model, dmodel, src, wavelet, rec) -> np.ndarray:
    model, dmodel, src, wavelet, rec = (_f64(model), _f64(dmodel), _i32(src), _f64(wavelet),
                                        _i32(rec))
    out = np.zeros((pb.nshots, pb.nt, pb.nrec, 2))
    _check(lib().orc_el_born(ctypes.byref(pb), _d(model), _d(dmodel), _i(src), _d(wavelet),
                             _i(rec), _d(out)), "el_born")
    return out


# ---------------------------------------------------------------- VTI
def vti_forward(pb: Problem, model, src, wavelet, rec) -> np.ndarray:
    """model [3][nz][nx] = (vv, v, eta)."""
    model, src, wavelet, rec = _f64(model), _i32(src), _f64(wavelet), _i32(rec)
    out = np.zeros((pb.nshots, pb.nt, pb.nrec))
    _check(lib().orc_vti_forward(ctypes.byref(pb), _d(model), _i(src), _d(wavelet), _i(rec),
                                 _d(out)), "vti_forward")
    return out


def vti_gradient(pb: Problem, model, src, wavelet, rec, resid, want_wavelet=False,
                 want_gathers=False):
    """Returns (grad [3][nz][nx] = dJ/d(vv, v, eta), grad_wavelet or None, gathers or None)."""
    model, src, wavelet, rec, resid = (_f64(model), _i32(src), _f64(wavelet), _i32(rec),
                                       _f64(resid))
    g = np.zeros((3, pb.nz, pb.nx))
    gw = np.zeros((pb.nshots, pb.nt)) if want_wavelet else None
    ga = np.zeros((pb.nshots, pb.nt, pb.nrec)) if want_gathers else None
    _check(lib().orc_vti_gradient(ctypes.byref(pb), _d(model), _i(src), _d(wavelet), _i(rec),
                                  _d(resid), _d(g), _d(gw) if gw is not None else None,
                                  _d(ga) if ga is not None else None), "vti_gradient")
    return g, gw, ga
