"""Pins for the first-order variable-density acoustic system (Eq. 1) as the
FP64 staggered oracle computes it: the elastic scheme (Eq. 12) with vs = 0,
where both normal stresses equal -p and the shear stress stays 0. CPU only.

* the closed-form field of an explosive (pressure) source in a homogeneous
  fluid, with the scheme's 4th-order convergence in time step;
* transpose identities with and without the pressure-release top;
* finite differences of the misfit in vp and rho, and an exact zero
  derivative in vs at vs = 0 (the gradient's (vp, rho) planes are those the
  GPU path returns).
"""
import numpy as np
import pytest

import synth
from tests.test_oracle_elastic import _explosive_error


def _fluid(nx, nz, seed):
    vp = synth.layered_anomaly(nx, nz, 1500.0, 3500.0, seed)
    rho = 310.0 * vp ** 0.25
    return np.stack([vp, np.zeros((nz, nx)), rho])


def _small(orc, fs, seed=0, nt=140):
    nx, nz, P, nshots, nrec = 34, 30, 8, 2, 9
    rng = np.random.default_rng(seed)
    m = _fluid(nx, nz, seed + 11)
    src = np.stack([rng.integers(2, nx - 2, nshots), rng.integers(1, nz - 2, nshots)], 1)
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))], 2)
    pb = orc.problem(nx, nz, P, 5.0, 0.5e-3, nt, 3500.0, 20.0, 1e-3, nshots=nshots, nrec=nrec,
                     free_surface=fs, ckpt_every=13)
    w = rng.standard_normal((nshots, nt))
    r = rng.standard_normal((nshots, nt, nrec, 2))
    return pb, m, src, rec, w, r, rng


def test_fluid_explosive_source_closed_form(orc):
    e1 = _explosive_error(orc, 1, vs=0.0)
    e2 = _explosive_error(orc, 2, vs=0.0)
    assert e1 < 5e-3
    assert e1 / e2 > 3.5


@pytest.mark.parametrize("fs", [0, 1])
def test_fluid_dot_product_source(orc, fs):
    pb, m, src, rec, w, r, _ = _small(orc, fs)
    d = orc.el_forward(pb, m, src, w, rec)
    _, gw, _ = orc.el_gradient(pb, m, src, w, rec, r, want_wavelet=True)
    lhs, rhs = np.sum(d * r), np.sum(w * gw)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("fs", [0, 1])
def test_fluid_dot_product_born(orc, fs):
    pb, m, src, rec, w, r, rng = _small(orc, fs, seed=3)
    dm = rng.standard_normal(m.shape) * np.array([100.0, 0.0, 50.0])[:, None, None]
    dd = orc.el_born(pb, m, dm, src, w, rec)
    g, _, _ = orc.el_gradient(pb, m, src, w, rec, r)
    lhs, rhs = np.sum(dd * r), np.sum(dm * g)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_fluid_gradient_matches_finite_differences(orc):
    nx, nz, nt = 32, 32, 150
    mt = _fluid(nx, nz, 21)
    m0 = mt.copy()
    m0[0] = synth.smooth(mt[0], 3.0)
    m0[2] = synth.smooth(mt[2], 3.0)
    src = np.array([[8, 3], [24, 3]])
    rec = np.stack([np.stack([np.arange(32), np.full(32, 2)], 1)] * 2)
    pb = orc.problem(nx, nz, 8, 5.0, 0.5e-3, nt, 3500.0, 25.0, 1e-3, nshots=2, nrec=32,
                     free_surface=1, ckpt_every=16)
    w = np.stack([synth.ricker(25.0, nt, 0.5e-3)] * 2)
    dobs = orc.el_forward(pb, mt, src, w, rec)

    def J(m):
        return 0.5 * np.sum((orc.el_forward(pb, m, src, w, rec) - dobs) ** 2)

    d0 = orc.el_forward(pb, m0, src, w, rec)
    g, _, _ = orc.el_gradient(pb, m0, src, w, rec, d0 - dobs)
    assert np.all(g[1] == 0.0)
    rng = np.random.default_rng(5)
    for c, scale in ((0, 50.0), (2, 20.0)):
        dm = np.zeros_like(m0)
        dm[c] = rng.standard_normal((nz, nx)) * scale
        an = np.sum(g * dm)
        eps = 1e-3
        fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
        assert abs(fd - an) <= 1e-6 * abs(an), (c, fd, an)
