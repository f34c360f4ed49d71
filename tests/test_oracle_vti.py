"""Pins for the FP64 pseudo-acoustic VTI oracle (Sec. 3.3.1, Eq. 5), CPU only.

* eta = 0 with v = vv is the isotropic acoustic equation: gathers equal the
  acoustic oracle's, and the gradients in vv and v add up to its gradient;
* the dot-product test of the source-to-data map and its adjoint;
* the model gradient (vv, v, eta) against central finite differences;
* plane-wave speeds of a homogeneous medium along the axes: v sqrt(1 + 2 eta)
  horizontally and vv vertically (the qP phase speed of Eq. 5 at 90 and 0
  degrees, where the slow artificial mode has zero speed);
* absorption: with eta > 0 inside and the eta = 0 pad, the field decays away.
"""
import math

import numpy as np
import pytest

import synth


def _vti_model(nx, nz, seed, eta_max=0.25):
    rng = np.random.default_rng(seed)
    vv = synth.layered_anomaly(nx, nz, 1500.0, 3000.0, seed + 1)
    vn = vv * (1.0 + 0.1 * rng.uniform(0.0, 1.0, (nz, nx)))
    eta = synth.smooth(rng.uniform(0.0, eta_max, (nz, nx)), 2.0)
    return np.stack([vv, vn, eta])


def _small(orc, nshots=2, nt=160, seed=0, ck=23, nx=36, nz=30, P=8):
    m = _vti_model(nx, nz, seed)
    rng = np.random.default_rng(seed + 10)
    src = np.stack([rng.integers(2, nx - 2, nshots), rng.integers(2, nz - 2, nshots)], 1)
    nrec = 9
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))], 2)
    vmax = float((m[1] * np.sqrt(1.0 + 2.0 * m[2])).max())
    pb = orc.problem(nx, nz, P, 10.0, 1e-3, nt, vmax, 15.0, 1e-3, nshots=nshots, nrec=nrec,
                     ckpt_every=ck)
    w = rng.standard_normal((nshots, nt))
    r = rng.standard_normal((nshots, nt, nrec))
    return pb, m, src, rec, w, r


def test_eta_zero_is_the_acoustic_equation(orc):
    pb, m, src, rec, w, r = _small(orc, seed=1)
    v = m[0]
    iso = np.stack([v, v, np.zeros_like(v)])
    d_vti = orc.vti_forward(pb, iso, src, w, rec)
    d_ac = orc.ac_forward(pb, v, src, w, rec)
    assert np.abs(d_vti - d_ac).max() <= 1e-12 * np.abs(d_ac).max()
    g_vti, _, _ = orc.vti_gradient(pb, iso, src, w, rec, r)
    g_ac, _, _ = orc.ac_gradient(pb, v, src, w, rec, r)
    np.testing.assert_allclose(g_vti[0] + g_vti[1], g_ac, rtol=0, atol=1e-12 * np.abs(g_ac).max())


def test_dot_product_source(orc):
    pb, m, src, rec, w, r = _small(orc, seed=2)
    d = orc.vti_forward(pb, m, src, w, rec)
    _, gw, ga = orc.vti_gradient(pb, m, src, w, rec, r, want_wavelet=True, want_gathers=True)
    lhs, rhs = np.sum(d * r), np.sum(w * gw)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.array_equal(ga, d)


def test_gradient_matches_finite_differences(orc):
    pb, m, src, rec, w, _ = _small(orc, seed=3, nt=150, nx=32, nz=32)
    w = np.stack([synth.ricker(15.0, pb.nt, pb.dt)] * pb.nshots)
    mt = m.copy()
    mt[:, 12:20, 10:22] *= 1.05
    dobs = orc.vti_forward(pb, mt, src, w, rec)

    def J(mm):
        return 0.5 * np.sum((orc.vti_forward(pb, mm, src, w, rec) - dobs) ** 2)

    d0 = orc.vti_forward(pb, m, src, w, rec)
    g, _, _ = orc.vti_gradient(pb, m, src, w, rec, d0 - dobs)
    rng = np.random.default_rng(7)
    dm = rng.standard_normal(m.shape) * np.array([30.0, 30.0, 0.01])[:, None, None]
    # each parameter on its own, then all together: the central difference
    # converges to the adjoint gradient as eps^2 (eta's direction is the most
    # curved, so the comparison is made at eps = 1e-4)
    for c in (0, 1, 2, None):
        dc = dm.copy() if c is None else np.zeros_like(dm)
        if c is not None:
            dc[c] = dm[c]
        an = np.sum(g * dc)
        err = [abs((J(m + e * dc) - J(m - e * dc)) / (2 * e) - an) / abs(an) for e in (1e-3, 1e-4)]
        assert err[1] <= 1e-6, (c, err)
        assert err[0] / err[1] > 30.0 or err[0] <= 1e-7, (c, err)


def _lag(a, b, dt):
    c = np.correlate(b, a, mode="full")
    k = int(np.argmax(c))
    y0, y1, y2 = c[k - 1], c[k], c[k + 1]
    return (k - (len(a) - 1) + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt


def test_axis_speeds_of_a_homogeneous_medium(orc):
    nx = nz = 161
    h, dt, nt, f0, P = 5.0, 0.5e-3, 700, 25.0, 20
    vv, vn, eta = 2000.0, 2200.0, 0.2
    vx = vn * math.sqrt(1.0 + 2.0 * eta)
    m = np.stack([np.full((nz, nx), vv), np.full((nz, nx), vn), np.full((nz, nx), eta)])
    c = 80
    d1, d2 = 25, 60
    rec = np.array([[[c + d1, c], [c + d2, c], [c, c + d1], [c, c + d2]]])
    pb = orc.problem(nx, nz, P, h, dt, nt, vx, f0, 1e-3, nshots=1, nrec=4)
    d = orc.vti_forward(pb, m, np.array([[c, c]]), synth.ricker(f0, nt, dt)[None], rec)[0]
    sx = (d2 - d1) * h / _lag(d[:, 0], d[:, 1], dt)
    sz = (d2 - d1) * h / _lag(d[:, 2], d[:, 3], dt)
    assert abs(sx / vx - 1.0) < 0.01, (sx, vx)
    assert abs(sz / vv - 1.0) < 0.01, (sz, vv)


def _energy(orc, m, nt):
    nz, nx = m.shape[1:]
    xs, zs = np.meshgrid(np.arange(0, nx, 5), np.arange(0, nz, 5))
    rec = np.stack([xs.ravel(), zs.ravel()], 1)[None]
    vmax = float((m[1] * np.sqrt(1.0 + 2.0 * m[2])).max())
    pb = orc.problem(nx, nz, 20, 10.0, 1e-3, nt, vmax, 15.0, 1e-3, nshots=1,
                     nrec=rec.shape[1])
    d = orc.vti_forward(pb, m, np.array([[nx // 2, nz // 2]]),
                        synth.ricker(15.0, nt, 1e-3)[None], rec)[0]
    return np.sum(d ** 2, axis=1)


def test_elliptic_medium_is_absorbed(orc):
    # eta = 0 with v != vv (elliptic anisotropy): the per-axis C-PML absorbs
    # the waves as in the isotropic case
    m = np.stack([np.full((80, 80), 2000.0), np.full((80, 80), 2300.0), np.zeros((80, 80))])
    e = _energy(orc, m, 3000)
    assert np.all(np.isfinite(e))
    assert e[-500:].max() / e.max() < 1e-6


def test_anisotropic_run_stays_bounded(orc):
    # eta > 0: the scheme also carries the slow artificial mode of the
    # pseudo-acoustic equation (the source sits in an isotropic patch, as the
    # qP formulation asks, but the eta contrasts still convert a little
    # energy into it), which the pad does not absorb at zero frequency. Over
    # 6000 steps the field stays finite and small and does not grow.
    m = np.stack([np.full((80, 80), 2000.0), np.full((80, 80), 2100.0),
                  np.full((80, 80), 0.25)])
    m[2, 30:50, 30:50] = 0.0
    e = _energy(orc, m, 6000)
    assert np.all(np.isfinite(e))
    assert e[3000:].max() / e.max() < 1e-3
    assert e[5000:].max() <= 3.0 * e[2000:3000].max()
