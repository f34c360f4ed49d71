"""Pins for the FP64 acoustic oracle (CPU only).

Each test checks the oracle against something other than itself: exactness on
polynomials, a conserved discrete energy, the closed-form 2-D Green's function,
absorption measured against a much larger domain, transpose identities
(dot-product tests, Sec. 1), finite differences, symmetry and time invariance.
"""
import numpy as np
import pytest

import synth
from tests.analytic import acoustic_trace


# ---------------------------------------------------------------- stencils
@pytest.mark.parametrize("deg", range(0, 10))
def test_d2_exact_on_polynomials(orc, deg):
    # the 8th-order second-derivative stencil is exact for degree <= 9
    h = 0.7
    x = (np.arange(40) - 17.3) * h
    f = x ** deg
    ref = deg * (deg - 1) * x ** (deg - 2) if deg >= 2 else np.zeros_like(x)
    got = orc.d2_1d(f, h)
    sl = slice(4, -4)  # away from the zero padding
    scale = np.abs(f[sl]).max() / h ** 2 + 1.0
    assert np.abs(got[sl] - ref[sl]).max() <= 1e-10 * scale


@pytest.mark.parametrize("deg", range(0, 9))
def test_d1_exact_on_polynomials(orc, deg):
    # the 8th-order first-derivative stencil is exact for degree <= 8
    h = 1.3
    x = (np.arange(40) - 21.7) * h
    f = x ** deg
    ref = deg * x ** (deg - 1) if deg >= 1 else np.zeros_like(x)
    got = orc.d1_1d(f, h)
    sl = slice(4, -4)
    scale = np.abs(f[sl]).max() / h + 1.0
    assert np.abs(got[sl] - ref[sl]).max() <= 1e-11 * scale


def test_stencils_see_zero_outside(orc):
    # a single spike at the first cell: its neighbours outside the array are zero
    f = np.zeros(12)
    f[0] = 1.0
    d2 = orc.d2_1d(f, 1.0)
    assert d2[0] == pytest.approx(-205.0 / 72.0, rel=1e-15)
    assert d2[1] == pytest.approx(8.0 / 5.0, rel=1e-15)
    assert d2[4] == pytest.approx(-1.0 / 560.0, rel=1e-15)
    assert d2[5] == 0.0
    d1 = orc.d1_1d(f, 1.0)
    assert d1[1] == pytest.approx(-4.0 / 5.0, rel=1e-15)  # (f_{i+1} - f_{i-1}) b1 at i=1
    assert d1[4] == pytest.approx(1.0 / 280.0, rel=1e-15)


# ---------------------------------------------------------------- PML profile
def test_pml_profile_shape(orc):
    n, P, h, dt, vmax, f0, R = 100, 20, 10.0, 1e-3, 3000.0, 10.0, 1e-3
    a, b = orc.pml_profile(n, P, P, h, dt, vmax, f0, R)
    interior = slice(P, n - P)
    assert np.all(a[interior] == 0.0)
    np.testing.assert_allclose(b[interior], np.exp(-np.pi * f0 * dt), rtol=1e-15)
    assert np.all(a[:P] < 0.0) and np.all(a[n - P:] < 0.0)
    # the memory-term weight a grows in magnitude towards the outer edge
    # (d rises quadratically, alpha falls linearly); the profile is symmetric
    assert np.all(np.diff(a[:P + 1]) > 0)
    np.testing.assert_allclose(a, a[::-1], rtol=0, atol=1e-15)
    # outermost cell: alpha = 0, d = d0 = -3 vmax ln R / (2 L)
    d0 = -3.0 * vmax * np.log(R) / (2.0 * P * h)
    assert b[0] == pytest.approx(np.exp(-d0 * dt), rel=1e-14)
    assert a[0] == pytest.approx(b[0] - 1.0, rel=1e-14)


def test_pml_profile_half_nodes(orc):
    # Half nodes (shift 0.5, the staggered elastic grid) sample the same profile
    # of position as the integer nodes: node i + 1/2 of an axis (n, P, h) is
    # integer node 2i + 1 of the axis refined by two (2n - 1, 2P, h/2), whose
    # pad has the same thickness and whose integer nodes are pinned above. A
    # half-cell error in where shift places the node fails this.
    n, P, h, dt, vmax, f0, R = 61, 12, 10.0, 1e-3, 3000.0, 10.0, 1e-3
    for lo in (P, 0):  # both pads, and no top pad (free surface)
        ah, bh = orc.pml_profile(n, lo, P, h, dt, vmax, f0, R, shift=0.5)
        ar, br = orc.pml_profile(2 * n - 1, 2 * lo, 2 * P, h / 2, dt, vmax, f0, R)
        np.testing.assert_allclose(ah[:-1], ar[1::2], rtol=1e-14, atol=0)
        np.testing.assert_allclose(bh[:-1], br[1::2], rtol=1e-14, atol=0)
    # with equal pads the half nodes i + 1/2 and (n - 2 - i) + 1/2 mirror each
    # other about the centre of the axis
    ah, bh = orc.pml_profile(n, P, P, h, dt, vmax, f0, R, shift=0.5)
    np.testing.assert_allclose(ah[:-1], ah[-2::-1], rtol=1e-14, atol=0)
    # the last half node of each pad sits half a cell in (damped, a < 0); the
    # first half node past it is undamped
    assert ah[P - 1] < 0.0 and ah[P] == 0.0
    assert ah[n - 1 - P] < 0.0 and ah[n - 2 - P] == 0.0


# ---------------------------------------------------------------- energy
def test_discrete_energy_is_conserved(orc):
    # Without damping or source, leapfrog with a symmetric Laplacian L conserves
    # E^{n+1/2} = sum (p^{n+1}-p^n)^2 / C - <p^{n+1}, L p^n>. With L p^n taken from
    # the recurrence itself this is sum (p^n p^n - p^{n+1} p^{n-1}) / C.
    nx, nz, nt, dt, h = 48, 40, 1500, 1e-3, 10.0
    v = synth.layered_anomaly(nx, nz, 1500.0, 3500.0, seed=3)
    w = synth.ricker(25.0, nt, dt)
    w[80:] = 0.0  # source switched off: energy must stay fixed from then on
    pb = orc.problem(nx, nz, 0, h, dt, nt, 3500.0, 25.0, nshots=1)
    snaps = orc.ac_wavefield(pb, v, np.array([[20, 17]]), w[None])
    C = (v * dt) ** 2
    E = [np.sum((snaps[n] ** 2 - snaps[n + 1] * snaps[n - 1]) / C) for n in range(100, nt - 1)]
    E = np.array(E)
    assert E[0] > 0
    assert np.abs(E - E[0]).max() / E[0] < 1e-11


# ---------------------------------------------------------------- closed form
def _point_source_trace(orc, dt_factor):
    nx = nz = 200
    dt = 1e-3 / dt_factor
    nt = 600 * dt_factor
    f0, v0 = 10.0, 2000.0
    pb = orc.problem(nx, nz, 20, 10.0, dt, nt, v0, f0, 1e-3, nshots=1, nrec=1)
    v = np.full((nz, nx), v0)
    d = orc.ac_forward(pb, v, np.array([[100, 100]]), synth.ricker(f0, nt, dt)[None],
                       np.array([[[150, 100]]]))[0, :, 0]
    times = (np.arange(nt) + 1) * dt  # gathers[n] = p^{n+1} ~ p(t_{n+1})
    ref = acoustic_trace(500.0, times, v0, f0)
    return np.linalg.norm(d - ref) / np.linalg.norm(ref)


def test_closed_form_green_function(orc):
    e1 = _point_source_trace(orc, 1)
    e2 = _point_source_trace(orc, 2)
    e4 = _point_source_trace(orc, 4)
    assert e1 < 1e-2
    # second order in time: each halving of dt cuts the error by ~4
    assert e1 / e2 > 3.5 and e2 / e4 > 3.5


# ---------------------------------------------------------------- absorption
def _grid_receivers(nx, nz, step, off=0):
    xs, zs = np.meshgrid(np.arange(0, nx, step), np.arange(0, nz, step))
    pts = np.stack([xs.ravel() + off, zs.ravel() + off], 1).astype(np.int32)
    return pts


def test_pml_energy_decay(orc):
    # interface model of the 200x200 workload, 20-cell pad, 2 s: the interior
    # field must fall below 1e-5 of its peak once the waves have left
    w = synth.workload("interface200")
    nt = 2000
    v = w.true_model()
    rec = _grid_receivers(w.nx, w.nz, 4)[None]
    pb = orc.problem(w.nx, w.nz, w.pml, w.h, w.dt, nt, 2500.0, w.f0, 1e-3, nshots=1,
                     nrec=rec.shape[1])
    d = orc.ac_forward(pb, v, np.array([[100, 100]]), synth.ricker(w.f0, nt, w.dt)[None], rec)[0]
    e = np.sum(d ** 2, axis=1)
    assert e[-1] / e.max() < 1e-5


def test_pml_matches_large_domain(orc):
    # same physical problem on a grid 150 cells larger on every side: no
    # reflection from the far boundary reaches the receivers within 1 s
    w = synth.workload("interface200")
    nt, ext = 1000, 150
    v = w.true_model()
    vbig = np.pad(v, ext, mode="edge")
    src = np.array([[100, 5]])
    rec = np.stack([np.arange(200), np.full(200, 5)], 1)[None]
    wav = synth.ricker(w.f0, nt, w.dt)[None]
    pb = orc.problem(w.nx, w.nz, w.pml, w.h, w.dt, nt, 2500.0, w.f0, 1e-3, nshots=1, nrec=200)
    pbb = orc.problem(w.nx + 2 * ext, w.nz + 2 * ext, w.pml, w.h, w.dt, nt, 2500.0, w.f0, 1e-3,
                      nshots=1, nrec=200)
    d = orc.ac_forward(pb, v, src, wav, rec)
    db = orc.ac_forward(pbb, vbig, src + ext, wav, rec + ext)
    assert np.linalg.norm(d - db) / np.linalg.norm(db) < 5e-3


# ---------------------------------------------------------------- adjoint
def _small_case(orc, nshots=2, nt=200, ckpt=17, seed=0):
    nx, nz, P = 40, 30, 10
    v = synth.layered_anomaly(nx, nz, 1500.0, 3000.0, seed + 1)
    rng = np.random.default_rng(seed)
    src = np.stack([rng.integers(0, nx, nshots), rng.integers(0, nz, nshots)], 1)
    nrec = 7
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))], 2)
    pb = orc.problem(nx, nz, P, 10.0, 1e-3, nt, 3000.0, 15.0, 1e-3, nshots=nshots, nrec=nrec,
                     ckpt_every=ckpt)
    w = rng.standard_normal((nshots, nt))
    r = rng.standard_normal((nshots, nt, nrec))
    return pb, v, src, rec, w, r, rng


def test_adjoint_dot_product_source(orc):
    # <F s, r> = <s, F^T r> for the linear map wavelet -> gathers
    pb, v, src, rec, w, r, _ = _small_case(orc)
    d = orc.ac_forward(pb, v, src, w, rec)
    _, gw, _ = orc.ac_gradient(pb, v, src, w, rec, r, want_wavelet=True)
    lhs, rhs = np.sum(d * r), np.sum(w * gw)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_dot_product_born(orc):
    # <J dv, r> = <dv, J^T r>: Born operator against the model gradient
    pb, v, src, rec, w, r, rng = _small_case(orc, seed=5)
    dv = rng.standard_normal(v.shape)
    dd = orc.ac_born(pb, v, dv, src, w, rec)
    g, _, _ = orc.ac_gradient(pb, v, src, w, rec, r)
    lhs, rhs = np.sum(dd * r), np.sum(dv * g)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_born_is_the_derivative(orc):
    pb, v, src, rec, w, r, rng = _small_case(orc, seed=2)
    dv = rng.standard_normal(v.shape)
    dd = orc.ac_born(pb, v, dv, src, w, rec)
    errs = []
    for eps in (1e-1, 1e-2):
        fd = (orc.ac_forward(pb, v + eps * dv, src, w, rec) -
              orc.ac_forward(pb, v - eps * dv, src, w, rec)) / (2 * eps)
        errs.append(np.linalg.norm(fd - dd) / np.linalg.norm(dd))
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 50  # O(eps^2)


def test_gradient_matches_finite_differences(orc):
    # J = 1/2 ||F(v) - d_obs||^2 on a 32x32 model (+10 pad), 150 steps
    nx = nz = 32
    nt = 150
    rng = np.random.default_rng(11)
    vt = synth.layered_anomaly(nx, nz, 1500.0, 3000.0, 4)
    v0 = synth.smooth(vt, 3.0)
    src = np.array([[8, 2], [24, 2]])
    rec = np.stack([np.stack([np.arange(32), np.full(32, 2)], 1)] * 2)
    pb = orc.problem(nx, nz, 10, 10.0, 1e-3, nt, 3000.0, 20.0, 1e-3, nshots=2, nrec=32,
                     ckpt_every=10)
    w = np.stack([synth.ricker(20.0, nt, 1e-3)] * 2)
    dobs = orc.ac_forward(pb, vt, src, w, rec)

    def J(v):
        return 0.5 * np.sum((orc.ac_forward(pb, v, src, w, rec) - dobs) ** 2)

    d0 = orc.ac_forward(pb, v0, src, w, rec)
    g, _, _ = orc.ac_gradient(pb, v0, src, w, rec, d0 - dobs)
    dv = rng.standard_normal(v0.shape)
    an = np.sum(g * dv)
    eps = 1e-3
    fd = (J(v0 + eps * dv) - J(v0 - eps * dv)) / (2 * eps)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_checkpointing_is_exact(orc):
    pb, v, src, rec, w, r, _ = _small_case(orc, nt=123, ckpt=10)
    g1, gw1, _ = orc.ac_gradient(pb, v, src, w, rec, r, want_wavelet=True)
    pb.ckpt_every = 0
    g0, gw0, _ = orc.ac_gradient(pb, v, src, w, rec, r, want_wavelet=True)
    assert np.array_equal(g0, g1) and np.array_equal(gw0, gw1)


# ---------------------------------------------------------------- invariances
def test_symmetry_homogeneous_centred_source(orc):
    n, nt = 41, 300
    v = np.full((n, n), 2000.0)
    pb = orc.problem(n, n, 10, 10.0, 1e-3, nt, 2000.0, 15.0, nshots=1)
    p = orc.ac_wavefield(pb, v, np.array([[20, 20]]), synth.ricker(15.0, nt, 1e-3)[None])
    scale = np.abs(p).max()
    for q in (p[:, :, ::-1], p[:, ::-1, :], np.swapaxes(p, 1, 2)):
        assert np.abs(q - p).max() <= 1e-12 * scale


def test_time_shift_and_linearity(orc):
    pb, v, src, rec, w, r, rng = _small_case(orc, nshots=1, nt=160)
    w = synth.ricker(15.0, pb.nt, 1e-3)[None]
    m = 23
    ws = np.zeros_like(w)
    ws[:, m:] = w[:, :-m]
    d = orc.ac_forward(pb, v, src, w, rec)
    ds = orc.ac_forward(pb, v, src, ws, rec)
    assert np.array_equal(ds[:, m:], d[:, :-m])
    assert np.all(ds[:, :m] == 0.0)
    w2 = rng.standard_normal(w.shape)
    d2 = orc.ac_forward(pb, v, src, w2, rec)
    dsum = orc.ac_forward(pb, v, src, 3.0 * w + w2, rec)
    assert np.abs(dsum - (3.0 * d + d2)).max() <= 1e-12 * np.abs(dsum).max()


def test_rejects_bad_geometry(orc):
    pb, v, src, rec, w, r, _ = _small_case(orc, nshots=1)
    bad = src.copy()
    bad[0, 0] = 40  # x == nx: outside the model
    with pytest.raises(ValueError):
        orc.ac_forward(pb, v, bad, w[:1], rec[:1])
