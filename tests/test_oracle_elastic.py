"""Pins for the FP64 elastic oracle (Sec. 3.5, Eq. 12), CPU only.

Transpose identities (dot-product tests) with and without the free surface,
finite differences of the Born operator and of the misfit, the closed-form
P-wave radiated by an explosive source in a homogeneous full space, the fluid
limit, the Rayleigh-wave speed along the free surface, and absorption.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth


def _small(orc, fs, nshots=2, nt=150, seed=0, ck=13):
    nx, nz, P = 36, 28, 8
    m = synth.elastic_model(nx, nz, seed + 3)
    rng = np.random.default_rng(seed)
    src = np.stack([rng.integers(2, nx - 2, nshots), rng.integers(1, nz - 2, nshots)], 1)
    nrec = 9
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))], 2)
    pb = orc.problem(nx, nz, P, 5.0, 0.4e-3, nt, 4500.0, 20.0, 1e-3, nshots=nshots, nrec=nrec,
                     free_surface=fs, ckpt_every=ck)
    w = rng.standard_normal((nshots, nt))
    r = rng.standard_normal((nshots, nt, nrec, 2))
    return pb, m, src, rec, w, r, rng


@pytest.mark.parametrize("fs", [0, 1])
def test_dot_product_source(orc, fs):
    pb, m, src, rec, w, r, _ = _small(orc, fs)
    d = orc.el_forward(pb, m, src, w, rec)
    _, gw, ga = orc.el_gradient(pb, m, src, w, rec, r, want_wavelet=True, want_gathers=True)
    assert np.array_equal(d, ga)
    lhs, rhs = np.sum(d * r), np.sum(w * gw)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("fs", [0, 1])
def test_dot_product_born(orc, fs):
    pb, m, src, rec, w, r, rng = _small(orc, fs, seed=4)
    dm = rng.standard_normal(m.shape) * np.array([100.0, 60.0, 50.0])[:, None, None]
    dd = orc.el_born(pb, m, dm, src, w, rec)
    g, _, _ = orc.el_gradient(pb, m, src, w, rec, r)
    lhs, rhs = np.sum(dd * r), np.sum(dm * g)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("fs", [0, 1])
def test_born_is_the_derivative(orc, fs):
    pb, m, src, rec, w, r, rng = _small(orc, fs, seed=7)
    dm = rng.standard_normal(m.shape) * np.array([100.0, 60.0, 50.0])[:, None, None]
    dd = orc.el_born(pb, m, dm, src, w, rec)
    errs = []
    for eps in (1e-2, 1e-3):
        fd = (orc.el_forward(pb, m + eps * dm, src, w, rec) -
              orc.el_forward(pb, m - eps * dm, src, w, rec)) / (2 * eps)
        errs.append(np.linalg.norm(fd - dd) / np.linalg.norm(dd))
    assert errs[1] < 1e-5
    assert errs[0] / errs[1] > 50


def test_gradient_matches_finite_differences(orc):
    nx, nz, nt = 32, 32, 160
    mt = synth.elastic_model(nx, nz, 5)
    m0 = np.stack([synth.smooth(c, 3.0) for c in mt])
    src = np.array([[8, 3], [24, 3]])
    rec = np.stack([np.stack([np.arange(32), np.full(32, 2)], 1)] * 2)
    pb = orc.problem(nx, nz, 8, 5.0, 0.4e-3, nt, 4500.0, 25.0, 1e-3, nshots=2, nrec=32,
                     free_surface=1, ckpt_every=16)
    w = np.stack([synth.ricker(25.0, nt, 0.4e-3)] * 2)
    dobs = orc.el_forward(pb, mt, src, w, rec)

    def J(m):
        return 0.5 * np.sum((orc.el_forward(pb, m, src, w, rec) - dobs) ** 2)

    d0 = orc.el_forward(pb, m0, src, w, rec)
    g, _, _ = orc.el_gradient(pb, m0, src, w, rec, d0 - dobs)
    rng = np.random.default_rng(3)
    for c, scale in enumerate((50.0, 30.0, 20.0)):
        dm = np.zeros_like(m0)
        dm[c] = rng.standard_normal((nz, nx)) * scale
        an = np.sum(g * dm)
        eps = 1e-3
        fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
        assert abs(fd - an) <= 1e-6 * abs(an), (c, fd, an)


def test_checkpointing_is_exact(orc):
    pb, m, src, rec, w, r, _ = _small(orc, 1, nt=97, ck=10)
    g1, gw1, _ = orc.el_gradient(pb, m, src, w, rec, r, want_wavelet=True)
    pb.ckpt_every = 0
    g0, gw0, _ = orc.el_gradient(pb, m, src, w, rec, r, want_wavelet=True)
    assert np.array_equal(g0, g1) and np.array_equal(gw0, gw1)


# ---------------------------------------------------------------- closed form
def _dG_dr(r, t, v, f0):
    """d/dr of (G * s)(r, t) for the 2-D Green's function and a Ricker s:
    -1/(2 pi v^3) int_0^{acosh(v t / r)} cosh(u) s'(t - (r/v) cosh u) du."""
    delay = 1.5 / f0
    if v * t <= r:
        return 0.0
    umax = math.acosh(v * t / r)

    def sp(tt):
        a = math.pi * f0 * (tt - delay)
        return math.pi * f0 * (-6 * a + 4 * a ** 3) * math.exp(-a * a)

    val, _ = quad(lambda u: math.cosh(u) * sp(t - r / v * math.cosh(u)), 0, umax, limit=400)
    return -val / (2 * math.pi * v ** 3)


def _explosive_error(orc, fac, vs=1732.0):
    # An explosive source s(t) on both normal stresses radiates only P: the
    # particle velocity is grad(G * s) / rho with G the 2-D Green's function at
    # vp, whatever vs (vs = 0 is the fluid).
    nx = nz = 160
    P, h, f0 = 20, 5.0, 15.0
    dt = 0.5e-3 / fac
    nt = int(round(0.3 / dt))
    vp, rho = 3000.0, 2000.0
    m = np.stack([np.full((nz, nx), vp), np.full((nz, nx), vs), np.full((nz, nx), rho)])
    pb = orc.problem(nx, nz, P, h, dt, nt, vp, f0, 1e-3, nshots=1, nrec=1)
    d = orc.el_forward(pb, m, np.array([[80, 80]]), synth.ricker(f0, nt, dt)[None],
                       np.array([[[120, 110]]]))[0, :, 0, :]
    t = np.arange(nt) * dt  # gathers[n] ~ v(t_n): s_n enters the stress update centred at t_{n+1/2}
    dxv, dzv = 40.5 * h, 30.0 * h  # vx node (i+1/2, j) relative to the source
    dxz, dzz = 40.0 * h, 30.5 * h  # vz node (i, j+1/2)
    rx, rz = math.hypot(dxv, dzv), math.hypot(dxz, dzz)
    ax = np.array([_dG_dr(rx, tt, vp, f0) * dxv / rx / rho for tt in t])
    az = np.array([_dG_dr(rz, tt, vp, f0) * dzz / rz / rho for tt in t])
    return math.sqrt((np.sum((d[:, 0] - ax) ** 2) + np.sum((d[:, 1] - az) ** 2)) /
                     (np.sum(ax ** 2) + np.sum(az ** 2)))


def test_explosive_source_closed_form(orc):
    e1 = _explosive_error(orc, 1)
    e2 = _explosive_error(orc, 2)
    assert e1 < 5e-3
    assert e1 / e2 > 3.5


def test_fluid_limit(orc):
    # vs = 0: txx and tzz receive identical increments and txz stays zero
    nx, nz, nt = 40, 36, 120
    m = np.stack([synth.layered_anomaly(nx, nz, 1500.0, 3000.0, 2), np.zeros((nz, nx)),
                  np.full((nz, nx), 1800.0)])
    pb = orc.problem(nx, nz, 8, 5.0, 0.5e-3, nt, 3000.0, 20.0, nshots=1)
    s = orc.el_wavefield(pb, m, np.array([[17, 15]]), synth.ricker(20.0, nt, 0.5e-3)[None])
    assert np.array_equal(s[:, 2], s[:, 3])
    assert np.all(s[:, 4] == 0.0)
    assert np.abs(s[:, 2]).max() > 0


def test_rayleigh_wave_speed(orc):
    # Poisson solid (vp/vs = sqrt 3): Rayleigh speed 0.9194 vs along the free surface
    nx, nz, P, h, dt, f0, nt = 300, 100, 30, 5.0, 0.5e-3, 15.0, 1500
    vp, vs, rho = 3000.0, 3000.0 / math.sqrt(3.0), 2000.0
    m = np.stack([np.full((nz, nx), vp), np.full((nz, nx), vs), np.full((nz, nx), rho)])
    x1, x2 = 120, 240
    pb = orc.problem(nx, nz, P, h, dt, nt, vp, f0, 1e-3, nshots=1, nrec=2, free_surface=1)
    d = orc.el_forward(pb, m, np.array([[40, 2]]), synth.ricker(f0, nt, dt)[None],
                       np.array([[[x1, 0], [x2, 0]]]))[0]
    a, b = d[:, 0, 1], d[:, 1, 1]
    c = np.correlate(b, a, mode="full")
    k = int(np.argmax(c))
    y0, y1, y2 = c[k - 1], c[k], c[k + 1]
    lag = (k - (nt - 1) + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt
    ratio = (x2 - x1) * h / lag / vs
    assert abs(ratio / 0.9194 - 1.0) < 0.02, ratio


def test_pml_energy_decay(orc):
    nx = nz = 100
    nt = 1600
    m = np.stack([np.full((nz, nx), 3000.0), np.full((nz, nx), 1700.0), np.full((nz, nx), 2200.0)])
    xs, zs = np.meshgrid(np.arange(0, nx, 4), np.arange(0, nz, 4))
    rec = np.stack([xs.ravel(), zs.ravel()], 1)[None]
    pb = orc.problem(nx, nz, 20, 5.0, 0.5e-3, nt, 3000.0, 20.0, 1e-3, nshots=1,
                     nrec=rec.shape[1])
    d = orc.el_forward(pb, m, np.array([[50, 50]]), synth.ricker(20.0, nt, 0.5e-3)[None], rec)[0]
    e = np.sum(d ** 2, axis=(1, 2))
    assert e[-1] / e.max() < 1e-4


def test_half_node_profiles_by_symmetry(orc):
    # Homogeneous square grid, equal pads on all sides, source on the centre
    # node. (i) Exchanging x and z maps vx onto vz, txx onto tzz and txz onto
    # itself; every operation has its transposed twin, so this holds exactly
    # and fails if any of the eight memory variables takes the profile of the
    # wrong axis. (ii) The mirror x -> -x maps txx onto itself and vx (half
    # nodes i + 1/2) onto -vx at (NX - 2 - i) + 1/2. It holds while each
    # memory variable takes its profile at its derivative's output node
    # (integer or half), up to the one vx node past the last integer node,
    # whose mirror lies outside the grid; taking the integer-node profile at a
    # half node instead (for the velocity or the stress terms) breaks it by
    # 100-1000 times more than that edge effect on this narrow pad.
    nx = nz = 41
    P, nt, dt = 6, 500, 0.5e-3
    m = np.stack([np.full((nz, nx), 3000.0), np.full((nz, nx), 1700.0),
                  np.full((nz, nx), 2200.0)])
    pb = orc.problem(nx, nz, P, 5.0, dt, nt, 3000.0, 20.0, 1e-3, nshots=1)
    s = orc.el_wavefield(pb, m, np.array([[20, 20]]), synth.ricker(25.0, nt, dt)[None])
    vx, vz, txx, tzz, txz = (s[:, k] for k in range(5))
    assert np.array_equal(vx, np.transpose(vz, (0, 2, 1)))
    assert np.array_equal(txx, np.transpose(tzz, (0, 2, 1)))
    assert np.array_equal(txz, np.transpose(txz, (0, 2, 1)))
    NX = nx + 2 * P
    mod = slice(P, P + nx)
    e_t = np.abs(txx - txx[:, :, ::-1])[:, mod, mod].max() / np.abs(txx[:, mod, mod]).max()
    e_v = (np.abs(vx[:, :, :NX - 1] + vx[:, :, NX - 2::-1])[:, mod, P:P + nx - 1].max() /
           np.abs(vx[:, mod, mod]).max())
    assert e_t < 2e-5 and e_v < 1e-4, (e_t, e_v)
