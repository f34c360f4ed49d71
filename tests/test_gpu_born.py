"""GPU: Born (tangent-linear) modelling, Eq. 16, against the FP64 oracle.

* parity: the Born gathers match the oracle's tangent-linear recurrence within
  the seismogram tolerance (1e-5 relative L2) on a ragged grid;
* transpose: the FP32 dot-product test <Born dv, r> = <dv, backward(r)> (the
  adjoint of Born modelling is the model gradient), on a small case and at the
  full 1000x300 / 64-shot / 3000-step size;
* the result does not depend on the tiling (bitwise); a zero perturbation
  gives zero gathers and the map is linear;
* least-squares RTM (CGLS over Born and its transpose) lowers the data
  residual at every iteration.
"""
import numpy as np
import pytest

import synth
from tests.helpers import case_from_workload, f32, random_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEIS_TOL = 1e-5
# normalised dot-test bound |<J dv, r> - <dv, J^T r>| / (|J dv| |r|): both sides
# are FP32 results within ~1e-6 of the exact operators
DOT_TOL = 1e-5


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.fixture(scope="module")
def sw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_14189_amd as sw
    sw.lib()
    return sw


def _dv(nz, nx, seed):
    """Model perturbation (m/s): white noise plus a smooth blob."""
    rng = np.random.default_rng(seed)
    z, x = np.mgrid[0:nz, 0:nx]
    blob = 60.0 * np.exp(-((x - 0.6 * nx) ** 2 + (z - 0.4 * nz) ** 2) / (2 * (0.1 * nx) ** 2))
    return f32(20.0 * rng.standard_normal((nz, nx)) + blob)


def _dot_error(plan, v, w, dv, r):
    jd = plan.born(v, dv, w)
    plan.forward(v, w, save=True)
    jt = plan.backward(r)
    torch.cuda.synchronize()
    lhs = float((jd.double() * r.double()).sum())
    rhs = float((dv.double().reshape(-1) * jt.double().reshape(-1)).sum())
    scale = float(jd.double().norm()) * float(r.double().norm())
    return abs(lhs - rhs) / scale, lhs, rhs


def test_born_parity_ragged(sw, orc):
    case = random_case(5, nt=200)
    dv = _dv(case.nz, case.nx, 3)
    dd = case.plan().born(_dev(case.v), _dev(dv), _dev(case.wav))
    ref = orc.ac_born(case.oracle_problem(orc), case.v, dv, case.src, case.wav, case.rec)
    err = rel_l2(_host(dd), ref)
    print("Born ragged rel L2", err, flush=True)
    assert np.linalg.norm(ref) > 0
    assert err <= SEIS_TOL


def test_born_transpose_is_the_gradient(sw):
    case = random_case(6, nt=160)
    r = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 9))
    e, lhs, rhs = _dot_error(case.plan(), _dev(case.v), _dev(case.wav),
                             _dev(_dv(case.nz, case.nx, 4)), r)
    print("Born dot test", lhs, rhs, e, flush=True)
    assert e <= DOT_TOL


@pytest.mark.parametrize("rz,prz", [(1, 1), (4, 4), (8, 2)])
def test_born_tilings_bitwise(sw, rz, prz):
    case = random_case(7, nt=120)
    v, w, dv = _dev(case.v), _dev(case.wav), _dev(_dv(case.nz, case.nx, 5))
    ref = case.plan().born(v, dv, w).clone()
    p = case.plan()
    p.set_tuning(rz=rz, pml_rz=prz)
    assert torch.equal(p.born(v, dv, w), ref)


def test_born_two_step_background_bitwise(sw):
    """Where the plan has deep tiles, the background field takes two-step
    passes (tblock 2) and the perturbation single steps; the Born gathers
    equal those with single background steps (tblock 1) bit for bit."""
    w = synth.batched_workloads()[1]  # 400 x 200, receivers and sources at depth 5
    case = case_from_workload(w, shots=[0, 7], nt=121)
    v, wv = _dev(case.v), _dev(case.wav)
    dv = _dev(_dv(case.nz, case.nx, 9))
    p2 = case.plan()
    assert p2.tiles()["deep"] > 0
    d2 = p2.born(v, dv, wv).clone()
    p1 = case.plan()
    p1.set_tuning(tblock=1)
    assert torch.equal(p1.born(v, dv, wv), d2)
    assert torch.any(d2 != 0)


def test_born_linear_and_zero(sw):
    """A zero perturbation gives exactly zero gathers; doubling dv doubles them
    (every operation of the perturbation recurrence scales exactly by 2 except
    where a value underflows the FP32 range, far below the tolerance)."""
    case = random_case(8, nt=100)
    v, w = _dev(case.v), _dev(case.wav)
    dv = _dev(_dv(case.nz, case.nx, 6))
    plan = case.plan()
    assert not torch.any(plan.born(v, torch.zeros_like(dv), w))
    d1 = plan.born(v, dv, w).clone()
    d2 = plan.born(v, 2.0 * dv, w)
    err = rel_l2(_host(d2), 2.0 * _host(d1))
    print("Born doubling rel L2", err, flush=True)
    assert err <= 1e-12


def test_born_full_size_dot_test(sw):
    """The 1000x300 layered workload at full size (64 shots, 3000 steps, the
    plan's default tiling): Born and the gradient are each other's transpose."""
    wl = synth.workload("layered1000x300")
    case = case_from_workload(wl)
    v = _dev(synth.smooth(case.v, 20.0))
    r = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), wl.f0, wl.dt, 11))
    dv = _dev(f32(case.v) - f32(synth.smooth(case.v, 20.0)))
    plan = case.plan()
    e, lhs, rhs = _dot_error(plan, v, _dev(case.wav), dv, r)
    plan.release_workspace()
    print("Born full-size dot test", lhs, rhs, e, flush=True)
    assert e <= DOT_TOL


def test_lsrtm_cgls_residual_falls(sw):
    """Least-squares RTM: CGLS over Born modelling and its transpose (the
    adjoint gradient), on data that Born modelling made from a known
    perturbation. The data residual falls at every iteration (CGLS minimises
    it over a growing Krylov space; slack for FP32 rounding), ends well below
    the data norm, and the recovered perturbation correlates with the true one
    (positive cosine)."""
    from paper_2604_14189_amd import fwi
    case = random_case(9, nt=160)
    v, w = _dev(case.v), _dev(case.wav)
    dv = _dev(_dv(case.nz, case.nx, 7))
    plan = case.plan()
    d = plan.born(v, dv, w).clone()
    ls = fwi.LSRTM(plan, v, w, d)
    for _ in range(6):
        ls.step()
    h = ls.history
    x = ls.perturbation.double()
    cos = float((x * dv.double()).sum() / (x.norm() * dv.double().norm()))
    print("LSRTM residual history", [f"{a / h[0]:.4f}" for a in h], "cosine", cos, flush=True)
    assert all(b <= a * (1 + 1e-4) for a, b in zip(h, h[1:]))
    assert h[-1] < 0.5 * h[0]
    assert cos > 0.0
