"""GPU: degenerate and extreme inputs.

Against the FP64 oracle (same tolerances as the parity tests):
* one and two time steps (receivers on the source cells, so the gathers are
  not zero), acoustic and elastic;
* a grid smaller than one tile (no interior rectangle: every tile is a frame
  tile) and a grid with no absorbing layer (pml = 0);
* no receivers: empty gathers, and a zero gradient with no residual array.

And the largest problem one call takes in this test: 4100 shots on a 1020x520
padded grid, i.e. 2.17e9 cells per wavefield buffer, past 2^31 (every shot
offset is 64-bit), checked bitwise against the same shot run alone; and
nearly the largest single plane (just under 2^29 cells), acoustic and VTI,
against a small grid around the same source.
"""
import dataclasses

import numpy as np
import pytest

import synth
from tests.helpers import f32, random_case, random_el_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEIS_TOL = 1e-5
GRAD_TOL = 1e-4


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


def _close(a, ref, tol):
    """rel L2 within tol; an all-zero reference must be matched exactly."""
    if not np.any(ref):
        return not np.any(a)
    return rel_l2(a, ref) <= tol


def _acoustic_round_trip(case, orc, seed):
    plan = case.plan()
    d = plan.forward(_dev(case.v), _dev(case.wav), save=True)
    resid = f32(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, seed))
    g = plan.backward(_dev(resid))
    gref, _, dref = orc.ac_gradient(case.oracle_problem(orc), case.v, case.src, case.wav,
                                    case.rec, resid, want_gathers=True)
    return _host(d), dref, _host(g)[0], gref


@pytest.mark.parametrize("nt", [1, 2])
def test_acoustic_one_and_two_steps(sw, orc, nt):
    case = random_case(11, nt=nt)
    case.rec = case.rec.copy()
    case.rec[:, 3] = case.src  # a receiver on each source cell
    d, dref, g, gref = _acoustic_round_trip(case, orc, 3)
    print("nt", nt, "max |d|", np.abs(dref).max(), "max |g|", np.abs(gref).max(), flush=True)
    assert np.any(dref)
    assert _close(d, dref, SEIS_TOL)
    assert _close(g, gref, GRAD_TOL)


@pytest.mark.parametrize("nx,nz,pml", [(20, 9, 6), (150, 77, 0)])
def test_acoustic_small_grid_and_no_pml(sw, orc, nx, nz, pml):
    case = random_case(13, nx=nx, nz=nz, pml=pml, nt=120, nshots=2, nrec=5)
    if pml == 6:
        assert case.plan().tiles()["interior"] == 0
    d, dref, g, gref = _acoustic_round_trip(case, orc, 5)
    e_d, e_g = rel_l2(d, dref), rel_l2(g, gref)
    print("grid", nx, nz, "pml", pml, "gathers", e_d, "gradient", e_g, flush=True)
    assert e_d <= SEIS_TOL and e_g <= GRAD_TOL


def test_acoustic_no_receivers(sw):
    case = random_case(12, nt=60)
    case.rec = case.rec[:, :0]
    plan = case.plan()
    d = plan.forward(_dev(case.v), _dev(case.wav), save=True)
    assert tuple(d.shape) == (case.nshots, case.nt, 0)
    g = plan.backward(torch.zeros((case.nshots, case.nt, 0), device="cuda"))
    torch.cuda.synchronize()
    assert torch.isfinite(g).all() and not torch.any(g)


@pytest.mark.parametrize("nt", [1, 2])
def test_elastic_one_and_two_steps(sw, orc, nt):
    case = random_el_case(31, nt=nt, nshots=2, nrec=6)
    case.rec = case.rec.copy()
    case.rec[:, 3] = case.src
    plan = case.plan()
    d = plan.forward(_dev(case.model), _dev(case.wav), save=True)
    resid = f32(np.random.default_rng(nt).standard_normal((case.nshots, case.nt, case.nrec, 2)))
    g = plan.backward(_dev(resid))
    gref, _, dref = orc.el_gradient(case.oracle_problem(orc), case.model, case.src, case.wav,
                                    case.rec, resid, want_gathers=True)
    assert _close(_host(d), dref, SEIS_TOL)
    assert _close(_host(g), gref, GRAD_TOL)


def test_elastic_no_receivers(sw):
    case = random_el_case(32, nt=40, nshots=2, nrec=4)
    case.rec = case.rec[:, :0]
    plan = case.plan()
    d = plan.forward(_dev(case.model), _dev(case.wav), save=True)
    assert d.numel() == 0
    g = plan.backward(torch.zeros((case.nshots, case.nt, 0, 2), device="cuda"))
    torch.cuda.synchronize()
    assert torch.isfinite(g).all() and not torch.any(g)


def test_offsets_past_2_31_elements(sw):
    """4100 shots x 530,400 padded cells = 2.17e9 elements per wavefield
    buffer (8.7 GB; about 145 GB of workspace with checkpoints). The last shot's
    gathers and gradient (residual on that shot only) equal the same shot run
    alone, bit for bit."""
    case = random_case(41, nx=1000, nz=500, pml=10, nt=6, nshots=4100, nrec=3, ckpt=3)
    case.rec = case.rec.copy()
    case.rec[:, 0] = case.src  # in 6 steps the field reaches only ~24 cells
    NX, NZ = case.nx + 2 * case.pml, case.nz + 2 * case.pml
    assert case.nshots * NX * NZ > 2 ** 31
    v, wav = _dev(case.v), _dev(case.wav)
    resid = np.zeros((case.nshots, case.nt, case.nrec), np.float32)
    resid[-1] = synth.bandlimited_noise((1, case.nt, case.nrec), 15.0, case.dt, 9)[0]
    big = case.plan()
    d = big.forward(v, wav, save=True)[-1].clone()
    g = big.backward(_dev(resid)).clone()
    big.release_workspace()
    del big
    torch.cuda.empty_cache()
    one = dataclasses.replace(case, src=case.src[-1:], rec=case.rec[-1:], wav=case.wav[-1:])
    p1 = one.plan()
    d1 = p1.forward(v, _dev(one.wav), save=True)[0]
    g1 = p1.backward(_dev(resid[-1:]))
    torch.cuda.synchronize()
    print("last-shot gathers max", float(d.abs().max()), "gradient max", float(g.abs().max()),
          flush=True)
    assert torch.any(d != 0) and torch.any(g != 0)
    assert torch.equal(d, d1)
    assert torch.equal(g, g1)


@pytest.mark.parametrize("physics", ["acoustic", "vti"])
def test_largest_plane_matches_a_small_grid(sw, physics):
    """One shot on nearly the largest plane a plan takes (23170 x 23170 padded
    cells, just under 2^29). The source sits 40 cells from the far corner, so
    the cells it reaches in 6 steps lie at the end of every plane: VTI's
    float64 planes are addressed there at byte offsets past 2^31, close to
    2^32. With a constant model, the same 6 steps on a 100 x 100 grid around
    the same source see the same neighbourhood, so the gathers and the
    gradient around the source must agree: bit for bit for acoustic; within
    1e-6 for VTI, whose interior and C-PML tile kernels round differently."""
    vti = physics == "vti"
    off = np.array([[0, 0], [7, -3], [-9, 5], [2, 9]])
    wav = np.array([[1.0, -0.5, 0.25, 0.75, -0.375, 0.125]], np.float32)
    resid = _dev(np.random.default_rng(3).standard_normal((1, 6, 4)))

    def run(n, xs):
        print(physics, "grid", n, "source", xs, flush=True)
        plan = sw.Plan(nx=n, nz=n, h=10.0, dt=1e-3, nt=6, pml=10,
                       src_xz=np.array([[xs, xs]], np.int32),
                       rec_xz=(np.array([[xs, xs]]) + off)[None].astype(np.int32),
                       pml_vmax=2400.0, pml_f0=15.0, ckpt_every=3,
                       physics=sw.VTI if vti else sw.ACOUSTIC)
        vals = (2000.0, 2100.0, 0.1) if vti else (2000.0,)
        m = torch.empty((len(vals), n, n), device="cuda")
        for i, val in enumerate(vals):
            m[i].fill_(val)
        d = plan.forward(m, _dev(wav), save=True).clone()
        g = plan.backward(resid)
        win = g[:, xs - 30:xs + 31, xs - 30:xs + 31].clone()
        del g, m
        plan.release_workspace()
        del plan
        torch.cuda.empty_cache()
        return d, win

    n_big = 23150
    assert (n_big + 20) ** 2 < 2 ** 29
    d_big, g_big = run(n_big, n_big - 40)
    d_small, g_small = run(100, 50)
    torch.cuda.synchronize()
    assert torch.any(d_small != 0) and torch.any(g_small != 0)
    print("largest plane", physics, "gathers max", float(d_small.abs().max()), flush=True)
    if vti:
        assert rel_l2(_host(d_big), _host(d_small)) <= 1e-6
        assert rel_l2(_host(g_big), _host(g_small)) <= 1e-6
    else:
        assert torch.equal(d_big, d_small)
        assert torch.equal(g_big, g_small)
