"""GPU parity: acoustic forward / adjoint (HIP, FP32) against the FP64 oracle.

Tolerances: seismograms <= 1e-5 and gradients <= 1e-4 relative L2. The
kernels run in FP32 with FP32 stencil sums; the oracle runs the same recurrence
in FP64, so the difference is FP32 rounding accumulated over the time loop.
"""
import os

import numpy as np
import pytest

import synth
from tests.helpers import case_from_workload, f32, random_case, rel_l2

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


def _gpu_forward(sw, case, save=False, tuning=None, plan=None):
    plan = plan or case.plan()
    if tuning:
        plan.set_tuning(**tuning)
    d = plan.forward(_dev(case.v), _dev(case.wav), save=save)
    return plan, d


def test_forward_parity_ragged(sw, orc):
    case = random_case(1)
    _, d = _gpu_forward(sw, case)
    ref = orc.ac_forward(case.oracle_problem(orc), case.v, case.src, case.wav, case.rec)
    err = rel_l2(_host(d), ref)
    print("forward ragged rel L2", err, flush=True)
    assert err <= SEIS_TOL


# (interior rows per thread, C-PML rows per thread): the tile height moves the
# boundary between interior and frame tiles and the frame kernel's split
TILINGS = [(1, 1), (2, 1), (2, 2), (4, 1), (4, 4), (8, 1), (8, 2), (8, 8)]


@pytest.mark.parametrize("rz,prz", TILINGS)
def test_forward_tilings_bitwise(sw, rz, prz):
    case = random_case(2, nx=200, nz=140, pml=12, nt=120)
    _, d0 = _gpu_forward(sw, case, tuning=dict(rz=8, pml_rz=4))
    _, d1 = _gpu_forward(sw, case, tuning=dict(rz=rz, pml_rz=prz))
    assert torch.equal(d0, d1)


def test_forward_parity_interface200(sw, orc):
    # 200x200 model, 20-cell pad, 1000 steps, source (100,5), 200 receivers at depth 5
    case = case_from_workload(synth.workload("interface200"))
    _, d = _gpu_forward(sw, case)
    ref = orc.ac_forward(case.oracle_problem(orc), case.v, case.src, case.wav, case.rec)
    err = rel_l2(_host(d), ref)
    print("interface200 rel L2", err, flush=True)
    assert err <= SEIS_TOL


def test_gradient_parity_ragged(sw, orc):
    case = random_case(3, nt=260, ckpt=17)
    plan, d = _gpu_forward(sw, case, save=True)
    resid = f32(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 7))
    g = plan.backward(_dev(resid))
    gref, _, dref = orc.ac_gradient(case.oracle_problem(orc), case.v, case.src, case.wav,
                                    case.rec, resid, want_gathers=True)
    e_d = rel_l2(_host(d), dref)
    e_g = rel_l2(_host(g)[0], gref)
    print("ragged gathers", e_d, "gradient", e_g, flush=True)
    assert e_d <= SEIS_TOL
    assert e_g <= GRAD_TOL


def test_gradient_parity_interface200(sw, orc):
    w = synth.workload("interface200")
    case = case_from_workload(w)
    plan, d = _gpu_forward(sw, case, save=True)
    # the residual is the oracle's (its own forward minus data from a smoothed
    # model) and feeds both adjoints
    pb = case.oracle_problem(orc)
    dobs = orc.ac_forward(pb, f32(synth.smooth(case.v, 5.0)), case.src, case.wav, case.rec)
    dref = orc.ac_forward(pb, case.v, case.src, case.wav, case.rec)
    resid = f32(dref - dobs)
    g = plan.backward(_dev(resid))
    gref, _, _ = orc.ac_gradient(pb, case.v, case.src, case.wav, case.rec, resid)
    e_g = rel_l2(_host(g)[0], gref)
    print("interface200 gradient", e_g, flush=True)
    assert e_g <= GRAD_TOL


def test_checkpoint_interval_invariance(sw):
    # Recomputation reproduces the forward bit for bit, so the adjoint sees the
    # same B^n for every checkpoint interval; only the grouping of the gradient
    # sum changes (FP32 partial per segment, folded into FP64 at segment ends).
    case = random_case(4, nt=150, ckpt=150)
    resid = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 2))
    grads = []
    for k in (150, 13, 1):
        case.ckpt = k
        plan, _ = _gpu_forward(sw, case, save=True)
        grads.append(_host(plan.backward(resid)))
    assert rel_l2(grads[1], grads[0]) <= 1e-6
    assert rel_l2(grads[2], grads[0]) <= 1e-6


@pytest.mark.parametrize("rz,prz", [(1, 1), (4, 2), (8, 8)])
def test_gradient_tilings_bitwise(sw, rz, prz):
    case = random_case(5, nx=170, nz=100, nt=90, ckpt=20)
    resid = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 3))
    out = []
    for t, tp in ((8, 2), (rz, prz)):
        plan, _ = _gpu_forward(sw, case, save=True, tuning=dict(rz=t, pml_rz=tp))
        out.append(plan.backward(resid).clone())
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("rz,ckpt", [(4, 50), (4, 17), (8, 17)])
def test_two_step_passes_bitwise(sw, rz, ckpt):
    """Deep interior tiles advanced two steps per pass give the same bits as
    single steps: gathers and gradient, with checkpoint intervals that leave
    single-step remainders (odd segment lengths)."""
    w = synth.workload("interface200")
    case = case_from_workload(w, nt=230)
    case.ckpt = ckpt
    resid = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 10.0, case.dt, 5))
    out = []
    for tb in (1, 2):
        plan, d = _gpu_forward(sw, case, save=True, tuning=dict(rz=rz, pml_rz=4, tblock=tb))
        if tb == 2:
            assert plan.tiles()["deep"] > 0
        out.append((d.clone(), plan.backward(resid).clone()))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("keep,tblock", [(1, 2), (3, 2), (99, 2), (99, 1)])
def test_stored_segments_bitwise(sw, keep, tblock):
    """Segments whose B'^n the saving forward stores (keep_b) are reversed
    without recomputation: gathers and gradient keep the bits of the full
    recomputation. 230 steps in segments of 17 (a ragged last one); 99 stores
    all of them. Segments recomputed after stored ones (keep 1, 3) write
    their B'^n into the first stored segment's slots, which the backward has
    consumed by then; the workspace changes by the stored segments less
    their checkpoints and the recomputation's own buffer."""
    w = synth.workload("interface200")
    case = case_from_workload(w, nt=230)
    case.ckpt = 17
    resid = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 10.0, case.dt, 6))
    plan, d0 = _gpu_forward(sw, case, save=True, tuning=dict(rz=4, pml_rz=4, tblock=tblock))
    d0, g0 = d0.clone(), plan.backward(resid).clone()
    base = plan.workspace_bytes(True)
    plan.release_workspace()
    kp, d1 = _gpu_forward(sw, case, save=True,
                          tuning=dict(rz=4, pml_rz=4, tblock=tblock, keep_b=keep))
    nseg = -(-case.nt // case.ckpt)
    n = min(keep, nseg)
    NX, NZ = kp.padded()
    ns, P2 = case.nshots, 2 * case.pml
    seg = case.ckpt * ns * NX * NZ * 4
    # a dropped checkpoint: p^n, p^(n-1) and the x- and z-strip memory variables
    slot = (2 * ns * NX * NZ + 2 * ns * NZ * P2 + 2 * ns * P2 * NX) * 4
    want = n * (seg - slot) - seg  # the recomputation's own buffer goes
    assert abs(kp.workspace_bytes(True) - base - want) < 4096
    assert torch.equal(d1, d0)
    assert torch.equal(kp.backward(resid), g0)


def test_stored_segments_graph_replays(sw):
    case = random_case(32, nt=140, ckpt=25)
    r = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 3))
    eager = case.plan()
    d0 = eager.forward(_dev(case.v), _dev(case.wav), save=True).clone()
    g0 = eager.backward(r).clone()
    gp = case.plan()
    gp.set_tuning(rz=8, use_graph=1, keep_b=3)
    # the workspace, stored segments included, allocated ahead of the first
    # forward and used as it is by every call
    assert gp.reserve_workspace(True) == gp.workspace_bytes(True)
    block = gp._work.data_ptr()
    v, w = _dev(case.v), _dev(case.wav)
    out, grad = torch.empty_like(d0), torch.empty_like(g0)
    for rep in range(3):
        gp.forward(v, w, save=True, out=out)
        gp.backward(r, out=grad)
        torch.cuda.synchronize()
        assert torch.equal(out, d0), rep
        assert torch.equal(grad, g0), rep
        assert gp._work.data_ptr() == block
        assert torch.isfinite(torch.randn(4096, device="cuda").sum())


def test_stored_segments_after_born(sw):
    """Born modelling on a plan with stored segments (Born lays out its state
    without them) and then a saving forward and backward on the same
    workspace: Born gathers and gradient equal those of a plan without stored
    segments, bit for bit."""
    case = random_case(33, nt=120, ckpt=20)
    v, w = _dev(case.v), _dev(case.wav)
    dv = _dev(np.random.default_rng(3).standard_normal((case.nz, case.nx)) * 10.0)
    r = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 7))
    ref = case.plan()
    dd0 = ref.born(v, dv, w).clone()
    ref.forward(v, w, save=True)
    g0 = ref.backward(r).clone()
    p = case.plan()
    p.set_tuning(rz=8, keep_b=4)
    p.reserve_workspace(True)
    assert torch.equal(p.born(v, dv, w), dd0)
    p.forward(v, w, save=True)
    assert torch.equal(p.backward(r), g0)
    assert torch.any(g0 != 0)


def test_repeatable(sw):
    case = random_case(6, nt=100, ckpt=30)
    resid = _dev(synth.bandlimited_noise((case.nshots, case.nt, case.nrec), 15.0, case.dt, 4))
    plan, d1 = _gpu_forward(sw, case, save=True)
    g1 = plan.backward(resid).clone()
    d1 = d1.clone()
    plan2, d2 = _gpu_forward(sw, case, save=True)
    g2 = plan2.backward(resid)
    assert torch.equal(d1, d2) and torch.equal(g1, g2)


def test_batched_equals_single_shot(sw):
    # batch modelling changes launch counts only, never results (Sec. 2.2)
    case = random_case(7, nt=120, nshots=4)
    _, dall = _gpu_forward(sw, case)
    for s in range(case.nshots):
        one = random_case(7, nt=120, nshots=4)
        one.src, one.rec, one.wav = one.src[s:s + 1], one.rec[s:s + 1], one.wav[s:s + 1]
        _, d1 = _gpu_forward(sw, one)
        assert torch.equal(d1[0], dall[s])


def test_misfit_kernel(sw):
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3, 777, 13)).astype(np.float32)
    b = rng.standard_normal((3, 777, 13)).astype(np.float32)
    r, J = sw.l2_misfit(_dev(a), _dev(b))
    np.testing.assert_array_equal(_host(r), (a - b).astype(np.float64))
    # J is the float64 sum of squares of the float32 residual the kernel returns
    ref = 0.5 * np.sum((a - b).astype(np.float64) ** 2)
    assert abs(J.item() - ref) <= 1e-12 * ref


def test_autograd_function(sw, orc):
    case = random_case(8, nt=150, ckpt=40)
    plan = case.plan()
    v = _dev(case.v).requires_grad_(True)
    d = sw.WaveFn.apply(v, _dev(case.wav), plan)
    target = _dev(np.zeros(d.shape))
    loss = 0.5 * ((d - target) ** 2).sum()
    loss.backward()
    gref, _, _ = orc.ac_gradient(case.oracle_problem(orc), case.v, case.src, case.wav, case.rec,
                                 f32(_host(d.detach())))
    assert rel_l2(_host(v.grad), gref) <= GRAD_TOL


def test_errors_are_reported(sw):
    case = random_case(9, nt=50)
    plan = case.plan()
    with pytest.raises(RuntimeError):
        plan.backward(_dev(np.zeros((case.nshots, case.nt, case.nrec))))
    bad = random_case(9, nt=50)
    bad.src = bad.src.copy()
    bad.src[0, 0] = bad.nx  # outside the model
    with pytest.raises(sw.SweepError):
        bad.plan()


# ------------------------------------------------------------- full size, sampled
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "layered1000x300_shot37.npz")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated")
@pytest.mark.parametrize("stored", [False, True])
def test_full_size_layered_sampled_shot(sw, stored):
    """All 64 shots of the 1000x300 / 3000-step workload in one launch sequence;
    the oracle values for shot 37 (sampled traces and gradient cells, written by
    tests/golden/make_golden.py) must match. `stored`: the benchmark's
    configuration, B'^n of as many of the last checkpoint segments as the free
    HBM holds (sized by the benchmark's own rule), the others recomputed;
    otherwise every segment is recomputed."""
    gold = np.load(GOLDEN)
    w = synth.workload("layered1000x300")
    case = case_from_workload(w)
    plan = case.plan()
    plan.set_tuning(rz=8, pml_rz=4, tblock=2)
    if stored:
        import bench
        keep = bench.fit_keep_b(torch, plan, w.nt, w.ckpt_every)
        print("stored segments", keep, "of", -(-w.nt // w.ckpt_every), flush=True)
        assert keep >= 1
    plan, d = _gpu_forward(sw, case, save=True, plan=plan)
    s = int(gold["shot"])
    traces = gold["trace_idx"]
    dg = d[s][:, torch.as_tensor(traces, device="cuda")]
    e_d = rel_l2(_host(dg), gold["traces"])
    resid = np.zeros((case.nshots, case.nt, case.nrec), np.float32)
    resid[s] = synth.bandlimited_noise((1, case.nt, case.nrec), w.f0, w.dt, 37)[0]
    g = _host(plan.backward(_dev(resid)))[0]
    cells = gold["grad_cells"]
    e_g = rel_l2(g.ravel()[cells], gold["grad"])
    e_gn = abs(np.linalg.norm(g) - float(gold["grad_norm"])) / float(gold["grad_norm"])
    print("full-size shot", s, "traces", e_d, "gradient", e_g, "norm", e_gn, flush=True)
    plan.release_workspace()
    assert e_d <= SEIS_TOL
    assert e_g <= GRAD_TOL and e_gn <= GRAD_TOL
