"""GPU parity: pseudo-acoustic VTI (Eq. 5) forward and adjoint (HIP, FP32)
against the FP64 oracle. Gathers <= 1e-5 and each of the three gradients
(vv, v, eta) <= 1e-4 relative L2, on a ragged grid with sources next to the
pad, coincident receivers and a ragged last checkpoint segment; eta = 0 with
v = vv gives the acoustic plan's results; edge cases (one step, a grid smaller
than one tile, no pad, no receivers); stored segments bitwise against
recomputation; and the full 1000x300 / 3000-step workload, one shot against
stored oracle values, with and without stored segments."""
import os

import numpy as np
import pytest

import synth
from tests.helpers import f32, random_case, rel_l2

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


def _vti_case(seed, nx=150, nz=77, pml=10, nt=240, nshots=3, nrec=41, ckpt=17, eta_max=0.2):
    """Ragged acoustic case with a VTI model: vv from the layered generator,
    v = vv (1 + up to 8 %), eta up to eta_max away from the sources (each
    source sits in an isotropic patch)."""
    c = random_case(seed, nx=nx, nz=nz, pml=pml, nt=nt, nshots=nshots, nrec=nrec, ckpt=ckpt)
    rng = np.random.default_rng(seed + 500)
    vv = c.v
    vn = f32(vv * (1.0 + 0.08 * synth.smooth(rng.uniform(0.0, 1.0, (nz, nx)), 3.0)))
    eta = synth.smooth(rng.uniform(0.0, eta_max, (nz, nx)), 3.0)
    jj, ii = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    for x, z in c.src:
        eta[np.hypot(ii - x, jj - z) < 6] = 0.0
    eta = f32(eta)
    c.model = np.stack([vv, vn, eta])
    c.vmax = float(np.max(vn * np.sqrt(1.0 + 2.0 * eta))) * 1.01
    return c


def _plan(sw, c, **kw):
    return sw.Plan(nx=c.nx, nz=c.nz, h=c.h, dt=c.dt, nt=c.nt, pml=c.pml, src_xz=c.src,
                   rec_xz=c.rec, pml_vmax=c.vmax, pml_f0=c.f0, pml_R=c.R, ckpt_every=c.ckpt,
                   physics=sw.VTI, **kw)


def _oracle(orc, c, resid):
    pb = orc.problem(c.nx, c.nz, c.pml, c.h, c.dt, c.nt, c.vmax, c.f0, c.R, nshots=c.nshots,
                     nrec=c.nrec, ckpt_every=c.ckpt)
    return orc.vti_gradient(pb, c.model, c.src, c.wav, c.rec, resid, want_gathers=True)


@pytest.mark.parametrize("seed", [1, 2])
def test_vti_parity(sw, orc, seed):
    c = _vti_case(seed)
    plan = _plan(sw, c)
    d = plan.forward(_dev(c.model), _dev(c.wav), save=True)
    resid = f32(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, seed + 7))
    g = _host(plan.backward(_dev(resid)))
    gref, _, dref = _oracle(orc, c, resid)
    e_d = rel_l2(_host(d), dref)
    errs = [rel_l2(g[q], gref[q]) for q in range(3)]
    print("vti seed", seed, "gathers", e_d, "grad vv, v, eta", errs, flush=True)
    assert e_d <= SEIS_TOL and max(errs) <= GRAD_TOL


def test_vti_isotropic_is_the_acoustic_plan(sw):
    c = _vti_case(3, nt=200)
    iso = np.stack([c.v, c.v, np.zeros_like(c.v)])
    p_vti = _plan(sw, c)
    d1 = p_vti.forward(_dev(iso), _dev(c.wav), save=True)
    p_ac = c.plan()
    d0 = p_ac.forward(_dev(c.v), _dev(c.wav), save=True)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 4))
    g1 = _host(p_vti.backward(r))
    g0 = _host(p_ac.backward(r))[0]
    # the two paths round differently (cx Bx + cz Bz against C (Bx + Bz)), and
    # each is within about 1e-6 of the oracle: they agree to the parity bar
    assert rel_l2(_host(d1), _host(d0)) <= SEIS_TOL
    assert rel_l2(g1[0] + g1[1], g0) <= GRAD_TOL


def test_vti_repeatable_and_checkpoint_interval(sw, orc):
    c = _vti_case(5, nt=180, ckpt=29)
    m, w = _dev(c.model), _dev(c.wav)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 9))
    plan = _plan(sw, c)
    outs = []
    for _ in range(2):
        d = plan.forward(m, w, save=True).clone()
        outs.append((d, plan.backward(r).clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    c2 = _vti_case(5, nt=180, ckpt=180)
    p2 = _plan(sw, c2)
    d2 = p2.forward(m, w, save=True)
    assert torch.equal(d2, outs[0][0])
    assert rel_l2(_host(p2.backward(r)), _host(outs[0][1])) <= 1e-6


@pytest.mark.parametrize("shape", [(1, 40, 30, 8), (120, 10, 12, 0), (60, 20, 14, 4)])
def test_vti_edge_cases(sw, orc, shape):
    """One step; a grid smaller than one tile without pad; a short run."""
    nt, nx, nz, pml = shape
    c = _vti_case(11, nx=nx, nz=nz, pml=pml, nt=nt, nshots=2, nrec=5, ckpt=7)
    # a wavelet with no quiet start and one receiver on each source, so that
    # even a single step records something
    c.wav = f32(np.random.default_rng(8).standard_normal((c.nshots, c.nt)))
    c.rec = c.rec.copy()
    c.rec[:, 3] = c.src
    plan = _plan(sw, c)
    d = plan.forward(_dev(c.model), _dev(c.wav), save=True)
    resid = f32(np.random.default_rng(3).standard_normal((c.nshots, c.nt, c.nrec)))
    g = _host(plan.backward(_dev(resid)))
    gref, _, dref = _oracle(orc, c, resid)
    def err(a, b):  # relative L2, or the size of a where the oracle's value is exactly 0
        nb = np.linalg.norm(b)
        return rel_l2(a, b) if nb > 0 else float(np.linalg.norm(a))

    errs = [err(_host(d), dref)] + [err(g[q], gref[q]) for q in range(3)]
    print("vti edge", shape, errs, flush=True)
    assert errs[0] <= SEIS_TOL and max(errs[1:]) <= GRAD_TOL


def test_vti_no_receivers(sw):
    c = _vti_case(12, nt=60, nrec=4)
    c.rec = c.rec[:, :0]
    plan = _plan(sw, c)
    d = plan.forward(_dev(c.model), _dev(c.wav), save=True)
    assert d.numel() == 0
    g = plan.backward(torch.zeros(plan.gathers_shape(), device="cuda"))
    torch.cuda.synchronize()
    assert not torch.any(g)


def test_vti_tuning_limits(sw):
    c = _vti_case(13, nt=20)
    plan = _plan(sw, c)
    with pytest.raises(sw.SweepError):
        plan.set_tuning(rz=8)


def test_vti_graph_replays_match_eager(sw):
    """use_graph = 1 on a VTI plan (both tile kernels, stored segments): every
    replay of the captured forward and backward, with other device work and
    synchronisation between them, equals the eager plan bit for bit."""
    c = _vti_case(9, nt=150)
    m, w = _dev(c.model), _dev(c.wav)
    eager = _plan(sw, c)
    d0 = eager.forward(m, w, save=True).clone()
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 16))
    g0 = eager.backward(r).clone()
    gp = _plan(sw, c)
    gp.set_tuning(use_graph=1, keep_b=3)
    gp.reserve_workspace(True)
    out, grad = torch.empty_like(d0), torch.empty_like(g0)
    for rep in range(3):
        gp.forward(m, w, save=True, out=out)
        gp.backward(r, out=grad)
        torch.cuda.synchronize()
        assert torch.equal(out, d0), rep
        assert torch.equal(grad, g0), rep
        nf, nb = gp.graph_nodes()
        assert nf > 0 and nb > 0, (nf, nb)
        assert torch.isfinite(torch.randn(4096, device="cuda").sum())


@pytest.mark.parametrize("keep", [3, 99])
def test_vti_stored_segments_bitwise(sw, keep):
    """Stored traces of the last `keep` checkpoint segments (some, or all of
    them; 240 steps in segments of 17, so the last one is ragged): gathers and
    the three gradients equal those of the plan that recomputes every
    segment, bit for bit."""
    c = _vti_case(7)
    m, w = _dev(c.model), _dev(c.wav)
    ref = _plan(sw, c)
    d0 = ref.forward(m, w, save=True).clone()
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 14))
    g0 = ref.backward(r).clone()
    p = _plan(sw, c)
    p.set_tuning(keep_b=keep)
    assert torch.equal(p.forward(m, w, save=True), d0)
    assert torch.equal(p.backward(r), g0)
    assert all(torch.any(g0[q] != 0) for q in range(3))


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "vti1000x300_shot23.npz")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated")
@pytest.mark.parametrize("stored", [False, True])
def test_full_size_vti_sampled_shot(sw, stored):
    """All 64 shots of the 1000x300 / 3000-step VTI workload (64 x 16 tiles,
    interior and C-PML tile kernels); shot 23 compared with stored oracle
    traces and with gradient samples for a residual on that shot only.
    `stored`: the bench's configuration, the traces of as many of the last
    checkpoint segments as the free HBM holds (the bench's own sizing rule),
    the others recomputed; otherwise every segment is recomputed."""
    gold = np.load(GOLDEN)
    w = synth.workload("vti1000x300")
    plan = sw.Plan(nx=w.nx, nz=w.nz, h=w.h, dt=w.dt, nt=w.nt, pml=w.pml, src_xz=w.sources(),
                   rec_xz=w.receivers(), pml_vmax=w.pml_vmax(), pml_f0=w.f0, pml_R=w.pml_R,
                   ckpt_every=w.ckpt_every, physics=sw.VTI)
    if stored:
        import bench
        keep = bench.fit_keep_b(torch, plan, w.nt, w.ckpt_every)
        print("stored segments", keep, "of", -(-w.nt // w.ckpt_every), flush=True)
        assert keep >= 1
    d = plan.forward(_dev(w.true_model()), _dev(w.wavelets()), save=True)
    s = int(gold["shot"])
    tr = torch.as_tensor(gold["trace_idx"], device="cuda")
    e_d = rel_l2(_host(d[s][:, tr]), gold["traces"])
    resid = np.zeros((w.nshots, w.nt, w.nrec), np.float32)
    resid[s] = f32(synth.bandlimited_noise((1, w.nt, w.nrec), w.f0, w.dt, 23))[0]
    g = _host(plan.backward(_dev(resid)))
    cells = gold["grad_cells"]
    errs = [rel_l2(g[c].ravel()[cells], gold["grad"][c]) for c in range(3)]
    norms = [abs(np.linalg.norm(g[c]) / gold["grad_norm"][c] - 1.0) for c in range(3)]
    print("full-size VTI shot", s, "traces", e_d, "grad (vv, v, eta)", errs, "norms", norms,
          flush=True)
    plan.release_workspace()
    assert e_d <= SEIS_TOL
    assert max(errs) <= GRAD_TOL
    assert max(norms) <= GRAD_TOL
