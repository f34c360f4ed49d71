"""GPU parity: first-order variable-density acoustic (Eq. 1), computed by the
fluid variants of the staggered elastic kernels, against the FP64 oracle (the
same scheme with vs = 0). Model (vp, rho), gathers (vx, vz), gradients (vp,
rho).

Tolerances as for the other physics: gathers <= 1e-5, gradients <= 1e-4
relative L2. The mode must also give exactly the elastic plan's results for
vs = 0 (the fluid variants drop only terms that are products with mu = 0).
The full 1000x300 / 3000-step workload with 64 shots (the benchmark's
configuration) is checked on one shot against stored oracle values.
"""
import os

import numpy as np
import pytest

import synth
from tests.helpers import f32, rel_l2

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


def _case(fs, seed=1, nx=110, nz=70, nt=260, nshots=3, nrec=17):
    rng = np.random.default_rng(seed)
    vp = f32(synth.layered_anomaly(nx, nz, 1500.0, 3500.0, seed + 30))
    rho = f32(310.0 * vp ** 0.25)
    src = np.stack([rng.integers(0, nx, nshots), rng.integers(0, nz, nshots)], 1).astype(np.int32)
    src[0] = [0, 0]
    rec = np.stack([rng.integers(0, nx, (nshots, nrec)), rng.integers(0, nz, (nshots, nrec))],
                   2).astype(np.int32)
    rec[:, 1] = rec[:, 0]
    wav = f32(np.stack([synth.ricker(20.0 + 2 * s, nt, 0.5e-3) for s in range(nshots)]))
    return dict(nx=nx, nz=nz, pml=10, h=5.0, dt=0.5e-3, nt=nt, f0=20.0, vmax=3500.0, fs=fs,
                vp=vp, rho=rho, src=src, rec=rec, wav=wav, ckpt=23)


def _plan(sw, c, physics):
    return sw.Plan(nx=c["nx"], nz=c["nz"], h=c["h"], dt=c["dt"], nt=c["nt"], pml=c["pml"],
                   src_xz=c["src"], rec_xz=c["rec"], pml_vmax=c["vmax"], pml_f0=c["f0"],
                   ckpt_every=c["ckpt"], physics=physics, free_surface=c["fs"])


@pytest.mark.parametrize("fs", [0, 1])
def test_vd_parity(sw, orc, fs):
    c = _case(fs)
    plan = _plan(sw, c, sw.ACOUSTIC_VD)
    d = plan.forward(_dev(np.stack([c["vp"], c["rho"]])), _dev(c["wav"]), save=True)
    resid = f32(np.random.default_rng(9).standard_normal(tuple(d.shape)))
    g = _host(plan.backward(_dev(resid)))
    m3 = np.stack([c["vp"], np.zeros_like(c["vp"]), c["rho"]])
    pb = orc.problem(c["nx"], c["nz"], c["pml"], c["h"], c["dt"], c["nt"], c["vmax"], c["f0"],
                     1e-3, nshots=len(c["src"]), nrec=c["rec"].shape[1], free_surface=fs,
                     ckpt_every=c["ckpt"])
    gref, _, dref = orc.el_gradient(pb, m3, c["src"], c["wav"], c["rec"], resid,
                                    want_gathers=True)
    e_d = rel_l2(_host(d), dref)
    e_v, e_r = rel_l2(g[0], gref[0]), rel_l2(g[1], gref[2])
    print("acoustic_vd fs", fs, "gathers", e_d, "grad vp", e_v, "grad rho", e_r, flush=True)
    assert tuple(g.shape) == (2, c["nz"], c["nx"])
    assert e_d <= SEIS_TOL and e_v <= GRAD_TOL and e_r <= GRAD_TOL


def test_vd_is_the_elastic_scheme_at_vs_zero(sw):
    c = _case(1, seed=4, nt=150)
    vd = _plan(sw, c, sw.ACOUSTIC_VD)
    el = _plan(sw, c, sw.ELASTIC)
    wav = _dev(c["wav"])
    d1 = vd.forward(_dev(np.stack([c["vp"], c["rho"]])), wav, save=True)
    d3 = el.forward(_dev(np.stack([c["vp"], np.zeros_like(c["vp"]), c["rho"]])), wav, save=True)
    assert torch.equal(d1, d3)
    r = _dev(np.random.default_rng(2).standard_normal(tuple(d1.shape)))
    g1, g3 = vd.backward(r), el.backward(r)
    assert torch.equal(g1[0], g3[0]) and torch.equal(g1[1], g3[2])
    assert not torch.any(g3[1])


@pytest.mark.parametrize("fs,keep", [(0, 3), (1, 3), (0, 99), (1, 99)])
def test_vd_stored_segments_bitwise(sw, fs, keep):
    """Stored traces of the last `keep` checkpoint segments (some, or all of
    them; 260 steps in segments of 23, so the last one is ragged): gathers and
    (vp, rho) gradients equal those of the plan that recomputes every segment,
    bit for bit."""
    c = _case(fs, seed=6)
    m, wav = _dev(np.stack([c["vp"], c["rho"]])), _dev(c["wav"])
    ref = _plan(sw, c, sw.ACOUSTIC_VD)
    d0 = ref.forward(m, wav, save=True).clone()
    r = _dev(np.random.default_rng(12).standard_normal(tuple(d0.shape)))
    g0 = ref.backward(r).clone()
    p = _plan(sw, c, sw.ACOUSTIC_VD)
    p.set_tuning(keep_b=keep)
    assert torch.equal(p.forward(m, wav, save=True), d0)
    assert torch.equal(p.backward(r), g0)
    assert torch.any(g0[0] != 0) and torch.any(g0[1] != 0)


def test_vd_graph_replays_match_eager(sw):
    """use_graph = 1 on a variable-density plan (fluid kernels, pressure-release
    top, stored segments): every replay of the captured forward and backward
    equals the eager plan bit for bit."""
    c = _case(1, seed=8, nt=150)
    m, wav = _dev(np.stack([c["vp"], c["rho"]])), _dev(c["wav"])
    eager = _plan(sw, c, sw.ACOUSTIC_VD)
    d0 = eager.forward(m, wav, save=True).clone()
    r = _dev(np.random.default_rng(6).standard_normal(tuple(d0.shape)))
    g0 = eager.backward(r).clone()
    gp = _plan(sw, c, sw.ACOUSTIC_VD)
    gp.set_tuning(use_graph=1, keep_b=2)
    gp.reserve_workspace(True)
    out, grad = torch.empty_like(d0), torch.empty_like(g0)
    for rep in range(3):
        gp.forward(m, wav, save=True, out=out)
        gp.backward(r, out=grad)
        torch.cuda.synchronize()
        assert torch.equal(out, d0), rep
        assert torch.equal(grad, g0), rep
        nf, nb = gp.graph_nodes()
        assert nf > 0 and nb > 0, (nf, nb)
        assert torch.isfinite(torch.randn(4096, device="cuda").sum())


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "vd1000x300_shot41.npz")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated")
@pytest.mark.parametrize("stored", [False, True])
def test_full_size_vd_sampled_shot(sw, stored):
    """All 64 shots of the 1000x300 / 3000-step layered workload with rho =
    310 vp^0.25; shot 41 compared with stored oracle traces and gradient
    samples for a residual on that shot only. `stored`: the benchmark's
    configuration, the traces of as many of the last checkpoint segments as
    the free HBM holds, the others recomputed."""
    gold = np.load(GOLDEN)
    w = synth.workload("layered1000x300")
    vp = f32(w.true_model())
    model = np.stack([vp, f32(310.0 * vp.astype(np.float64) ** 0.25)])
    plan = sw.Plan(nx=w.nx, nz=w.nz, h=w.h, dt=w.dt, nt=w.nt, pml=w.pml, src_xz=w.sources(),
                   rec_xz=w.receivers(), pml_vmax=w.pml_vmax(), pml_f0=w.f0, pml_R=w.pml_R,
                   ckpt_every=w.ckpt_every, physics=sw.ACOUSTIC_VD)
    if stored:
        import bench
        keep = bench.fit_keep_b(torch, plan, w.nt, w.ckpt_every)
        print("stored segments", keep, "of", -(-w.nt // w.ckpt_every), flush=True)
        assert keep >= 1
    d = plan.forward(_dev(model), _dev(w.wavelets()), save=True)
    s = int(gold["shot"])
    tr = torch.as_tensor(gold["trace_idx"], device="cuda")
    e_d = rel_l2(_host(d[s][:, tr, :]), gold["traces"])
    resid = np.zeros((w.nshots, w.nt, w.nrec, 2), np.float32)
    resid[s] = f32(synth.bandlimited_noise((1, w.nt, w.nrec * 2), w.f0, w.dt, 41)
                   .reshape(w.nt, w.nrec, 2))
    g = _host(plan.backward(_dev(resid)))
    cells = gold["grad_cells"]
    errs = [rel_l2(g[c].ravel()[cells], gold["grad"][c]) for c in range(2)]
    norms = [abs(np.linalg.norm(g[c]) / gold["grad_norm"][c] - 1.0) for c in range(2)]
    print("full-size variable-density shot", s, "traces", e_d, "grad (vp, rho)", errs, "norms",
          norms, flush=True)
    plan.release_workspace()
    assert e_d <= SEIS_TOL
    assert max(errs) <= GRAD_TOL
    assert max(norms) <= GRAD_TOL
