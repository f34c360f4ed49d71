"""GPU: encoded shots (source encoding; several sources per simulation, each
with its own wavelet, e.g. a random sign times the shot's wavelet) against the
FP64 oracle, on a grid with deep tiles (two-step passes) and frame tiles.

* gathers <= 1e-5 and gradient <= 1e-4 relative L2 of the oracle, with two
  coincident sources and receivers on source cells;
* one source given as [nshots, 1, 2] is the plain path, bit for bit;
* an encoded shot equals the sum of its sources run one by one (FP32);
* the result does not depend on the tiling or the time blocking (bitwise);
* graph replays and stored B'^n segments give the eager, recomputing bits.
"""
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


def _encoded(seed, nsrc=4, nt=160, nx=300, nz=200):
    c = random_case(seed, nx=nx, nz=nz, nt=nt, nshots=2, nrec=9, ckpt=17)
    rng = np.random.default_rng(seed)
    src = np.stack([np.stack([rng.integers(0, nx, nsrc), rng.integers(0, 12, nsrc)], 1)
                    for _ in range(c.nshots)]).astype(np.int32)
    src[:, 1] = src[:, 0]                 # two coincident sources
    rec = c.rec.copy()
    rec[:, 0] = src[:, 2]                 # a receiver on a source cell
    signs = rng.choice([-1.0, 1.0], size=(c.nshots, nsrc))
    wav = f32(np.stack([[signs[s, k] * synth.ricker(15.0 + 2 * k, nt, c.dt)
                         for k in range(nsrc)] for s in range(c.nshots)]))
    c.rec = rec
    return c, src, wav


def _plan(c, src):
    import paper_2604_14189_amd as sw
    return sw.Plan(nx=c.nx, nz=c.nz, h=c.h, dt=c.dt, nt=c.nt, pml=c.pml, src_xz=src,
                   rec_xz=c.rec, pml_vmax=c.vmax, pml_f0=c.f0, pml_R=c.R, ckpt_every=c.ckpt)


@pytest.mark.parametrize("tblock", [2, 1])
def test_encoded_parity(sw, orc, tblock):
    c, src, wav = _encoded(61)
    plan = _plan(c, src)
    plan.set_tuning(rz=4, pml_rz=4, tblock=tblock)
    if tblock == 2:
        assert plan.tiles()["deep"] > 0
    d = plan.forward(_dev(c.v), _dev(wav), save=True)
    resid = f32(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 3))
    g = _host(plan.backward(_dev(resid)))[0]
    pb = c.oracle_problem(orc)
    dref = orc.ac_forward_encoded(pb, c.v, src, wav, c.rec)
    gref = orc.ac_gradient_encoded(pb, c.v, src, wav, c.rec, resid)
    e_d, e_g = rel_l2(_host(d), dref), rel_l2(g, gref)
    print("encoded tblock", tblock, "gathers", e_d, "gradient", e_g, flush=True)
    assert np.any(dref[:, :, 0])
    assert e_d <= SEIS_TOL and e_g <= GRAD_TOL


def test_one_source_as_encoded_is_plain(sw):
    c = random_case(62, nt=120)
    v, w = _dev(c.v), _dev(c.wav)
    d0 = c.plan().forward(v, w).clone()
    d1 = _plan(c, c.src[:, None]).forward(v, w[:, None].contiguous())
    assert torch.equal(d0, d1)


def test_encoded_shot_is_the_sum_of_its_sources(sw):
    c, src, wav = _encoded(63, nt=140)
    v = _dev(c.v)
    d = _host(_plan(c, src).forward(v, _dev(wav)))
    parts = sum(_host(_plan(c, src[:, k:k + 1]).forward(v, _dev(wav[:, k:k + 1])))
                for k in range(src.shape[1]))
    e = rel_l2(d, parts)
    print("encoded superposition", e, flush=True)
    assert e <= 1e-6


@pytest.mark.parametrize("rz,prz,tblock", [(1, 1, 1), (8, 2, 2), (8, 4, 1)])
def test_encoded_tilings_bitwise(sw, rz, prz, tblock):
    c, src, wav = _encoded(64, nt=100)
    v, w = _dev(c.v), _dev(wav)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 4))
    ref = _plan(c, src)
    d0 = ref.forward(v, w, save=True).clone()
    g0 = ref.backward(r).clone()
    p = _plan(c, src)
    p.set_tuning(rz=rz, pml_rz=prz, tblock=tblock)
    assert torch.equal(p.forward(v, w, save=True), d0)
    assert torch.equal(p.backward(r), g0)


def test_encoded_born_and_batch_rules(sw):
    c, src, wav = _encoded(65, nt=90, nx=150, nz=77)
    plan = _plan(c, src)
    v, w = _dev(c.v), _dev(wav)
    dv = _dev(np.random.default_rng(1).standard_normal((c.nz, c.nx)) * 20.0)
    dd = plan.born(v, dv, w)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 5))
    plan.forward(v, w, save=True)
    g = plan.backward(r)
    lhs = float((dd.double() * r.double()).sum())
    rhs = float((dv.double().reshape(-1) * g.double().reshape(-1)).sum())
    assert abs(lhs - rhs) <= 1e-5 * float(dd.double().norm()) * float(r.double().norm())
    with pytest.raises(sw.SweepError):
        sw.Batch([_plan(c, src), c.plan()])


def test_encoded_graph_replays_match_eager(sw):
    """The per-step source injection of encoded shots is captured with the
    rest of the time loop: every replay gives the eager bits."""
    c, src, wav = _encoded(66, nt=80, nx=150, nz=77)
    v, w = _dev(c.v), _dev(wav)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 6))
    eager = _plan(c, src)
    d0 = eager.forward(v, w, save=True).clone()
    g0 = eager.backward(r).clone()
    gp = _plan(c, src)
    gp.set_tuning(rz=8, use_graph=1)
    out, grad = torch.empty_like(d0), torch.empty_like(g0)
    for rep in range(3):
        gp.forward(v, w, save=True, out=out)
        gp.backward(r, out=grad)
        torch.cuda.synchronize()
        assert torch.equal(out, d0), rep
        assert torch.equal(grad, g0), rep
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()


@pytest.mark.parametrize("keep", [3, 99])
def test_encoded_stored_segments_bitwise(sw, keep):
    """Encoded shots with stored B'^n segments (some, or all of them): the
    per-step source injection follows the step kernels that write B'^n, so
    gathers and gradient are those of the plan that recomputes every
    segment, bit for bit."""
    c, src, wav = _encoded(67, nt=120)
    v, w = _dev(c.v), _dev(wav)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 8))
    ref = _plan(c, src)
    d0 = ref.forward(v, w, save=True).clone()
    g0 = ref.backward(r).clone()
    p = _plan(c, src)
    p.set_tuning(rz=8, keep_b=keep)
    assert torch.equal(p.forward(v, w, save=True), d0)
    assert torch.equal(p.backward(r), g0)
    assert torch.any(g0 != 0)
