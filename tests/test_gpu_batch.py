"""GPU: batched uneven plans, hipGraph replay and the autotuner.

Batch modelling changes the number of launches, never the results (Sec. 2.2):
a batch of plans with different grids, shot counts and step counts must give
bit-identical gathers and gradients to each plan run alone. Captured graphs are
replayed several times with eager work in between and every replay is checked
against the eager result.
"""
import json
import os

import numpy as np
import pytest

import synth
from tests.helpers import case_from_workload, f32, random_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


@pytest.fixture(scope="module")
def sw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_14189_amd as sw
    sw.lib()
    return sw


def _cases():
    # uneven: different grids (ragged tiles), shots, steps, checkpoint intervals
    return [random_case(21, nx=150, nz=77, nt=130, nshots=3, ckpt=17),
            random_case(22, nx=96, nz=120, nt=90, nshots=2, ckpt=20),
            random_case(23, nx=200, nz=64, nt=111, nshots=4, ckpt=50)]


def _resids(cases):
    return [_dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 40 + i))
            for i, c in enumerate(cases)]


def _single(cases, resids):
    out = []
    for c, r in zip(cases, resids):
        plan = c.plan()
        d = plan.forward(_dev(c.v), _dev(c.wav), save=True).clone()
        g = plan.backward(r).clone()
        out.append((d, g))
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_plans(sw, graph):
    cases = _cases()
    resids = _resids(cases)
    ref = _single(cases, resids)
    plans = [c.plan() for c in cases]
    batch = sw.Batch(plans, use_graph=graph)
    for rep in range(3 if graph else 1):
        ds = batch.forward([_dev(c.v) for c in cases], [_dev(c.wav) for c in cases], save=True)
        gs = batch.backward(resids)
        torch.cuda.synchronize()
        for q in range(len(cases)):
            assert torch.equal(ds[q], ref[q][0]), (rep, q)
            assert torch.equal(gs[q], ref[q][1]), (rep, q)
        # eager work between replays
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()


def test_batch_two_step_passes(sw):
    """Plans with deep tiles take batched two-step passes (ragged step counts and
    odd checkpoint intervals force single steps in between); the results are
    bitwise those of each plan alone with single steps."""
    cases = [random_case(51, nx=300, nz=200, nt=101, nshots=2, nrec=6, ckpt=17),
             random_case(52, nx=260, nz=150, nt=76, nshots=3, nrec=5, ckpt=25),
             random_case(53, nx=120, nz=90, nt=90, nshots=2, nrec=4, ckpt=50)]
    resids = _resids(cases)
    ref = []
    for c, r in zip(cases, resids):
        p = c.plan()
        p.set_tuning(rz=4, pml_rz=4, tblock=1)
        ref.append((p.forward(_dev(c.v), _dev(c.wav), save=True).clone(), p.backward(r).clone()))
    plans = [c.plan() for c in cases]
    for p in plans:
        p.set_tuning(rz=4, pml_rz=4, tblock=2)
    assert sum(p.tiles()["deep"] > 0 for p in plans) >= 2
    batch = sw.Batch(plans)
    ds = batch.forward([_dev(c.v) for c in cases], [_dev(c.wav) for c in cases], save=True)
    gs = batch.backward(resids)
    torch.cuda.synchronize()
    for q in range(len(cases)):
        assert torch.equal(ds[q], ref[q][0]), q
        assert torch.equal(gs[q], ref[q][1]), q


@pytest.mark.parametrize("graph", [False, True])
def test_batch_stored_segments(sw, graph):
    """Stored B'^n segments in a batch, each plan with its own count (some,
    all, none; ragged last segments), with two-step passes and with graph
    replays: gathers and gradients are bitwise those of each plan alone
    recomputing every segment."""
    cases = [random_case(51, nx=300, nz=200, nt=101, nshots=2, nrec=6, ckpt=17),
             random_case(52, nx=260, nz=150, nt=76, nshots=3, nrec=5, ckpt=25),
             random_case(53, nx=120, nz=90, nt=90, nshots=2, nrec=4, ckpt=50),
             random_case(21, nx=150, nz=77, nt=130, nshots=3, ckpt=17)]
    resids = _resids(cases)
    ref = _single(cases, resids)
    plans = [c.plan() for c in cases]
    base = sw.Batch(plans).workspace_bytes(True)
    for p, keep in zip(plans, (2, 99, 0, 3)):
        p.set_tuning(rz=4, pml_rz=4, tblock=2, keep_b=keep)
    assert sum(p.tiles()["deep"] > 0 for p in plans) >= 2
    batch = sw.Batch(plans, use_graph=graph)
    assert batch.workspace_bytes(True) > base
    for rep in range(3 if graph else 1):
        ds = batch.forward([_dev(c.v) for c in cases], [_dev(c.wav) for c in cases], save=True)
        gs = batch.backward(resids)
        torch.cuda.synchronize()
        for q in range(len(cases)):
            assert torch.equal(ds[q], ref[q][0]), (rep, q)
            assert torch.equal(gs[q], ref[q][1]), (rep, q)
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()


def test_batch_autotune_picks_and_caches(sw, tmp_path):
    """The batch autotuner sets one tuning on every plan, caches it under the
    batch's shapes, and the results keep the bits of single-step plans."""
    cases = [random_case(61, nx=260, nz=150, nt=40, nshots=2, nrec=5, ckpt=20),
             random_case(62, nx=120, nz=90, nt=30, nshots=2, nrec=4, ckpt=50)]
    plans = [c.plan() for c in cases]
    batch = sw.Batch(plans)
    cache = str(tmp_path / "btune.jsonl")
    vs, ws = [_dev(c.v) for c in cases], [_dev(c.wav) for c in cases]
    t = batch.autotune(vs, ws, steps=6, cache_path=cache)
    assert t["rz"] in (1, 2, 4, 8) and t["pml_rz"] <= t["rz"] and t["tblock"] in (1, 2)
    for p in plans:
        tp = p.tuning
        assert (tp["rz"], tp["pml_rz"], tp["tblock"]) == (t["rz"], t["pml_rz"], t["tblock"])
    with open(cache) as f:
        lines = f.read().strip().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["mode"] == "batch-gradient" and rec["physics"] == "acoustic"
    assert rec["shapes"] == " ".join(f"{p.padded()[0]}x{p.padded()[1]}x{c.nshots}x{c.pml}"
                                     for p, c in zip(plans, cases))
    assert (rec["rz"], rec["pml_rz"], rec["tblock"]) == (t["rz"], t["pml_rz"], t["tblock"])
    assert rec["us_per_step"] > 0
    assert sw.Batch([c.plan() for c in cases]).autotune(vs, ws, steps=6, cache_path=cache) == t
    resids = _resids(cases)
    ds = batch.forward(vs, ws, save=True)
    gs = batch.backward(resids)
    for q, (c, r) in enumerate(zip(cases, resids)):
        p = c.plan()
        p.set_tuning(rz=4, pml_rz=4, tblock=1)
        assert torch.equal(ds[q], p.forward(vs[q], ws[q], save=True)), q
        assert torch.equal(gs[q], p.backward(r)), q


def test_plan_graph_replays_match_eager(sw):
    c = random_case(31, nt=140, ckpt=25)
    r = _dev(synth.bandlimited_noise((c.nshots, c.nt, c.nrec), 15.0, c.dt, 3))
    eager = c.plan()
    d0 = eager.forward(_dev(c.v), _dev(c.wav), save=True).clone()
    g0 = eager.backward(r).clone()
    gp = c.plan()
    gp.set_tuning(rz=8, use_graph=1)
    v, w = _dev(c.v), _dev(c.wav)
    out = torch.empty_like(d0)
    grad = torch.empty_like(g0)
    for rep in range(4):
        gp.forward(v, w, save=True, out=out)
        gp.backward(r, out=grad)
        torch.cuda.synchronize()
        assert torch.equal(out, d0), rep
        assert torch.equal(grad, g0), rep
        x = torch.randn(4096, device="cuda")
        assert torch.isfinite(x.sum())


def test_autotune_picks_a_tiling_and_caches(sw, tmp_path):
    c = random_case(41, nx=300, nz=180, nt=60, nshots=4)
    plan = c.plan()
    cache = str(tmp_path / "tune.jsonl")
    rz = plan.autotune(_dev(c.v), _dev(c.wav), steps=10, cache_path=cache)
    assert rz in (1, 2, 4, 8)
    assert plan.tuning["rz"] == rz
    with open(cache) as f:
        lines = f.read().strip().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    NX, NZ = plan.padded()
    assert rec["mode"] == "plan-forward" and rec["shapes"] == f"{NX}x{NZ}x{c.nshots}x{c.pml}"
    assert rec["rz"] == rz and rec["pml_rz"] == plan.tuning["pml_rz"]
    assert rec["tblock"] == plan.tuning["tblock"] and rec["tblock"] in (1, 2)
    assert plan.tuning["pml_rz"] <= rz
    d1 = plan.forward(_dev(c.v), _dev(c.wav)).clone()
    plan2 = c.plan()
    assert plan2.autotune(_dev(c.v), _dev(c.wav), steps=10, cache_path=cache) == rz
    d0 = c.plan().forward(_dev(c.v), _dev(c.wav))
    assert torch.equal(d0, d1)


# ------------------------------------------------- the eight uneven workloads
BATCH_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch_uneven8_short.npz")


@pytest.mark.skipif(not os.path.exists(BATCH_GOLDEN), reason="golden file not generated")
@pytest.mark.parametrize("graph", [False, True])
def test_batch_uneven8_against_oracle(sw, graph):
    """The eight uneven workloads (grids 200x200 ... 1200x400 with 40-cell
    pads, 16 ... 48 shots, 256 shots in all) in one batch with the benchmark's
    launch configuration (rz 8, pml_rz 4, two-step passes, stored segments on
    half of the plans), their runs shortened to 125 ... 250 steps. The middle
    shot of each model is compared with the oracle's traces and gradient
    samples (written by tests/golden/make_golden.py: the largest cells, and
    random others measured against the gradient's norm); the residual is non-zero
    on that shot only, so the batch gradient is that shot's gradient. With a
    captured graph, three replays with eager work between them each match."""
    from tests.golden.make_golden import batch_short_nt
    gold = np.load(BATCH_GOLDEN)
    ws = synth.batched_workloads()
    cases, plans, models, wavs, resids = [], [], [], [], []
    for m, w in enumerate(ws):
        nt = batch_short_nt(m)
        assert int(gold[f"m{m}_nt"]) == nt
        c = case_from_workload(w.replace(nt=nt))
        p = c.plan()
        p.set_tuning(rz=8, pml_rz=4, tblock=2, keep_b=m % 2)
        s = int(gold[f"m{m}_shot"])
        r = np.zeros((c.nshots, nt, c.nrec), np.float32)
        r[s] = synth.bandlimited_noise((1, nt, w.nrec), w.f0, w.dt, 100 + m)[0]
        cases.append(c)
        plans.append(p)
        models.append(_dev(c.v))
        wavs.append(_dev(c.wav))
        resids.append(_dev(r))
    assert sum(c.nshots for c in cases) == 256
    batch = sw.Batch(plans, use_graph=graph)
    first = None
    for rep in range(3 if graph else 1):
        print("batch uneven8 graph", graph, "replay", rep, flush=True)
        ds = batch.forward(models, wavs, save=True)
        gs = batch.backward(resids)
        torch.cuda.synchronize()
        if first is None:
            first = [(d.clone(), g.clone()) for d, g in zip(ds, gs)]
            for m in range(len(ws)):
                s = int(gold[f"m{m}_shot"])
                tr = torch.as_tensor(gold[f"m{m}_trace_idx"], device="cuda")
                e_d = rel_l2(ds[m][s][:, tr].double().cpu().numpy(), gold[f"m{m}_traces"])
                g = gs[m][0].double().cpu().numpy().ravel()
                gn = float(gold[f"m{m}_grad_norm"])
                # the 2000 largest cells carry the gradient's norm; the random
                # others' error, scaled to the cells they stand for, is their
                # estimated share of the whole gradient's relative L2
                e_top = rel_l2(g[gold[f"m{m}_top_cells"]], gold[f"m{m}_top"])
                rc = gold[f"m{m}_rand_cells"]
                e_rest = (np.linalg.norm(g[rc] - gold[f"m{m}_rand"]) *
                          np.sqrt((g.size - 2000) / len(rc)) / gn)
                e_n = abs(np.linalg.norm(g) - gn) / gn
                print("model", m, "shot", s, "traces", e_d, "gradient top", e_top, "rest", e_rest,
                      "norm", e_n, flush=True)
                assert e_d <= 1e-5 and e_top <= 1e-4 and e_rest <= 1e-4 and e_n <= 1e-4, m
        else:
            for m in range(len(ws)):
                assert torch.equal(ds[m], first[m][0]) and torch.equal(gs[m], first[m][1])
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()


def test_batch_refuses_member_tuning_changes(sw):
    """A member's tuning change after the saving forward makes the batch's
    backward fail (its saved layout no longer holds) instead of reading
    checkpoints the forward never wrote; a changed tiling makes the forward
    fail; re-tuning every plan alike restores the batch's results."""
    cases = _cases()
    resids = _resids(cases)
    ref = _single(cases, resids)
    plans = [c.plan() for c in cases]
    batch = sw.Batch(plans)
    models, wavs = [_dev(c.v) for c in cases], [_dev(c.wav) for c in cases]
    batch.forward(models, wavs, save=True)
    plans[1].set_tuning(keep_b=2)
    with pytest.raises(sw.SweepError) as e:
        batch.backward(resids)
    assert e.value.rc == sw._lib.ESTATE
    plans[0].set_tuning(rz=4)
    with pytest.raises(sw.SweepError) as e:
        batch.forward(models, wavs, save=True)
    assert e.value.rc == sw._lib.EINVAL
    for p in plans:
        p.set_tuning(rz=8)
    ds = batch.forward(models, wavs, save=True)
    gs = batch.backward(resids)
    torch.cuda.synchronize()
    for q in range(len(cases)):
        assert torch.equal(ds[q], ref[q][0]) and torch.equal(gs[q], ref[q][1])
