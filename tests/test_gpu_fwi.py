"""GPU: full-waveform inversion through the solver's adjoint, on the grid
parameterisation and through the MLP velocity model.

(1) Chain rule: dJ/dtheta from MLP forward -> modelling -> misfit -> adjoint ->
MLP backward on the GPU against the same chain composed from the oracles (FP64
acoustic gradient, bf16-emulating FP64 MLP), every input generated on the host.
(2) A small inversion: both methods lower the misfit; the run reports what the
network gains or loses against grid FWI on model error and data misfit.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from tests.helpers import Case, f32, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_14189_amd as sw
    from paper_2604_14189_amd import fwi, mlp
    sw.lib()
    return sw, mlp, fwi


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def _case(w: synth.Workload, v) -> Case:
    return Case(w.nx, w.nz, w.pml, w.h, w.dt, w.nt, w.f0, w.vmax, f32(v),
                w.sources().astype(np.int32), w.receivers().astype(np.int32), f32(w.wavelets()),
                ckpt=w.ckpt_every, R=w.pml_R)


def test_neural_gradient_chain_matches_oracles(sw, orc):
    _, mlp, _ = sw
    w = synth.Workload("chain", "acoustic", 48, 32, 10.0, 1e-3, 300, 10, 12.0, 2, 48, 3, 3,
                       ckpt_every=40, seed=5)
    case = _case(w, w.true_model())
    pb = case.oracle_problem(orc)
    dobs = orc.ac_forward(pb, case.v, case.src, case.wav, case.rec)
    B = f32(synth.rff_frequencies(seed=1))
    theta = f32(omlp.init_params(2))

    # GPU chain
    net = mlp.MLPVelocity(w.nx, w.nz, B, theta)
    plan = case.plan()
    v = net.forward()
    d = plan.forward(v, _dev(case.wav), save=True)
    r, _ = sw[0].l2_misfit(d, _dev(dobs))
    gv = plan.backward(r)
    gt = net.backward(gv[0]).double().cpu().numpy()
    torch.cuda.synchronize()

    # oracle chain on the same host inputs
    vo, cache = omlp.forward(theta, omlp.encode(B, w.nx, w.nz))
    vo = vo.reshape(w.nz, w.nx)
    do = orc.ac_forward(pb, vo, case.src, case.wav, case.rec)
    gvo, _, _ = orc.ac_gradient(pb, vo, case.src, case.wav, case.rec, do - dobs)
    gto = omlp.backward(theta, cache, gvo.ravel())

    e_v = rel_l2(v.double().cpu().numpy() - 1500.0, vo - 1500.0)
    e_gv = rel_l2(gv[0].double().cpu().numpy(), gvo)
    e_gt = rel_l2(gt, gto)
    print("chain: v", e_v, "dJ/dv", e_gv, "dJ/dtheta", e_gt, flush=True)
    assert e_v <= 1e-5
    assert e_gv <= 1e-4
    assert e_gt <= 1e-3


def test_grid_and_neural_fwi_reduce_misfit(sw):
    sw_, mlp, fwi = sw
    w = synth.Workload("fwi_small", "acoustic", 160, 60, 10.0, 1e-3, 700, 20, 10.0, 6, 160, 3, 3,
                       seed=3)
    v_true = w.true_model()
    v_init = synth.smooth(v_true, 8.0)
    plan = sw_.Plan.from_workload(w)
    wav = _dev(w.wavelets())
    d_obs = plan.forward(_dev(v_true), wav).clone()
    v0 = _dev(v_init)
    net = mlp.MLPVelocity(w.nx, w.nz, f32(synth.rff_frequencies(seed=0)),
                          f32(omlp.init_params(4)))
    fit = fwi.prefit(net, v0, 400)
    r0 = {"grid": fwi.rmse(v0, v_true), "mlp": fwi.rmse(net.forward(), v_true)}
    runs = {"grid": fwi.GridFWI(plan, v0, wav, d_obs, lr=10.0),
            "mlp": fwi.NeuralFWI(plan, net, wav, d_obs, lr=1e-3)}
    out = {}
    for name, opt in runs.items():
        Js = [opt.step() for _ in range(30)]
        out[name] = {"J_rel": Js[-1] / Js[0], "rmse0": r0[name],
                     "rmse": fwi.rmse(opt.velocity, v_true)}
    print("prefit rms", fit, "fwi", out, flush=True)
    for name in out:
        assert np.isfinite(out[name]["J_rel"]) and out[name]["J_rel"] < 0.9, name
    assert out["grid"]["rmse"] < out["grid"]["rmse0"]
