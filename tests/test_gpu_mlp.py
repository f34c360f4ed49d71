"""GPU: MLP velocity model (bf16 MFMA, float32 accumulation) against the
bf16-emulating FP64 oracle, and Adam against the oracle's Adam.

Forward and gradients <= 1e-3 relative L2: both sides round to bfloat16 at
the same points, but the float32 (GPU) and float64 (oracle) sums can put a
value on different sides of a bfloat16 rounding boundary or of a ReLU kink."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from tests.helpers import f32, rel_l2
from tests.mlp_decisions import gradient_on_decisions

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_14189_amd as sw
    from paper_2604_14189_amd import mlp
    sw.lib()
    return mlp


def _blocks(g):
    out, o = [], 0
    for s in omlp.SHAPES:
        n = int(np.prod(s))
        out.append(g[o:o + n])
        o += n
    return out


def _setup(sw, nx, nz):
    B = f32(synth.rff_frequencies(seed=0))
    theta = f32(omlp.init_params(1) +
                0.01 * np.random.default_rng(2).standard_normal(omlp.n_params()))
    net = sw.MLPVelocity(nx, nz, B, theta)
    v = net.forward()
    dv = f32(np.random.default_rng(3).standard_normal((nz, nx)) * 1e-3)
    g = net.backward(torch.tensor(dv, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    torch.cuda.synchronize()
    return B, theta, net, v.double().cpu().numpy().ravel(), dv, g


def test_end_to_end_small(sw):
    # small grid: every ReLU and rounding decision of the float32 kernels agrees
    # with the float64 oracle closely enough for a direct comparison
    nx, nz = 67, 41
    B, theta, net, v, dv, g = _setup(sw, nx, nz)
    vref, cache = omlp.forward(theta, omlp.encode(B, nx, nz))
    gref = omlp.backward(theta, cache, dv.ravel())
    errs = [rel_l2(a, b) for a, b in zip(_blocks(g), _blocks(gref))]
    print("mlp small v", rel_l2(v - 1500.0, vref - 1500.0), "grad", max(errs), flush=True)
    assert rel_l2(v - 1500.0, vref - 1500.0) <= 1e-3
    assert max(errs) <= 1e-3


def _within_sum_bound(got, exact, scale, K):
    """True where got is a bf16 rounding of some value within the float32
    recursive-summation error bound (K + 2) u scale of exact (u = 2^-24; the two
    extra terms cover the bias add and the final product). bf16 rounding is
    monotone, so that set is the interval [bf16(exact - E), bf16(exact + E)]."""
    E = (K + 2) * 2.0 ** -24 * scale
    return (got >= omlp.bf16(exact - E)) & (got <= omlp.bf16(exact + E))


def test_full_size_decisions_and_gradient(sw):
    """300k points. ReLU masks and bf16 roundings are discrete decisions taken in
    float32 by the kernels; a few of them fall on the other side in float64.
    Forward: every layer's activations are recomputed by the oracle from the
    kernel's previous layer; mismatches must be rare and each must be a correct
    rounding of a value within the float32 summation error bound. Backward: the
    same for every pre-activation gradient, recomputed from the kernel's next
    one. Then the gradient is compared with the oracle run on the kernel's
    activations and pre-activation gradients (same decisions), to 1e-4."""
    nx, nz = 1000, 300
    M = nx * nz
    B, theta, net, v, dv, g = _setup(sw, nx, nz)
    gamma = omlp.encode(B, nx, nz)
    hs = [h.double().cpu().numpy() for h in net.activations()]
    dzs = [d.double().cpu().numpy() for d in net.pre_activation_grads()]
    feats = ((net.feats.view(M, 128).to(torch.int32) << 16).view(torch.float32)
             .double().cpu().numpy())
    # features: cos / sin computed in float64 on both sides, then rounded to bf16
    fbad = feats != gamma
    print("features mismatch fraction", fbad.mean(), flush=True)
    assert fbad.mean() < 1e-5
    p = omlp.unpack(theta)
    prev = feats
    for l in range(4):
        W = omlp.bf16(p[2 * l])
        z = prev @ W.T + p[2 * l + 1]
        S = np.abs(prev) @ np.abs(W).T + np.abs(p[2 * l + 1])
        bad = omlp.bf16(np.maximum(z, 0.0)) != hs[l]
        # relu then bf16 is monotone too: compare against relu of the interval
        ok = _within_sum_bound(hs[l], z, S, prev.shape[1]) | (
            (hs[l] == 0.0) & (z <= (prev.shape[1] + 2) * 2.0 ** -24 * S))
        ok &= hs[l] >= 0.0
        print("forward layer", l + 1, "mismatch fraction", bad.mean(), "valid", bool(ok.all()),
              flush=True)
        assert bad.mean() < 2e-3 and ok.all()
        prev = hs[l]
    w5 = omlp.bf16(p[8])
    y = hs[3] @ w5 + p[9][0]
    vref = 1500.0 + 3200.0 / (1.0 + np.exp(-y))
    assert rel_l2(v - 1500.0, vref - 1500.0) <= 1e-5
    s = 1.0 / (1.0 + np.exp(-y))
    # head: dZ4 = bf16(dy w5 [h4 > 0]); dy carries the float32 error of y
    # (scaled by |1 - 2s|) and of a few float32 operations around expf
    dy = dv.ravel() * 3200.0 * s * (1.0 - s)
    Ey = (256 + 2) * 2.0 ** -24 * (np.abs(hs[3]) @ np.abs(w5) + abs(p[9][0]))
    rel = np.abs(1.0 - 2.0 * s) * Ey + 2.0 ** -24 * (16.0 + 8.0 * s / (1.0 - s))
    t = np.outer(dy, w5) * (hs[3] > 0)
    E = np.abs(t) * rel[:, None]
    ok = (dzs[3] >= omlp.bf16(t - E)) & (dzs[3] <= omlp.bf16(t + E))
    print("backward dZ4 mismatch fraction", (omlp.bf16(t) != dzs[3]).mean(), "valid",
          bool(ok.all()), flush=True)
    assert ok.all()
    for l in (3, 2, 1):
        W = omlp.bf16(p[2 * l])
        mask = hs[l - 1] > 0
        t = (dzs[l] @ W) * mask
        S = (np.abs(dzs[l]) @ np.abs(W)) * mask
        bad = omlp.bf16(t) != dzs[l - 1]
        ok = _within_sum_bound(dzs[l - 1], t, S, 256) & ((dzs[l - 1] == 0.0) | mask)
        print("backward dZ%d mismatch fraction" % l, bad.mean(), "valid", bool(ok.all()),
              flush=True)
        assert bad.mean() < 2e-3 and ok.all()
    gref = gradient_on_decisions(theta, [feats] + hs, s, dzs, dv.ravel())
    errs = [rel_l2(a, b) for a, b in zip(_blocks(g), _blocks(gref))]
    print("mlp full-size gradient (same decisions)", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-4


def test_deterministic(sw):
    B = f32(synth.rff_frequencies(seed=5))
    theta = f32(omlp.init_params(6))
    outs = []
    for _ in range(2):
        net = sw.MLPVelocity(130, 70, B, theta)
        v = net.forward()
        g = net.backward(torch.ones((70, 130), device="cuda") * 1e-3)
        outs.append((v.clone(), g.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_adam_matches_oracle(sw):
    rng = np.random.default_rng(7)
    n = 10007
    th, g1, g2 = (f32(rng.standard_normal(n)) for _ in range(3))
    t_th = torch.tensor(th, dtype=torch.float32, device="cuda")
    t_m = torch.zeros(n, device="cuda")
    t_v = torch.zeros(n, device="cuda")
    o_th, o_m, o_v = th.copy(), np.zeros(n), np.zeros(n)
    for t, g in ((1, g1), (2, g2)):
        sw.adam_step(t_th, t_m, t_v, torch.tensor(g, dtype=torch.float32, device="cuda"), t,
                     1e-2, 0.9, 0.999, 1e-8)
        o_th, o_m, o_v = omlp.adam(o_th, o_m, o_v, g, t, 1e-2, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    assert rel_l2(t_th.double().cpu().numpy() - th, o_th - th) <= 1e-5
