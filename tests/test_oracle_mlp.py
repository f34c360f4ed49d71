"""Pins for the MLP velocity-model oracle (CPU): bfloat16 rounding against
torch's conversion, the network against torch.nn in float64 (forward and
autograd gradient), finite differences, special cases, and Adam's first step."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        # exact ties between two bf16 values: even mantissa wins
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0])])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def _torch_net(theta):
    p = [torch.tensor(a) for a in mlp.unpack(theta)]
    layers = []
    for l in range(mlp.DEPTH):
        lin = torch.nn.Linear(p[2 * l].shape[1], p[2 * l].shape[0]).double()
        lin.weight.data[:] = p[2 * l]
        lin.bias.data[:] = p[2 * l + 1]
        layers += [lin, torch.nn.ReLU()]
    last = torch.nn.Linear(mlp.WIDTH, 1).double()
    last.weight.data[0] = p[2 * mlp.DEPTH]
    last.bias.data[:] = p[2 * mlp.DEPTH + 1]
    return torch.nn.Sequential(*layers, last)


def test_forward_and_gradient_match_torch_nn():
    theta = mlp.init_params(3)
    theta[np.random.default_rng(1).integers(0, len(theta), 50)] += 0.3  # non-zero biases
    g = mlp.encode(synth.rff_frequencies(seed=2), 13, 7, emulate=False)
    v, cache = mlp.forward(theta, g, emulate=False)
    net = _torch_net(theta)
    x = torch.tensor(g)
    vt = 1500.0 + 3200.0 * torch.sigmoid(net(x)[:, 0])
    np.testing.assert_allclose(v, vt.detach().numpy(), rtol=1e-13)
    dv = np.random.default_rng(4).standard_normal(len(v))
    grad = mlp.backward(theta, cache, dv, emulate=False)
    (vt * torch.tensor(dv)).sum().backward()
    tg = []
    for l in range(mlp.DEPTH):
        tg += [net[2 * l].weight.grad.numpy().ravel(), net[2 * l].bias.grad.numpy().ravel()]
    tg += [net[-1].weight.grad.numpy().ravel(), net[-1].bias.grad.numpy().ravel()]
    np.testing.assert_allclose(grad, np.concatenate(tg), rtol=1e-10, atol=1e-12)


def test_gradient_finite_differences():
    theta = mlp.init_params(5)
    g = mlp.encode(synth.rff_frequencies(seed=6), 9, 5, emulate=False)
    dv = np.random.default_rng(7).standard_normal(45)
    _, cache = mlp.forward(theta, g, emulate=False)
    grad = mlp.backward(theta, cache, dv, emulate=False)
    # the output layer is smooth in its parameters (no ReLU kink can be crossed);
    # the whole network is pinned against torch.nn above
    d = np.zeros(len(theta))
    d[-257:] = np.random.default_rng(8).standard_normal(257)
    eps = 1e-5
    fp = np.sum(dv * mlp.forward(theta + eps * d, g, emulate=False)[0])
    fm = np.sum(dv * mlp.forward(theta - eps * d, g, emulate=False)[0])
    assert abs((fp - fm) / (2 * eps) - grad @ d) <= 1e-7 * abs(grad @ d)


def test_special_cases():
    n = mlp.n_params()
    assert n == 230657
    theta = np.zeros(n)
    theta[-1] = 0.7  # only the output bias
    g = mlp.encode(np.zeros((64, 2)), 4, 3)
    assert np.all(g[:, :64] == 1.0) and np.all(g[:, 64:] == 0.0)
    v, _ = mlp.forward(theta, g)
    np.testing.assert_allclose(v, 1500.0 + 3200.0 / (1.0 + np.exp(-0.7)), rtol=1e-15)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(9)
    theta = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    new, m, v = mlp.adam(theta, np.zeros(1000), np.zeros(1000), g, 1, lr=1e-3, eps=1e-12)
    np.testing.assert_allclose(new - theta, -1e-3 * np.sign(g), rtol=1e-6)


def test_encode_closed_form():
    # one frequency per axis fixes the orientation, the point order
    # (m = j nx + i) and the 2 pi: row 0 = (1, 0) gives cos / sin(2 pi i/(nx-1)),
    # row 1 = (0, 1/2) gives cos / sin(pi j/(nz-1)); the other rows are 0
    nx, nz = 5, 3
    B = np.zeros((64, 2))
    B[0] = (1.0, 0.0)
    B[1] = (0.0, 0.5)
    g = mlp.encode(B, nx, nz, emulate=False)
    assert g.shape == (nx * nz, 128)
    i = np.tile(np.arange(nx), nz)
    j = np.repeat(np.arange(nz), nx)
    cos_x = np.array([1.0, 0.0, -1.0, 0.0, 1.0])[i]
    sin_x = np.array([0.0, 1.0, 0.0, -1.0, 0.0])[i]
    cos_z = np.array([1.0, 0.0, -1.0])[j]
    sin_z = np.array([0.0, 1.0, 0.0])[j]
    np.testing.assert_allclose(g[:, 0], cos_x, atol=1e-15)
    np.testing.assert_allclose(g[:, 64], sin_x, atol=1e-15)
    np.testing.assert_allclose(g[:, 1], cos_z, atol=1e-15)
    np.testing.assert_allclose(g[:, 65], sin_z, atol=1e-15)
    assert np.all(g[:, 2:64] == 1.0) and np.all(g[:, 66:] == 0.0)
    # the emulating encoder stores the same features rounded to bf16
    assert np.array_equal(mlp.encode(B, nx, nz), mlp.bf16(g))


def test_gradient_on_decisions_matches_oracle():
    # the test-side gradient from stored decisions (used by the full-size GPU
    # test) equals the oracle's backward when given the oracle's own decisions
    from tests.mlp_decisions import gradient_on_decisions
    theta = mlp.init_params(11)
    theta[np.random.default_rng(12).integers(0, len(theta), 80)] += 0.2
    g = mlp.encode(synth.rff_frequencies(seed=13), 17, 9)
    v, cache = mlp.forward(theta, g)
    dv = np.random.default_rng(14).standard_normal(len(v))
    ref, dzs = mlp.backward(theta, cache, dv, return_dz=True)
    got = gradient_on_decisions(theta, cache["hs"], cache["s"], dzs, dv)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)
