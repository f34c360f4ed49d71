"""Host logic of the least-squares RTM driver (no GPU).

fwi.LSRTM runs conjugate gradients on the normal equations (CGLS) with Born
modelling as the operator L and the adjoint gradient as L^T. Here a dense
matrix with its exact transpose stands in for both, so the iteration itself
is checked against linear algebra: after as many iterations as unknowns it
reaches the least-squares solution numpy's lstsq gives (exact arithmetic
reaches it then; float64 stays within 1e-8 for a well-conditioned matrix),
the data residual it reports never rises, and each iteration applies L once
and L^T once (the latter after a saving forward, as the solver requires).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


class MatrixPlan:
    """Plan stand-in: born(v0, dv, w) = A dv, backward(r) = A^T r after a
    saving forward; born() leaves no saved state, as the solver's does."""

    def __init__(self, A, shape):
        self.A = torch.as_tensor(A, dtype=torch.float64)
        self.shape = shape
        self.saved = False
        self.calls = {"born": 0, "forward": 0, "backward": 0}

    def born(self, v0, dv, wavelet):
        self.calls["born"] += 1
        self.saved = False
        return self.A @ dv.reshape(-1)

    def forward(self, v0, wavelet, save=False):
        self.calls["forward"] += 1
        self.saved = save

    def backward(self, r):
        assert self.saved, "backward() without a saving forward"
        self.calls["backward"] += 1
        return (self.A.T @ r.reshape(-1)).reshape((1,) + self.shape)


def _system(seed, m=30, shape=(3, 4)):
    rng = np.random.default_rng(seed)
    n = shape[0] * shape[1]
    # well conditioned: orthonormal columns scaled by singular values in [1, 3]
    q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    v, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = q @ np.diag(np.linspace(1.0, 3.0, n)) @ v.T
    return A, rng


def _driver(A, shape, d):
    from paper_2604_14189_amd import fwi
    plan = MatrixPlan(A, shape)
    v0 = torch.zeros(shape, dtype=torch.float64)
    ls = fwi.LSRTM(plan, v0, None, torch.as_tensor(d, dtype=torch.float64))
    return plan, ls


def test_cgls_reaches_the_least_squares_solution():
    shape = (3, 4)
    A, rng = _system(1, shape=shape)
    d = rng.standard_normal(A.shape[0])  # not in the range of A
    plan, ls = _driver(A, shape, d)
    n = A.shape[1]
    for _ in range(n):
        ls.step()
    x_ls = np.linalg.lstsq(A, d, rcond=None)[0]
    x = ls.perturbation.numpy().reshape(-1)
    assert np.linalg.norm(x - x_ls) <= 1e-8 * np.linalg.norm(x_ls)
    h = ls.history
    assert len(h) == n + 1 and h[0] == pytest.approx(np.linalg.norm(d))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(h, h[1:]))
    assert h[-1] == pytest.approx(np.linalg.norm(A @ x_ls - d), rel=1e-8)
    assert plan.calls == {"born": n, "forward": n + 1, "backward": n + 1}


def test_cgls_recovers_a_perturbation_from_consistent_data():
    shape = (3, 4)
    A, rng = _system(2, shape=shape)
    x_true = rng.standard_normal(A.shape[1])
    plan, ls = _driver(A, shape, A @ x_true)
    for _ in range(A.shape[1]):
        ls.step()
    x = ls.perturbation.numpy().reshape(-1)
    assert np.linalg.norm(x - x_true) <= 1e-8 * np.linalg.norm(x_true)
    assert ls.history[-1] <= 1e-8 * ls.history[0]


def test_cgls_zero_data_stays_at_zero():
    shape = (2, 3)
    A, _ = _system(3, m=10, shape=shape)
    plan, ls = _driver(A, shape, np.zeros(A.shape[0]))
    assert ls.step() == 0.0
    assert not torch.any(ls.perturbation)
    assert plan.calls["born"] == 1 and plan.calls["backward"] == 1
