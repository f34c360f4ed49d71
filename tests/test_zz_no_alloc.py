"""GPU: the allocation-free forward (static per-GPU workspace) against the
forward with a caller workspace, called through the C ABI: two calls in a
row, the second on a smaller problem, each bit for bit equal; an elastic plan
too; a plan whose workspace does not fit is refused with an error."""
import ctypes

import numpy as np
import pytest

from tests.helpers import random_case, random_el_case

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


def _noalloc(sw, plan, model, wav):
    out = torch.full(plan.gathers_shape(), float("nan"), device="cuda")
    L = sw.lib()
    rc = L.sweep_forward_noalloc(plan._h, ctypes.c_void_p(model.data_ptr()),
                                 ctypes.c_void_p(wav.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.sweep_last_error()
    torch.cuda.synchronize()
    return out


def test_noalloc_forward_equals_workspace_forward(sw):
    big = random_case(61, nx=150, nz=77, nt=180, nshots=3, nrec=41)
    small = random_case(62, nx=96, nz=60, nt=120, nshots=2, nrec=17)
    for case in (big, small):
        plan = case.plan()
        assert plan.workspace_bytes(False) <= 32 << 20
        m, w = _dev(case.v)[None], _dev(case.wav)
        print("noalloc acoustic", case.nx, case.nz, case.nshots, flush=True)
        got = _noalloc(sw, plan, m, w)
        ref = case.plan().forward(m, w)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.any(ref != 0)


def test_noalloc_elastic_and_limit(sw):
    c = random_el_case(63, fs=1, nx=80, nz=50, nt=150, nshots=2, nrec=11)
    plan = c.plan()
    m, w = _dev(c.model), _dev(c.wav)
    print("noalloc elastic", flush=True)
    got = _noalloc(sw, plan, m, w)
    ref = c.plan().forward(m, w)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    # a forward workspace beyond 32 MiB is refused before any launch
    huge = random_case(64, nx=600, nz=400, nt=20, nshots=8, nrec=5).plan()
    assert huge.workspace_bytes(False) > 32 << 20
    out = torch.empty(huge.gathers_shape(), device="cuda")
    with pytest.raises(sw.SweepError) as e:
        huge.forward_noalloc(_dev(np.full((400, 600), 2000.0)), _dev(np.zeros((8, 20))), out)
    assert e.value.rc == sw._lib.EINVAL and "32" in str(e.value)
