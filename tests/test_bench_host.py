"""Host logic of the benchmark (no GPU): how many checkpoint segments it
stores for a plan, and its refusal of more than one GPU.

The workspace sizes come from the C library's host-side layout; the device
calls (free memory, allocation) are stand-ins, so the sizing and the
step-down after an allocation failure are checked exactly.
"""
import os
import subprocess
import sys
import types

import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GiB = 1 << 30


@pytest.fixture(scope="module")
def bench():
    import paper_2604_14189_amd as sw
    sw.lib()  # the plan's host-side layout comes from the built library
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def _plan(nshots=64):
    import synth
    from tests.helpers import case_from_workload
    w = synth.workload("layered1000x300")
    p = case_from_workload(w, shots=list(range(nshots))).plan()
    p.set_tuning(rz=8, pml_rz=4, tblock=2)
    return w, p


def _fake_torch(free_bytes):
    cuda = types.SimpleNamespace(mem_get_info=lambda: (free_bytes, free_bytes),
                                 empty_cache=lambda: None, synchronize=lambda: None,
                                 memory_reserved=lambda: 0, memory_allocated=lambda: 0)
    return types.SimpleNamespace(cuda=cuda, OutOfMemoryError=torch.OutOfMemoryError)


def test_keep_b_fills_free_memory(bench):
    w, plan = _plan()
    nseg = -(-w.nt // w.ckpt_every)
    sizes = {}
    for k in range(nseg + 1):
        plan.set_tuning(rz=8, pml_rz=4, tblock=2, keep_b=k)
        sizes[k] = plan.workspace_bytes(True)
    plan.set_tuning(rz=8, pml_rz=4, tblock=2)
    plan.reserve_workspace = lambda fb=True: plan.workspace_bytes(fb)
    free = 287 * GiB
    keep = bench.fit_keep_b(_fake_torch(free), plan, w.nt, w.ckpt_every)
    # the largest count whose workspace leaves the 8 GiB reserve free
    assert keep == max(k for k in range(1, nseg + 1) if sizes[k] <= free - 8 * GiB)
    assert 0 < keep < nseg
    assert plan.tuning["keep_b"] == keep
    assert plan.workspace_bytes(True) <= free - 8 * GiB
    plan.set_tuning(rz=8, pml_rz=4, tblock=2, keep_b=keep + 1)
    assert plan.workspace_bytes(True) > free - 8 * GiB
    # a stored segment costs less than its planes: its checkpoint is dropped;
    # and the first one also takes over the recomputation's buffer
    net = sizes[nseg] - sizes[nseg - 1]
    assert net < w.ckpt_every * w.nshots * w.NX * w.NZ * 4
    assert sizes[1] < sizes[0]


def test_keep_b_caps_at_the_segment_count(bench):
    w, plan = _plan(nshots=8)
    plan.reserve_workspace = lambda fb=True: plan.workspace_bytes(fb)
    keep = bench.fit_keep_b(_fake_torch(287 * GiB), plan, w.nt, w.ckpt_every)
    assert keep == -(-w.nt // w.ckpt_every)


def test_keep_b_steps_down_on_allocation_failure(bench):
    w, plan = _plan()
    tried = []

    def reserve(fb=True):
        tried.append(plan.tuning["keep_b"])
        if len(tried) < 3:
            raise torch.OutOfMemoryError("stand-in")
        return plan.workspace_bytes(fb)

    plan.reserve_workspace = reserve
    keep = bench.fit_keep_b(_fake_torch(287 * GiB), plan, w.nt, w.ckpt_every)
    assert tried == [tried[0], tried[0] - 2, tried[0] - 4] and keep == tried[0] - 4
    assert plan.tuning["keep_b"] == keep


def test_keep_b_gives_up_at_zero(bench):
    w, plan = _plan()

    def reserve(fb=True):
        raise torch.OutOfMemoryError("stand-in")

    plan.reserve_workspace = reserve
    with pytest.raises(torch.OutOfMemoryError):
        bench.fit_keep_b(_fake_torch(40 * GiB), plan, w.nt, w.ckpt_every)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


class _FakeAlloc:
    """torch stand-in whose allocations fail above `limit` bytes."""

    def __init__(self, free_bytes, limit):
        self.OutOfMemoryError = torch.OutOfMemoryError
        self.uint8 = torch.uint8
        self.cuda = _fake_torch(free_bytes).cuda
        self.limit, self.tried = limit, []

    def empty(self, n, dtype=None, device=None):
        self.tried.append(n)
        if n > self.limit:
            raise torch.OutOfMemoryError("stand-in")
        return types.SimpleNamespace(numel=lambda: n)


def _batch():
    import paper_2604_14189_amd as sw
    import synth
    from tests.helpers import case_from_workload
    ws = synth.batched_workloads()
    plans = [case_from_workload(w).plan() for w in ws]
    return ws, plans, sw.Batch(plans), [-(-w.nt // w.ckpt_every) for w in ws]


def test_batch_keep_b_same_fraction_that_fits(bench):
    ws, plans, batch, nsegs = _batch()
    free = 280 * GiB
    t = _FakeAlloc(free, limit=free)
    keeps = bench.fit_batch_keep_b(t, batch, plans, nsegs)
    need = batch.workspace_bytes(True)
    assert need <= free - 8 * GiB and t.tried == [need]
    assert keeps == [p.tuning["keep_b"] for p in plans]
    assert all(0 < k < n for k, n in zip(keeps, nsegs))
    # one common fraction f (logged to 4 digits): each count is floor(f * nseg)
    f = bench.FIT_LOG[-1]["first_fraction"]
    assert all(abs(k - f * n) <= 1 for k, n in zip(keeps, nsegs))
    # a slightly larger fraction would not fit
    for p, n in zip(plans, nsegs):
        p.set_tuning(**dict(p.tuning, keep_b=int((f + 0.01) * n)))
    assert batch.workspace_bytes(True) > free - 8 * GiB


def test_batch_keep_b_all_when_it_fits(bench):
    ws, plans, batch, nsegs = _batch()
    keeps = bench.fit_batch_keep_b(_FakeAlloc(4096 * GiB, 4096 * GiB), batch, plans, nsegs)
    assert keeps == nsegs


def test_batch_keep_b_steps_down_on_allocation_failure(bench):
    ws, plans, batch, nsegs = _batch()
    free = 280 * GiB
    t = _FakeAlloc(free, limit=200 * GiB)
    keeps = bench.fit_batch_keep_b(t, batch, plans, nsegs)
    assert len(t.tried) > 1 and t.tried[-1] <= 200 * GiB < t.tried[0]
    assert batch.workspace_bytes(True) == t.tried[-1]
    assert bench.FIT_LOG[-1]["failed_tries"] == len(t.tried) - 1
    assert keeps == [p.tuning["keep_b"] for p in plans]
