"""Host-only checks of the C-ABI boundary: the built library loads without a
GPU, exports exactly the entry points include/sweep.h declares, and its
argument validation, which runs before any HIP call, rejects bad problems."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sweep.h")
LIB = os.path.join(ROOT, "paper_2604_14189_amd", "libsweep.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sweep_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsweep.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("sweep_plan_create", "sweep_forward", "sweep_backward", "sweep_batch_create",
                 "sweep_batch_forward", "sweep_batch_backward", "sweep_l2_misfit",
                 "sweep_mlp_forward", "sweep_mlp_backward", "sweep_adam_step",
                 "sweep_plan_autotune", "sweep_last_error"):
        assert core in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(shutil.which("nm") is None, reason="nm not available")
def test_no_undeclared_c_exports():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines()
                       if ln.split() and ln.split()[-1].startswith("sweep_")})
    assert exported == _declared()


def test_argument_validation_needs_no_gpu(lib):
    from paper_2604_14189_amd._lib import Problem, EINVAL, ECFL
    lib.sweep_plan_create.restype = ctypes.c_int
    lib.sweep_plan_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.sweep_last_error.restype = ctypes.c_char_p
    src = (ctypes.c_int32 * 2)(5, 5)
    rec = (ctypes.c_int32 * 2)(7, 5)

    def create(**kw):
        pb = dict(physics=0, nx=32, nz=32, pml=10, free_surface=0, h=10.0, dt=1e-3, nt=10,
                  pml_vmax=2000.0, pml_f0=10.0, pml_R=1e-3, ckpt_every=5, nshots=1, nrec=1)
        pb.update(kw)
        out = ctypes.c_void_p()
        rc = lib.sweep_plan_create(None, ctypes.byref(Problem(**pb)), src, rec, ctypes.byref(out))
        return rc, lib.sweep_last_error().decode()

    rc, msg = create(nt=0)
    assert rc == EINVAL and msg
    rc, msg = create(nx=-3)
    assert rc == EINVAL
    # Courant number vmax dt / h above the 8th-order leapfrog limit
    rc, msg = create(pml_vmax=6000.0)
    assert rc == ECFL and msg
    rc, msg = create(physics=7)
    assert rc == EINVAL


def test_stored_segments_workspace_accounting(lib):
    """keep_b adds exactly its stored B'^n segments to the backward workspace
    and drops their checkpoint slots (host-side layout, no GPU): per stored
    segment ckpt * nshots * NX * NZ floats, less two fields per shot and the
    C-PML memory variables of a checkpoint, up to the carve alignment; with
    any stored, the recomputation's own B'^n buffer (one segment) goes, since
    it reuses the first stored segment's slots; never more segments than the
    run has."""
    import paper_2604_14189_amd as sw
    nx, nz, pml, nt, k, ns = 70, 40, 10, 100, 17, 3
    src = [[5 + 20 * s, 3] for s in range(ns)]
    rec = [[[x, 2] for x in range(0, nx, 7)] for _ in range(ns)]
    plan = sw.Plan(nx=nx, nz=nz, h=10.0, dt=1e-3, nt=nt, pml=pml, src_xz=src, rec_xz=rec,
                   pml_vmax=3000.0, pml_f0=10.0, ckpt_every=k)
    base = plan.workspace_bytes(True)
    fwd = plan.workspace_bytes(False)
    NX, NZ = nx + 2 * pml, nz + 2 * pml
    seg = k * ns * NX * NZ * 4
    # checkpoint slot: p^n and p^(n-1) per shot, and psi/zeta of the x strips
    # ([NZ][2P]) and z strips ([2P][NX]) per shot
    slot = (2 * ns * NX * NZ + 2 * ns * NZ * 2 * pml + 2 * ns * 2 * pml * NX) * 4
    nseg = -(-nt // k)
    for keep in (1, 2, nseg, nseg + 5):
        plan.set_tuning(keep_b=keep)
        extra = plan.workspace_bytes(True) - base
        want = min(keep, nseg) * (seg - slot) - seg
        assert abs(extra - want) < 4096, (keep, extra, want)
        assert plan.workspace_bytes(False) == fwd
        assert plan.tuning["keep_b"] == keep
    with pytest.raises(sw.SweepError):
        plan.set_tuning(keep_b=-1)


def test_batch_stored_segments_workspace_accounting(lib):
    """A batch lays out each plan with that plan's stored segments: its
    backward workspace grows by exactly what each plan's own grows by, and
    its forward part is unchanged (host-side layout, no GPU)."""
    import paper_2604_14189_amd as sw
    from tests.helpers import random_case
    cases = [random_case(51, nx=300, nz=200, nt=101, nshots=2, nrec=6, ckpt=17),
             random_case(52, nx=260, nz=150, nt=76, nshots=3, nrec=5, ckpt=25),
             random_case(53, nx=120, nz=90, nt=90, nshots=2, nrec=4, ckpt=50)]
    plans = [c.plan() for c in cases]
    base, fbase = sw.Batch(plans).workspace_bytes(True), sw.Batch(plans).workspace_bytes(False)
    want = 0
    for p, keep in zip(plans, (2, 99, 0)):
        w0 = p.workspace_bytes(True)
        p.set_tuning(keep_b=keep)
        want += p.workspace_bytes(True) - w0
    b = sw.Batch(plans)
    assert want > 0
    assert b.workspace_bytes(True) - base == want
    assert b.workspace_bytes(False) == fbase


def test_elastic_stored_segments_workspace_accounting(lib):
    """Elastic plans store the five trace planes of each stored segment and
    need no checkpoint for it: per stored segment ckpt * 5 * nshots * NX * NZ
    floats more backward workspace, less one 13-plane state checkpoint
    (5 fields and 8 memory variables per shot), the forward part unchanged
    (host-side layout, no GPU)."""
    from tests.helpers import random_el_case
    c = random_el_case(5, fs=1, nt=300, ckpt=23)
    p = c.plan()
    NX, NZ = p.padded()
    w0, f0 = p.workspace_bytes(True), p.workspace_bytes(False)
    nseg = -(-c.nt // c.ckpt)
    for keep in (2, nseg, nseg + 3):
        p.set_tuning(keep_b=keep)
        want = min(keep, nseg) * (c.ckpt * 5 - 13) * c.nshots * NX * NZ * 4
        assert abs(p.workspace_bytes(True) - w0 - want) < 4096, keep
        assert p.workspace_bytes(False) == f0


def test_vti_stored_segments_workspace_accounting(lib):
    """VTI plans store the three trace planes of each stored segment and need
    no checkpoint for it: per stored segment ckpt * 3 * nshots * NX * NZ
    floats more backward workspace, less one checkpoint slot (P^n, P^{n-1},
    G^n, G^{n-1} in float64 and the four C-PML memory-variable strips), the
    forward part unchanged (host-side layout, no GPU)."""
    import paper_2604_14189_amd as sw
    from tests.helpers import random_case
    c = random_case(8, nx=150, nz=77, pml=10, nt=240, nshots=3, nrec=9, ckpt=17)
    p = sw.Plan(nx=c.nx, nz=c.nz, h=c.h, dt=c.dt, nt=c.nt, pml=c.pml, src_xz=c.src,
                rec_xz=c.rec, pml_vmax=c.vmax * 1.3, pml_f0=c.f0, ckpt_every=c.ckpt,
                physics=sw.VTI)
    NX, NZ = p.padded()
    P = c.pml
    w0, f0 = p.workspace_bytes(True), p.workspace_bytes(False)
    nseg = -(-c.nt // c.ckpt)
    slot = 8 * c.nshots * NX * NZ + c.nshots * (2 * NZ * 2 * P + 2 * 2 * P * NX)
    for keep in (2, nseg, nseg + 3):
        p.set_tuning(keep_b=keep)
        want = min(keep, nseg) * (c.ckpt * 3 * c.nshots * NX * NZ - slot) * 4
        assert abs(p.workspace_bytes(True) - w0 - want) < 4096, keep
        assert p.workspace_bytes(False) == f0


def test_batch_membership_and_tuning_checks(lib):
    """Batches hold any number of distinct plans of one tiling (launches carry
    up to eight plans each), and refuse (before any device call) a forward
    whose member changed its tiling, and a backward after a member's tuning
    changed since the saving forward (host-side checks, no GPU)."""
    import paper_2604_14189_amd as sw
    from tests.helpers import random_case
    plans = [random_case(70 + q, nx=90 + 7 * q, nz=60, nt=40, nshots=1, nrec=3, ckpt=20).plan()
             for q in range(12)]
    b = sw.Batch(plans)
    assert b.workspace_bytes(True) >= sum(p.workspace_bytes(True) for p in plans)
    with pytest.raises(sw.SweepError) as e:
        sw.Batch([plans[0], plans[1], plans[0]])
    assert e.value.rc == sw._lib.EINVAL
    plans[3].set_tuning(rz=4)
    with pytest.raises(sw.SweepError):
        sw.Batch(plans)
    # the batch was made for rz 8: its forward refuses the changed member
    fake = ctypes.c_void_p(256)
    arr = (ctypes.c_void_p * len(plans))(*([256] * len(plans)))
    L = sw.lib()
    rc = L.sweep_batch_forward(b._h, arr, arr, arr, fake, 1 << 40, 1, None)
    assert rc == sw._lib.EINVAL and b"rz" in L.sweep_last_error()
    rc = L.sweep_batch_backward(b._h, arr, arr, fake, 1 << 40, None)
    assert rc == sw._lib.ESTATE


def test_set_tuning_keeps_unnamed_fields(lib):
    from tests.helpers import random_case
    p = random_case(3, nt=40).plan()
    p.set_tuning(rz=4, pml_rz=2, tblock=1)
    p.set_tuning(keep_b=2)
    t = p.tuning
    assert (t["rz"], t["pml_rz"], t["tblock"], t["keep_b"]) == (4, 2, 1, 2)
    p.set_tuning(rz=8)
    assert (p.tuning["rz"], p.tuning["pml_rz"], p.tuning["keep_b"]) == (8, 4, 2)


def test_context_outside_device_range_is_an_error(lib):
    import paper_2604_14189_amd as sw
    h = ctypes.c_void_p()
    rc = sw.lib().sweep_ctx_create(ctypes.byref(h), 1 << 20)
    assert rc in (sw._lib.EINVAL, sw._lib.EHIP) and not h.value
    assert sw.lib().sweep_last_error()


def test_autotune_cache_lines_are_json(lib, tmp_path):
    """A cached search (one JSON object per line) is taken without timing
    anything: the plan gets the line's choice; lines of other shapes, modes
    or malformed fields are skipped (host-side: no device call is made)."""
    import json
    import torch
    import paper_2604_14189_amd as sw
    from tests.helpers import random_case
    c = random_case(5, nx=140, nz=90, nt=30, nshots=2, nrec=3)
    p = c.plan()
    NX, NZ = p.padded()
    arch = (torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
            if torch.cuda.is_available() else "unknown")
    key = {"arch": arch, "physics": "acoustic", "mode": "plan-forward",
           "shapes": f"{NX}x{NZ}x{c.nshots}x{c.pml}"}
    lines = [dict(key, shapes=f"{NX}x{NZ}x{c.nshots}x{c.pml + 1}", rz=1, pml_rz=1, tblock=1),
             dict(key, mode="batch-forward", rz=1, pml_rz=1, tblock=1),
             dict(key, rz=3, pml_rz=1, tblock=1),
             dict(key, rz=2, pml_rz=2, tblock=1, us_per_step=12.5),
             dict(key, rz=4, pml_rz=4, tblock=2, us_per_step=10.0)]
    path = tmp_path / "tune.jsonl"
    path.write_text("".join(json.dumps(x, separators=(",", ":")) + "\n" for x in lines))
    L = sw.lib()
    fake = ctypes.c_void_p(256)
    rz = ctypes.c_int()
    rc = L.sweep_plan_autotune(p._h, fake, fake, fake, 1 << 40, 5, str(path).encode(), None,
                               ctypes.byref(rz))
    assert rc == 0, L.sweep_last_error()
    assert rz.value == 2
    assert (p.tuning["rz"], p.tuning["pml_rz"], p.tuning["tblock"]) == (2, 2, 1)
