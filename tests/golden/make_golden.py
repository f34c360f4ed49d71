"""Writes the stored oracle values used by the full-size parity test.

Calls only the FP64 oracle (oracle/) and the seeded input generators (synth);
nothing here touches the HIP library.

    python tests/golden/make_golden.py

layered1000x300_shot37.npz: shot 37 of the 1000x300 / 3000-step / 40-cell-pad
acoustic workload (64 shots, 1000 receivers at depth 5, 8 Hz Ricker). Stores
8 complete receiver traces and the model gradient for a band-limited seeded
residual on that shot (20 000 sampled cells plus the full gradient norm).

batch_uneven8_short.npz: the eight uneven batched workloads (grids 200x200 ...
1200x400, 16 ... 48 shots each, 40-cell pads) with their runs shortened to
125 ... 250 steps (the full 2000 ... 4000 spread divided by 16, so segments of
50 steps end ragged). For the middle shot of each model: 8 complete receiver
traces within 32 cells of the source and the model gradient for a band-limited seeded residual on that shot
(the 2000 cells of largest magnitude and 2000 random others, plus the
gradient norm).

elastic600x300_shot11.npz: shot 11 of the 600x300 / 4000-step elastic workload
(30-cell pad, free surface, 32 explosive 15 Hz shots, 600 two-component
receivers): 8 complete (vx, vz) traces and the (vp, vs, rho) gradient for a
band-limited seeded residual on that shot at 20 000 sampled cells.

vti1000x300_shot23.npz: shot 23 of the 1000x300 / 3000-step pseudo-acoustic
VTI workload (the layered benchmark's grid, shots and receivers; eta up to
0.12 below an isotropic top zone): 8 complete receiver traces and the
(vv, v, eta) gradient for a band-limited seeded residual on that shot at
20 000 sampled cells, with the norm of each gradient plane.

vd1000x300_shot41.npz: shot 41 of the 1000x300 / 3000-step layered workload
as a first-order variable-density acoustic problem (rho = 310 vp^0.25, the
elastic oracle with vs = 0, no free surface): 8 complete (vx, vz) traces and
the (vp, rho) gradient for a band-limited seeded residual on that shot at
20 000 sampled cells, with the norm of each gradient plane.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from synth.cases import case_from_workload, f32  # noqa: E402


def layered_shot37(path):
    w = synth.workload("layered1000x300")
    s = 37
    case = case_from_workload(w, shots=[s])
    pb = case.oracle_problem(oracle)
    resid = f32(synth.bandlimited_noise((1, w.nt, w.nrec), w.f0, w.dt, 37))
    t = time.time()
    g, _, d = oracle.ac_gradient(pb, case.v, case.src, case.wav, case.rec, resid,
                                 want_gathers=True)
    print("oracle gradient took %.1f s" % (time.time() - t), flush=True)
    trace_idx = np.linspace(0, w.nrec - 1, 8).round().astype(np.int64)
    cells = np.random.default_rng(37).choice(g.size, 20000, replace=False)
    np.savez_compressed(path, shot=s, trace_idx=trace_idx, traces=d[0][:, trace_idx],
                        grad_cells=cells, grad=g.ravel()[cells],
                        grad_norm=np.linalg.norm(g))


def elastic_shot11(path):
    from synth.cases import el_case_from_workload
    w = synth.workload("elastic600x300")
    s = 11
    case = el_case_from_workload(w, shots=[s])
    pb = case.oracle_problem(oracle)
    resid = f32(synth.bandlimited_noise((1, w.nt, w.nrec * 2), w.f0, w.dt, 11)
                .reshape(1, w.nt, w.nrec, 2))
    t = time.time()
    g, _, d = oracle.el_gradient(pb, case.model, case.src, case.wav, case.rec, resid,
                                 want_gathers=True)
    print("oracle elastic gradient took %.1f s" % (time.time() - t), flush=True)
    trace_idx = np.linspace(0, w.nrec - 1, 8).round().astype(np.int64)
    cells = np.random.default_rng(11).choice(g[0].size, 20000, replace=False)
    np.savez_compressed(path, shot=s, trace_idx=trace_idx, traces=d[0][:, trace_idx, :],
                        grad_cells=cells, grad=np.stack([g[c].ravel()[cells] for c in range(3)]))


def vti_shot23(path):
    w = synth.workload("vti1000x300")
    s = 23
    sl = slice(s, s + 1)
    src, rec, wav = w.sources()[sl], w.receivers()[sl], f32(w.wavelets()[sl])
    model = f32(w.true_model())
    pb = oracle.problem(w.nx, w.nz, w.pml, w.h, w.dt, w.nt, w.pml_vmax(), w.f0, w.pml_R,
                        nshots=1, nrec=w.nrec, ckpt_every=w.ckpt_every)
    resid = f32(synth.bandlimited_noise((1, w.nt, w.nrec), w.f0, w.dt, 23))
    t = time.time()
    g, _, d = oracle.vti_gradient(pb, model, src, wav, rec, resid, want_gathers=True)
    print("oracle VTI gradient took %.1f s" % (time.time() - t), flush=True)
    trace_idx = np.linspace(0, w.nrec - 1, 8).round().astype(np.int64)
    cells = np.random.default_rng(23).choice(g[0].size, 20000, replace=False)
    np.savez_compressed(path, shot=s, trace_idx=trace_idx, traces=d[0][:, trace_idx],
                        grad_cells=cells, grad=np.stack([g[c].ravel()[cells] for c in range(3)]),
                        grad_norm=np.array([np.linalg.norm(g[c]) for c in range(3)]))


def vd_shot41(path):
    """First-order variable-density acoustic: the elastic oracle with vs = 0."""
    w = synth.workload("layered1000x300")
    s = 41
    sl = slice(s, s + 1)
    vp = f32(w.true_model())
    rho = f32(310.0 * vp.astype(np.float64) ** 0.25)
    model = np.stack([vp, np.zeros_like(vp), rho])
    src, rec, wav = w.sources()[sl], w.receivers()[sl], f32(w.wavelets()[sl])
    pb = oracle.problem(w.nx, w.nz, w.pml, w.h, w.dt, w.nt, w.pml_vmax(), w.f0, w.pml_R,
                        nshots=1, nrec=w.nrec, ckpt_every=w.ckpt_every)
    resid = f32(synth.bandlimited_noise((1, w.nt, w.nrec * 2), w.f0, w.dt, 41)
                .reshape(1, w.nt, w.nrec, 2))
    t = time.time()
    g, _, d = oracle.el_gradient(pb, model, src, wav, rec, resid, want_gathers=True)
    print("oracle variable-density gradient took %.1f s" % (time.time() - t), flush=True)
    trace_idx = np.linspace(0, w.nrec - 1, 8).round().astype(np.int64)
    cells = np.random.default_rng(41).choice(g[0].size, 20000, replace=False)
    gvd = np.stack([g[0], g[2]])  # (vp, rho)
    np.savez_compressed(path, shot=s, trace_idx=trace_idx, traces=d[0][:, trace_idx, :],
                        grad_cells=cells, grad=np.stack([gvd[c].ravel()[cells] for c in range(2)]),
                        grad_norm=np.array([np.linalg.norm(gvd[c]) for c in range(2)]))


def batch_short_nt(m: int) -> int:
    """Shortened run of batched workload m (125 ... 250 steps)."""
    return 125 + int(round(125 * m / 7))


def batch_uneven8_short(path):
    out = {}
    t = time.time()
    for m, w in enumerate(synth.batched_workloads()):
        nt = batch_short_nt(m)
        s = w.nshots // 2
        case = case_from_workload(w.replace(nt=nt), shots=[s])
        pb = case.oracle_problem(oracle)
        resid = f32(synth.bandlimited_noise((1, nt, w.nrec), w.f0, w.dt, 100 + m))
        g, _, d = oracle.ac_gradient(pb, case.v, case.src, case.wav, case.rec, resid,
                                     want_gathers=True)
        # a short run reaches the receivers within about 30 cells of the
        # source (one receiver per column): the traces are taken there
        sx = int(case.src[0, 0])
        trace_idx = np.clip(sx + np.array([-32, -16, -8, -2, 0, 4, 12, 24]), 0,
                            w.nrec - 1).astype(np.int64)
        assert np.all(case.rec[0, trace_idx, 0] == case.src[0, 0] + trace_idx - sx)
        # a short run concentrates the gradient near the source and the
        # receivers: the cells of the 2000 largest oracle values carry the
        # comparison, 2000 random cells check the rest
        top = np.sort(np.argsort(np.abs(g.ravel()))[-2000:])
        rest = np.setdiff1d(np.arange(g.size), top)
        rand = np.sort(np.random.default_rng(200 + m).choice(rest, 2000, replace=False))
        out.update({f"m{m}_shot": s, f"m{m}_nt": nt, f"m{m}_trace_idx": trace_idx,
                    f"m{m}_traces": d[0][:, trace_idx], f"m{m}_top_cells": top,
                    f"m{m}_top": g.ravel()[top], f"m{m}_rand_cells": rand,
                    f"m{m}_rand": g.ravel()[rand], f"m{m}_grad_norm": np.linalg.norm(g)})
    print("oracle batch gradients took %.1f s" % (time.time() - t), flush=True)
    np.savez_compressed(path, **out)


if __name__ == "__main__":
    oracle.build(force=False)
    which = sys.argv[1:] or ["layered", "elastic", "batch", "vti", "vd"]
    if "layered" in which:
        layered_shot37(os.path.join(HERE, "layered1000x300_shot37.npz"))
    if "elastic" in which:
        elastic_shot11(os.path.join(HERE, "elastic600x300_shot11.npz"))
    if "batch" in which:
        batch_uneven8_short(os.path.join(HERE, "batch_uneven8_short.npz"))
    if "vti" in which:
        vti_shot23(os.path.join(HERE, "vti1000x300_shot23.npz"))
    if "vd" in which:
        vd_shot41(os.path.join(HERE, "vd1000x300_shot41.npz"))
