"""Pins for encoded shots (source encoding, Sec. 1): several sources in one
simulation, each with its own wavelet. CPU only, FP64 oracle.

* the recurrence is linear in the sources: an encoded shot equals the sum of
  its sources simulated one by one (to rounding);
* one source per shot is the plain modelling, bit for bit;
* two sources on one cell act as one source with the summed wavelet;
* the model gradient of an encoded shot matches central differences.
"""
import numpy as np

import synth
from tests.helpers import random_case


def _encoded(seed, nsrc=3, nt=140):
    c = random_case(seed, nt=nt, nshots=2, nrec=11)
    rng = np.random.default_rng(seed)
    src = np.stack([np.stack([rng.integers(0, c.nx, nsrc), rng.integers(0, c.nz, nsrc)], 1)
                    for _ in range(c.nshots)]).astype(np.int32)
    signs = rng.choice([-1.0, 1.0], size=(c.nshots, nsrc))
    wav = np.stack([[signs[s, k] * synth.ricker(12.0 + 2 * k, nt, c.dt) for k in range(nsrc)]
                    for s in range(c.nshots)])
    return c, src, wav


def test_encoded_shot_is_the_sum_of_its_sources(orc):
    c, src, wav = _encoded(1)
    pb = c.oracle_problem(orc)
    d = orc.ac_forward_encoded(pb, c.v, src, wav, c.rec)
    parts = sum(orc.ac_forward(pb, c.v, src[:, k], wav[:, k], c.rec) for k in range(src.shape[1]))
    assert np.linalg.norm(d - parts) <= 1e-12 * np.linalg.norm(d)


def test_one_source_is_the_plain_modelling(orc):
    c = random_case(2, nt=120)
    pb = c.oracle_problem(orc)
    d0 = orc.ac_forward(pb, c.v, c.src, c.wav, c.rec)
    d1 = orc.ac_forward_encoded(pb, c.v, c.src[:, None], c.wav[:, None], c.rec)
    assert np.array_equal(d0, d1)


def test_coincident_sources_add(orc):
    c, src, wav = _encoded(3, nsrc=2)
    src[:, 1] = src[:, 0]
    pb = c.oracle_problem(orc)
    d = orc.ac_forward_encoded(pb, c.v, src, wav, c.rec)
    d1 = orc.ac_forward(pb, c.v, src[:, 0], wav[:, 0] + wav[:, 1], c.rec)
    assert np.linalg.norm(d - d1) <= 1e-12 * np.linalg.norm(d)


def test_encoded_gradient_matches_finite_differences(orc):
    nx = nz = 32
    c = random_case(4, nx=nx, nz=nz, pml=8, nt=150, nshots=1, nrec=32, ckpt=16)
    c.rec = np.stack([np.stack([np.arange(nx), np.full(nx, 2)], 1)]).astype(np.int32)
    src = np.array([[[6, 3], [16, 3], [26, 3]]], np.int32)
    wav = np.stack([[s * synth.ricker(25.0, c.nt, c.dt) for s in (1.0, -1.0, 1.0)]])
    pb = c.oracle_problem(orc)
    vt = c.v
    v0 = synth.smooth(vt, 3.0)
    dobs = orc.ac_forward_encoded(pb, vt, src, wav, c.rec)

    def J(v):
        return 0.5 * np.sum((orc.ac_forward_encoded(pb, v, src, wav, c.rec) - dobs) ** 2)

    r = orc.ac_forward_encoded(pb, v0, src, wav, c.rec) - dobs
    g = orc.ac_gradient_encoded(pb, v0, src, wav, c.rec, r)
    dv = np.random.default_rng(5).standard_normal((nz, nx)) * 20.0
    an = np.sum(g * dv)
    # the misfit is far from quadratic here (smooth start model): the central
    # difference converges as eps^2 to the adjoint value
    errs = []
    for eps in (1e-4, 1e-5):
        fd = (J(v0 + eps * dv) - J(v0 - eps * dv)) / (2 * eps)
        errs.append(abs(fd - an) / abs(an))
    assert errs[1] <= 1e-6, errs
    assert errs[0] / errs[1] > 50, errs
