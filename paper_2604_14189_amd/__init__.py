"""MI355X (gfx950) implementation of the SWEEP hot path (arXiv 2604.14189).

The 2-D finite-difference time loop (acoustic Eq. 2 with C-PML; elastic Eq. 12
with C-PML and a free surface; first-order variable-density acoustic Eq. 1;
pseudo-acoustic VTI Eq. 5), its exact adjoint and the resulting FWI
gradients, in hand-written HIP kernels behind the C-ABI of include/sweep.h.
"""
from ._lib import SweepError, lib  # noqa: F401
from .propagator import (ACOUSTIC, ACOUSTIC_VD, ELASTIC, VTI, Batch, Plan,  # noqa: F401
                         WaveFn, l2_misfit)
