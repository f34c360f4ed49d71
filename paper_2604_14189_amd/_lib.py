"""ctypes binding to libsweep.so (argument marshalling only).

Every step of the wave-equation path runs in the library's HIP kernels; this
module only checks shapes, passes device pointers and the current HIP stream,
and raises on a non-zero status. If the library has not been built the import
of any entry point fails loudly: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsweep.so")

OK, EINVAL, EHIP, ENOMEM, ECFL, ESTATE = 0, -1, -2, -3, -4, -5
ACOUSTIC, ELASTIC, ACOUSTIC_VD, VTI = 0, 1, 2, 3


class SweepError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"libsweep error {rc}: {msg}")
        self.rc = rc


class Problem(ctypes.Structure):
    """Mirror of sweep_problem (include/sweep.h)."""
    _fields_ = [
        ("physics", ctypes.c_int), ("nx", ctypes.c_int), ("nz", ctypes.c_int),
        ("pml", ctypes.c_int), ("free_surface", ctypes.c_int), ("h", ctypes.c_double),
        ("dt", ctypes.c_double), ("nt", ctypes.c_int), ("pml_vmax", ctypes.c_double),
        ("pml_f0", ctypes.c_double), ("pml_R", ctypes.c_double), ("ckpt_every", ctypes.c_int),
        ("nshots", ctypes.c_int), ("nrec", ctypes.c_int), ("nsrc", ctypes.c_int),
    ]


class Tuning(ctypes.Structure):
    """Mirror of sweep_tuning."""
    _fields_ = [("rz", ctypes.c_int), ("pml_rz", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("tblock", ctypes.c_int),
                ("keep_b", ctypes.c_int)]


_lib = None

_SIGS = {
    "sweep_last_error": (ctypes.c_char_p, []),
    "sweep_ctx_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "sweep_ctx_destroy": (None, [ctypes.c_void_p]),
    "sweep_ctx_device": (ctypes.c_int, [ctypes.c_void_p]),
    "sweep_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Problem),
                                         ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "sweep_plan_destroy": (None, [ctypes.c_void_p]),
    "sweep_plan_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sweep_plan_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sweep_plan_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int]),
    "sweep_plan_padded": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)]),
    "sweep_plan_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]),
    "sweep_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_int, ctypes.c_void_p]),
    "sweep_forward_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "sweep_born_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "sweep_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "sweep_plan_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sweep_plan_graph_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "sweep_plan_kernel_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_double)]),
    "sweep_plan_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                           ctypes.c_char_p, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_int)]),
    "sweep_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "sweep_batch_destroy": (None, [ctypes.c_void_p]),
    "sweep_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sweep_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int]),
    "sweep_batch_graph_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "sweep_batch_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]),
    "sweep_batch_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_void_p]),
    "sweep_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_char_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_int)]),
    "sweep_l2_misfit_scratch_bytes": (ctypes.c_size_t, [ctypes.c_size_t]),
    "sweep_l2_misfit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_void_p]),
}


def lib():
    """Load libsweep.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} not found: build it with `python -m paper_2604_14189_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if hasattr(L, name):
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
        _lib = L
    return _lib


_contexts = {}


def context(device_index: int) -> ctypes.c_void_p:
    """The library context of HIP device `device_index` (created once, kept
    for the life of the process; plans and batches made with it run on that
    device)."""
    h = _contexts.get(device_index)
    if h is None:
        h = ctypes.c_void_p()
        check(lib().sweep_ctx_create(ctypes.byref(h), int(device_index)))
        _contexts[device_index] = h
    return h


def check(rc: int):
    if rc != OK:
        msg = lib().sweep_last_error()
        raise SweepError(rc, msg.decode() if msg else "")
