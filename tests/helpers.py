"""Shared helpers for the parity tests. The seeded cases come from
synth.cases (inputs only); this module adds the comparison measure."""
from __future__ import annotations

import numpy as np

from synth.cases import (Case, ElCase, case_from_workload, el_case_from_workload,  # noqa: F401
                         f32, random_case, random_el_case)


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
