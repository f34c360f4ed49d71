"""Closed-form references used to pin the oracle (independent of it).

2-D acoustic Green's function convolved with a Ricker wavelet. For
p_tt = v^2 (p_xx + p_zz) + s(t) delta(x) (the continuous limit of Eq. 2 with a
point source of amplitude s), the causal solution at distance r is

    p(r, t) = 1 / (2 pi v^2) * integral_0^{acosh(v t / r)} s(t - (r / v) cosh u) du,

obtained from G = H(v t - r) / (2 pi v sqrt(v^2 t^2 - r^2)) with the substitution
v tau = r cosh u, which removes the square-root singularity at the wavefront.

For an explosive source in a homogeneous elastic full space the displacement
potential obeys the same scalar equation with speed vp, and the particle
velocity is the gradient of the potential's time derivative; the elastic pin
builds it from the same integral (see elastic_explosive_velocity).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad


def _ricker(t, f0, delay):
    a = (math.pi * f0 * (t - delay)) ** 2
    return (1.0 - 2.0 * a) * math.exp(-a)


def green2d_ricker(r: float, t: float, v: float, f0: float, delay: float | None = None,
                   deriv: int = 0) -> float:
    """(G * s)(r, t) for a Ricker s; deriv=1 uses s' instead of s."""
    if delay is None:
        delay = 1.5 / f0
    if v * t <= r:
        return 0.0
    umax = math.acosh(v * t / r)
    if deriv == 0:
        s = lambda tt: _ricker(tt, f0, delay)
    else:
        def s(tt):
            a = math.pi * f0 * (tt - delay)
            # d/dt [(1 - 2 a^2) e^{-a^2}] = pi f0 * (-6 a + 4 a^3) e^{-a^2}
            return math.pi * f0 * (-6.0 * a + 4.0 * a ** 3) * math.exp(-a * a)
    val, _ = quad(lambda u: s(t - r / v * math.cosh(u)), 0.0, umax, limit=400)
    return val / (2.0 * math.pi * v * v)


def acoustic_trace(r: float, times: np.ndarray, v: float, f0: float) -> np.ndarray:
    return np.array([green2d_ricker(r, float(t), v, f0) for t in times])
