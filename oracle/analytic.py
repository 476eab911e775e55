"""Closed-form references for the oracle's pins -- TEST INFRASTRUCTURE ONLY.

Homogeneous medium, constant density, point source f_p = s(t) delta(x) in eq. (1):
eliminating v gives  p_tt - c^2 lap p = s'(t) delta(x),  so p = G * s' with the free-space
Green's function of the scalar wave equation:
  2D:  G2(r, t) = H(t - r/c) / (2 pi c^2 sqrt(t^2 - r^2/c^2))
  3D:  G3(r, t) = delta(t - r/c) / (4 pi c^2 r)
The stepper adds dt*stf[n]/dV to p after the p update of step n, i.e. the source acts at
t = (n + 1/2) dt, so s(t) = w(t - dt/2) for stf[n] = w(n dt); dcal[n] samples t = (n+1) dt.
"""
from __future__ import annotations

import math

import numpy as np


def ricker(t: np.ndarray, fm: float, t0: float) -> np.ndarray:
    u = (math.pi * fm * (np.asarray(t, np.float64) - t0)) ** 2
    return (1.0 - 2.0 * u) * np.exp(-u)


def ricker_dot(t: np.ndarray, fm: float, t0: float) -> np.ndarray:
    """Time derivative of the Ricker wavelet: pi fm exp(-u^2) (4u^3 - 6u), u = pi fm (t-t0)."""
    u = math.pi * fm * (np.asarray(t, np.float64) - t0)
    return math.pi * fm * np.exp(-u * u) * (4.0 * u ** 3 - 6.0 * u)


def green2d_trace(r: float, c: float, t: np.ndarray, fm: float, t0: float, dt: float,
                  ntau: int = 200000) -> np.ndarray:
    """p(r, t) = int G2(r, tau) s'(t - tau) d tau with s(t) = w(t - dt/2).

    The kernel's square-root singularity is integrated exactly per bin,
    int_{a}^{b} G2 dtau = (arccosh(b c / r) - arccosh(a c / r)) / (2 pi c^2),
    and s' is taken at the bin midpoint."""
    tmax = float(np.max(t))
    ta = r / c
    edges = np.linspace(ta, max(tmax, ta) + 1e-12, ntau + 1)
    w = (np.arccosh(np.maximum(edges[1:] * c / r, 1.0))
         - np.arccosh(np.maximum(edges[:-1] * c / r, 1.0))) / (2.0 * math.pi * c * c)
    mid = 0.5 * (edges[1:] + edges[:-1])
    out = np.zeros(len(t))
    for k, tk in enumerate(t):
        m = mid < tk
        out[k] = np.sum(w[m] * ricker_dot(tk - mid[m] - 0.5 * dt, fm, t0))
    return out


def green3d_trace(r: float, c: float, t: np.ndarray, fm: float, t0: float, dt: float) -> np.ndarray:
    """p(r, t) = s'(t - r/c) / (4 pi c^2 r) with s(t) = w(t - dt/2)."""
    return ricker_dot(np.asarray(t) - r / c - 0.5 * dt, fm, t0) / (4.0 * math.pi * c * c * r)
