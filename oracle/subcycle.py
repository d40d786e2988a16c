"""CPU reference of the sub-cycled explicit comparison baseline.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The baseline is not the
method: it replaces the analytic solution of the windowed chain (Sec. 3) by
nsub classical fourth-order Runge-Kutta substeps of dt/nsub on
dN/dt = A N (Eq. (3) restricted to the window, top absorbing), with the
rates of Eq. (1) frozen over the step and the window shift at the start of
the step as in the analytic step.  Sub-cycled time stepping of the rate
equations is what the paper's exact solution avoids (Sec. 1).
"""
from __future__ import annotations

import numpy as np

from .mlp import window_shift


def chain_deriv(x, y):
    """A y for the windowed chain: x[w][n] (rates times dt), y[w+1][n]."""
    d = np.zeros_like(y)
    w = x.shape[0]
    d[0] = -x[0] * y[0]
    for j in range(1, w):
        d[j] = x[j - 1] * y[j - 1] - x[j] * y[j]
    d[w] = x[w - 1] * y[w - 1]
    return d


def rk4(x, y, nsub):
    """nsub RK4 steps of size 1/nsub (time in units of dt)."""
    h = 1.0 / nsub
    y = np.array(y, np.float64)
    for _ in range(nsub):
        k1 = chain_deriv(x, y)
        k2 = chain_deriv(x, y + 0.5 * h * k1)
        k3 = chain_deriv(x, y + 0.5 * h * k2)
        k4 = chain_deriv(x, y + h * k3)
        y = y + (h / 6.0) * (k1 + 2.0 * (k2 + k3) + k4)
    return y


def subcycle_step(orc, spec, E, dt, pops, lo, w, eps, nsub):
    """The baseline step for every cell (compact layout [w+1][n]); returns
    (pops, lo) and the window rates times dt x[w][n]."""
    Z = spec.Z
    E = np.abs(np.asarray(E, np.float64))
    N, p = window_shift(pops, lo, Z, eps)
    Wall = orc.rates(spec, np.where(np.isfinite(E), E, 0.0))  # [Z][n], 1/s
    n = E.size
    x = np.zeros((w, n))
    for s in range(w):
        k = p + s
        ok = k < Z
        x[s, ok] = Wall[k[ok], np.nonzero(ok)[0]] * dt
    y = rk4(x, N, nsub)
    bad = ~np.isfinite(E) & (p < Z)
    y[:, bad] = np.nan
    for s in range(w + 1):
        y[s, p + s > Z] = 0.0
    return y, p.astype(np.uint8), x
