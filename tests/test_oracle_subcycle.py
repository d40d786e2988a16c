"""Pins of the sub-cycled RK4 comparison baseline's CPU reference: the
single-level closed form (the RK4 stability polynomial to the power nsub),
conservation, and fourth-order convergence to the exact step."""
import numpy as np

from oracle import subcycle
from paper_2202_10647_amd import workloads as wl


def test_single_level_closed_form(orc):
    Z = 7
    t = wl.synthetic_gas(Z)
    spec = orc.GasSpec(t.U, t.l, t.m)
    E = wl.loguniform_field(300, 10.0, 400.0, seed=1)
    dt = 1.3e-16
    N = np.zeros((2, E.size))
    N[0] = 1.0
    lo = np.zeros(E.size, np.uint8)
    for nsub in (1, 7, 40):
        y, p, x = subcycle.subcycle_step(orc, spec, E, dt, N, lo, 1, 0.0, nsub)
        z = x[0] / nsub
        R = 1 - z + z ** 2 / 2 - z ** 3 / 6 + z ** 4 / 24
        assert np.allclose(y[0], R ** nsub, rtol=1e-12, atol=1e-300)
        assert np.allclose(y[0] + y[1], 1.0, atol=1e-13)
    assert np.allclose(x[0], orc.rates(spec, E, 0, 1)[0] * dt, rtol=1e-15)


def test_conservation_and_fourth_order_convergence(orc):
    Z = 18
    t = wl.synthetic_gas(Z)
    spec = orc.GasSpec(t.U, t.l, t.m)
    w = 3
    comp, lo = wl.random_window_state(400, Z, w, seed=4)
    E = wl.loguniform_field(400, 10.0, 150.0, seed=5)
    dt = 1.3e-16
    exact, elo = orc.ionize_step(spec, E, dt, comp, lo, w, 1e-8)
    errs = []
    for nsub in (16, 32, 64):
        y, p, x = subcycle.subcycle_step(orc, spec, E, dt, comp, lo, w, 1e-8, nsub)
        assert np.array_equal(p, elo)
        assert np.allclose(y.sum(axis=0), comp.sum(axis=0), atol=1e-13)
        stable = (x.max(axis=0) / nsub) < 1.0
        errs.append(np.max(np.abs(y - exact)[:, stable]))
    assert x.max() > 1.0  # the inputs exercise real sub-cycling
    # fourth order: halving the substep divides the error by ~16
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs
