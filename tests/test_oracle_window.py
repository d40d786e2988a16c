"""Pins of the oracle's locally-reduced window (Sec. 3, reduced system and
cut-off criterion after Eq. (9)) and its step driver."""
import numpy as np
import pytest

from paper_2202_10647_amd import workloads as wl

DT = 1.334e-16


def spec_of(orc, Z):
    g = wl.synthetic_gas(Z)
    return orc.GasSpec(g.U, g.l, g.m)


def test_shift_folds_residual_and_moves_window(orc):
    """E = 0 freezes the chain, so only the start-of-step shift acts."""
    spec = spec_of(orc, 7)
    pops = np.array([[1e-9, 5e-9, 0.2], [0.5, 0.3, 0.3], [0.5, 0.7, 0.5], [0.0, 0.0, 0.0]])
    lo = np.array([0, 2, 4], np.uint8)
    out, lo2 = orc.ionize_step(spec, np.zeros(3), DT, pops, lo, w=3, eps=1e-8)
    # cell 0: one shift, residual folded into level 1
    assert lo2[0] == 1
    assert out[:, 0].tolist() == [0.5 + 1e-9, 0.5, 0.0, 0.0]
    # cell 1: one shift (5e-9 < eps), then 0.3+5e-9 >= eps stops
    assert lo2[1] == 3 and out[0, 1] == 0.3 + 5e-9
    # cell 2: no shift
    assert lo2[2] == 4 and np.array_equal(out[:, 2], pops[:, 2])


def test_multiple_shifts_in_one_step(orc):
    spec = spec_of(orc, 7)
    pops = np.array([[1e-10], [2e-10], [3e-10], [1.0 - 6e-10]])
    out, lo2 = orc.ionize_step(spec, np.zeros(1), DT, pops, np.zeros(1, np.uint8), w=3, eps=1e-8)
    assert lo2[0] == 3
    assert out[0, 0] == pytest.approx(1.0, abs=1e-16)
    assert out[1:, 0].tolist() == [0.0, 0.0, 0.0]


def test_window_stops_at_Z(orc):
    spec = spec_of(orc, 7)
    # all mass in level 7 = Z: window [7, 7], nothing evolves
    pops = np.array([[1.0], [0.0], [0.0], [0.0]])
    out, lo2 = orc.ionize_step(spec, np.full(1, 3000.0), DT, pops, np.full(1, 7, np.uint8), w=3, eps=1e-8)
    assert lo2[0] == 7 and out[:, 0].tolist() == [1.0, 0.0, 0.0, 0.0]
    # lo above Z is read as Z
    out, lo2 = orc.ionize_step(spec, np.full(1, 3000.0), DT, pops, np.full(1, 200, np.uint8), w=3, eps=1e-8)
    assert lo2[0] == 7


def test_window_top_clipped_at_Z(orc):
    """lo + w > Z: the window is [lo, Z] and level Z absorbs."""
    spec = spec_of(orc, 7)
    E = np.array([900.0])
    pops = np.array([[0.6], [0.4], [0.0], [0.0]])
    out, lo2 = orc.ionize_step(spec, E, DT, pops, np.full(1, 6, np.uint8), w=3, eps=0.0)
    W = orc.rates(spec, E, k0=6, nk=1)
    ref = orc.chain_advance(W, DT, np.array([[0.6], [0.4]]))
    assert out[:2, 0] == pytest.approx(ref[:, 0], abs=1e-16)
    assert out[2:, 0].tolist() == [0.0, 0.0]


@pytest.mark.parametrize("Z,w", [(7, 7), (7, 4), (18, 3)])
def test_window_equals_full_chain_when_it_covers_the_rest(orc, Z, w):
    """w >= Z - lo: the reduced system is the full system of Eq. (3) (exact)."""
    spec = spec_of(orc, Z)
    rng = np.random.default_rng(Z + w)
    n = 300
    lo = rng.integers(max(0, Z - w), Z + 1, n).astype(np.uint8)
    E = wl.loguniform_field(n, 10, 3000, 11)
    full = rng.random((Z + 1, n))
    full[np.arange(Z + 1)[:, None] < lo[None, :]] = 0.0
    full /= full.sum(axis=0)
    comp = np.zeros((w + 1, n))
    for c in range(n):
        k = np.arange(lo[c], Z + 1)
        comp[k - lo[c], c] = full[k, c]
    outc, loc = orc.ionize_step(spec, E, DT, comp, lo, w=w, eps=0.0, layout=0)
    outf, lof = orc.ionize_step(spec, E, DT, full, lo, w=Z, eps=0.0, layout=1)
    # the same chain solved as a general matrix exponential, level by level
    for c in range(0, n, 37):
        k = np.arange(lo[c], Z + 1)
        W = orc.rates(spec, [E[c]], k0=int(lo[c]), nk=Z - int(lo[c])) if lo[c] < Z else np.zeros((0, 1))
        A = np.zeros((k.size, k.size))
        for i in range(k.size - 1):
            A[i, i] = -W[i, 0] * DT
            A[i + 1, i] = W[i, 0] * DT
        ref = orc.expm(A) @ full[k, c]
        assert np.max(np.abs(outf[k, c] - ref)) < 1e-15
    for c in range(n):
        k = np.arange(lo[c], Z + 1)
        assert np.max(np.abs(outc[k - lo[c], c] - outf[k, c])) < 1e-15
    assert np.array_equal(loc, lof)


def test_compact_and_full_layouts_agree(orc):
    """Under the fold rule levels outside the window stay zero, so the compact
    and full layouts hold the same state after any step."""
    Z, w = 18, 3
    spec = spec_of(orc, Z)
    n = 400
    comp, lo = wl.random_window_state(n, Z, w, seed=3)
    full = np.zeros((Z + 1, n))
    for c in range(n):
        for s in range(w + 1):
            if lo[c] + s <= Z:
                full[lo[c] + s, c] = comp[s, c]
    E = wl.loguniform_field(n, 10, 5000, 4)
    oc, lc = orc.ionize_step(spec, E, DT, comp, lo, w=w, eps=1e-8, layout=0)
    of, lf = orc.ionize_step(spec, E, DT, full, lo, w=w, eps=1e-8, layout=1)
    assert np.array_equal(lc, lf)
    for c in range(n):
        k = np.arange(lc[c], min(lc[c] + w, Z) + 1)
        assert np.array_equal(oc[k - lc[c], c], of[k, c])
        mask = np.ones(Z + 1, bool)
        mask[k] = False
        assert np.all(of[mask, c] == 0.0)


def test_conservation_and_nonnegativity_over_a_pulse(orc):
    """Fifty steps of a laser pulse at a few on-axis points: sum N = 1 to
    rounding, N >= 0, the window moves up monotonically."""
    Z, w = 18, 3
    spec = spec_of(orc, Z)
    mesh = wl.mesh_2d()
    idx = np.array([512 * 1024 + 100, 512 * 1024 + 200, 500 * 1024 + 150])
    pops, lo = wl.neutral_state(idx.size, w + 1)
    last_lo = lo.copy()
    for step in range(0, 1000, 20):
        E = mesh.field_at(step, idx)
        pops, lo = orc.ionize_step(spec, E, mesh.dt * 20, pops, lo, w=w, eps=1e-8)
        assert np.max(np.abs(pops.sum(axis=0) - 1.0)) < 1e-13
        assert pops.min() >= -1e-18
        assert np.all(lo >= last_lo)
        last_lo = lo.copy()
    assert lo.max() > 0


def test_reduced_window_tracks_full_chain(orc):
    """Sec. 3 replaces the full system by a 3- or 4-level window per cell and
    reports (Fig. 2b/2c, krypton) small errors for the 4-level system and
    larger ones for the 3-level system.  On the synthetic 18-level gas at two
    on-axis points of the 2D pulse: the 4-population window (w = 3) stays
    within 2e-2 of the full chain and the 5-population window within 1e-4,
    while the 3-population window (w = 2) is clearly worse."""
    Z = 18
    spec = spec_of(orc, Z)
    mesh = wl.mesh_2d()
    idx = np.array([512 * 1024 + 300, 540 * 1024 + 300])
    ws = (2, 3, 4)
    red = {w: wl.neutral_state(idx.size, w + 1) for w in ws}
    pf, lf = wl.neutral_state(idx.size, Z + 1)
    worst = {w: 0.0 for w in ws}
    for step in range(0, 1000):
        E = mesh.field_at(step, idx)
        pf, lf = orc.ionize_step(spec, E, mesh.dt, pf, lf, w=Z, eps=0.0, layout=1)
        for w in ws:
            pr, lr = orc.ionize_step(spec, E, mesh.dt, *red[w], w=w, eps=1e-8)
            red[w] = (pr, lr)
            for c in range(idx.size):
                full = np.zeros(Z + 1)
                k = np.arange(lr[c], min(lr[c] + w, Z) + 1)
                full[k] = pr[k - lr[c], c]
                worst[w] = max(worst[w], np.max(np.abs(full - pf[:, c])))
    assert min(red[3][1]) >= 8
    assert worst[3] < 2e-2
    assert worst[4] < 1e-4
    assert worst[2] > 10 * worst[3]


def test_electron_yield_closed_forms(orc):
    """Electron yield of a step: one level from the neutral state gives
    1 - exp(-W dt) (Eq. (6)); a shift without field moves the folded residual
    up one charge; in general the yield equals sum_k k (N'_k - N_k) over the
    full chain (full layout, Sec. 3)."""
    Z = 7
    t = wl.synthetic_gas(Z)
    spec = orc.GasSpec(t.U, t.l, t.m)
    dt = 1.3e-16
    E = wl.loguniform_field(500, 10.0, 2000.0, seed=3)
    N = np.zeros((2, E.size))
    N[0] = 1.0
    lo = np.zeros(E.size, np.uint8)
    out, lo2 = orc.ionize_step(spec, E, dt, N, lo, 1, 0.0)
    x = orc.rates(spec, E, 0, 1)[0] * dt
    y = orc.electron_yield(N, lo, out, lo2, Z)
    assert np.allclose(y, -np.expm1(-x), rtol=1e-13, atol=1e-300)
    # shift only: N_lo = 3e-9 < eps at zero field
    N = np.array([[3e-9], [0.4], [0.6 - 3e-9], [0.0]])
    lo = np.array([2], np.uint8)
    out, lo2 = orc.ionize_step(spec, np.zeros(1), dt, N, lo, 3, 1e-8)
    assert lo2[0] == 3
    assert abs(orc.electron_yield(N, lo, out, lo2, Z)[0] - 3e-9) < 2e-15  # rounding of sums near 3
    # random windows: compact yield = full-chain charge change
    w = 3
    comp, lo = wl.random_window_state(2000, Z, w, seed=11)
    E = wl.loguniform_field(2000, 10.0, 3000.0, seed=12)
    full = np.zeros((Z + 1, 2000))
    for s in range(w + 1):
        ok = lo.astype(int) + s <= Z
        full[lo[ok].astype(int) + s, np.nonzero(ok)[0]] = comp[s, ok]
    outc, loc = orc.ionize_step(spec, E, dt, comp, lo, w, 1e-8)
    outf, _ = orc.ionize_step(spec, E, dt, full, lo, w, 1e-8, layout=1)
    k = np.arange(Z + 1)[:, None]
    yf = (k * outf).sum(axis=0) - (k * full).sum(axis=0)
    assert np.max(np.abs(orc.electron_yield(comp, lo, outc, loc, Z) - yf)) < 1e-13
