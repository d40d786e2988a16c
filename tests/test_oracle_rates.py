"""Pins of the oracle's ADK rate (Eq. (1), Sec. 2) against closed forms and
exact scaling laws that do not reuse the oracle's code path."""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
OMEGA_A = GOLD["omega_a_per_s"]
E_A = GOLD["E_a_GV_per_m"]
U_H = 27.21 / 2


def hydrogen_closed_form(E):
    """Eq. (1) with Q = 1, n* = 1, l = m = 0, simplified by hand:
    sqrt(3E/(pi E_a)) * (1/2) * (2e)^2 * exp(-2E_a/(3E)) * 1/(2 pi) * (2 E_a/E)."""
    return OMEGA_A * (math.e ** 2 / math.pi) * math.sqrt(3 * E / (math.pi * E_A)) * (2 * E_A / E) * \
        math.exp(-2 * E_A / (3 * E))


def test_paper_constants_are_oracle_defaults(orc):
    assert orc.OMEGA_A == OMEGA_A and orc.E_A == E_A


@pytest.mark.parametrize("E", [5.0, 30.0, 100.0, 510.0, 2000.0, 5000.0])
def test_hydrogen_closed_form(orc, E):
    w = orc.rate_lm(U_H, 1, 0, 0, E)
    assert w == pytest.approx(hydrogen_closed_form(E), rel=1e-13)


@pytest.mark.parametrize("Q", [2, 3, 5, 11])
@pytest.mark.parametrize("ns", [1.0, 1.7, 3.2])
@pytest.mark.parametrize("E", [20.0, 700.0])
def test_hydrogenic_scaling_law(orc, Q, ns, E):
    """Atomic-unit scaling: at fixed n*, W(lam Q, lam^3 E) = lam^2 W(Q, E)
    (every field factor of Eq. (1) depends on E/Q^3, the prefactor on Q^2)."""
    lam = Q
    # U chosen so that n* = Q sqrt(U_H/U) equals ns for charge 1 and charge Q
    U1 = U_H * (1.0 / ns) ** 2
    UQ = U_H * (Q / ns) ** 2
    for l, am in [(0, 0), (1, 1), (2, 1)]:
        w1 = orc.rate_lm(U1, 1, l, am, E)
        wq = orc.rate_lm(UQ, Q, l, am, lam ** 3 * E)
        assert wq == pytest.approx(lam ** 2 * w1, rel=1e-12)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_projection_ratio_closed_form(orc, l):
    """W_l|m| / W_l0 = (l+|m|)!/(2^|m| |m|! (l-|m|)! l!/l!) * (E n*^3/(2 E_a Q^3))^|m|."""
    U, Q, E = 180.0, 4, 350.0
    ns = Q * math.sqrt(U_H / U)
    w0 = orc.rate_lm(U, Q, l, 0, E)
    for am in range(1, l + 1):
        ratio = math.factorial(l + am) / (2 ** am * math.factorial(am) * math.factorial(l - am)) \
            * (E * ns ** 3 / (2 * E_A * Q ** 3)) ** am
        assert orc.rate_lm(U, Q, l, am, E) / w0 == pytest.approx(ratio, rel=1e-12)


def test_orbital_factor(orc):
    """|m| = 0: W is proportional to (2l+1)."""
    w0 = orc.rate_lm(40.0, 2, 0, 0, 120.0)
    for l in range(1, 4):
        assert orc.rate_lm(40.0, 2, l, 0, 120.0) / w0 == pytest.approx(2 * l + 1, rel=1e-13)


def test_projection_average(orc):
    """m-average = (W_0 + 2 sum_{|m|>=1} W_|m|) / (2l + 1)."""
    U, Q, E, l = 95.0, 3, 260.0, 2
    parts = [orc.rate_lm(U, Q, l, am, E) for am in range(l + 1)]
    want = (parts[0] + 2 * sum(parts[1:])) / (2 * l + 1)
    assert orc.level_rate(U, Q, l, -1, E) == pytest.approx(want, rel=1e-14)


def test_zero_sign_and_nan(orc):
    assert orc.rate_lm(20.0, 1, 1, 0, 0.0) == 0.0
    assert orc.rate_lm(20.0, 1, 1, 0, -150.0) == orc.rate_lm(20.0, 1, 1, 0, 150.0)
    assert math.isnan(orc.rate_lm(20.0, 1, 1, 0, float("nan")))
    # tunnelling factor underflows: exactly zero, never 0 * inf
    assert orc.rate_lm(5000.0, 30, 1, 0, 1e-3) == 0.0


def test_weak_field_monotone(orc):
    """Below the barrier-suppression regime W rises steeply with E."""
    E = np.geomspace(1.0, 100.0, 40)
    w = np.array([orc.rate_lm(U_H, 1, 0, 0, e) for e in E])
    assert np.all(np.diff(w) > 0)


def test_rates_array_matches_scalar(orc):
    from paper_2202_10647_amd import workloads as wl
    g = wl.synthetic_gas(36)
    spec = orc.GasSpec(g.U, g.l, g.m)
    E = np.array([15.0, 300.0, 4000.0])
    W = orc.rates(spec, E, k0=3, nk=5)
    for j in range(5):
        k = 3 + j
        for i, e in enumerate(E):
            assert W[j, i] == orc.level_rate(g.U[k], k + 1, g.l[k], g.m[k], e)


@pytest.mark.parametrize("U,Q,l", [(15.76, 1, 1), (40.74, 3, 1), (422.4, 8, 1), (520.0, 10, 2), (8.0, 1, 0)])
@pytest.mark.parametrize("E1,E2", [(150.0, 900.0), (400.0, 3000.0)])
def test_field_dependence_at_noninteger_nstar(orc, U, Q, l, E1, E2):
    """Eq. (1) depends on the field only through E^(1/2) (the square-root
    factor), E^-(2n*-|m|-1) (the power factor) and exp(-2 E_a (Q/n*)^3 / (3E))
    (the tunnelling factor), so the log-ratio of two rates of one level is, at
    any n*, (1/2 - (2n*-|m|-1)) ln(E2/E1) - (2/3) E_a (Q/n*)^3 (1/E2 - 1/E1).
    Every n* here is non-integer; a wrong exponent on E or a wrong power of
    Q/n* in the tunnelling factor changes the ratio by orders of magnitude."""
    ns = Q * math.sqrt(U_H / U)
    assert abs(ns - round(ns)) > 0.05
    for am in range(l + 1):
        w1 = orc.rate_lm(U, Q, l, am, E1)
        w2 = orc.rate_lm(U, Q, l, am, E2)
        assert w1 > 0.0 and w2 > 0.0
        want = (0.5 - (2 * ns - am - 1)) * math.log(E2 / E1) - (2.0 / 3.0) * E_A * (Q / ns) ** 3 * (1 / E2 - 1 / E1)
        assert math.log(w2 / w1) == pytest.approx(want, rel=1e-12, abs=1e-11)


@pytest.mark.parametrize("E", [30.0, 60.0, 100.0, 200.0])
def test_hydrogen_step_closed_form(orc, E):
    """The step driver on a one-level gas (hydrogen: U = U_H, so Q = 1 and
    n* = 1, l = m = 0): the neutral fraction falls to exp(-W dt) with W the
    hand-simplified Eq. (1), the rest is ionized (Eq. (3) with one rate).
    Pins which charge and level the driver evaluates Eq. (1) at, and dt."""
    dt = 1.334e-16
    spec = orc.GasSpec([U_H], [0], [0])
    x = hydrogen_closed_form(E) * dt
    assert 1e-3 < x < 10.0
    pops = np.array([[1.0, 0.25], [0.0, 0.75]])
    out, lo = orc.ionize_step(spec, np.array([E, -E]), dt, pops, np.zeros(2, np.uint8), w=1, eps=1e-8)
    assert lo.tolist() == [0, 0]
    for c, n0 in enumerate((1.0, 0.25)):
        assert out[0, c] == pytest.approx(n0 * math.exp(-x), rel=1e-13)
        assert out[1, c] == pytest.approx(1.0 - n0 * math.exp(-x), rel=1e-13)


def closed_form_nstar2(E, Q, l, am):
    """Eq. (1) at n* = 2, simplified by hand for the two charges that give
    n* = 2 exactly: Q = 1 with U = U_H/4 and Q = 2 with U = U_H.  With n* = 2
    the factors are sqrt(24 E/(pi Q^3 E_a)), Q^2/8, e^4,
    exp(-E_a Q^3/(12 E)), (2l+1)(l+|m|)!/(4 pi 2^|m| |m|! (l-|m|)!) and
    (E_a Q^3/(4 E))^(3-|m|); below they are multiplied out per case."""
    e = math.e
    if Q == 1:
        s = OMEGA_A * e ** 4 / (32 * math.pi) * math.sqrt(24 * E / (math.pi * E_A)) * (E_A / (4 * E)) ** 3 \
            * math.exp(-E_A / (12 * E))
        return {(0, 0): s, (1, 0): 3 * s, (1, 1): 3 * s * 4 * E / E_A}[(l, am)]
    if Q == 2:
        s = OMEGA_A * e ** 4 / (8 * math.pi) * math.sqrt(3 * E / (math.pi * E_A)) * (2 * E_A / E) ** 3 \
            * math.exp(-2 * E_A / (3 * E))
        return {(0, 0): s, (1, 0): 3 * s, (1, 1): 3 * s * E / (2 * E_A)}[(l, am)]
    raise ValueError(Q)


def closed_form_nstar3(E, l, am):
    """Eq. (1) at n* = 3 (Q = 3, U = U_H), simplified by hand: the square-root
    factor is sqrt(3E/(pi E_a)), Q^2/(2 n*^2) = 1/2, (2e/3)^6,
    exp(-2 E_a/(3E)), angular factor (2l+1)(l+|m|)!/(6 pi 2^|m| |m|! (l-|m|)!)
    and (2 E_a/E)^(5-|m|)."""
    s = OMEGA_A * (2 * math.e / 3) ** 6 / (12 * math.pi) * math.sqrt(3 * E / (math.pi * E_A)) \
        * (2 * E_A / E) ** 5 * math.exp(-2 * E_A / (3 * E))
    r = E / (2 * E_A)
    return {(0, 0): s, (1, 0): 3 * s, (1, 1): 3 * s * r, (2, 0): 5 * s, (2, 1): 15 * s * r,
            (2, 2): 15 * s * r * r}[(l, am)]


@pytest.mark.parametrize("E", [5.0, 40.0, 300.0, 2000.0])
def test_integer_nstar_closed_forms(orc, E):
    """The n* dependence of Eq. (1)'s field-independent factor: at n* = 2
    (two charges) and n* = 3 every factor is an elementary number, and the
    oracle must give the hand-simplified value (a factor n*^3 dropped from the
    square root, a wrong power of 2e/n* or of n* in the angular factor all
    move these by integer ratios)."""
    for Q, U in ((1, U_H / 4), (2, U_H)):
        for l, am in ((0, 0), (1, 0), (1, 1)):
            assert orc.rate_lm(U, Q, l, am, E) == pytest.approx(closed_form_nstar2(E, Q, l, am), rel=1e-13)
        want = (closed_form_nstar2(E, Q, 1, 0) + 2 * closed_form_nstar2(E, Q, 1, 1)) / 3
        assert orc.level_rate(U, Q, 1, -1, E) == pytest.approx(want, rel=1e-13)
    for l, am in ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)):
        assert orc.rate_lm(U_H, 3, l, am, E) == pytest.approx(closed_form_nstar3(E, l, am), rel=1e-13)
