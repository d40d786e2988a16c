"""Pins of the oracle's chain solution (Eqs. (2)-(9), Sec. 2-3) against closed
forms, invariants and brute-force high-precision arithmetic."""
import math

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 50


def chain_matrix(x):
    """dt*A of Eq. (3) restricted to len(x)+1 levels, top absorbing."""
    n = len(x) + 1
    A = np.zeros((n, n))
    for i, xi in enumerate(x):
        A[i, i] = -xi
        A[i + 1, i] = xi
    return A


def mp_expm_chain(x):
    n = len(x) + 1
    A = mp.zeros(n, n)
    for i, xi in enumerate(x):
        A[i, i] = -mp.mpf(float(xi))
        A[i + 1, i] = mp.mpf(float(xi))
    T = mp.expm(A)
    return np.array([[float(T[i, j]) for j in range(n)] for i in range(n)])


def mp_bateman(x):
    """Eigen-expansion of Eqs. (4)-(5) for distinct rates, in 50-digit
    arithmetic: T[j][i] = prod_{k=i}^{j-1} x_k sum_{m=i}^{j} e^{-x_m} /
    prod_{l != m} (x_l - x_m), with x_top = 0."""
    pts = [mp.mpf(float(v)) for v in x] + [mp.mpf(0)]
    n = len(pts)
    T = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            prod = mp.mpf(1)
            for k in range(i, j):
                prod *= pts[k]
            s = mp.mpf(0)
            for m in range(i, j + 1):
                d = mp.mpf(1)
                for l in range(i, j + 1):
                    if l != m:
                        d *= pts[l] - pts[m]
                s += mp.e ** (-pts[m]) / d
            T[j, i] = float(prod * s)
    return T


def oracle_T(orc, x):
    return orc.expm(chain_matrix(x))


def rand_cases(rng, w, n):
    out = []
    for c in range(n):
        kind = c % 6
        if kind == 0:
            x = np.exp(rng.uniform(np.log(1e-6), np.log(50), w))
        elif kind == 1:
            c0 = np.exp(rng.uniform(np.log(1e-2), np.log(20)))
            x = np.abs(c0 * (1 + 10.0 ** rng.uniform(-12, -1, w) * rng.standard_normal(w)))
        elif kind == 2:
            x = np.full(w, np.exp(rng.uniform(np.log(1e-3), np.log(20))))
        elif kind == 3:
            x = np.exp(rng.uniform(np.log(1e-3), np.log(5), w))
            x[rng.random(w) < 0.4] = 0.0
        elif kind == 4:
            x = rng.uniform(0, 3, w)
        else:
            x = rng.uniform(0, 10, w)
            x[-1] = x[0] * (1 + 1e-9)
        out.append(x)
    return out


def test_expm_general_matrices(orc):
    """orc.expm against mpmath's expm on random dense matrices."""
    rng = np.random.default_rng(7)
    for n in (1, 2, 3, 5, 8):
        for scale in (0.1, 3.0, 40.0):
            M = rng.standard_normal((n, n)) * scale / n
            T = orc.expm(M)
            Tm = mp.expm(mp.matrix(M.tolist()))
            ref = np.array([[float(Tm[i, j]) for j in range(n)] for i in range(n)])
            assert np.max(np.abs(T - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("x", [1e-12, 1e-5, 0.3, 1.0, 7.5, 60.0])
def test_single_level_closed_form(orc, x):
    """Eq. (6) plus its absorbing partner: N0' = N0 e^{-x}, N1' = N1 + N0 (1 - e^{-x})."""
    W = np.array([[x / 1e-16]])
    pops = np.array([[0.7], [0.3]])
    out = orc.chain_advance(W, 1e-16, pops)
    assert out[0, 0] == pytest.approx(0.7 * math.exp(-x), rel=1e-14, abs=1e-300)
    assert out[1, 0] == pytest.approx(0.3 + 0.7 * -math.expm1(-x), rel=1e-14)


@pytest.mark.parametrize("a,b", [(0.4, 1.3), (2.0, 0.05), (5.0, 4.5), (1e-3, 3.0)])
def test_two_level_eq7(orc, a, b):
    """Eq. (7) with the exponent sign of its second term read as negative:
    n_{p+1}' = n_p a/(a-b) (e^{-b} - e^{-a}) + n_{p+1} e^{-b}."""
    n0, n1, n2 = 0.5, 0.3, 0.2
    T = oracle_T(orc, [a, b])
    N = T @ np.array([n0, n1, n2])
    want1 = n0 * a / (a - b) * (math.exp(-b) - math.exp(-a)) + n1 * math.exp(-b)
    assert N[0] == pytest.approx(n0 * math.exp(-a), rel=1e-14)
    assert N[1] == pytest.approx(want1, rel=1e-13)
    # as printed, with e^{+W_{p+1} dt}, the result differs at O(1)
    printed = n0 * a / (a - b) * (math.exp(-b) - math.exp(-a)) + n1 * math.exp(+b)
    assert abs(N[1] - printed) > 1e-3


def four_level_corrected(a, b, c):
    """Eqs. (6)-(9) with the removable factors of Eq. (8) cancelled and the
    e^{-W_{p+2} dt} terms of Eq. (9) taken with negative sign."""
    Ea, Eb, Ec = math.exp(-a), math.exp(-b), math.exp(-c)
    T = np.zeros((4, 4))
    T[0, 0] = Ea
    T[1, 0] = a / (a - b) * (Eb - Ea)
    T[1, 1] = Eb
    T[2, 0] = a * b * (Ec / ((a - c) * (b - c)) - Eb / ((a - b) * (b - c)) + Ea / ((a - b) * (a - c)))
    T[2, 1] = b * (Ec - Eb) / (b - c)
    T[2, 2] = Ec
    T[3, 0] = 1 - b * c * Ea / ((a - b) * (a - c)) + a * c * Eb / ((a - b) * (b - c)) - a * b * Ec / ((a - c) * (b - c))
    T[3, 1] = 1 + (c * Eb - b * Ec) / (b - c)
    T[3, 2] = 1 - Ec
    T[3, 3] = 1.0
    return T


def four_level_printed_top_row(a, b, c):
    Ea, Eb, Ec = math.exp(-a), math.exp(-b), math.exp(-c)
    t30 = 1 + a * b * Ec / ((a - c) * (b - c)) + a * c * Eb / ((a - b) * (b - c)) - b * c * Ea / ((a - b) * (a - c))
    t31 = 1 + (a * b - b * c) * Ec / ((a - c) * (b - c)) + (a * c - b * c) * Eb / ((a - b) * (b - c))
    t32 = 1 + (c * c + a * b - a * c - b * c) * Ec / ((a - c) * (b - c))
    return np.array([t30, t31, t32])


@pytest.mark.parametrize("abc", [(3.0, 0.8, 0.05), (0.4, 1.7, 0.9), (12.0, 2.5, 0.3), (0.02, 0.3, 5.0)])
def test_four_level_eqs6_9(orc, abc):
    a, b, c = abc
    T = oracle_T(orc, [a, b, c])
    ref = four_level_corrected(a, b, c)
    assert np.max(np.abs(T - ref)) < 1e-13
    # the printed signs of Eq. (9) are not the solution (error of order one)
    assert np.max(np.abs(four_level_printed_top_row(a, b, c) - T[3, :3])) > 1e-2


@pytest.mark.parametrize("w", [1, 3, 6])
@pytest.mark.parametrize("x", [1e-4, 0.7, 4.0, 30.0])
def test_erlang_equal_rates(orc, w, x):
    """All rates equal: T[j][0] = x^j e^{-x} / j! below the top, the top gets the rest."""
    T = oracle_T(orc, [x] * w)
    for j in range(w):
        assert T[j, 0] == pytest.approx(x ** j * math.exp(-x) / math.factorial(j), rel=1e-12, abs=1e-300)
    rest = 1 - sum(x ** j * math.exp(-x) / math.factorial(j) for j in range(w))
    assert T[w, 0] == pytest.approx(rest, abs=1e-14)


def test_zero_rates_identity(orc):
    for w in (1, 4, 8):
        T = oracle_T(orc, [0.0] * w)
        assert np.array_equal(T, np.eye(w + 1))


@pytest.mark.parametrize("w", [1, 2, 3, 4, 6, 8])
def test_mpmath_brute_force(orc, w):
    rng = np.random.default_rng(100 + w)
    for x in rand_cases(rng, w, 24):
        T = oracle_T(orc, x)
        ref = mp_expm_chain(x)
        assert np.max(np.abs(T - ref)) < 1e-14, x


@pytest.mark.parametrize("w", [2, 3, 5])
def test_bateman_large_rates(orc, w):
    """Well separated large rates (up to 1e10 per step) against the 50-digit
    eigen expansion of Eqs. (4)-(5)."""
    rng = np.random.default_rng(200 + w)
    for _ in range(12):
        x = np.sort(np.exp(rng.uniform(np.log(0.5), np.log(1e10), w)))[::-1]
        T = oracle_T(orc, x)
        ref = mp_bateman(x)
        assert np.max(np.abs(T - ref)) < 1e-15, x


@pytest.mark.parametrize("w", [1, 3, 7])
def test_invariants(orc, w):
    """Column sums 1 (columns of Eq. (3) sum to zero), nonnegative entries,
    semigroup T(dt) = T(dt/2)^2, dt -> 0 gives I + dt A."""
    rng = np.random.default_rng(300 + w)
    for x in rand_cases(rng, w, 18):
        T = oracle_T(orc, x)
        assert np.max(np.abs(T.sum(axis=0) - 1)) < 1e-14
        assert T.min() > -1e-16
        Th = oracle_T(orc, np.asarray(x) / 2)
        assert np.max(np.abs(Th @ Th - T)) < 1e-13
        h = 1e-9
        Ts = oracle_T(orc, np.asarray(x) * h)
        assert np.max(np.abs(Ts - (np.eye(w + 1) + h * chain_matrix(x)))) < 3e-16 + (h * max(x.max(), 1)) ** 2


def test_chain_advance_matches_matrix(orc):
    rng = np.random.default_rng(5)
    w, n = 4, 50
    W = np.exp(rng.uniform(np.log(1e10), np.log(1e17), (w, n)))
    pops = rng.random((w + 1, n))
    pops /= pops.sum(axis=0)
    dt = 1.3e-16
    out = orc.chain_advance(W, dt, pops)
    for c in range(n):
        T = oracle_T(orc, W[:, c] * dt)
        assert np.max(np.abs(out[:, c] - T @ pops[:, c])) < 1e-15
