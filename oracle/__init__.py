"""Plain FP64 CPU oracle for the multi-level ADK ionization step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package.  The product package
never imports it, and it imports nothing from the product package: the two
share no code.  The arithmetic lives in ``adk_oracle.c`` (Eq. (1) in product
form; expm of the windowed rate matrix of Eq. (3) by Taylor series with
scaling and squaring; window shift with upward fold at the start of a step).

Every function here takes and returns numpy arrays; nothing touches a GPU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

#: Paper constants of Eq. (1) (Sec. 2): omega_a [1/s], E_a [GV/m]; U_H [eV]
#: is half the atomic energy unit 27.21 eV, so that n* = Q / sqrt(2 U / 27.21 eV).
OMEGA_A = 4.13e16
E_A = 510.0
U_H = 27.21 / 2.0
M_AVERAGE = -1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-shared", "-fPIC",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i8p = ctypes.POINTER(ctypes.c_int8)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.orc_rate_lm.restype = ctypes.c_double
    lib.orc_rate_lm.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, dp]
    lib.orc_level_rate.restype = ctypes.c_double
    lib.orc_level_rate.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, dp]
    lib.orc_rates.restype = None
    lib.orc_rates.argtypes = [ctypes.c_int, dp, i8p, i8p, dp, dp, ctypes.c_int64,
                              ctypes.c_int, ctypes.c_int, dp]
    lib.orc_expm.restype = None
    lib.orc_expm.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_chain_advance.restype = None
    lib.orc_chain_advance.argtypes = [ctypes.c_int, ctypes.c_int64, dp, ctypes.c_double, dp]
    lib.orc_ionize_step.restype = None
    lib.orc_ionize_step.argtypes = [ctypes.c_int, dp, i8p, i8p, dp, ctypes.c_int64, dp,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, dp, u8p]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_adaptive_step.restype = None
    lib.orc_adaptive_step.argtypes = [ctypes.c_int, dp, i8p, i8p, dp, ctypes.c_int64, dp, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, u8p, u8p,
                                      ip, ip, dp, dp, dp]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _consts(consts):
    if consts is None:
        consts = (OMEGA_A, E_A, U_H)
    return np.ascontiguousarray(np.asarray(consts, dtype=np.float64))


class GasSpec:
    """Level table of a gas: U[k] (eV) ionizes charge k -> k+1, with orbital
    number l[k] and projection m[k] (|m|; M_AVERAGE averages over m = -l..l)."""

    def __init__(self, U, l, m):
        self.U = np.ascontiguousarray(np.asarray(U, dtype=np.float64))
        self.l = np.ascontiguousarray(np.asarray(l, dtype=np.int8))
        self.m = np.ascontiguousarray(np.asarray(m, dtype=np.int8))
        self.Z = int(self.U.shape[0])
        assert self.l.shape == (self.Z,) and self.m.shape == (self.Z,)

    def _ptrs(self):
        return (_dp(self.U), self.l.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                self.m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))


def rate_lm(U, Q, l, am, E, consts=None) -> float:
    """Eq. (1) for one (l, |m|) at one field value, in 1/s."""
    c = _consts(consts)
    return _load().orc_rate_lm(float(U), int(Q), int(l), int(am), float(E), _dp(c))


def level_rate(U, Q, l, m, E, consts=None) -> float:
    """Rate of one level (m < 0: averaged over m = -l..l), in 1/s."""
    c = _consts(consts)
    return _load().orc_level_rate(float(U), int(Q), int(l), int(m), float(E), _dp(c))


def rates(gas: GasSpec, E, k0=0, nk=None, consts=None) -> np.ndarray:
    """W[j][i] = rate of level k0 + j at field E[i] (1/s)."""
    if nk is None:
        nk = gas.Z - k0
    assert 0 <= k0 and k0 + nk <= gas.Z
    E = np.ascontiguousarray(np.asarray(E, dtype=np.float64).ravel())
    out = np.zeros((nk, E.size), dtype=np.float64)
    c = _consts(consts)
    _load().orc_rates(gas.Z, *gas._ptrs(), _dp(c), _dp(E), E.size, k0, nk, _dp(out))
    return out


def expm(M) -> np.ndarray:
    """exp(M) of a small square matrix (Taylor + scaling and squaring)."""
    M = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
    n = M.shape[0]
    assert M.shape == (n, n) and n <= 72
    T = np.zeros_like(M)
    _load().orc_expm(n, _dp(M), _dp(T))
    return T


def chain_advance(W, dt, pops) -> np.ndarray:
    """Advance pops[(w+1)][n] over dt with rates W[w][n] (1/s); top absorbing;
    no window shift.  Returns a new array."""
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    pops = np.array(pops, dtype=np.float64, order="C", copy=True)
    w = W.shape[0]
    n = pops.shape[1]
    assert pops.shape == (w + 1, n) and W.shape == (w, n)
    _load().orc_chain_advance(w, n, _dp(W), float(dt), _dp(pops))
    return pops


def ionize_step(gas: GasSpec, E, dt, pops, lo, w, eps, layout=0, consts=None):
    """One ionization step over all cells.  Returns (new_pops, new_lo) as new
    arrays.  layout 0: pops[(w+1)][n] (slot s = level lo+s); layout 1:
    pops[(Z+1)][n]."""
    E = np.ascontiguousarray(np.asarray(E, dtype=np.float64).ravel())
    n = E.size
    pops = np.array(pops, dtype=np.float64, order="C", copy=True)
    lo = np.array(lo, dtype=np.uint8, order="C", copy=True).ravel()
    rows = (w + 1) if layout == 0 else (gas.Z + 1)
    assert pops.shape == (rows, n), (pops.shape, rows, n)
    assert lo.shape == (n,)
    c = _consts(consts)
    _load().orc_ionize_step(gas.Z, *gas._ptrs(), _dp(c), n, _dp(E), float(dt), int(w),
                            float(eps), int(layout), _dp(pops),
                            lo.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return pops, lo


def adaptive_step(gas: GasSpec, E, dt, pops, lo, wc, wmin, wmax, eps, tol, force_top=None, consts=None):
    """One step with an adaptive window (see orc_adaptive_step): pops[(wmax+1)][n],
    lo[n] and wc[n] (rates in each cell's window) in; returns (pops, lo, wc,
    info) as new arrays, info = dict(top, leak_top, leak_below, leaks) per cell
    (leaks[(wmax+1)][n]: leak(t) for the slots the criterion may test, -1
    elsewhere).  force_top[n] (optional, int): where >= 0, the top slot to
    take instead of the leak criterion."""
    E = np.ascontiguousarray(np.asarray(E, dtype=np.float64).ravel())
    n = E.size
    pops = np.array(pops, dtype=np.float64, order="C", copy=True)
    lo = np.array(lo, dtype=np.uint8, order="C", copy=True).ravel()
    wc = np.array(wc, dtype=np.uint8, order="C", copy=True).ravel()
    assert pops.shape == (wmax + 1, n), (pops.shape, wmax, n)
    assert lo.shape == (n,) and wc.shape == (n,)
    assert 0 <= wmin <= wmax <= 63
    top = np.zeros(n, np.int32)
    lt = np.zeros(n)
    lb = np.zeros(n)
    lk = np.zeros((wmax + 1, n))
    ip = ctypes.POINTER(ctypes.c_int)
    ft = None
    if force_top is not None:
        ft = np.ascontiguousarray(np.asarray(force_top, np.int32).ravel())
        assert ft.shape == (n,)
    c = _consts(consts)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    _load().orc_adaptive_step(gas.Z, *gas._ptrs(), _dp(c), n, _dp(E), float(dt), int(wmin), int(wmax), float(eps),
                              float(tol), _dp(pops), lo.ctypes.data_as(u8), wc.ctypes.data_as(u8),
                              ft.ctypes.data_as(ip) if ft is not None else None, top.ctypes.data_as(ip),
                              _dp(lt), _dp(lb), _dp(lk))
    return pops, lo, wc, dict(top=top, leak_top=lt, leak_below=lb, leaks=lk)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def electron_yield(pops_in, lo_in, pops_out, lo_out, Z):
    """Electron yield of a step per atom, compact layout: the change of the
    mean charge sum_k k N_k (the electron density of Fig. 2(c) per atom),
    sum_s (lo' + s) N'_s - sum_s (lo + s) N_s, with lo read as min(lo, Z)."""
    Pi = np.asarray(pops_in, np.float64)
    Po = np.asarray(pops_out, np.float64)
    li = np.minimum(np.asarray(lo_in, np.int64), Z)
    lq = np.asarray(lo_out, np.int64)
    s = np.arange(Pi.shape[0])[:, None]
    return ((lq[None, :] + s) * Po).sum(axis=0) - ((li[None, :] + s) * Pi).sum(axis=0)
