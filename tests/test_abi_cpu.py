"""CPU-side checks of the C-ABI library: it loads, exports every function the
header declares, validates arguments on the host before any device call,
and its host-built coefficient table reproduces the oracle's Eq. (1)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2202_10647_amd import adkion, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adkion.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(adkion.LIB_PATH):
        from paper_2202_10647_amd import build
        build.build()
    return adkion.lib()


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M))


def test_exports_every_declared_function(L):
    declared = header_functions()
    assert declared == set(adkion.EXPORTS), declared
    out = subprocess.run(["nm", "-D", "--defined-only", adkion.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = declared - exported
    assert not missing, missing
    for name in declared:
        assert hasattr(L, name)


def test_version_and_strerror(L):
    assert "adkion" in adkion.version()
    assert adkion.status_text(adkion.ADK_EINVAL) == "invalid argument"
    assert adkion.status_text(12345) == "unknown status"


def gas_desc(Z=7):
    g = wl.synthetic_gas(Z)
    return g.U, g.l, g.m


@pytest.mark.parametrize("bad,status", [
    (dict(U=[-1.0]), adkion.ADK_EINVAL),
    (dict(U=[float("nan")]), adkion.ADK_EINVAL),
    (dict(l=[4]), adkion.ADK_EINVAL),
    (dict(l=[-1]), adkion.ADK_EINVAL),
    (dict(l=[1], m=[2]), adkion.ADK_EINVAL),
    (dict(l=[1], m=[-2]), adkion.ADK_EINVAL),
])
def test_gas_validation(L, bad, status):
    U, l, m = [13.6], [0], [0]
    U = bad.get("U", U)
    l = bad.get("l", l)
    m = bad.get("m", m)
    with pytest.raises(adkion.AdkError) as e:
        adkion.gas_coeffs(U, l, m)
    assert e.value.status == status


def test_gas_z_range(L):
    with pytest.raises(adkion.AdkError) as e:
        adkion.gas_coeffs(np.full(65, 20.0), np.zeros(65), np.zeros(65))
    assert e.value.status == adkion.ADK_ERANGE
    d = adkion._GasDesc(0, None, None, None)
    assert L.adk_gas_coeffs(ctypes.byref(d), None, None) == adkion.ADK_ERANGE
    assert L.adk_gas_coeffs(None, None, None) == adkion.ADK_EINVAL
    with pytest.raises(adkion.AdkError):
        adkion.gas_coeffs([13.6], [0], [0], consts=(-1.0, 510.0, 13.6))


@pytest.mark.parametrize("Z", [1, 7, 18, 36, 54])
def test_coefficients_reproduce_eq1(L, orc, Z):
    """ln W = A + alpha L - B R + ln(1 + sum c_j u^j) from the host table
    against the oracle's literal product form."""
    g = wl.synthetic_gas(Z)
    coef = adkion.gas_coeffs(g.U, g.l, g.m)
    spec = orc.GasSpec(g.U, g.l, g.m)
    E = np.geomspace(5.0, 20000.0, 37)
    W = orc.rates(spec, E)
    u = E / orc.E_A
    for k in range(Z):
        A, al, B, c1, c2, c3 = coef[k, :6]
        lnW = A + al * np.log(u) - B / u + np.log1p(c1 * u + c2 * u ** 2 + c3 * u ** 3)
        ok = W[k] > 1e-250
        if not ok.any():
            continue
        assert np.max(np.abs(lnW[ok] - np.log(W[k, ok]))) < 1e-12 * max(1.0, np.max(np.abs(lnW[ok])))


def test_default_constants_are_paper_values(L):
    U, l, m = gas_desc(7)
    a = adkion.gas_coeffs(U, l, m)
    b = adkion.gas_coeffs(U, l, m, consts=(4.13e16, 510.0, 27.21 / 2))
    assert np.array_equal(a, b)


def test_chain_advance_validation_before_device(L):
    """Every rejected argument returns before any HIP call (no GPU here)."""
    f = L.adk_chain_advance
    p = ctypes.c_void_p(16)
    assert f(0, p, 10, 1e-16, p, 0, None) == adkion.ADK_ERANGE
    assert f(64, p, 10, 1e-16, p, 0, None) == adkion.ADK_ERANGE
    assert f(3, p, -1, 1e-16, p, 0, None) == adkion.ADK_EINVAL
    assert f(3, p, 10, 0.0, p, 0, None) == adkion.ADK_EINVAL
    assert f(3, p, 10, float("inf"), p, 0, None) == adkion.ADK_EINVAL
    assert f(3, None, 10, 1e-16, p, 0, None) == adkion.ADK_EINVAL
    assert f(3, p, 10, 1e-16, p, 7, None) == adkion.ADK_EINVAL
    # zero cells is a no-op that touches no device
    assert f(3, None, 0, 1e-16, None, 0, None) == adkion.ADK_OK


def test_step_and_rates_reject_null_gas(L):
    win = adkion._Window(3, 1e-8, 0, 0)
    p = ctypes.c_void_p(16)
    assert L.ionize_step(None, p, 10, 1e-16, p, p, ctypes.byref(win), None) == adkion.ADK_EINVAL
    assert L.ionize_step(p, p, 10, 1e-16, p, p, None, None) == adkion.ADK_EINVAL
    assert L.adk_rates(None, p, 10, 0, 1, p, 0, None) == adkion.ADK_EINVAL
    assert L.adk_gas_levels(None) == adkion.ADK_EINVAL
    assert L.adk_gas_destroy(None) == adkion.ADK_OK


def test_gas_create_out_pointer_required(L):
    U, l, m = gas_desc(7)
    d, keep = adkion._desc(U, l, m)
    assert L.adk_gas_create(ctypes.byref(d), None, None) == adkion.ADK_EINVAL
    h = ctypes.c_void_p(1234)
    bad, keep2 = adkion._desc([-5.0], [0], [0])
    assert L.adk_gas_create(ctypes.byref(bad), None, ctypes.byref(h)) == adkion.ADK_EINVAL
    assert h.value is None


def test_plan_validation_before_device(L):
    vp = ctypes.c_void_p
    out = vp()
    one = (vp * 1)(vp(16))
    cg = np.zeros(4, np.uint8)
    cw = np.ones(4, np.uint8)
    f = L.adk_plan_create
    c = lambda a: a.ctypes.data_as(vp)
    assert f(one, 1, c(cg), c(cw), 4, 0, 1e-8, 0, 0, None) == adkion.ADK_EINVAL
    assert f(None, 1, c(cg), c(cw), 4, 0, 1e-8, 0, 0, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 0, c(cg), c(cw), 4, 0, 1e-8, 0, 0, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 9, c(cg), c(cw), 4, 0, 1e-8, 0, 0, ctypes.byref(out)) == adkion.ADK_ERANGE
    assert f(one, 1, c(cg), c(cw), -1, 0, 1e-8, 0, 0, ctypes.byref(out)) == adkion.ADK_ERANGE
    assert f(one, 1, None, c(cw), 4, 0, 1e-8, 0, 0, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 1, c(cg), c(cw), 4, 5, 1e-8, 0, 0, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 1, c(cg), c(cw), 4, 0, -1.0, 0, 0, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 1, c(cg), c(cw), 4, 0, 1e-8, 3, 0, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 1, c(cg), c(cw), 4, 0, 1e-8, 0, 2, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert f(one, 1, c(cg), c(cw), 4, 0, 1e-8, 0, -1, ctypes.byref(out)) == adkion.ADK_EINVAL
    assert out.value is None
    info = adkion._PlanInfo()
    assert L.adk_plan_get_info(None, ctypes.byref(info)) == adkion.ADK_EINVAL
    assert L.adk_plan_order(None, vp(16)) == adkion.ADK_EINVAL
    assert L.adk_plan_step(None, vp(16), 1e-16, vp(16), vp(16), None) == adkion.ADK_EINVAL
    assert L.adk_plan_destroy(None) == adkion.ADK_OK
    fh = L.adk_field_hash
    assert fh(vp(16), -1, 1, 0, 10.0, 20.0, 0, None) == adkion.ADK_EINVAL
    assert fh(vp(16), 4, 1, -1, 10.0, 20.0, 0, None) == adkion.ADK_EINVAL
    assert fh(vp(16), 4, 1, 0, 0.0, 20.0, 0, None) == adkion.ADK_EINVAL
    assert fh(vp(16), 4, 1, 0, 30.0, 20.0, 0, None) == adkion.ADK_EINVAL
    assert fh(None, 0, 1, 0, 10.0, 20.0, 0, None) == adkion.ADK_OK


def test_batched_cells_generator():
    g, w = wl.batched_cells(200000, seed=4)
    assert abs((g > 0).mean() - 0.01) < 0.002
    assert np.all(w[g == 0] == 1)
    zs = np.array((1,) + wl.DOPANT_Z)
    assert np.all(w <= np.minimum(6, zs[g]))
    assert set(np.unique(g[g > 0])) == {1, 2, 3, 4}


def test_hash_field_is_loguniform():
    E = wl.hash_field(200000, 4, 0)
    assert E.min() >= 10.0 and E.max() <= 5000.0
    u = np.log(E / 10.0) / np.log(500.0)
    assert abs(u.mean() - 0.5) < 0.005 and abs(u.var() - 1 / 12) < 0.002
    assert not np.array_equal(wl.hash_field(100, 4, 0), wl.hash_field(100, 4, 1))


def test_mlp_host_validation(L):
    """Surrogate entry points reject bad arguments before touching a device."""
    for Z in (1, 36, 64):
        assert L.adk_mlp_nparams(Z) == 16 * Z + 9796 == wl.mlp_nparams(Z)
    assert L.adk_mlp_nparams(0) == -1 and L.adk_mlp_nparams(65) == -1
    h = ctypes.c_void_p()
    prm = (ctypes.c_float * 10)()
    assert L.adk_mlp_create(None, prm, None, ctypes.byref(h)) == adkion.ADK_EINVAL
    assert L.adk_mlp_destroy(None) == adkion.ADK_OK
    assert L.adk_mlp_get_state(None, None, None, None, None) == adkion.ADK_EINVAL
    assert L.adk_band_columns(None, None, None, None, 5, None, None) == adkion.ADK_EINVAL
    assert L.adk_mlp_forward(None, None, None, None, 5, None, None) == adkion.ADK_EINVAL
    assert L.adk_mlp_loss_grad(None, None, None, None, None, 5, None, None, None) == adkion.ADK_EINVAL
    assert L.adk_mlp_train(None, None, None, None, None) == adkion.ADK_EINVAL
    assert L.adk_mlp_save(None, b"/nonexistent") == adkion.ADK_EINVAL
    assert L.adk_mlp_load(None, b"/nonexistent", ctypes.byref(h)) == adkion.ADK_EINVAL
    win = adkion._Window(3, 1e-8, adkion.ADK_LAYOUT_COMPACT, adkion.ADK_MIXED)
    assert L.adk_surrogate_step(None, None, None, 4, 1e-16, None, None, ctypes.byref(win), None,
                                None) == adkion.ADK_EINVAL


def test_yield_host_validation(L):
    win = adkion._Window(3, 1e-8, adkion.ADK_LAYOUT_FULL, adkion.ADK_MIXED)
    assert L.ionize_step_yield(None, None, 4, 1e-16, None, None, ctypes.byref(win), None, None) == adkion.ADK_EINVAL
    win = adkion._Window(3, 1e-8, adkion.ADK_LAYOUT_COMPACT, adkion.ADK_MIXED)
    assert L.ionize_step_yield(None, None, 4, 1e-16, None, None, ctypes.byref(win), None, None) == adkion.ADK_EINVAL
    assert L.ionize_step_yield(None, None, 0, 1e-16, None, None, None, None, None) == adkion.ADK_EINVAL


def test_ceiling_host_validation(L):
    """The measurement harness entry points reject bad arguments on the host
    (no device call is made for any of these)."""
    E = adkion.ADK_EINVAL
    assert L.adk_ceiling_copy(None, None, 40, 1, None) == E      # not a multiple of 16
    assert L.adk_ceiling_copy(None, None, 32, 1, None) == E      # null buffers
    assert L.adk_ceiling_copy(None, None, 32, 0, None) == E      # reps < 1
    assert L.adk_ceiling_copy(None, None, -16, 1, None) == E
    assert L.adk_ceiling_copy(None, None, 0, 1, None) == adkion.ADK_OK  # nothing to copy
    assert L.adk_ceiling_valu(3, 10, None, 256, None) == E       # kind
    assert L.adk_ceiling_valu(0, 10, None, 256, None) == E       # null out
    buf = ctypes.c_void_p(1)
    assert L.adk_ceiling_valu(0, -1, buf, 256, None) == E        # iters < 0
    assert L.adk_ceiling_valu(0, 10, buf, 100, None) == E        # lanes not a multiple of 256
    assert L.adk_ceiling_valu(0, 10, buf, 0, None) == E


def test_plan_graph_replay_host_validation(L):
    assert L.adk_plan_graph_replay(None, 1, None) == adkion.ADK_EINVAL
    assert L.adk_plan_graph_replay(None, -1, None) == adkion.ADK_EINVAL


def test_adaptive_host_validation(L):
    """Workspace size and the host-side rejections of ionize_step_adaptive
    that need no gas on a device."""
    assert L.adk_adaptive_work_bytes(0) == 256
    assert L.adk_adaptive_work_bytes(1000) == 256 + 32 * 4 + 8000
    assert L.adk_adaptive_work_bytes(1024) == 256 + 32 * 4 + 8192
    win = adkion._Adaptive(1, 8, 1e-8, 1e-9, adkion.ADK_MIXED)
    E = adkion.ADK_EINVAL
    assert L.ionize_step_adaptive(None, None, 4, 1e-16, None, None, None, ctypes.byref(win), None, 0, None,
                                  None) == E
    assert L.ionize_step_adaptive(None, None, 0, 1e-16, None, None, None, None, None, 0, None, None) == E
