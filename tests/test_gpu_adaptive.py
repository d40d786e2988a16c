"""Adaptive windows on the GPU (ionize_step_adaptive) against the oracle's
adaptive step (oracle.adaptive_step).

The top of each cell's window is an integer that floating point decides
(the leak criterion against the tolerance), and the two sides evaluate the
rates and the leak in different orders (the mixed path from float rates), so
near the threshold they may choose different tops.  The tests therefore take
the device's top as the result to check: it must be the lowest slot at or
above the starting top whose oracle leak is within the tolerance (up to a
relative margin for rounding), or the storage limit when none is; the
populations must then equal the oracle's step forced to that top, to the
per-call tolerance (1e-12 FP64, 1e-6 mixed).  The window index is compared
bit for bit."""
import numpy as np
import pytest

from paper_2202_10647_amd import workloads as wl

pytestmark = pytest.mark.gpu

DT = 1.334e-16
TOL = {"f64": 1e-12, "mixed": 1e-6}


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2202_10647_amd import adkion
    assert torch.cuda.is_available()
    gases = {}
    for Z in (7, 18, 36):
        t = wl.synthetic_gas(Z)
        gases[Z] = (adkion.Gas.from_table(t), orc.GasSpec(t.U, t.l, t.m))
    return torch, adkion, gases


def adaptive_state(n, Z, wmax, seed):
    """Random windows: lo in [0, Z], wc in [0, wmax] (clipped to Z - lo),
    populations on slots 0..wc (exact zeros and sub-threshold slots)."""
    r = np.random.default_rng(seed)
    lo = r.integers(0, Z + 1, n).astype(np.uint8)
    wc = np.minimum(r.integers(0, wmax + 1, n), Z - lo.astype(int)).astype(np.uint8)
    P = r.exponential(size=(wmax + 1, n))
    kill = r.random((wmax + 1, n))
    P[kill < 0.2] = 0.0
    P[(kill >= 0.2) & (kill < 0.3)] *= 1e-9
    P[np.arange(wmax + 1)[:, None] > wc[None, :]] = 0.0
    s = P.sum(axis=0)
    P[0, s == 0] = 1.0
    return P / P.sum(axis=0), lo, wc


def run_device(torch, ak, gas, E, P, lo, wc, wmin, wmax, eps, tol, prec, counters=False, dt=DT):
    tdt = torch.float32 if prec == "mixed" else torch.float64
    n = E.size
    Et = torch.from_numpy(E).to(tdt).cuda()
    Pt = torch.from_numpy(P).to(tdt).cuda()
    Lt = torch.from_numpy(lo.copy()).cuda()
    Wt = torch.from_numpy(wc.copy()).cuda()
    work = ak.adaptive_workspace(n)
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda") if counters else None
    print(f"adaptive step: n={n} wmin={wmin} wmax={wmax} tol={tol} prec={prec}", flush=True)
    ak.ionize_step_adaptive(gas, Et, dt, Pt, Lt, Wt, wmin, wmax, eps=eps, tol=tol, work=work, counters=cnt)
    torch.cuda.synchronize()
    out = (Pt.cpu().numpy().astype(np.float64), Lt.cpu().numpy(), Wt.cpu().numpy())
    return out + ((cnt.cpu().numpy(),) if counters else ())


def check_against_oracle(orc, spec, E, P, lo, wc, wmin, wmax, eps, tol, prec, got, glo, gwc, margin, dt=DT):
    """Window index bit for bit, the device's top valid for the oracle's
    leaks, populations equal to the oracle forced to the device's top."""
    Z = spec.Z
    npdt = np.float32 if prec == "mixed" else np.float64
    E_in = E.astype(npdt).astype(np.float64)
    P_in = P.astype(npdt).astype(np.float64)
    ref, rlo, rwc, info = orc.adaptive_step(spec, E_in, dt, P_in, lo, wc, wmin, wmax, eps, tol)
    assert np.array_equal(glo, rlo)
    leaks = info["leaks"]
    room = np.minimum(wmax, Z - rlo.astype(int))
    # lowest slot with a leak within the tolerance on the oracle's numbers;
    # for every slot between the starting top and the device's top the leak
    # must exceed the tolerance (up to the margin), at the device's top it
    # must be within it (or the top is the storage limit)
    tested = leaks >= 0
    for c in np.nonzero(rwc != gwc)[0]:
        t = int(gwc[c])
        assert tested[t, c] or t == room[c], (c, t)
        below = [s for s in range(wmax + 1) if tested[s, c] and s < t and s < room[c]]
        assert all(leaks[s, c] > tol * (1 - margin) for s in below), (c, t, leaks[:, c])
        if t < room[c]:
            assert leaks[t, c] <= tol * (1 + margin), (c, t, leaks[:, c])
    frac = float(np.mean(rwc != gwc))
    forced, flo, fwc, _ = orc.adaptive_step(spec, E_in, dt, P_in, lo, wc, wmin, wmax, eps, tol,
                                            force_top=gwc.astype(np.int32))
    assert np.array_equal(fwc, gwc) and np.array_equal(flo, glo)
    fin = np.isfinite(E)
    err = float(np.max(np.abs(got[:, fin] - forced[:, fin]), initial=0.0))
    return err, frac


@pytest.mark.parametrize("prec", ["f64", "mixed"])
@pytest.mark.parametrize("Z,wmax,tol", [(7, 7, 1e-9), (18, 8, 1e-6), (18, 18, 1e-9), (36, 12, 1e-9),
                                        (36, 36, 1e-12), (36, 2, 1e-9)])
def test_random_states_match_oracle(env, orc, prec, Z, wmax, tol):
    torch, ak, gases = env
    gas, spec = gases[Z]
    n = 3000 + 37
    P, lo, wc = adaptive_state(n, Z, wmax, seed=Z * 100 + wmax)
    E = wl.loguniform_field(n, 10.0, 5000.0, seed=Z + wmax)
    E[::97] = 0.0
    E[5::89] *= -1.0
    got, glo, gwc, cnt = run_device(torch, ak, gas, E, P, lo, wc, 1, wmax, 1e-8, tol, prec, counters=True)
    err, frac = check_against_oracle(orc, spec, E, P, lo, wc, 1, wmax, 1e-8, tol, prec, got, glo, gwc,
                                     margin=1e-9 if prec == "f64" else 1e-5)
    print(f"max |dN| {err:.2e}, top differs from the oracle's own choice in {100 * frac:.3f} % of cells, "
          f"counters {cnt.tolist()}")
    assert err <= TOL[prec]
    assert frac <= 0.01
    # slots above each window hold zero; totals conserved
    assert np.all(got[np.arange(wmax + 1)[:, None] > gwc[None, :]] == 0.0)
    assert np.allclose(got.sum(axis=0), P.sum(axis=0), atol=1e-12 if prec == "f64" else 3e-6)
    # every cell whose window widened beyond eight rates went through the
    # wavefront tier, and no cell whose window was and stays within eight did
    assert cnt[0] >= int(np.sum((gwc > 8) & (gwc > wc)))
    assert cnt[0] <= int(np.sum((gwc > 8) | (np.minimum(wc, wmax) > 8)))


@pytest.mark.parametrize("prec", ["f64", "mixed"])
@pytest.mark.parametrize("w", [1, 2, 3, 5])
def test_fixed_width_is_the_fixed_window(env, orc, prec, w):
    """wmin = wmax = w: the oracle's fixed window of w rates."""
    torch, ak, gases = env
    Z = 18
    gas, spec = gases[Z]
    n = 4096 + 11
    P, lo = wl.random_window_state(n, Z, w, seed=70 + w)
    E = wl.loguniform_field(n, 10.0, 5000.0, seed=71 + w)
    wc = np.minimum(w, Z - lo.astype(int)).astype(np.uint8)
    got, glo, gwc = run_device(torch, ak, gas, E, P, lo, wc, w, w, 1e-8, 1e-9, prec)
    npdt = np.float32 if prec == "mixed" else np.float64
    ref, rlo = orc.ionize_step(spec, E.astype(npdt).astype(np.float64), DT, P.astype(npdt).astype(np.float64),
                               lo, w, 1e-8)
    assert np.array_equal(glo, rlo)
    assert np.array_equal(gwc, np.minimum(w, Z - rlo.astype(int)))
    assert np.max(np.abs(got - ref)) <= TOL[prec]


@pytest.mark.parametrize("Z", [7, 18])
def test_zero_tolerance_is_the_full_chain(env, orc, Z):
    """tol = 0 with room for every level: the oracle's full chain (FP64)."""
    torch, ak, gases = env
    gas, spec = gases[Z]
    n = 2000 + 5
    P, lo, wc = adaptive_state(n, Z, Z, seed=Z)
    E = wl.loguniform_field(n, 10.0, 5000.0, seed=Z + 1)
    got, glo, gwc = run_device(torch, ak, gas, E, P, lo, wc, 1, Z, 1e-8, 0.0, "f64")
    full = np.zeros((Z + 1, n))
    for s in range(Z + 1):
        k = lo.astype(int) + s
        ok = k <= Z
        full[k[ok], np.nonzero(ok)[0]] += P[s, ok]
    ref, rlo = orc.ionize_step(spec, E, DT, full, np.zeros(n, np.uint8), Z, 1e-8, layout=1)
    assert np.array_equal(glo, rlo)
    gfull = np.zeros_like(ref)
    for s in range(Z + 1):
        k = glo.astype(int) + s
        ok = k <= Z
        gfull[k[ok], np.nonzero(ok)[0]] += got[s, ok]
    assert np.max(np.abs(gfull - ref)) <= 1e-12


def test_nonfinite_fields_and_stripped_cells(env, orc):
    torch, ak, gases = env
    Z = 18
    gas, spec = gases[Z]
    n = 640
    P, lo, wc = adaptive_state(n, Z, 10, seed=5)
    E = wl.loguniform_field(n, 10.0, 5000.0, seed=6)
    E[:64] = np.nan
    E[64:128] = np.inf
    lo[128:192] = 200  # past Z: read as Z
    got, glo, gwc = run_device(torch, ak, gas, E, P, lo, wc, 1, 10, 1e-8, 1e-9, "f64")
    active = glo[:128] < Z
    assert np.all(np.isnan(got[:, :128][:, active][0]))
    assert np.all(glo[128:192] == Z) and np.all(gwc[128:192] == 0)
    assert np.array_equal(got[:, 128:192], P[:, 128:192])
    err, _ = check_against_oracle(orc, spec, E[192:], P[:, 192:], lo[192:], wc[192:], 1, 10, 1e-8, 1e-9, "f64",
                                  got[:, 192:], glo[192:], gwc[192:], 1e-9)
    assert err <= 1e-12


def test_pulse_trajectory_tracks_the_full_chain(env, orc):
    """Cells on the axis of the 3D pulse that it reaches gradually (36 levels,
    m averaged), the whole 500-step run from neutral cells, FP64: the
    adaptive window (tolerance 1e-9 per step) stays within 1e-6 of the
    device's full chain (w = Z, no shift) at every step, and every 50 steps
    one step is recomputed by the oracle from the device's input bits."""
    torch, ak, gases = env
    Z = 36
    gas, spec = gases[Z]
    mesh = wl.mesh_3d()
    nx, ny, nz = mesh.shape
    idx = np.concatenate([((nx // 2 + dx) * ny + ny // 2) * nz + np.arange(300, 512, 4) for dx in (0, 8, 24)])
    n = idx.size
    Pa = torch.zeros((Z + 1, n), dtype=torch.float64, device="cuda")
    Pa[0] = 1.0
    La = torch.zeros(n, dtype=torch.uint8, device="cuda")
    Wa = torch.ones(n, dtype=torch.uint8, device="cuda")
    Pf = Pa.clone()
    Lf = La.clone()
    work = ak.adaptive_workspace(n)
    lev = torch.arange(Z + 1, dtype=torch.float64, device="cuda")[:, None]
    worst = 0.0
    checked = 0
    for t in range(mesh.steps):
        E = torch.from_numpy(mesh.field_at(t, idx)).cuda()
        if t % 50 == 25:
            pre = (Pa.cpu().numpy(), La.cpu().numpy(), Wa.cpu().numpy())
        ak.ionize_step_adaptive(gas, E, mesh.dt, Pa, La, Wa, 1, Z, eps=1e-8, tol=1e-9, work=work)
        ak.ionize_step(gas, E, mesh.dt, Pf, Lf, w=Z, eps=0.0)
        if t % 50 == 25:
            got = (Pa.cpu().numpy(), La.cpu().numpy(), Wa.cpu().numpy())
            err, _ = check_against_oracle(orc, spec, E.cpu().numpy(), pre[0], pre[1], pre[2], 1, Z, 1e-8, 1e-9,
                                          "f64", *got, margin=1e-9, dt=mesh.dt)
            assert err <= 1e-12, (t, err)
            checked += 1
        full = torch.zeros_like(Pf)
        full.scatter_add_(0, (La.to(torch.int64)[None, :] + torch.arange(Z + 1, device="cuda")[:, None]).clamp(max=Z),
                          torch.where(La.to(torch.int64)[None, :] + torch.arange(Z + 1, device="cuda")[:, None] <= Z,
                                      Pa, torch.zeros_like(Pa)))
        worst = max(worst, float((full - Pf).abs().max()))
    ne = (lev * Pf).sum(0)
    print(f"max |dN| adaptive vs full chain over the run: {worst:.2e}; final mean charge {float(ne.mean()):.2f}")
    assert float(ne.max()) > 5.0
    assert worst <= 1e-6
    assert checked == 10


def test_graph_replay_matches_eager(env):
    torch, ak, gases = env
    Z = 36
    gas, _ = gases[Z]
    n = 20000 + 3
    wmax = 16
    P, lo, wc = adaptive_state(n, Z, wmax, seed=9)
    fields = torch.stack([torch.from_numpy(wl.loguniform_field(n, 10.0, 5000.0, seed=20 + s)) for s in range(4)]).cuda()
    P0 = torch.from_numpy(P).cuda()
    L0 = torch.from_numpy(lo).cuda()
    W0 = torch.from_numpy(wc).cuda()
    work = ak.adaptive_workspace(n)
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    Pt, Lt, Wt = P0.clone(), L0.clone(), W0.clone()
    for s in range(4):
        ak.ionize_step_adaptive(gas, fields[s], DT, Pt, Lt, Wt, 1, wmax, tol=1e-9, work=work, counters=cnt)
    torch.cuda.synchronize()
    want = (Pt.clone(), Lt.clone(), Wt.clone(), cnt.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for s in range(4):
            ak.ionize_step_adaptive(gas, fields[s], DT, Pt, Lt, Wt, 1, wmax, tol=1e-9, work=work, counters=cnt)
    for rep in range(3):
        Pt.copy_(P0)
        Lt.copy_(L0)
        Wt.copy_(W0)
        cnt.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Pt, want[0]) and torch.equal(Lt, want[1]) and torch.equal(Wt, want[2]), rep
        assert torch.equal(cnt, want[3]), rep
        _ = float(Pt.sum().item())
    assert int(want[3][0]) > 0
    del g


def test_argument_errors(env):
    torch, ak, gases = env
    gas, _ = gases[18]
    n = 64
    E = torch.ones(n, dtype=torch.float64, device="cuda") * 100
    P = torch.zeros((9, n), dtype=torch.float64, device="cuda")
    L = torch.zeros(n, dtype=torch.uint8, device="cuda")
    W = torch.ones(n, dtype=torch.uint8, device="cuda")
    work = ak.adaptive_workspace(n)
    small = ak.adaptive_workspace(n - 1)
    for kw, status in ((dict(wmin=1, wmax=8, work=small), ak.ADK_EINVAL),
                       (dict(wmin=9, wmax=8, work=work), ak.ADK_ERANGE),
                       (dict(wmin=1, wmax=8, tol=float("nan"), work=work), ak.ADK_EINVAL),
                       (dict(wmin=1, wmax=8, tol=-1.0, work=work), ak.ADK_EINVAL),
                       (dict(wmin=1, wmax=8, eps=-1.0, work=work), ak.ADK_EINVAL)):
        with pytest.raises(ak.AdkError) as e:
            ak.ionize_step_adaptive(gas, E, DT, P, L, W, **kw)
        assert e.value.status == status, kw
    P19 = torch.zeros((20, n), dtype=torch.float64, device="cuda")
    with pytest.raises(ak.AdkError) as e:
        ak.ionize_step_adaptive(gas, E, DT, P19, L, W, 1, 19, work=work)  # wmax > Z
    assert e.value.status == ak.ADK_ERANGE
