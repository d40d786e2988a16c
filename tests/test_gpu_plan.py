"""Batched plan (cells of several gases with uneven windows, one launch per
launch group) against the oracle, per (gas, window) group, from identical inputs."""
import numpy as np
import pytest

from paper_2202_10647_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "mixed": 1e-6}
DT = 1.334e-16
ZS = (1,) + wl.DOPANT_Z


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2202_10647_amd import adkion
    assert torch.cuda.is_available()
    tables = [wl.synthetic_gas(z) for z in ZS]
    gases = [adkion.Gas.from_table(t) for t in tables]
    specs = [orc.GasSpec(t.U, t.l, t.m) for t in tables]
    return torch, adkion, gases, specs


def plan_state(cell_gas, cell_w, rows, seed):
    return wl.plan_window_state(cell_gas, cell_w, ZS, rows, seed)


def oracle_plan(orc, specs, cell_gas, cell_w, E, pops, lo, eps):
    ref = pops.copy()
    rlo = lo.copy()
    for g in range(len(ZS)):
        for w in range(1, 7):
            idx = np.nonzero((cell_gas == g) & (cell_w == w))[0]
            if idx.size == 0:
                continue
            p2, l2 = orc.ionize_step(specs[g], E[idx], DT, pops[: w + 1, idx], lo[idx], w, eps)
            ref[: w + 1, idx] = p2
            rlo[idx] = l2
    return ref, rlo


@pytest.mark.parametrize("prec", ["mixed", "f64"])
@pytest.mark.parametrize("cpl", [1, 2, 4, 0])
def test_plan_matches_oracle(env, orc, prec, cpl):
    torch, ak, gases, specs = env
    n = 40000 + 123
    cell_gas, cell_w = wl.batched_cells(n, seed=9, dopant_fraction=0.3)
    plan = ak.Plan(gases, cell_gas, cell_w, prec=prec, eps=1e-8, cells_per_lane=cpl)
    info = plan.info
    assert info["rows"] == 7 and info["ngas"] == 5
    if cpl:
        assert info["cells_per_lane"] == cpl
    else:
        assert info["cells_per_lane"] in (1, 2, 4)
    npdt = np.float32 if prec == "mixed" else np.float64
    tdt = torch.float32 if prec == "mixed" else torch.float64
    pops, lo = plan_state(cell_gas, cell_w, info["rows"], seed=100 + cpl)
    pops = pops.astype(npdt)
    E = wl.hash_field(n, seed=17, step=3, dtype=npdt)
    E[::41] = 0.0
    Pt = torch.from_numpy(pops).cuda()
    Lt = torch.from_numpy(lo).cuda()
    plan.step(torch.from_numpy(E).cuda(), DT, Pt, Lt)
    torch.cuda.synchronize()
    out, l2 = Pt.cpu().numpy().astype(np.float64), Lt.cpu().numpy()
    ref, rlo = oracle_plan(orc, specs, cell_gas, cell_w, E.astype(np.float64), pops.astype(np.float64), lo, 1e-8)
    assert np.array_equal(l2, rlo)
    err = np.max(np.abs(out - ref))
    assert err <= TOL[prec], err
    # rows above each cell's window are untouched
    for w in range(1, 6):
        idx = np.nonzero(cell_w == w)[0]
        assert np.all(out[w + 1:, idx] == np.float64(npdt(0.625)))
    # a second launch of the same plan
    plan.step(torch.from_numpy(E).cuda(), DT, Pt, Lt)
    torch.cuda.synchronize()
    ref2, rlo2 = oracle_plan(orc, specs, cell_gas, cell_w, E.astype(np.float64), out.astype(npdt).astype(np.float64),
                             l2, 1e-8)
    assert np.array_equal(Lt.cpu().numpy(), rlo2)
    assert np.max(np.abs(Pt.cpu().numpy().astype(np.float64) - ref2)) <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["mixed", "f64"])
def test_plan_launch_groups(env, orc, prec):
    """Widths with many cells get launches of their own (compiled for that
    width), runs of sparse widths share one: 600k cells w = 1 and 600k cells
    w = 3 (solo), sparse w = 2 and w = 4..6 (two shared launches), interleaved
    at random over the mesh.  Sampled cells of every (gas, w) group against
    the oracle, launch by launch as reported in the plan's info."""
    torch, ak, gases, specs = env
    rng = np.random.default_rng(77)
    na, nb, nc = 600_000, 600_000, 120_000
    g = np.concatenate([np.zeros(na, np.uint8), np.full(nb, 2, np.uint8), rng.integers(1, 5, nc).astype(np.uint8)])
    w = np.concatenate([np.ones(na, np.uint8), np.full(nb, 3, np.uint8), rng.integers(2, 7, nc).astype(np.uint8)])
    order = rng.permutation(g.size)
    cell_gas, cell_w = g[order], w[order]
    n = cell_gas.size
    plan = ak.Plan(gases, cell_gas, cell_w, prec=prec, eps=1e-8, cells_per_lane=0)
    info = plan.info
    assert info["nlaunches"] == 4
    assert info["launch_wmax"] == [6, 3, 2, 1]
    cells = info["launch_cells"]
    assert cells[1] == int(np.sum(cell_w == 3)) and cells[3] == int(np.sum(cell_w == 1))
    assert cells[0] == int(np.sum(cell_w >= 4)) and cells[2] == int(np.sum(cell_w == 2))
    assert sum(info["launch_tiles"]) == info["ntiles"]
    assert all(c in (1, 2, 4) for c in info["launch_cpl"])
    npdt = np.float32 if prec == "mixed" else np.float64
    pops, lo = plan_state(cell_gas, cell_w, info["rows"], seed=123)
    pops = pops.astype(npdt)
    E = wl.hash_field(n, seed=19, step=1, dtype=npdt)
    Pt = torch.from_numpy(pops).cuda()
    Lt = torch.from_numpy(lo).cuda()
    plan.step(torch.from_numpy(E).cuda(), DT, Pt, Lt)
    torch.cuda.synchronize()
    samp = np.unique(np.concatenate([rng.choice(np.nonzero((cell_gas == gi) & (cell_w == wi))[0], 400)
                                     for gi in range(len(ZS)) for wi in range(1, 7)
                                     if np.any((cell_gas == gi) & (cell_w == wi))]))
    idx = torch.from_numpy(samp).cuda()
    out, l2 = Pt[:, idx].cpu().numpy().astype(np.float64), Lt[idx].cpu().numpy()
    sg, sw = cell_gas[samp], cell_w[samp]
    ref, rlo = oracle_plan(orc, specs, sg, sw, E[samp].astype(np.float64), pops[:, samp].astype(np.float64),
                           lo[samp], 1e-8)
    assert np.array_equal(l2, rlo)
    assert np.max(np.abs(out - ref)) <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("n,nlaunches", [(30000, 1), (600000, 2)])
def test_plan_graph_replay(env, orc, n, nlaunches):
    """Eight plan steps captured in one HIP graph, replayed three times with
    eager work in between: bitwise equal to eager launches.  With two launch
    groups (a solo w = 1 group of the host gas and one shared group of the
    dopants) each step forks the dopant launch onto the plan's side stream and
    joins it back, captured as parallel branches."""
    torch, ak, gases, specs = env
    cell_gas, cell_w = wl.batched_cells(n, seed=3, dopant_fraction=0.2 if n < 100000 else 0.05)
    plan = ak.Plan(gases, cell_gas, cell_w, prec="mixed", cells_per_lane=2)
    assert plan.info["nlaunches"] == nlaunches
    rows = plan.info["rows"]
    pops, lo = plan_state(cell_gas, cell_w, rows, seed=5)
    P0 = torch.from_numpy(pops.astype(np.float32)).cuda()
    L0 = torch.from_numpy(lo).cuda()
    fields = torch.stack([torch.from_numpy(wl.hash_field(n, 11, s, dtype=np.float32)) for s in range(8)]).cuda()
    P, L = P0.clone(), L0.clone()
    for s in range(8):
        plan.step(fields[s], DT, P, L)
    torch.cuda.synchronize()
    want_p, want_l = P.clone(), L.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for s in range(8):
            plan.step(fields[s], DT, P, L)
    for rep in range(3):
        P.copy_(P0)
        L.copy_(L0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(P, want_p) and torch.equal(L, want_l), rep
        _ = float(P.sum().item())
    del g
    plan.close()


@pytest.mark.parametrize("prec", ["mixed", "f64"])
def test_field_hash_matches_host_definition(env, prec):
    torch, ak, gases, specs = env
    n = 100003
    tdt = torch.float32 if prec == "mixed" else torch.float64
    E = torch.empty(n, dtype=tdt, device="cuda")
    ak.field_hash(E, seed=4, step=12, E_lo=10.0, E_hi=5000.0)
    g = E.cpu().numpy().astype(np.float64)
    h = wl.hash_field(n, 4, 12, 10.0, 5000.0, dtype=np.float64)
    rel = np.abs(g - h) / h
    # exp of an argument up to ~8.5 rounded two ways: a few double ulps
    assert rel.max() < (1.2e-7 if prec == "mixed" else 5e-15)
    assert g.min() >= 10.0 * (1 - 1e-6) and g.max() <= 5000.0 * (1 + 1e-6)


def test_plan_errors(env):
    torch, ak, gases, specs = env
    with pytest.raises(ak.AdkError) as e:
        ak.Plan(gases[:2], np.array([0, 2], np.uint8), np.array([1, 1], np.uint8))
    assert e.value.status == ak.ADK_ERANGE  # gas index out of range
    with pytest.raises(ak.AdkError) as e:
        ak.Plan(gases[:1], np.array([0], np.uint8), np.array([2], np.uint8))
    assert e.value.status == ak.ADK_ERANGE  # w > Z
    with pytest.raises(ak.AdkError) as e:
        ak.Plan(gases, np.array([3], np.uint8), np.array([7], np.uint8))
    assert e.value.status == ak.ADK_ERANGE  # w > ADK_PLAN_MAX_W
    p = ak.Plan(gases, np.zeros(0, np.uint8), np.zeros(0, np.uint8))
    assert p.info["ntiles"] == 0
    p.close()


def test_plan_graph_replay_entry_point(env, orc):
    """adk_plan_graph_replay: one step, then seven more replayed as the plan's
    own captured graph (two launch groups: fork and join inside the graph),
    bitwise equal to eight eager steps; the cached graph is replayed again,
    captured anew for new arrays, and inside a caller's capture the steps join
    the caller's graph.  Errors before any step and for nsteps < 0."""
    torch, ak, gases, specs = env
    n = 600000
    cell_gas, cell_w = wl.batched_cells(n, seed=8, dopant_fraction=0.05)
    plan = ak.Plan(gases, cell_gas, cell_w, prec="mixed", cells_per_lane=2)
    assert plan.info["nlaunches"] == 2
    with pytest.raises(ak.AdkError) as e:
        plan.graph_replay(3)  # no step yet
    assert e.value.status == ak.ADK_EINVAL
    rows = plan.info["rows"]
    pops, lo = plan_state(cell_gas, cell_w, rows, seed=9)
    P0 = torch.from_numpy(pops.astype(np.float32)).cuda()
    L0 = torch.from_numpy(lo).cuda()
    E = torch.from_numpy(wl.hash_field(n, 21, 1, dtype=np.float32)).cuda()
    P, L = P0.clone(), L0.clone()
    for _ in range(8):
        plan.step(E, DT, P, L)
    torch.cuda.synchronize()
    want_p, want_l = P.clone(), L.clone()
    for rep in range(2):  # captured on the first pass, cached on the second
        P.copy_(P0)
        L.copy_(L0)
        plan.step(E, DT, P, L)
        plan.graph_replay(7)
        torch.cuda.synchronize()
        assert torch.equal(P, want_p) and torch.equal(L, want_l), rep
    P2, L2 = P0.clone(), L0.clone()  # new arrays: captured again
    plan.step(E, DT, P2, L2)
    plan.graph_replay(7)
    torch.cuda.synchronize()
    assert torch.equal(P2, want_p) and torch.equal(L2, want_l)
    P2.copy_(P0)
    L2.copy_(L0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.step(E, DT, P2, L2)
        plan.graph_replay(7)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(P2, want_p) and torch.equal(L2, want_l)
    del g
    with pytest.raises(ak.AdkError) as e:
        plan.graph_replay(-1)
    assert e.value.status == ak.ADK_EINVAL
    plan.close()


@pytest.mark.parametrize("prec", ["mixed", "f64"])
def test_plan_full_size_sampled(env, orc, prec):
    """The benchmark's batched mix at full size: 16,777,216 cells, 1 %
    dopants of 7, 18, 36 and 54 levels with w = 1..6, the launch groups and
    cells per lane the autotuner picks (the launch configuration the
    benchmark times).  One step from a seeded window state in a host-made
    log-uniform field; 10,000 host cells and 10,000 dopant cells are
    recomputed by the oracle."""
    torch, ak, gases, specs = env
    n = 1 << 24
    cell_gas, cell_w = wl.batched_cells(n, seed=4)
    plan = ak.Plan(gases, cell_gas, cell_w, prec=prec, eps=1e-8, cells_per_lane=0)
    rows = plan.info["rows"]
    npdt = np.float32 if prec == "mixed" else np.float64
    pops, lo = plan_state(cell_gas, cell_w, rows, seed=31)
    pops = pops.astype(npdt)
    E = wl.hash_field(n, seed=19, step=3, dtype=npdt)
    Pt = torch.from_numpy(pops).cuda()
    Lt = torch.from_numpy(lo).cuda()
    plan.step(torch.from_numpy(E).cuda(), DT, Pt, Lt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    dop = np.nonzero(cell_gas > 0)[0]
    host = np.nonzero(cell_gas == 0)[0]
    samp = np.unique(np.concatenate([rng.choice(host, 10000, replace=False), rng.choice(dop, 10000, replace=False)]))
    idx = torch.from_numpy(samp).cuda()
    out, l2 = Pt[:, idx].cpu().numpy().astype(np.float64), Lt[idx].cpu().numpy()
    ref, rlo = oracle_plan(orc, specs, cell_gas[samp], cell_w[samp], E[samp].astype(np.float64),
                           pops[:, samp].astype(np.float64), lo[samp], 1e-8)
    assert np.array_equal(l2, rlo)
    assert np.max(np.abs(out - ref)) <= TOL[prec]
    # rows above a cell's window are left as they were
    above = np.arange(rows)[:, None] > cell_w[samp][None, :]
    assert np.array_equal(out[above], pops[:, samp].astype(np.float64)[above])
    del Pt, Lt, idx
    plan.close()
    torch.cuda.empty_cache()


def test_tune_cache_file(env, orc, tmp_path, monkeypatch):
    """ADK_TUNE_CACHE: a first plan is tuned and stores one entry per launch
    group; the same plan again takes every choice from the file (from_cache
    = 1, same cells per lane); a corrupt file is tuned again and appended to;
    valid entries after corrupt lines are still used, and a choice written
    into the file is the one the plan runs with (checked against the oracle)."""
    torch, ak, gases, specs = env
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("ADK_TUNE_CACHE", str(path))
    n = 40000 + 123
    cell_gas, cell_w = wl.batched_cells(n, seed=9, dopant_fraction=0.3)
    p1 = ak.Plan(gases, cell_gas, cell_w, prec="mixed", eps=1e-8, cells_per_lane=0)
    i1 = p1.info
    p1.close()
    nl = i1["nlaunches"]
    assert i1["from_cache"] == 0 and i1["tuned_us"] > 0.0
    lines = path.read_text().splitlines()
    assert len(lines) == nl
    assert sorted(int(l.split()[1]) for l in lines) == sorted(i1["launch_cpl"])
    p2 = ak.Plan(gases, cell_gas, cell_w, prec="mixed", eps=1e-8, cells_per_lane=0)
    i2 = p2.info
    p2.close()
    assert i2["from_cache"] == 1 and i2["launch_cpl"] == i1["launch_cpl"]
    assert len(path.read_text().splitlines()) == nl  # nothing appended on a hit
    # corrupt file: tuned again, entries appended
    path.write_text("not a cache file\n\x00garbage 7\n")
    p3 = ak.Plan(gases, cell_gas, cell_w, prec="mixed", eps=1e-8, cells_per_lane=0)
    i3 = p3.info
    p3.close()
    assert i3["from_cache"] == 0
    assert len(path.read_text().splitlines()) == 2 + nl
    # valid entries after corrupt lines, each set to a choice of our own
    keys = [l.split()[0] for l in lines]
    forced = [4 if int(l.split()[1]) != 4 else 1 for l in lines]
    path.write_text("junk line\n" + "".join(f"{k} {c}\n" for k, c in zip(keys, forced)) + keys[0][:10])
    p4 = ak.Plan(gases, cell_gas, cell_w, prec="mixed", eps=1e-8, cells_per_lane=0)
    i4 = p4.info
    assert i4["from_cache"] == 1
    assert sorted(i4["launch_cpl"]) == sorted(forced)
    pops, lo = plan_state(cell_gas, cell_w, i4["rows"], seed=321)
    pops = pops.astype(np.float32)
    E = wl.hash_field(n, seed=23, step=2, dtype=np.float32)
    Pt = torch.from_numpy(pops).cuda()
    Lt = torch.from_numpy(lo).cuda()
    p4.step(torch.from_numpy(E).cuda(), DT, Pt, Lt)
    torch.cuda.synchronize()
    ref, rlo = oracle_plan(orc, specs, cell_gas, cell_w, E.astype(np.float64), pops.astype(np.float64), lo, 1e-8)
    assert np.array_equal(Lt.cpu().numpy(), rlo)
    assert np.max(np.abs(Pt.cpu().numpy().astype(np.float64) - ref)) <= TOL["mixed"]
    p4.close()


@pytest.mark.parametrize("prec", ["mixed", "f64"])
def test_plan_grouped_layout(env, orc, prec):
    """ADK_PLAN_GROUPED: the arrays hold the cells in the plan's order (each
    (gas, w) group contiguous).  The order is a permutation whose groups are
    contiguous runs in mesh order within each; a grouped step equals the
    mesh-order step of the same cells bit for bit, and the oracle."""
    torch, ak, gases, specs = env
    n = 60000 + 77
    cell_gas, cell_w = wl.batched_cells(n, seed=12, dopant_fraction=0.2)
    pm = ak.Plan(gases, cell_gas, cell_w, prec=prec, eps=1e-8, cells_per_lane=2)
    pg = ak.Plan(gases, cell_gas, cell_w, prec=prec, eps=1e-8, cells_per_lane=2, layout="grouped")
    assert pg.info["layout"] == ak.ADK_PLAN_GROUPED and pm.info["layout"] == ak.ADK_PLAN_MESH_ORDER
    order = pg.order()
    assert np.array_equal(order, pm.order())
    assert np.array_equal(np.sort(order), np.arange(n))
    key = cell_gas[order].astype(np.int64) * 8 + cell_w[order]
    runs = np.count_nonzero(np.diff(key)) + 1
    assert runs == np.unique(key).size  # one contiguous run per (gas, w)
    same = np.diff(key) == 0
    assert np.all(np.diff(order)[same] > 0)  # mesh order kept within a group
    npdt = np.float32 if prec == "mixed" else np.float64
    rows = pg.info["rows"]
    pops, lo = plan_state(cell_gas, cell_w, rows, seed=55)
    pops = pops.astype(npdt)
    E = wl.hash_field(n, seed=29, step=4, dtype=npdt)
    E[::37] = 0.0
    Pm, Lm = torch.from_numpy(pops).cuda(), torch.from_numpy(lo).cuda()
    pm.step(torch.from_numpy(E).cuda(), DT, Pm, Lm)
    Pg = torch.from_numpy(np.ascontiguousarray(pops[:, order])).cuda()
    Lg = torch.from_numpy(np.ascontiguousarray(lo[order])).cuda()
    pg.step(torch.from_numpy(np.ascontiguousarray(E[order])).cuda(), DT, Pg, Lg)
    torch.cuda.synchronize()
    outm, outg = Pm.cpu().numpy(), Pg.cpu().numpy()
    assert np.array_equal(outg, outm[:, order]) and np.array_equal(Lg.cpu().numpy(), Lm.cpu().numpy()[order])
    ref, rlo = oracle_plan(orc, specs, cell_gas, cell_w, E.astype(np.float64), pops.astype(np.float64), lo, 1e-8)
    assert np.array_equal(Lm.cpu().numpy(), rlo)
    assert np.max(np.abs(outm.astype(np.float64) - ref)) <= TOL[prec]
    pm.close()
    pg.close()
