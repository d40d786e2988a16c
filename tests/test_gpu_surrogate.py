"""Band-column surrogate on the GPU against the CPU references: exact band
columns (FP64 analytic solver) against the oracle, network output and
gradient against the FP64 network with bfloat16 operands, one Adam step,
deterministic and resumable training, the surrogate-form step against its
reference, graph replay, fallback, and what training gains.

Tolerances of the network comparisons.  The device network rounds h1, h2 and
h3 to bfloat16 after FP32 arithmetic, the reference after FP64 arithmetic.
The pre-rounding values differ by ~1e-7 relative, so on a small fraction of
the activations the two sides round to neighbouring bfloat16 values (one
unit in the 8th bit, 0.4-0.8 % of the value); such a sample's output moves
by up to ~1e-3.  Elsewhere the outputs agree to FP32 rounding (~1e-6).  The
tests therefore bound a high quantile tightly and the maximum loosely."""
import numpy as np
import pytest

from oracle import mlp
from paper_2202_10647_amd import workloads as wl

pytestmark = pytest.mark.gpu

DT = 1.334e-16
RNG = mlp.Range()


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2202_10647_amd import adkion
    assert torch.cuda.is_available()
    gases = {}
    for Z in (7, 36):
        t = wl.synthetic_gas(Z)
        gases[Z] = (adkion.Gas.from_table(t), orc.GasSpec(t.U, t.l, t.m))
    return torch, adkion, gases


def _dev(torch, E, dt, k):
    return (torch.from_numpy(np.ascontiguousarray(E, np.float64)).cuda(),
            torch.from_numpy(np.array(np.broadcast_to(dt, np.shape(E)), np.float64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(k, np.int32)).cuda())


@pytest.mark.parametrize("Z", [7, 36])
def test_band_columns_match_oracle(env, orc, Z):
    torch, ak, gases = env
    gas, spec = gases[Z]
    n = 3000
    E, dt, k = wl.surrogate_samples(n, 21, Z)
    k[:40] = Z - 1
    k[40:80] = Z - 2
    E[80:90] = 0.0
    E[90:100] = 2e5
    dt[100:110] = 1e-22
    ref = mlp.exact_band_columns(orc, spec, Z, E, dt, k)
    got = ak.band_columns(gas, *_dev(torch, E, dt, k)).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12
    assert np.allclose(got.sum(axis=0), 1.0, atol=1e-14)
    # invalid level or step: NaN columns, nothing else touched
    kk = np.array([-1, Z, 0], np.int32)
    bad = ak.band_columns(gas, *_dev(torch, np.array([100.0] * 3), np.array([DT, DT, -1.0]), kk)).cpu().numpy()
    assert np.all(np.isnan(bad))


def test_forward_matches_oracle(env, orc):
    torch, ak, gases = env
    Z = 36
    gas, _ = gases[Z]
    params = wl.mlp_init(Z, 5)
    net = ak.Mlp(gas, params)
    n = 20000 + 7
    E, dt, k = wl.surrogate_samples(n, 22, Z)
    Q = net.forward(*_dev(torch, E, dt, k)).cpu().numpy().astype(np.float64)
    u, v = RNG.features(E, dt)
    Qo, _ = mlp.forward(params.astype(np.float64), Z, u, v, k)
    d = np.abs(Q - Qo.T).max(axis=0)
    assert np.quantile(d, 0.9) <= 1e-5, np.quantile(d, [0.5, 0.9, 0.99])
    assert d.max() <= 1e-2
    assert np.all(Q >= 0) and np.allclose(Q.sum(axis=0), 1.0, atol=1e-6)
    net.close()


def test_loss_grad_matches_oracle(env, orc):
    torch, ak, gases = env
    Z = 36
    gas, spec = gases[Z]
    params = wl.mlp_init(Z, 6)
    b = mlp.unpack(params.astype(np.float64).copy(), Z)
    r = np.random.default_rng(3)
    for name in ("b1", "b2", "b3", "b4"):  # non-zero biases exercise every bias gradient path
        b[name][:] = r.uniform(-0.2, 0.2, b[name].shape)
    params = mlp.pack(b, Z).astype(np.float32)
    net = ak.Mlp(gas, params)
    n = 2048 + 13
    E, dt, k = wl.surrogate_samples(n, 23, Z)
    P = mlp.exact_band_columns(orc, spec, Z, E, dt, k).T
    u, v = RNG.features(E, dt)
    Lo, go = mlp.loss_and_grad(params.astype(np.float64), Z, u, v, k, P)
    L, g = net.loss_grad(*_dev(torch, E, dt, k))
    L = float(L.item())
    g = g.cpu().numpy().astype(np.float64)
    assert abs(L - Lo) <= 1e-4 * Lo, (L, Lo)
    off = 0
    for name, shape in mlp.block_shapes(Z):
        m = int(np.prod(shape))
        a, o = g[off:off + m], go[off:off + m]
        assert np.linalg.norm(a - o) <= 2e-3 * np.linalg.norm(o) + 1e-9, (name, np.linalg.norm(a - o), np.linalg.norm(o))
        off += m
    net.close()


def test_one_training_step_is_adam_on_the_oracle_gradient(env, orc):
    """First Adam step from the seeded network on the seeded training set:
    the device sampler, the targets, the gradient and the update together
    against the references (update lr g/(|g| + eps) is insensitive to small
    gradient differences wherever |g| >> eps)."""
    torch, ak, gases = env
    Z = 7
    gas, spec = gases[Z]
    p0 = wl.mlp_init(Z, 9)
    lr = 1e-3
    net = ak.Mlp(gas, p0)
    net.train(1, nsamples=1024, batch=1024, lr=lr, lr_min=lr, seed=31)
    gp, gm, gv, step = net.state()
    assert step == 1
    E, dt, k = wl.surrogate_samples(1024, 31, Z)
    P = mlp.exact_band_columns(orc, spec, Z, E, dt, k).T
    u, v = RNG.features(E, dt)
    _, g = mlp.loss_and_grad(p0.astype(np.float64), Z, u, v, k, P)
    p1, m1, v1 = mlp.adam_step(p0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    big = np.abs(g) > 1e-5
    assert big.mean() > 0.5
    assert np.max(np.abs(gp[big] - p1[big])) <= 1e-3 * lr + 1e-7
    assert np.max(np.abs(gp - p0)) <= lr * (1 + 1e-6) + 1e-7
    assert np.linalg.norm(gm - m1) <= 2e-3 * np.linalg.norm(m1)
    net.close()


def test_training_is_deterministic_and_resumes_bitwise(env, tmp_path):
    torch, ak, gases = env
    Z = 7
    gas, _ = gases[Z]
    p0 = wl.mlp_init(Z, 8)
    kw = dict(nsamples=8192, batch=512, total_iters=60, seed=4, lr=3e-3)
    a = ak.Mlp(gas, p0)
    la = a.train(60, **kw)
    b = ak.Mlp(gas, p0)
    lb1 = b.train(25, **kw)
    path = str(tmp_path / "net.bin")
    b.save(path)
    b.close()
    c = ak.Mlp.load(gas, path)
    lb2 = c.train(35, **kw)
    sa, sc = a.state(), c.state()
    assert sa[3] == sc[3] == 60
    for x, y in zip(sa[:3], sc[:3]):
        assert np.array_equal(x, y)
    assert np.array_equal(la, np.concatenate([lb1, lb2]))
    d = ak.Mlp(gas, p0)
    assert np.array_equal(d.train(60, **kw), la)
    assert np.array_equal(d.state()[0], sa[0])
    assert la[-10:].mean() < 0.5 * la[:5].mean()
    # a corrupt or foreign file is rejected
    with open(path, "r+b") as f:
        f.write(b"XXXX")
    with pytest.raises(ak.AdkError):
        ak.Mlp.load(gas, path)
    with pytest.raises(ak.AdkError):
        ak.Mlp.load(gases[36][0], str(tmp_path / "missing.bin"))
    for net in (a, c, d):
        net.close()


def _mixed_fields(n, seed):
    """70 % in the trained range, 10 % zero, 10 % in (2, 10) GV/m, 10 % above
    the range; float32 values."""
    r = np.random.default_rng(seed)
    E = np.exp(r.uniform(np.log(10.0), np.log(5000.0), n))
    sel = r.random(n)
    E[sel < 0.1] = 0.0
    m = (sel >= 0.1) & (sel < 0.2)
    E[m] = r.uniform(2.0, 9.9, m.sum())
    m = (sel >= 0.2) & (sel < 0.3)
    E[m] = r.uniform(5100.0, 9000.0, m.sum())
    return E.astype(np.float32)


@pytest.mark.parametrize("w", [1, 2, 3])
def test_surrogate_step_matches_reference(env, orc, w):
    torch, ak, gases = env
    Z = 36
    gas, spec = gases[Z]
    # below 10 GV/m every rate of this gas gives W dt < 1e-30 (under the
    # field cutoff: identity on either path, not counted); above the range
    # the analytic fallback is counted
    assert (orc.rates(spec, np.array([10.0])) * DT).max() < 1e-30
    params = wl.mlp_init(Z, 12)
    net = ak.Mlp(gas, params)
    n = 20000 + 37
    N, lo = wl.random_window_state(n, Z, w, seed=40 + w, dtype=np.float32)
    E = _mixed_fields(n, 50 + w)
    eps = 1e-8
    Pt = torch.from_numpy(N).cuda()
    Lt = torch.from_numpy(lo).cuda()
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    ak.surrogate_step(gas, net, torch.from_numpy(E).cuda(), DT, Pt, Lt, w=w, eps=eps, counters=cnt)
    got, glo = Pt.cpu().numpy().astype(np.float64), Lt.cpu().numpy()
    ref, rlo, use, x = mlp.surrogate_step(orc, spec, Z, params.astype(np.float64), RNG, E.astype(np.float64), DT,
                                          N.astype(np.float64), lo, w, eps)
    assert np.array_equal(glo, rlo)
    ana = ~use
    assert np.max(np.abs(got[:, ana] - ref[:, ana])) <= 1e-6
    # a source whose W dt lies within a factor 3 of the negligible threshold
    # may be judged either way by the two sides' rate evaluations
    th = mlp.NEGLIGIBLE_XDT
    clear = ~np.any((x > th / 3) & (x < 3 * th), axis=0)
    sel = use & clear
    assert sel.sum() > 0.9 * use.sum()
    d = np.abs(got[:, sel] - ref[:, sel]).max(axis=0)
    assert np.quantile(d, 0.9) <= 1e-5 and d.max() <= 1e-2, np.quantile(d, [0.5, 0.9, 0.99, 1.0])
    # negligible sources keep their population exactly (identity columns)
    negl = sel & np.all((x < th) | (np.arange(w)[:, None] >= np.minimum(w, Z - rlo.astype(int))[None, :]), axis=0)
    assert np.max(np.abs(got[:, negl] - ref[:, negl]), initial=0.0) <= 1e-6
    # conservation and non-negativity of the network columns
    assert np.allclose(got[:, use].sum(axis=0), N[:, use].astype(np.float64).sum(axis=0), atol=3e-6)
    assert np.all(got[:, use] >= 0)
    c = cnt.cpu().numpy()
    _, p_shift = mlp.window_shift(N, lo, Z, eps)
    E64 = E.astype(np.float64)
    fb = (~use) & (p_shift < Z) & (E64 > 5000.0)
    assert c[0] == fb.sum()
    top = np.minimum(w, Z - p_shift)
    needed = (np.arange(w)[:, None] < top[None, :]) & (x >= th)
    assert abs(int(c[1]) - int(needed[:, use].sum())) <= int((~clear & use).sum()) * w
    net.close()


def test_surrogate_outside_step_range_is_the_analytic_step(env):
    torch, ak, gases = env
    Z = 36
    gas, _ = gases[Z]
    net = ak.Mlp(gas, wl.mlp_init(Z, 13))
    n = 30000
    N, lo = wl.random_window_state(n, Z, 3, seed=60, dtype=np.float32)
    E = torch.from_numpy(_mixed_fields(n, 61)).cuda()
    dt = 5e-16  # above the trained 0.2 fs
    P1, L1 = torch.from_numpy(N).cuda(), torch.from_numpy(lo).cuda()
    P2, L2 = P1.clone(), L1.clone()
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    ak.surrogate_step(gas, net, E, dt, P1, L1, w=3, counters=cnt)
    ak.ionize_step(gas, E, dt, P2, L2, 3)
    assert torch.equal(L1, L2)
    assert float((P1 - P2).abs().max()) <= 1e-7
    assert int(cnt[1]) == 0 and int(cnt[0]) > 0
    net.close()


def test_surrogate_graph_replay(env):
    torch, ak, gases = env
    Z = 36
    gas, _ = gases[Z]
    net = ak.Mlp(gas, wl.mlp_init(Z, 14))
    n = 50000
    N, lo = wl.random_window_state(n, Z, 3, seed=70, dtype=np.float32)
    P0, L0 = torch.from_numpy(N).cuda(), torch.from_numpy(lo).cuda()
    fields = torch.stack([torch.from_numpy(_mixed_fields(n, 80 + s)) for s in range(4)]).cuda()
    zero = torch.zeros(2, dtype=torch.int64, device="cuda")
    cnt = zero.clone()
    P, L = P0.clone(), L0.clone()
    for s in range(4):
        ak.surrogate_step(gas, net, fields[s], DT, P, L, counters=cnt)
    torch.cuda.synchronize()
    want_p, want_l, want_c = P.clone(), L.clone(), cnt.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for s in range(4):
            ak.surrogate_step(gas, net, fields[s], DT, P, L, counters=cnt)
    for rep in range(3):
        P.copy_(P0)
        L.copy_(L0)
        cnt.copy_(zero)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(P, want_p) and torch.equal(L, want_l) and torch.equal(cnt, want_c), rep
        _ = float(P.sum().item())
    del g
    net.close()


def test_surrogate_argument_errors(env):
    torch, ak, gases = env
    g36, _ = gases[36]
    g7, _ = gases[7]
    net = ak.Mlp(g36, wl.mlp_init(36, 1))
    n = 64
    E = torch.ones(n, dtype=torch.float32, device="cuda") * 100
    P = torch.zeros((5, n), dtype=torch.float32, device="cuda")
    L = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(ak.AdkError) as e:
        ak.surrogate_step(g36, net, E, DT, P, L, w=4)
    assert e.value.status == ak.ADK_ERANGE
    with pytest.raises(ak.AdkError) as e:
        ak.surrogate_step(g7, net, E, DT, P[:4], L, w=3)
    assert e.value.status == ak.ADK_EINVAL
    with pytest.raises(ak.AdkError) as e:
        ak.surrogate_step(g36, net, E, 0.0, P[:4], L, w=3)
    assert e.value.status == ak.ADK_EINVAL
    with pytest.raises(ak.AdkError):
        ak.Mlp(g36, wl.mlp_init(36, 1), E_range=(10.0, 5.0))
    bad = wl.mlp_init(36, 1)
    bad[7] = np.nan
    with pytest.raises(ak.AdkError):
        ak.Mlp(g36, bad)
    with pytest.raises(ak.AdkError):
        net.train(5, nsamples=100, batch=200)
    net.close()


def test_trained_network_gain(env, orc):
    """What training gives: on held-out samples the trained network's band
    columns are far closer to the exact ones than the initial network's and
    than the no-ionization column (1, 0, 0, 0)."""
    torch, ak, gases = env
    Z = 36
    gas, spec = gases[Z]
    p0 = wl.mlp_init(Z, 2022)
    net = ak.Mlp(gas, p0)
    losses = net.train(1500, nsamples=262144, batch=2048, lr=3e-3, seed=1)
    assert np.all(np.isfinite(losses))
    E, dt, k = wl.surrogate_samples(4000, 999, Z)
    exact = mlp.exact_band_columns(orc, spec, Z, E, dt, k)
    dev = _dev(torch, E, dt, k)
    Qt = net.forward(*dev).cpu().numpy().astype(np.float64)
    init = ak.Mlp(gas, p0)
    Qi = init.forward(*dev).cpu().numpy().astype(np.float64)
    ident = np.zeros_like(exact)
    ident[0] = 1.0
    err = {name: np.abs(Q - exact).max(axis=0) for name, Q in (("trained", Qt), ("init", Qi), ("identity", ident))}
    print({k: (float(v.mean()), float(np.quantile(v, 0.99)), float(v.max())) for k, v in err.items()})
    assert err["trained"].mean() <= 0.05 * err["init"].mean()
    assert err["trained"].mean() <= 0.2 * err["identity"].mean()
    net.close()
    init.close()


def test_surrogate_full_size_sampled(env, orc):
    """The surrogate form at the 3D mesh's full size (33,554,432 cells, 36
    levels m averaged, w = 3) in the pulse (t = 210 dt), from a seeded window
    state, in the launch configuration the benchmark times; 65,536 sampled
    cells against the CPU reference of the same network (tolerances as in the
    small-mesh comparison above)."""
    torch, ak, gases = env
    Z, w, eps = 36, 3, 1e-8
    gas, spec = gases[Z]
    params = wl.mlp_init(Z, 12)
    net = ak.Mlp(gas, params)
    mesh = wl.mesh_3d()
    n = mesh.ncells
    N, lo = wl.random_window_state(n, Z, w, seed=77, dtype=np.float32)
    E = mesh.field(210, dtype=np.float32)
    Pt = torch.from_numpy(N).cuda()
    Lt = torch.from_numpy(lo).cuda()
    ak.surrogate_step(gas, net, torch.from_numpy(E).cuda(), mesh.dt, Pt, Lt, w=w, eps=eps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(210)
    samp = np.sort(rng.choice(n, 65536, replace=False))
    idx = torch.from_numpy(samp).cuda()
    got, glo = Pt[:, idx].cpu().numpy().astype(np.float64), Lt[idx].cpu().numpy()
    ref, rlo, use, x = mlp.surrogate_step(orc, spec, Z, params.astype(np.float64), RNG, E[samp].astype(np.float64),
                                          mesh.dt, N[:, samp].astype(np.float64), lo[samp], w, eps)
    assert np.array_equal(glo, rlo)
    assert use.sum() > 10000  # the pulse puts many sampled cells in the network's range
    ana = ~use
    assert np.max(np.abs(got[:, ana] - ref[:, ana])) <= 1e-6
    th = mlp.NEGLIGIBLE_XDT
    clear = ~np.any((x > th / 3) & (x < 3 * th), axis=0)
    sel = use & clear
    d = np.abs(got[:, sel] - ref[:, sel]).max(axis=0)
    assert np.quantile(d, 0.9) <= 1e-5 and d.max() <= 1e-2, np.quantile(d, [0.5, 0.9, 0.99, 1.0])
    assert np.allclose(got[:, use].sum(axis=0), N[:, samp][:, use].astype(np.float64).sum(axis=0), atol=3e-6)
    del Pt, Lt, idx
    net.close()
    torch.cuda.empty_cache()
