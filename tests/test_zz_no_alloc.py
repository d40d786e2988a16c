"""adk_mlp_loss_grad_noalloc (the entry point for callers that cannot
allocate) against adk_mlp_loss_grad on the same network and samples: two
calls in a row, the second with fewer samples, each bit for bit equal to the
allocating entry point (same kernels, same summation order); sizes above the
maximum are rejected."""
import numpy as np
import pytest

from paper_2202_10647_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_noalloc_loss_grad_matches_allocating_entry_point():
    import torch
    from paper_2202_10647_amd import adkion as ak
    assert torch.cuda.is_available()
    Z = 36
    gas = ak.Gas.from_table(wl.synthetic_gas(Z))
    net = ak.Mlp(gas, wl.mlp_init(Z, 17))
    g = torch.empty(net.nparams, dtype=torch.float32, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    for n, seed in ((ak.ADK_MLP_NOALLOC_MAX_SAMPLES, 41), (1000 + 7, 42)):
        E, dt, k = wl.surrogate_samples(n, seed, Z)
        dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (E, dt, k.astype(np.int32))]
        g.fill_(np.nan)
        L.fill_(np.nan)
        print(f"noalloc loss_grad: n={n}", flush=True)
        net.loss_grad_noalloc(*dev, g, L)
        Lr, gr = net.loss_grad(*dev)
        torch.cuda.synchronize()
        assert torch.isfinite(g).all() and torch.isfinite(L).all()
        assert torch.equal(L, Lr), (float(L), float(Lr))
        assert torch.equal(g, gr), float((g - gr).abs().max())
    E, dt, k = wl.surrogate_samples(ak.ADK_MLP_NOALLOC_MAX_SAMPLES + 1, 43, Z)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (E, dt, k.astype(np.int32))]
    with pytest.raises(ak.AdkError) as e:
        net.loss_grad_noalloc(*dev, g, L)
    assert e.value.status == ak.ADK_ERANGE
    net.close()
    gas.close()
