#!/usr/bin/env python3
"""Throughput of the multi-level ADK ionization step on one MI355X.

Metric: cell-level updates per second of ionize_step, one unit being one
population of a cell's active window advanced by one step (sum over cells
of top - lo + 1), for the mixed-precision path, next to the plain FP64 path
on the same GPU and the CPU oracle on the host.

Headline workload: the 3D laser-pulse mesh (256 x 256 x 512 = 33,554,432
cells, 36-level synthetic chain with m-averaged rates, window of 4
populations, w = 3, 500 steps of 0.05 laser periods), the largest
single-GPU configuration and the one whose state (1.3 GB per step) streams
from HBM.  The pulse is run in from neutral cells for 200 steps (untimed),
then K consecutive steps (default 300, the rest of the run) are timed as one
replay of a HIP graph, with the field of every step already resident in
device memory.  The 2D mesh (1024 x 1024 cells, 18 levels), whose state
stays in the 256 MB Infinity Cache, is reported under "mesh2d".

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "cell·level updates/s of ionize_step vs plain FP64 at max |ΔN_k| ≤ 1e-6"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILE_3D_BYTES = "step_compact_w3_mesh3d_bytes.txt"
PROFILE_2D_BYTES = "step_compact_mixed_w3_mesh2d_bytes.txt"


def measured_traffic(key, profile=PROFILE_3D_BYTES):
    """HBM bytes per launch of a step kernel from a committed byte-counter
    summary under profiles/, or None when the step kernel's sources changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    csrc = os.path.join(ROOT, "paper_2202_10647_amd", "csrc")
    try:
        vals = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        h = hashlib.sha256()
        for f in ("kernels.hpp", "chain.hpp", "inst.hip"):
            h.update(open(os.path.join(csrc, f), "rb").read())
        if h.hexdigest() != vals.get("kernel_sources_sha256"):
            return None
        return float(vals[key])
    except (OSError, KeyError, ValueError):
        return None


def bytes_per_cell(w, prec):
    """Algorithmic HBM bytes per cell per step, compact layout: E read, window
    index read + write, w+1 populations read + written."""
    s = 4 if prec == "mixed" else 8
    return s + 1 + 1 + 2 * (w + 1) * s


def window_units(lo, w, Z):
    import torch
    top = torch.clamp(lo.to(torch.int64) + w, max=Z)
    return int((top - lo.to(torch.int64) + 1).sum().item())


def run_steps(ak, gas, fields, dt, pops, lo, w, eps, t0=0, nsteps=None, per_launch=False, count_units=False,
              Z=None):
    """Advance nsteps steps with fields[t0 + i].  Returns (elapsed_ms between
    events on the launch stream, per-launch average ms or None, units)."""
    import torch
    nsteps = fields.shape[0] - t0 if nsteps is None else nsteps
    stream = torch.cuda.current_stream()
    units = 0
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nsteps)] if per_launch else None
    start.record(stream)
    for i in range(nsteps):
        if per_launch:
            evs[i][0].record(stream)
        ak.ionize_step(gas, fields[t0 + i], dt, pops, lo, w=w, eps=eps)
        if per_launch:
            evs[i][1].record(stream)
        if count_units:
            units += window_units(lo, w, Z)
    end.record(stream)
    torch.cuda.synchronize()
    total = start.elapsed_time(end)
    avg = float(np.mean([a.elapsed_time(b) for a, b in evs])) if per_launch else None
    return total, avg, units


def capture_steps(ak, gas, fields, dt, pops, lo, w, eps):
    """Capture len(fields) consecutive ionize_step launches into one HIP graph
    (the launches read the per-step field tensors in place)."""
    import torch
    ak.ionize_step(gas, fields[0], dt, pops, lo, w=w, eps=eps)  # host-side caches before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for t in range(fields.shape[0]):
            ak.ionize_step(gas, fields[t], dt, pops, lo, w=w, eps=eps)
    torch.cuda.synchronize()
    return graph


def measure_path(ak, gas, mesh, fields, prec, w, eps, Z, warmup, label):
    """Time the run as one graph replay (events on the replay stream), time it
    again with eager per-call launches, count window units in a replay."""
    import torch
    tdt = torch.float32 if prec == "mixed" else torch.float64
    n = mesh.ncells
    K = fields.shape[0]
    p = torch.zeros((w + 1, n), dtype=tdt, device="cuda")
    lo = torch.zeros(n, dtype=torch.uint8, device="cuda")

    def reset():
        p.zero_()
        p[0] = 1.0
        lo.zero_()
        torch.cuda.synchronize()

    reset()
    run_steps(ak, gas, fields, mesh.dt, p, lo, w, eps, nsteps=min(warmup, K))
    reset()
    eager_ms, _, _ = run_steps(ak, gas, fields, mesh.dt, p, lo, w, eps)
    graph = capture_steps(ak, gas, fields, mesh.dt, p, lo, w, eps)
    reset()
    graph.replay()  # warm replay
    reset()
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    graph.replay()
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    # untimed eager replay counting the window populations advanced per step
    reset()
    _, _, units = run_steps(ak, gas, fields, mesh.dt, p, lo, w, eps, count_units=True, Z=Z)
    final_lo = int(lo.max().item())
    del graph
    ms_per_step = total_ms / K
    value = units / (total_ms * 1e-3)
    gbps = bytes_per_cell(w, prec) * n / (ms_per_step * 1e-3) / 1e9
    log(f"[{label}] {prec}: {ms_per_step * 1e3:.2f} us/step (graph), {eager_ms / K * 1e3:.2f} us/step eager, "
        f"{value:.3e} cell-level/s, {gbps:.0f} GB/s algorithmic, max lo {final_lo}")
    return dict(value=value, ms_per_step=ms_per_step, kernel_ms=ms_per_step, units=units, achieved_gbps=gbps,
                max_lo=final_lo, eager_ms_per_step=eager_ms / K)


def parity_check(ak, orc, gas, spec, mesh, w, eps, step, seed):
    """One call from a seeded synthetic state at full mesh size; sampled cells
    recomputed by the oracle from the same input bits."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    n = mesh.ncells
    rng = np.random.default_rng(seed)
    sample = np.unique(np.concatenate([rng.choice(n, min(n, 65536), replace=False),
                                       np.arange(n // 2, n // 2 + mesh.shape[-1])]))
    E64 = mesh.field(step)
    comp, lo = wl.random_window_state(n, spec.Z, w, seed=seed)
    out = {}
    for prec, npdt, tdt in (("mixed", np.float32, torch.float32), ("f64", np.float64, torch.float64)):
        E = E64.astype(npdt)
        P = comp.astype(npdt)
        Pt, Lt = torch.from_numpy(P).cuda(), torch.from_numpy(lo.copy()).cuda()
        dne = torch.empty(n, dtype=tdt, device="cuda")
        ak.ionize_step(gas, torch.from_numpy(E).cuda(), mesh.dt, Pt, Lt, w=w, eps=eps, dne=dne)
        idx = torch.from_numpy(sample).cuda()
        g = Pt[:, idx].cpu().numpy().astype(np.float64)
        gl = Lt[idx].cpu().numpy()
        gy = dne[idx].cpu().numpy().astype(np.float64)
        ref, rlo = orc.ionize_step(spec, E[sample].astype(np.float64), mesh.dt, P[:, sample].astype(np.float64),
                                   lo[sample], w, eps)
        yref = orc.electron_yield(P[:, sample].astype(np.float64), lo[sample], ref, rlo, spec.Z)
        out[prec] = dict(max_abs_err=float(np.max(np.abs(g - ref))), lo_mismatch=int(np.sum(gl != rlo)),
                         cells=int(sample.size), electron_yield_max_abs_err=float(np.max(np.abs(gy - yref))),
                         per_level_max_abs_err=per_level_error(g, gl, ref, rlo, spec.Z))
        log(f"[parity] {prec}: max |dN| = {out[prec]['max_abs_err']:.2e} over {sample.size} cells, "
            f"lo mismatches {out[prec]['lo_mismatch']}, electron yield max err "
            f"{out[prec]['electron_yield_max_abs_err']:.2e}")
    return out


def _probe_rate(fn, probe):
    t = time.perf_counter()
    fn(probe)
    return probe / max(time.perf_counter() - t, 1e-6)


def cpu_baseline(orc, spec, mesh, w, eps, step, seed, target_s):
    """The oracle as it stands, on the host cores, on the 2D mesh: one
    ionize_step over a bounded sample of the mesh cells (sized for about
    target_s seconds) from a seeded random window state."""
    from paper_2202_10647_amd import workloads as wl
    n = mesh.ncells
    E = mesh.field(step)
    comp, lo = wl.random_window_state(n, spec.Z, w, seed=seed)
    rate = _probe_rate(lambda m: orc.ionize_step(spec, E[:m], mesh.dt, comp[:, :m], lo[:m], w, eps), 8192)
    m = int(min(n, max(8192, rate * target_s)))
    t = time.perf_counter()
    _, lo2 = orc.ionize_step(spec, E[:m], mesh.dt, comp[:, :m], lo[:m], w, eps)
    el = time.perf_counter() - t
    units = int(np.sum(np.minimum(lo2.astype(np.int64) + w, spec.Z) - lo2.astype(np.int64) + 1))
    log(f"[cpu] oracle, 2D mesh: {m} cells in {el:.2f} s on {orc.max_threads()} threads")
    return dict(value=units / el, unit="cell·level updates/s", cores=orc.max_threads(), kind="oracle",
                workload=f"laser2d_1024x1024_Z{spec.Z}_w{w}",
                sample=f"one ionize_step (w={w}, {spec.Z} levels, FP64 rates, binary128 expm) over the first "
                       f"{m} cells of the {mesh.shape[0]}x{mesh.shape[1]} mesh at t={step} dt from a seeded "
                       f"random window state; OpenMP over cells; {el:.1f} s")


def cpu_baseline_3d(orc, spec36, mesh, mid_state, w, eps, seed, target_s):
    """The oracle on the headline workload: one ionize_step of a seeded random
    sample of the 3D mesh's cells, from the run state the GPU read before the
    middle timed step (float32 bits widened to double), sized for about
    target_s seconds of host time."""
    E, P, lo, step = mid_state
    n = mesh.ncells
    perm = np.random.default_rng(seed).permutation(n)

    def run(m):
        idx = np.sort(perm[:m])
        return orc.ionize_step(spec36, E[idx], mesh.dt, P[:, idx], lo[idx], w, eps)

    rate = _probe_rate(run, 16384)
    m = int(min(n, max(16384, rate * target_s)))
    t = time.perf_counter()
    _, lo2 = run(m)
    el = time.perf_counter() - t
    units = int(np.sum(np.minimum(lo2.astype(np.int64) + w, spec36.Z) - lo2.astype(np.int64) + 1))
    log(f"[cpu] oracle, 3D mesh: {m} cells in {el:.2f} s on {orc.max_threads()} threads")
    return dict(value=units / el, unit="cell·level updates/s", cores=orc.max_threads(), kind="oracle",
                workload=f"laser3d_256x256x512_Z36mavg_w{w}",
                sample=f"plain oracle (FP64 rates, binary128 expm, OpenMP over cells): one ionize_step (w={w}, 36 "
                       f"levels m averaged) of {m} randomly sampled cells of the 256x256x512 mesh from the run state "
                       f"before step {step} (the bits the GPU read); {el:.1f} s")


def cpu_baseline_chain7(orc, target_s):
    """The oracle on the 7-level chain workload: 4096 cells, full chain w = 7,
    fields log-uniform in [10, 2000] GV/m, dt = 0.1 fs, neutral cells; the
    4096-cell step repeated for about target_s seconds."""
    from paper_2202_10647_amd import workloads as wl
    g = wl.synthetic_gas(7)
    spec = orc.GasSpec(g.U, g.l, g.m)
    n, w, dt = 4096, 7, 1e-16
    E = wl.loguniform_field(n, 10.0, 2000.0, seed=1)
    P, lo = wl.neutral_state(n, w + 1)
    reps, el = 0, 0.0
    t = time.perf_counter()
    while el < target_s or reps == 0:
        orc.ionize_step(spec, E, dt, P, lo, w, 0.0)
        reps += 1
        el = time.perf_counter() - t
    units = reps * n * (w + 1)
    log(f"[cpu] oracle, 7-level chain: {reps} x {n} cells in {el:.2f} s")
    return dict(value=units / el, unit="cell·level updates/s", cores=orc.max_threads(), kind="oracle",
                workload="chain7_4096_cells_full_chain",
                sample=f"plain oracle: {reps} repetitions of one full-chain step (w = 7) of all {n} cells; {el:.1f} s")


def cpu_baseline_batched(orc, ncells, target_s, seed=4):
    """The oracle on the batched mixed-gas workload: one step of a seeded
    random sample of its cells (host gas and dopants as they occur), from the
    seeded window states and hashed field of the GPU parity check."""
    from paper_2202_10647_amd import workloads as wl
    tables = [wl.synthetic_gas(z) for z in (1,) + wl.DOPANT_Z]
    specs = [orc.GasSpec(t.U, t.l, t.m) for t in tables]
    cell_gas, cell_w = wl.batched_cells(ncells, seed=seed)
    perm = np.random.default_rng(seed + 1).permutation(ncells)
    dt = 1.334e-16
    E_all = wl.hash_field(ncells, 99, 7)

    def run(m):
        idx = np.sort(perm[:m])
        cg, cw = cell_gas[idx], cell_w[idx]
        pops, lo = wl.plan_window_state(cg, cw, [t.Z for t in tables], 7, seed=31)
        E = E_all[idx]
        t = time.perf_counter()
        units = 0
        for gi, spec in enumerate(specs):
            for w in range(1, 7):
                sel = np.nonzero((cg == gi) & (cw == w))[0]
                if sel.size == 0:
                    continue
                _, l2 = orc.ionize_step(spec, E[sel], dt, pops[: w + 1, sel], lo[sel], w, 1e-8)
                units += int(np.sum(np.minimum(l2.astype(np.int64) + w, spec.Z) - l2.astype(np.int64) + 1))
        return time.perf_counter() - t, units

    el, _ = run(65536)
    m = int(min(ncells, max(65536, 65536 / max(el, 1e-6) * target_s)))
    el, units = run(m)
    log(f"[cpu] oracle, batched mixed gases: {m} cells in {el:.2f} s")
    return dict(value=units / el, unit="cell·level updates/s", cores=orc.max_threads(), kind="oracle",
                workload=f"batched_{ncells}_cells_1pct_dopants_Z7_18_36_54_w1to6",
                sample=f"plain oracle: one step of {m} randomly sampled cells of the {ncells}-cell mixed-gas mesh "
                       f"(per (gas, w) group), seeded window states; {el:.1f} s")


def full_levels_np(P, lo, Z):
    """Compact windows P[w+1][n] at lo -> populations of every level [Z+1][n]."""
    w = P.shape[0] - 1
    n = P.shape[1]
    full = np.zeros((Z + 1, n))
    l64 = np.minimum(np.asarray(lo, np.int64), Z)
    cols = np.arange(n)
    for s_ in range(w + 1):
        k = l64 + s_
        ok = k <= Z
        np.add.at(full, (k[ok], cols[ok]), np.asarray(P[s_], np.float64)[ok])
    return full


def per_level_error(got, glo, ref, rlo, Z):
    """max over cells of |dN_k| for every level k = 0..Z (windows mapped to
    their levels on each side)."""
    d = np.abs(full_levels_np(got, glo, Z) - full_levels_np(ref, rlo, Z))
    return [float(v) for v in d.max(axis=1)]


def sampled_parity(ak, orc, gas, spec, E_np, P_np, lo_np, dt, w, eps, sample, prec, Z):
    """One ionize_step call on the device from the given state (all cells),
    sampled cells recomputed by the oracle from the same input bits; returns
    the max error, the per-level max error and the window-index mismatches."""
    import torch
    npdt = np.float32 if prec == "mixed" else np.float64
    E = E_np.astype(npdt)
    P = P_np.astype(npdt)
    Pt, Lt = torch.from_numpy(P).cuda(), torch.from_numpy(lo_np.copy()).cuda()
    ak.ionize_step(gas, torch.from_numpy(E).cuda(), dt, Pt, Lt, w=w, eps=eps)
    idx = torch.from_numpy(sample).cuda()
    g = Pt[:, idx].cpu().numpy().astype(np.float64)
    gl = Lt[idx].cpu().numpy()
    del Pt, Lt
    ref, rlo = orc.ionize_step(spec, E[sample].astype(np.float64), dt, P[:, sample].astype(np.float64),
                               lo_np[sample], w, eps)
    return dict(max_abs_err=float(np.max(np.abs(g - ref))), lo_mismatch=int(np.sum(gl != rlo)),
                cells=int(sample.size), per_level_max_abs_err=per_level_error(g, gl, ref, rlo, Z))


def headline_3d(ak, orc, gas36, spec36, mesh, K, warmup, w, eps, t0=200, parity_cells=65536, seed=2031):
    """The headline: K consecutive steps of the 3D pulse run (33.5M cells,
    36 levels, w = 3), mixed precision and FP64.  Per precision: fields of
    steps t0..t0+K-1 resident on the device; the pulse run in from neutral
    cells over steps 0..t0-1 (untimed, eager); `warmup` untimed eager steps
    from that state on a copy; the K steps captured in one HIP graph, replayed
    once untimed and once timed (HIP events on the replay stream) from the
    run-in state; an untimed eager pass counts the window populations of
    every step.  Parity: one call from the run state at the middle of the
    timed steps and one from a seeded random window state, 65,536 sampled
    cells recomputed by the oracle from the same bits, per-level errors."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    n = mesh.ncells
    Z = 36
    t0 = min(t0, max(0, mesh.steps - K))
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(n, min(n, parity_cells), replace=False))
    res = {"workload": f"laser3d_256x256x512_Z36mavg_w{w}", "cells": n, "levels": Z, "window_w": w, "eps": eps,
           "t0": t0, "timed_steps": f"steps {t0}..{t0 + K - 1} of the {mesh.steps}-step run, after {t0} steps "
                                     f"of run-in from neutral cells"}
    stream = torch.cuda.current_stream()
    for prec, tdt in (("mixed", torch.float32), ("f64", torch.float64)):
        fields = torch.empty((K, n), dtype=tdt, device="cuda")
        for i in range(K):
            fields[i] = mesh.field_torch(t0 + i, "cuda", tdt)
        p = torch.zeros((w + 1, n), dtype=tdt, device="cuda")
        p[0] = 1.0
        lo = torch.zeros(n, dtype=torch.uint8, device="cuda")
        for t in range(t0):
            ak.ionize_step(gas36, mesh.field_torch(t, "cuda", tdt), mesh.dt, p, lo, w=w, eps=eps)
        p0, l0 = p.clone(), lo.clone()

        def restore():
            p.copy_(p0)
            lo.copy_(l0)
            torch.cuda.synchronize()

        for i in range(min(warmup, K)):
            ak.ionize_step(gas36, fields[i], mesh.dt, p, lo, w=w, eps=eps)
        restore()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for i in range(K):
                ak.ionize_step(gas36, fields[i], mesh.dt, p, lo, w=w, eps=eps)
        restore()
        graph.replay()  # warm replay
        restore()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        graph.replay()
        b.record(stream)
        torch.cuda.synchronize()
        total_ms = a.elapsed_time(b)
        del graph
        # untimed eager pass: window populations advanced per step, and the
        # run state at the middle of the timed steps for the parity check
        restore()
        units = 0
        mid = K // 2
        for i in range(K):
            if i == mid:
                mid_state = (fields[i].cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64),
                             lo.cpu().numpy())
            ak.ionize_step(gas36, fields[i], mesh.dt, p, lo, w=w, eps=eps)
            units += window_units(lo, w, Z)  # the window after the step's start-of-step shift
        torch.cuda.synchronize()
        max_lo = int(lo.max().item())
        del fields, p, lo, p0, l0
        torch.cuda.empty_cache()
        ms = total_ms / K
        gbps = bytes_per_cell(w, prec) * n / (ms * 1e-3) / 1e9
        r = dict(value=units / (total_ms * 1e-3), ms_per_step=ms, kernel_avg_us=ms * 1e3, units=units,
                 achieved_gbps=gbps, frac_hbm=gbps / HBM_PEAK_GBPS, max_lo=max_lo,
                 bytes_per_cell=bytes_per_cell(w, prec))
        log(f"[mesh3d] {prec}: {ms * 1e3:.1f} us/step (graph of {K} steps), {r['value']:.3e} cell-level/s, "
            f"{gbps:.0f} GB/s algorithmic ({gbps / HBM_PEAK_GBPS:.2f} of 8 TB/s), max lo {max_lo}")
        # parity from the run state (the bits the timed steps read) and from a
        # seeded random window state (every window position, shifts due)
        E_mid, P_mid, l_mid = mid_state
        r["parity_run_state"] = sampled_parity(ak, orc, gas36, spec36, E_mid, P_mid, l_mid, mesh.dt, w, eps,
                                               sample, prec, Z)
        r["parity_run_state"]["state"] = f"run state before step {t0 + mid}"
        comp, lr = wl.random_window_state(n, Z, w, seed=seed + 1)
        r["parity_random_state"] = sampled_parity(ak, orc, gas36, spec36, E_mid, comp, lr, mesh.dt, w, eps,
                                                  sample, prec, Z)
        r["parity_random_state"]["state"] = f"seeded random window states, field of step {t0 + mid}"
        if prec == "mixed":
            res["_mid_state"] = (E_mid, P_mid, l_mid, t0 + mid)
        del comp, lr, mid_state
        for key in ("parity_run_state", "parity_random_state"):
            q = r[key]
            log(f"[mesh3d] {prec} parity ({q['state']}): max |dN| {q['max_abs_err']:.2e} over {q['cells']} "
                f"cells, lo mismatches {q['lo_mismatch']}")
        res[prec] = r
    res["speedup_mixed_vs_f64"] = res["mixed"]["value"] / res["f64"]["value"]
    return res


def adaptive_measure(ak, gas36, mesh, steps, eps, wmax=24, tol=1e-9, t0=200):
    """Adaptive windows (ionize_step_adaptive, mixed precision) on the whole
    3D mesh: widths 1..wmax per cell and step (leak tolerance tol per step),
    the pulse run in from neutral cells over steps 0..t0-1, then `steps`
    steps timed as one graph replay (HIP events); an untimed eager pass
    counts window populations (wc + 1 per live cell) and the cells the wide
    tiers solved (16 lanes per cell, or a wavefront when its slots do not
    fit)."""
    import torch
    n = mesh.ncells
    Z = 36
    fields = torch.empty((steps, n), dtype=torch.float32, device="cuda")
    for i in range(steps):
        fields[i] = mesh.field_torch(t0 + i, "cuda", torch.float32)
    P = torch.zeros((wmax + 1, n), dtype=torch.float32, device="cuda")
    P[0] = 1.0
    L = torch.zeros(n, dtype=torch.uint8, device="cuda")
    Wc = torch.ones(n, dtype=torch.uint8, device="cuda")
    work = ak.adaptive_workspace(n)
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    t_run = time.perf_counter()
    for t in range(t0):
        ak.ionize_step_adaptive(gas36, mesh.field_torch(t, "cuda", torch.float32), mesh.dt, P, L, Wc, 1, wmax, eps=eps,
                                tol=tol, work=work, counters=cnt)
    torch.cuda.synchronize()
    run_in_s = time.perf_counter() - t_run
    held_run_in = int(cnt[1])
    P0, L0, W0 = P.clone(), L.clone(), Wc.clone()

    def restore():
        P.copy_(P0)
        L.copy_(L0)
        Wc.copy_(W0)
        cnt.zero_()
        torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for i in range(steps):
            ak.ionize_step_adaptive(gas36, fields[i], mesh.dt, P, L, Wc, 1, wmax, eps=eps, tol=tol, work=work,
                                    counters=cnt)
    restore()
    graph.replay()
    restore()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    graph.replay()
    b.record(stream)
    torch.cuda.synchronize()
    total_ms = a.elapsed_time(b)
    wide_cells, held = (int(v) for v in cnt.cpu().numpy())
    del graph
    restore()
    units = 0
    wsum = wlive = 0.0
    for i in range(steps):
        ak.ionize_step_adaptive(gas36, fields[i], mesh.dt, P, L, Wc, 1, wmax, eps=eps, tol=tol, work=work)
        live = L < Z
        units += int((Wc.to(torch.int64) + 1)[live].sum()) + int((~live).sum())
        wsum += float(Wc[live].double().sum())
        wlive += float(live.sum())
    torch.cuda.synchronize()
    live = L < Z
    hist = torch.bincount(Wc[live].to(torch.int64), minlength=wmax + 1).cpu().numpy()
    ms = total_ms / steps
    res = {"workload": f"laser3d_256x256x512_Z36mavg_adaptive_w1to{wmax}_mixed", "tolerance_per_step": tol,
           "width_histogram_last_step": [int(v) for v in hist],
           "timed_steps": f"steps {t0}..{t0 + steps - 1} after {t0} steps of run-in (run-in {run_in_s:.1f} s eager)",
           "ms_per_step": ms, "value": units / (total_ms * 1e-3), "unit": "cell·level updates/s",
           "mean_width_live_cells": wsum / max(wlive, 1.0), "max_width": int(Wc.max()),
           "wide_tier_cells_per_step": wide_cells / steps, "held_by_wmax_timed_steps": held,
           "held_by_wmax_run_in": held_run_in,
           "launches_per_step": 5}
    log(f"[adaptive] mixed, widths 1..{wmax}, tol {tol:g}: {ms * 1e3:.1f} us/step, {res['value']:.3e} cell-level/s, "
        f"mean width {res['mean_width_live_cells']:.2f} (max {res['max_width']}), {wide_cells / steps:.0f} "
        f"cells/step on the wide tiers, held by wmax: {held} (timed) {held_run_in} (run-in); widths "
        f"{res['width_histogram_last_step']}")
    del fields, P, L, Wc, P0, L0, W0, work
    torch.cuda.empty_cache()
    return res


def yield_measure(ak, gas36, w, eps, steps):
    """Cost of the fused electron yield on the 3D mesh (mixed): the same
    steps with and without the dne output, per-launch HIP events."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    mesh = wl.mesh_3d()
    n = mesh.ncells
    t_first = 200
    fields = torch.empty((steps, n), dtype=torch.float32, device="cuda")
    for i in range(steps):
        fields[i] = mesh.field_torch(t_first + i, "cuda", torch.float32)
    p0 = torch.zeros((w + 1, n), dtype=torch.float32, device="cuda")
    p0[0] = 1.0
    l0 = torch.zeros(n, dtype=torch.uint8, device="cuda")
    for i in range(t_first):
        ak.ionize_step(gas36, mesh.field_torch(i, "cuda", torch.float32), mesh.dt, p0, l0, w=w, eps=eps)
    dne = torch.empty(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for name, d in (("without", None), ("with_yield", dne)):
        p, lo = p0.clone(), l0.clone()
        ak.ionize_step(gas36, fields[0], mesh.dt, p.clone(), lo.clone(), w=w, eps=eps, dne=d)  # warm
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for i in range(steps):
            evs[i][0].record(stream)
            ak.ionize_step(gas36, fields[i], mesh.dt, p, lo, w=w, eps=eps, dne=d)
            evs[i][1].record(stream)
        torch.cuda.synchronize()
        res[name] = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e3
    res["overhead"] = res["with_yield"] / res["without"] - 1.0
    res["bytes_per_cell"] = {"without": bytes_per_cell(w, "mixed"), "with_yield": bytes_per_cell(w, "mixed") + 4}
    res["workload"] = "laser3d_256x256x512_Z36mavg_w3_mixed"
    log(f"[yield] mesh3d mixed: {res['without']:.1f} us/launch without, {res['with_yield']:.1f} us with the "
        f"fused electron yield ({100 * res['overhead']:+.1f} %)")
    del fields, p0, l0, dne
    torch.cuda.empty_cache()
    return res


def subcycle_measure(ak, orc, gas, spec, mesh, w, eps, step, seed, nsubs=(8, 64, 512)):
    """What the analytic solution avoids: one full-size FP64 step of the 2D
    mesh from a seeded state, analytic vs sub-cycled explicit RK4 with nsub
    substeps, timed with HIP events; errors against the oracle's exact step
    on sampled cells; the share of sampled cells whose RK4 substep exceeds
    the stability limit (max W dt / nsub > 2.78)."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    n = mesh.ncells
    E = mesh.field(step)
    comp, lo = wl.random_window_state(n, spec.Z, w, seed=seed)
    rng = np.random.default_rng(seed + 1)
    sample = np.sort(rng.choice(n, 65536, replace=False))
    exact, elo = orc.ionize_step(spec, E[sample], mesh.dt, comp[:, sample], lo[sample], w, eps)
    Wall = orc.rates(spec, np.abs(E[sample]))
    from oracle import mlp as omlp
    _, p = omlp.window_shift(comp[:, sample], lo[sample], spec.Z, eps)
    xmax = np.zeros(sample.size)
    for s in range(w):
        k = p + s
        ok = k < spec.Z
        xmax[ok] = np.maximum(xmax[ok], Wall[k[ok], np.nonzero(ok)[0]] * mesh.dt)
    Et = torch.from_numpy(E).cuda()
    idx = torch.from_numpy(sample).cuda()
    stream = torch.cuda.current_stream()

    def timed(fn):
        P, L = torch.from_numpy(comp).cuda(), torch.from_numpy(lo.copy()).cuda()
        fn(P.clone(), L.clone())  # warm
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn(P, L)
        b.record(stream)
        torch.cuda.synchronize()
        d = np.abs(P[:, idx].cpu().numpy() - exact)
        fin = np.isfinite(d).all(axis=0)
        err = float(np.max(d[:, fin])) if fin.any() else None
        return a.elapsed_time(b) * 1e3, (err, int((~fin).sum()))

    res = {"workload": f"laser2d_1024x1024_Z{spec.Z}_w{w}_f64_one_call_t{step}", "sampled_cells": int(sample.size)}
    us, (err, nonfin) = timed(lambda P, L: ak.ionize_step(gas, Et, mesh.dt, P, L, w=w, eps=eps))
    res["analytic"] = {"us": us, "max_abs_err": err, "nonfinite_cells": nonfin}
    log(f"[subcycle] analytic FP64: {us:.1f} us, max |dN| {err:.1e}")
    for k in nsubs:
        us, (err, nonfin) = timed(lambda P, L: ak.subcycle_step(gas, Et, mesh.dt, P, L, w, k, eps=eps))
        unstable = float(np.mean(xmax / k > 2.78))
        res[f"rk4_nsub_{k}"] = {"us": us, "max_abs_err_finite_cells": err, "nonfinite_cells": nonfin,
                                "unstable_cell_fraction": unstable}
        log(f"[subcycle] RK4 x {k}: {us:.1f} us, max |dN| over finite cells {err}, non-finite {nonfin}, "
            f"unstable cells {100 * unstable:.2f} %")
    del Et
    torch.cuda.empty_cache()
    return res


def _to_full(P, L, w, Z):
    """Compact windows [w+1][n] at lo -> all levels [Z+1][n] (device)."""
    import torch
    full = torch.zeros((Z + 1, P.shape[1]), dtype=P.dtype, device=P.device)
    L64 = L.to(torch.int64)
    for s in range(w + 1):
        k = L64 + s
        full.scatter_add_(0, k.clamp(max=Z)[None], torch.where(k <= Z, P[s], torch.zeros_like(P[s]))[None])
    return full


def window_study(ak, mesh, eps, widths=(2, 3, 4, 8), every=10):
    """Full-vs-reduced study on the whole 2D mesh over the whole pulse (the
    synthetic stand-in for Fig. 2b/2c): FP64 windows of w = 2, 3, 4, 8 rates
    against the full chain (w = Z = 18 on the wide path, no shift; it tracks
    the oracle's full chain, tests/test_gpu_study.py), sampled every `every`
    steps: max |dN_k| per level and the relative error of the electron
    density n_e = sum_k k N_k; then the orbital-number variants of the gas
    table (Sec. 3 remark on alternative couplings) at w = 3."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    Z = 18
    ref_w, ref_eps = Z, 0.0
    g = wl.synthetic_gas(Z)
    gas = ak.Gas.from_table(g)
    n = mesh.ncells
    lev = torch.arange(Z + 1, dtype=torch.float64, device="cuda")[:, None]
    ws = tuple(widths) + (ref_w,)
    st = {}
    for w in ws:
        P = torch.zeros((w + 1, n), dtype=torch.float64, device="cuda")
        P[0] = 1.0
        st[w] = (P, torch.zeros(n, dtype=torch.uint8, device="cuda"))
    # cells whose field over the first laser period (20 steps) already
    # exceeds 1 GV/m start ionizing in a strong field (the pulse is partly
    # inside the mesh at t = 0): a neutral cell can then climb more levels in
    # one step than a window holds, which no reduced system follows.  They are
    # reported apart from the cells the pulse reaches gradually.
    e0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    for t in range(21):
        e0 = torch.maximum(e0, mesh.field_torch(t, "cuda", torch.float64).abs())
    gradual = e0 < 1.0
    del e0
    lvl_max = {w: torch.zeros(Z + 1, dtype=torch.float64, device="cuda") for w in widths}
    cell_max = {w: torch.zeros(n, dtype=torch.float64, device="cuda") for w in widths}
    ne_max = {w: torch.zeros(n, dtype=torch.float64, device="cuda") for w in widths}
    t0 = time.perf_counter()
    ref_s = 0.0
    ne_prev = torch.zeros(n, dtype=torch.float64, device="cuda")
    jump = torch.zeros(n, dtype=torch.float64, device="cuda")  # largest charge gain of the full chain in one step
    for t in range(mesh.steps):
        E = mesh.field_torch(t, "cuda", torch.float64)
        for w in ws:
            if w == ref_w:
                torch.cuda.synchronize()
                tr = time.perf_counter()
            ak.ionize_step(gas, E, mesh.dt, *st[w], w=w, eps=ref_eps if w == ref_w else eps)
            if w == ref_w:
                torch.cuda.synchronize()
                ref_s += time.perf_counter() - tr
        ne_now = (lev * st[ref_w][0]).sum(0)
        jump = torch.maximum(jump, ne_now - ne_prev)
        ne_prev = ne_now
        if t % every == 0 or t == mesh.steps - 1:
            ref = _to_full(*st[ref_w], ref_w, Z)
            ne_ref = (lev * ref).sum(0)
            for w in widths:
                full = _to_full(*st[w], w, Z)
                d = (full - ref).abs()
                lvl_max[w] = torch.maximum(lvl_max[w], d[:, gradual].amax(dim=1))
                cell_max[w] = torch.maximum(cell_max[w], d.amax(dim=0))
                ne = (lev * full).sum(0)
                ne_max[w] = torch.maximum(ne_max[w], torch.where(ne_ref > 1e-3, (ne - ne_ref).abs() / ne_ref,
                                                                 torch.zeros_like(ne)))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ne_final = (lev * _to_full(*st[ref_w], ref_w, Z)).sum(0)
    res = {"workload": f"laser2d_1024x1024_Z18_full_pulse_{mesh.steps}_steps_f64",
           "reference": f"full chain: w = Z = {ref_w} (one wavefront per cell), no shift", "eps": eps,
           "sampled_every": every, "seconds": el, "full_chain_seconds": ref_s,
           "full_chain_us_per_step": ref_s / mesh.steps * 1e6, "gradual_onset_cells": int(gradual.sum()), "strong_start_cells": int((~gradual).sum()),
           "final_mean_charge": {"max": float(ne_final.max()), "mean": float(ne_final.mean())},
           "largest_charge_gain_in_one_step": {
               "gradual": {"median": float(jump[gradual].median()), "max": float(jump[gradual].max())},
               "strong_start": {"median": float(jump[~gradual].median()), "max": float(jump[~gradual].max())}}}

    def stats(v):
        v = v.double()
        return {"max": float(v.max()), "p99_9": float(torch.quantile(v[::7].float(), 0.999)),
                "frac_above_1e-3": float((v > 1e-3).double().mean()), "frac_above_1e-4": float((v > 1e-4).double().mean())}

    for w in widths:
        lm = lvl_max[w].cpu().numpy()
        res[f"w{w}"] = {"gradual": {"max_abs_dN": stats(cell_max[w][gradual]), "max_rel_err_ne": stats(ne_max[w][gradual]),
                                    "max_abs_dN_per_level": [float(v) for v in lm]},
                        "strong_start": {"max_abs_dN": stats(cell_max[w][~gradual]),
                                         "max_rel_err_ne": stats(ne_max[w][~gradual])}}
        gr = res[f"w{w}"]["gradual"]
        log(f"[study] w={w}: gradual-onset cells max |dN| {gr['max_abs_dN']['max']:.2e} (p99.9 "
            f"{gr['max_abs_dN']['p99_9']:.1e}), max rel n_e error {gr['max_rel_err_ne']['max']:.2e}; strong-start "
            f"cells max |dN| {res[f'w{w}']['strong_start']['max_abs_dN']['max']:.2e}")
    # orbital-number variants of the table, w = 3
    variants = {"l_by_shell_m0": (g.l, g.m), "m_averaged": (g.l, np.full(Z, -1, np.int8)),
                "outer_shell_as_s": (np.where(np.arange(Z) < 6, 0, g.l).astype(np.int8), g.m)}
    ne_v = {}
    for name, (l, m) in variants.items():
        gv = ak.Gas(g.U, l, m)
        P = torch.zeros((4, n), dtype=torch.float64, device="cuda")
        P[0] = 1.0
        L = torch.zeros(n, dtype=torch.uint8, device="cuda")
        for t in range(mesh.steps):
            ak.ionize_step(gv, mesh.field_torch(t, "cuda", torch.float64), mesh.dt, P, L, w=3, eps=eps)
        ne_v[name] = (lev * _to_full(P, L, 3, Z)).sum(0)
        gv.close()
    base = ne_v["l_by_shell_m0"]
    res["orbital_variants"] = {name: {"mesh_mean_charge": float(v.mean()),
                                      "max_abs_diff_vs_l_by_shell": float((v - base).abs().max())}
                               for name, v in ne_v.items()}
    log("[study] orbital variants, final mesh-mean charge: " +
        ", ".join(f"{k} {v['mesh_mean_charge']:.4f}" for k, v in res["orbital_variants"].items()))
    gas.close()
    torch.cuda.empty_cache()
    return res


def window_study_3d(ak, mesh, eps, steps, widths=(2, 3, 4), every=10, half_width=32, tols=(1e-9, 1e-6)):
    """Full-vs-reduced study on the 3D mesh (256 x 256 x 512 cells, 36 levels,
    m averaged): FP64 windows of w = 2, 3, 4 rates and the adaptive window
    (ionize_step_adaptive: width 1..36 per cell and step, leak tolerances
    `tols` per step) against the full 36-level chain (w = Z on the wide path,
    no shift), `steps` steps of the pulse from t = 0, on the central
    transverse box of (2 half_width)^2 x 512 cells (the strongest fields:
    |x|, |y| < 10 um around the axis).  Every `every` steps: max |dN_k| per
    cell and the relative error of n_e = sum_k k N_k, and the adaptive
    windows' widths; the step times of the full chain and of the adaptive
    window."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    Z = 36
    gas = ak.Gas.from_table(wl.synthetic_gas(Z))
    nx, ny, nz = mesh.shape
    ix = torch.arange(nx // 2 - half_width, nx // 2 + half_width, device="cuda")
    iy = torch.arange(ny // 2 - half_width, ny // 2 + half_width, device="cuda")
    iz = torch.arange(nz, device="cuda")
    idx = ((ix[:, None, None] * ny + iy[None, :, None]) * nz + iz[None, None, :]).reshape(-1)
    n = idx.numel()
    lev = torch.arange(Z + 1, dtype=torch.float64, device="cuda")[:, None]
    ws = tuple(widths) + (Z,)
    st = {}
    for w in ws:
        P = torch.zeros((w + 1, n), dtype=torch.float64, device="cuda")
        P[0] = 1.0
        st[w] = (P, torch.zeros(n, dtype=torch.uint8, device="cuda"))
    # adaptive windows, one run per tolerance: storage for every level,
    # widths start at 1
    work = ak.adaptive_workspace(n)
    ada = {}
    for tol in tols:
        Pa = torch.zeros((Z + 1, n), dtype=torch.float64, device="cuda")
        Pa[0] = 1.0
        ada[tol] = dict(P=Pa, L=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                        W=torch.ones(n, dtype=torch.uint8, device="cuda"),
                        cnt=torch.zeros(2, dtype=torch.int64, device="cuda"), s=0.0, wsum=0.0, wcells=0.0, wmax=0,
                        dmax=torch.zeros(n, dtype=torch.float64, device="cuda"),
                        nemax=torch.zeros(n, dtype=torch.float64, device="cuda"))
    # cells whose field over the first laser period already exceeds 1 GV/m
    # start ionizing in a strong field (the pulse is partly inside the mesh at
    # t = 0); reported apart from the cells the pulse reaches gradually
    e0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    for t in range(21):
        e0 = torch.maximum(e0, mesh.field_torch(t, "cuda", torch.float64)[idx].abs())
    gradual = e0 < 1.0
    del e0
    dmax = {w: torch.zeros(n, dtype=torch.float64, device="cuda") for w in widths}
    nemax = {w: torch.zeros(n, dtype=torch.float64, device="cuda") for w in widths}
    ref_s = 0.0
    ne_prev = torch.zeros(n, dtype=torch.float64, device="cuda")
    jump = torch.zeros(n, dtype=torch.float64, device="cuda")  # largest charge gain of the full chain in one step
    t0 = time.perf_counter()
    for t in range(steps):
        E = mesh.field_torch(t, "cuda", torch.float64)[idx].contiguous()
        for w in ws:
            if w == Z:
                torch.cuda.synchronize()
                tr = time.perf_counter()
            ak.ionize_step(gas, E, mesh.dt, *st[w], w=w, eps=0.0 if w == Z else eps)
            if w == Z:
                torch.cuda.synchronize()
                ref_s += time.perf_counter() - tr
        for tol, a in ada.items():
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ak.ionize_step_adaptive(gas, E, mesh.dt, a["P"], a["L"], a["W"], 1, Z, eps=eps, tol=tol, work=work,
                                    counters=a["cnt"])
            torch.cuda.synchronize()
            a["s"] += time.perf_counter() - ta
        ne_now = (lev * st[Z][0]).sum(0)
        jump = torch.maximum(jump, ne_now - ne_prev)
        ne_prev = ne_now
        if t % every == 0 or t == steps - 1:
            ref = st[Z][0]
            ne_ref = (lev * ref).sum(0)
            for w in widths:
                full = _to_full(*st[w], w, Z)
                dmax[w] = torch.maximum(dmax[w], (full - ref).abs().amax(dim=0))
                ne = (lev * full).sum(0)
                nemax[w] = torch.maximum(nemax[w], torch.where(ne_ref > 1e-3, (ne - ne_ref).abs() / ne_ref,
                                                               torch.zeros_like(ne)))
            for a in ada.values():
                full = _to_full(a["P"], a["L"], Z, Z)
                a["dmax"] = torch.maximum(a["dmax"], (full - ref).abs().amax(dim=0))
                ne = (lev * full).sum(0)
                a["nemax"] = torch.maximum(a["nemax"], torch.where(ne_ref > 1e-3, (ne - ne_ref).abs() / ne_ref,
                                                                   torch.zeros_like(ne)))
                live = a["L"] < Z
                a["wsum"] += float(a["W"][live].double().sum())
                a["wcells"] += float(live.sum())
                a["wmax"] = max(a["wmax"], int(a["W"].max()))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ne_final = (lev * st[Z][0]).sum(0)
    res = {"workload": f"laser3d_256x256x512_Z36mavg_central_{2 * half_width}x{2 * half_width}x{nz}_{steps}_steps_f64",
           "reference": "full chain: w = Z = 36 (one wavefront per cell), no shift", "eps": eps,
           "cells": int(n), "gradual_onset_cells": int(gradual.sum()), "strong_start_cells": int((~gradual).sum()),
           "sampled_every": every, "seconds": el, "full_chain_seconds": ref_s,
           "full_chain_us_per_step": ref_s / steps * 1e6,
           "final_mean_charge": {"max": float(ne_final.max()), "mean": float(ne_final.mean())},
           "largest_charge_gain_in_one_step": {
               "gradual": {"median": float(jump[gradual].median()), "max": float(jump[gradual].max())},
               "strong_start": {"median": float(jump[~gradual].median()), "max": float(jump[~gradual].max())}}}
    def stats(d, e):
        if d.numel() == 0:
            return None
        return {"max_abs_dN": float(d.max()), "p99_9_abs_dN": float(torch.quantile(d[::3].float(), 0.999)),
                "frac_cells_above_1e-4": float((d > 1e-4).double().mean()),
                "max_rel_err_ne": float(e.max()), "p99_9_rel_err_ne": float(torch.quantile(e[::3].float(), 0.999))}

    for w in widths:
        gr, ss = stats(dmax[w][gradual], nemax[w][gradual]), stats(dmax[w][~gradual], nemax[w][~gradual])
        res[f"w{w}"] = {"gradual": gr, "strong_start": ss}
        log(f"[study3d] w={w}: gradual-onset cells max |dN| {gr['max_abs_dN']:.2e} (p99.9 {gr['p99_9_abs_dN']:.1e}), "
            f"max rel n_e error {gr['max_rel_err_ne']:.2e}; strong-start cells max |dN| "
            f"{ss['max_abs_dN'] if ss else float('nan'):.2e}")
    for tol, a in ada.items():
        ga, sa = stats(a["dmax"][gradual], a["nemax"][gradual]), stats(a["dmax"][~gradual], a["nemax"][~gradual])
        c = a["cnt"].cpu().numpy()
        key = "adaptive" if tol == tols[0] else f"adaptive_tol_{tol:g}"
        r = {"tolerance_per_step": tol, "wmin": 1, "wmax": Z, "gradual": ga, "strong_start": sa,
             "mean_width": a["wsum"] / max(a["wcells"], 1.0), "max_width": a["wmax"],
             "width_sampling": f"every {every} steps over cells with lo < Z",
             "us_per_step": a["s"] / steps * 1e6,
             "wide_tier_cells_per_step": float(c[0]) / steps, "held_by_wmax": int(c[1]),
             "storage": "Z + 1 rows allotted (wmax = Z); a cell uses wc + 1 of them"}
        res[key] = r
        log(f"[study3d] adaptive (tol {tol:g}/step): gradual-onset cells max |dN| {ga['max_abs_dN']:.2e}, max rel "
            f"n_e error {ga['max_rel_err_ne']:.2e}; strong-start cells max |dN| "
            f"{sa['max_abs_dN'] if sa else float('nan'):.2e}; mean width {r['mean_width']:.2f} (max {a['wmax']}); "
            f"{r['us_per_step']:.0f} us/step against {res['full_chain_us_per_step']:.0f} for the full chain; "
            f"{r['wide_tier_cells_per_step']:.0f} cells/step on the wide tiers")
    jg = res["largest_charge_gain_in_one_step"]["gradual"]
    log(f"[study3d] largest charge gain of the full chain in one step (gradual-onset cells): median "
        f"{jg['median']:.2f}, max {jg['max']:.2f} levels")
    log(f"[study3d] full 36-level chain: {res['full_chain_us_per_step']:.0f} us/step on {n} cells; "
        f"final mean charge {res['final_mean_charge']['mean']:.3f} (max {res['final_mean_charge']['max']:.2f})")
    del st, dmax, nemax, ada, work
    gas.close()
    torch.cuda.empty_cache()
    return res


MLP_FLOPS_PER_EVAL = 2 * (2 * 64 * 64 + 64 * 4) + 2 * 64  # layers 2-4 on MFMA, layer 1 one FMA per unit
BF16_MFMA_PEAK_TFLOPS = 2500.0


def surrogate_measure(ak, orc, gas36, spec36, w, eps, steps, train_iters, nsamples=1_000_000):
    """Surrogate form on the 3D mesh: train the band-column network on the
    device (analytic FP64 targets), check its columns on held-out samples
    against the oracle, time surrogate steps over the mesh like mesh3d, and
    check one full-size call against the FP64 oracle (sampled cells) and
    against the FP64 analytic step on the GPU (all cells)."""
    import torch
    from oracle import mlp as omlp
    from paper_2202_10647_amd import workloads as wl
    res = {"workload": "laser3d_256x256x512_Z36mavg_w3_surrogate",
           "network": "3 x 64 ReLU, 16-dim level embedding, band-4 softmax; layers 2-4 BF16 MFMA, FP32 accumulate"}
    net = ak.Mlp(gas36, wl.mlp_init(36, 2022))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(train_iters, nsamples=nsamples, batch=4096, lr=3e-3, lr_min=1e-5, seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    res["training"] = dict(samples=nsamples, iters=train_iters, batch=4096, seconds=train_s,
                           ms_per_iter=train_s / max(train_iters, 1) * 1e3,
                           final_loss=float(np.mean(losses[-100:])), first_loss=float(losses[0]))
    log(f"[surrogate] trained {train_iters} iters on {nsamples} samples in {train_s:.1f} s, "
        f"loss {losses[0]:.4f} -> {np.mean(losses[-100:]):.5f}")
    # held-out band columns against the oracle's exact columns
    E, dt, k = wl.surrogate_samples(20000, 999, 36)
    exact = omlp.exact_band_columns(orc, spec36, 36, E, dt, k)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (E, dt, k.astype(np.int32))]
    Q = net.forward(*dev).cpu().numpy().astype(np.float64)
    err = np.abs(Q - exact).max(axis=0)
    res["heldout_column_error"] = dict(samples=int(err.size), mean=float(err.mean()),
                                       p50=float(np.quantile(err, 0.5)), p99=float(np.quantile(err, 0.99)),
                                       max=float(err.max()))
    log(f"[surrogate] held-out column error: mean {err.mean():.2e}, p99 {np.quantile(err, 0.99):.2e}, "
        f"max {err.max():.2e}")

    mesh = wl.mesh_3d()
    n = mesh.ncells
    t_first = 200
    fields = torch.empty((steps, n), dtype=torch.float32, device="cuda")
    for i in range(steps):
        fields[i] = mesh.field_torch(t_first + i, "cuda", torch.float32)
    p = torch.zeros((w + 1, n), dtype=torch.float32, device="cuda")
    p[0] = 1.0
    lo = torch.zeros(n, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    for i in range(t_first):  # run the pulse in (untimed), surrogate form throughout
        ak.surrogate_step(gas36, net, mesh.field_torch(i, "cuda", torch.float32), mesh.dt, p, lo, w=w, eps=eps)
    ak.surrogate_step(gas36, net, fields[0], mesh.dt, p.clone(), lo.clone(), w=w, eps=eps)  # warm
    cnt.zero_()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(steps):
        evs[i][0].record(stream)
        ak.surrogate_step(gas36, net, fields[i], mesh.dt, p, lo, w=w, eps=eps, counters=cnt)
        evs[i][1].record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    total = start.elapsed_time(end)
    avg = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    units = window_units(lo, w, 36) * steps
    fb, evals = (int(x) for x in cnt.cpu().numpy())
    tflops = evals / steps * MLP_FLOPS_PER_EVAL / (avg * 1e-3) / 1e12
    res.update(value=units / (total * 1e-3), unit="cell·level updates/s", ms_per_step=total / steps,
               kernel_avg_us=avg * 1e3, timed_steps=f"{steps} steps from t={t_first} dt",
               network_evals_per_step=evals / steps, fallback_cells_per_step=fb / steps,
               mfma=dict(bound="mfma", achieved=tflops, peak=BF16_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                         frac=tflops / BF16_MFMA_PEAK_TFLOPS, flops_per_eval=MLP_FLOPS_PER_EVAL))
    log(f"[surrogate] {total / steps * 1e3:.1f} us/step, kernel {avg * 1e3:.1f} us, {res['value']:.3e} "
        f"cell-level/s, {evals / steps:.3e} network evals/step ({tflops:.1f} TFLOP/s BF16), "
        f"{fb / steps:.0f} fallback cells/step")
    del fields
    # error of one full-size call from a seeded state: oracle on sampled cells,
    # FP64 analytic GPU step on all cells
    step = t_first + steps // 2
    E64 = mesh.field(step)
    comp, lo0 = wl.random_window_state(n, 36, w, seed=77)
    E32 = E64.astype(np.float32)
    P32 = comp.astype(np.float32)
    Ps, Ls = torch.from_numpy(P32).cuda(), torch.from_numpy(lo0.copy()).cuda()
    ak.surrogate_step(gas36, net, torch.from_numpy(E32).cuda(), mesh.dt, Ps, Ls, w=w, eps=eps)
    Pf = torch.from_numpy(P32.astype(np.float64)).cuda()
    Lf = torch.from_numpy(lo0.copy()).cuda()
    ak.ionize_step(gas36, torch.from_numpy(E32.astype(np.float64)).cuda(), mesh.dt, Pf, Lf, w=w, eps=eps)
    dfull = (Ps.to(torch.float64) - Pf).abs().amax(dim=0)
    active = torch.from_numpy((np.abs(E32) >= 10.0) & (np.abs(E32) <= 5000.0)).cuda()
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(n, 65536, replace=False))
    idx = torch.from_numpy(sample).cuda()
    g = Ps[:, idx].cpu().numpy().astype(np.float64)
    ref, rlo = orc.ionize_step(spec36, E32[sample].astype(np.float64), mesh.dt, P32[:, sample].astype(np.float64),
                               lo0[sample], w, eps)
    d_or = np.abs(g - ref).max(axis=0)
    gl = Ls[idx].cpu().numpy()
    res["error_vs_fp64"] = dict(
        oracle_sample=dict(cells=int(sample.size), max_abs=float(d_or.max()), mean_abs=float(d_or.mean()),
                           p99=float(np.quantile(d_or, 0.99)),
                           lo_mismatch=int(np.sum(gl != rlo)),
                           per_level_max_abs_err=per_level_error(g, gl, ref, rlo, 36)),
        gpu_fp64_all_cells=dict(cells=n, max_abs=float(dfull.max()), mean_abs=float(dfull.mean()),
                                in_range_cells=int(active.sum()),
                                max_abs_in_range=float(dfull[active].max()) if bool(active.any()) else 0.0),
        state="seeded random window states, field of step %d" % step)
    log(f"[surrogate] one call vs FP64: oracle sample max {d_or.max():.2e} mean {d_or.mean():.2e}; "
        f"GPU FP64 all cells max {float(dfull.max()):.2e} mean {float(dfull.mean()):.2e}")
    # the method without the network on the same cells: the mixed analytic step
    Pm, Lm = torch.from_numpy(P32.copy()).cuda(), torch.from_numpy(lo0.copy()).cuda()
    ak.ionize_step(gas36, torch.from_numpy(E32).cuda(), mesh.dt, Pm, Lm, w=w, eps=eps)
    gm, glm = Pm[:, idx].cpu().numpy().astype(np.float64), Lm[idx].cpu().numpy()
    res["error_vs_fp64"]["mixed_analytic_same_cells"] = dict(
        max_abs=float(np.abs(gm - ref).max()), per_level_max_abs_err=per_level_error(gm, glm, ref, rlo, 36))
    del Pm, Lm
    del Ps, Ls, Pf, Lf, p, lo
    net.close()
    torch.cuda.empty_cache()
    return res


def batched_measure(ak, orc, steps, ncells, parity_cells=20000, layouts=("mesh", "grouped")):
    """Mixed gases with uneven windows (1-level host gas, 1 % dopants of 7, 18,
    36 and 54 levels, w in 1..6): one launch per launch group per step.  Each
    step's field is generated on the device by the hash harness; the timed
    graph holds [field, step] x steps and the field-only graph is timed
    separately and subtracted.  Layout "mesh": arrays indexed by mesh cell
    (the dopants scattered over the mesh); "grouped": the arrays in the plan's
    order (each gas and width contiguous, as in species-major storage), the
    same cells, the field drawn per storage position."""
    import torch
    from paper_2202_10647_amd import workloads as wl
    tables = [wl.synthetic_gas(z) for z in (1,) + wl.DOPANT_Z]
    gases = [ak.Gas.from_table(t) for t in tables]
    cell_gas, cell_w = wl.batched_cells(ncells, seed=4)
    dt = 1.334e-16
    res = {"workload": f"batched_{ncells}_cells_1pct_dopants_Z7_18_36_54_w1to6", "steps": steps}
    for prec, tdt, layout in [(p, t, lay) for p, t in (("mixed", torch.float32), ("f64", torch.float64))
                              for lay in layouts]:
        rk = prec if layout == "mesh" else f"{prec}_{layout}"
        t0 = time.perf_counter()
        plan = ak.Plan(gases, cell_gas, cell_w, prec=prec, eps=1e-8, cells_per_lane=0, layout=layout)
        create_s = time.perf_counter() - t0
        info = plan.info
        order = plan.order() if layout == "grouped" else None
        rows = info["rows"]
        E = torch.empty(ncells, dtype=tdt, device="cuda")
        P = torch.zeros((rows, ncells), dtype=tdt, device="cuda")
        L = torch.zeros(ncells, dtype=torch.uint8, device="cuda")

        def reset():
            P.zero_()
            P[0] = 1.0
            L.zero_()
            torch.cuda.synchronize()

        reset()
        ak.field_hash(E, 4, 0)
        plan.step(E, dt, P, L)  # host caches before capture
        torch.cuda.synchronize()
        g_all, g_field = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_all):
            for s in range(steps):
                ak.field_hash(E, 4, s)
                plan.step(E, dt, P, L)
        with torch.cuda.graph(g_field):
            for s in range(steps):
                ak.field_hash(E, 4, s)
        stream = torch.cuda.current_stream()
        times = {}
        for name, g in (("all", g_all), ("field", g_field)):
            reset()
            g.replay()  # warm
            reset()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.replay()
            b.record(stream)
            torch.cuda.synchronize()
            times[name] = a.elapsed_time(b)
        step_ms = (times["all"] - times["field"]) / steps
        sg, sw = (cell_gas, cell_w) if order is None else (cell_gas[order], cell_w[order])  # storage order
        top = np.minimum(L.cpu().numpy().astype(np.int64) + sw, np.array([t.Z for t in tables])[sg])
        units_last = int((top - L.cpu().numpy().astype(np.int64) + 1).sum())
        es = 4 if prec == "mixed" else 8
        bytes_step = int(ncells * (es + 2 + 4) + 2 * es * int((cell_w.astype(np.int64) + 1).sum()))
        res[rk] = dict(layout=layout, ms_per_step=step_ms, field_ms_per_step=times["field"] / steps,
                       value=units_last / (step_ms * 1e-3), achieved_gbps=bytes_step / (step_ms * 1e-3) / 1e9,
                       algorithmic_bytes_per_step=bytes_step, plan_create_s=create_s,
                       cells_per_lane=info["cells_per_lane"], grid=info["grid"], tiles=info["ntiles"],
                       buckets=info["nbuckets"], tuned_us=info["tuned_us"], launch_cpl=info["launch_cpl"],
                       launch_cells=info["launch_cells"])
        log(f"[batched] {prec} ({layout} order): {step_ms * 1e3:.1f} us/step (+{times['field'] / steps * 1e3:.1f} us "
            f"field), {res[rk]['value']:.3e} cell-level/s (final windows), {res[rk]['achieved_gbps']:.0f} GB/s, "
            f"cells/lane {info['launch_cpl']}, {info['ntiles']} tiles, {info['nbuckets']} groups")
        # parity of one launch from a seeded synthetic state and host-generated
        # field (the same bits go to the oracle), on sampled cells
        rng = np.random.default_rng(5)
        dop = np.nonzero(cell_gas > 0)[0]
        samp = np.unique(np.concatenate([rng.choice(ncells, parity_cells // 2, replace=False),
                                         rng.choice(dop, min(dop.size, parity_cells // 2), replace=False)]))
        npdt = np.float32 if prec == "mixed" else np.float64
        zs = [t.Z for t in tables]
        pops0, lo0 = wl.plan_window_state(cell_gas, cell_w, zs, rows, seed=31, dtype=npdt)
        E0 = wl.hash_field(ncells, 99, 7, dtype=npdt)
        if order is None:
            P.copy_(torch.from_numpy(pops0))
            L.copy_(torch.from_numpy(lo0))
            E.copy_(torch.from_numpy(E0))
            pos = samp
        else:  # the same mesh cells stored in the plan's order
            P.copy_(torch.from_numpy(np.ascontiguousarray(pops0[:, order])))
            L.copy_(torch.from_numpy(np.ascontiguousarray(lo0[order])))
            E.copy_(torch.from_numpy(np.ascontiguousarray(E0[order])))
            inv = np.empty(ncells, np.int64)
            inv[order] = np.arange(ncells)
            pos = inv[samp]
        plan.step(E, dt, P, L)
        torch.cuda.synchronize()
        idx = torch.from_numpy(pos).cuda()
        out, l2 = P[:, idx].cpu().numpy().astype(np.float64), L[idx].cpu().numpy()
        pre_p, pre_l, e_s = pops0[:, samp], lo0[samp], E0[samp]
        del pops0
        err, mism = 0.0, 0
        per_level = {}
        for gi, t in enumerate(tables):
            spec = orc.GasSpec(t.U, t.l, t.m)
            lv = np.zeros(t.Z + 1)
            for w in range(1, 7):
                sel = np.nonzero((cell_gas[samp] == gi) & (cell_w[samp] == w))[0]
                if sel.size == 0:
                    continue
                ref, rlo = orc.ionize_step(spec, e_s[sel].astype(np.float64), dt,
                                           pre_p[: w + 1, sel].astype(np.float64), pre_l[sel], w, 1e-8)
                err = max(err, float(np.max(np.abs(out[: w + 1, sel] - ref))))
                mism += int(np.sum(l2[sel] != rlo))
                lv = np.maximum(lv, per_level_error(out[: w + 1, sel], l2[sel], ref, rlo, t.Z))
            per_level[f"Z{t.Z}"] = [float(v) for v in lv]
        res[rk]["parity_max_abs_err"] = err
        res[rk]["parity_lo_mismatch"] = mism
        res[rk]["per_level_max_abs_err"] = per_level
        log(f"[batched] {prec} ({layout} order) parity on {samp.size} sampled cells (seeded state, host field): "
            f"max |dN| {err:.2e}, lo mismatches {mism}")
        del g_all, g_field, P, L, E
        plan.close()
        torch.cuda.empty_cache()
    res["speedup_mixed_vs_f64"] = res["f64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    if "mixed_grouped" in res:
        res["speedup_grouped_vs_mesh_order_mixed"] = res["mixed"]["ms_per_step"] / res["mixed_grouped"]["ms_per_step"]
    for g in gases:
        g.close()
    return res


def measure_ceilings(ak):
    """The device's own ceilings (best of 3 launches each): streaming copies
    of 1, 2 and 4 GiB with the library's harness kernel and with the runtime's
    device-to-device copy (HBM: the best of both), 50 passes of a 32 MiB copy
    (resident in the 256 MB Infinity Cache), and chains of float FMA, double
    FMA and float exp2 on every wavefront slot of the chip."""
    import torch
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best_ms(fn):
        fn()
        torch.cuda.synchronize()
        t = float("inf")
        for _ in range(3):
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            t = min(t, a.elapsed_time(b))
        return t

    res = {}
    own, rt = 0.0, 0.0
    for nb in (1 << 30, 2 << 30, 4 << 30):
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        own = max(own, 2 * nb / (best_ms(lambda: ak.ceiling_copy(dst, src)) * 1e-3) / 1e9)
        rt = max(rt, 2 * nb / (best_ms(lambda: dst.copy_(src)) * 1e-3) / 1e9)
        del src, dst
    res["hbm_copy_gbps"] = max(own, rt)
    res["hbm_copy_own_kernel_gbps"] = own
    res["hbm_copy_runtime_gbps"] = rt
    nb, reps = 32 << 20, 50
    src = torch.ones(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    t = best_ms(lambda: ak.ceiling_copy(dst, src, reps))
    res["cache_copy_gbps"] = 2 * nb * reps / (t * 1e-3) / 1e9
    del src, dst
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    lanes = cus * 32 * 64  # 32 wavefront slots per CU
    iters = 4096
    for kind, key, tdt, per in ((0, "valu_fp32_fma_tflops", torch.float32, 16), (1, "valu_fp64_fma_tflops",
                                torch.float64, 16), (2, "valu_exp2_f32_tops", torch.float32, 8)):
        out = torch.empty(lanes, dtype=tdt, device="cuda")
        t = best_ms(lambda: ak.ceiling_valu(kind, iters, out))
        assert bool(torch.all(out == 8)), key
        res[key] = per * iters * lanes / (t * 1e-3) / 1e12
    res["method"] = ("HBM: best of the library's 16-byte copy (one 4 KiB block per workgroup, in address order) "
                     "and the runtime's device-to-device copy "
                     "over 1, 2 and 4 GiB; cache: the library's copy of 32 MiB x 50 passes; VALU: "
                     "8 dependent chains per lane of fma(x, 1, 0) or exp2(fma(x, 0, 0)) on every wavefront slot; "
                     "best of 3 launches")
    log(f"[ceilings] HBM copy {res['hbm_copy_gbps']:.0f} GB/s, cache copy {res['cache_copy_gbps']:.0f} GB/s, "
        f"FP32 FMA {res['valu_fp32_fma_tflops']:.1f} TFLOP/s, FP64 FMA {res['valu_fp64_fma_tflops']:.1f} TFLOP/s, "
        f"exp2 {res['valu_exp2_f32_tops']:.2f} T/s")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=300, help="timed steps of the 3D run (after the run-in)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--window", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-mesh2d", action="store_true")
    ap.add_argument("--mesh2d-steps", type=int, default=2000)
    ap.add_argument("--yield-steps", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-extra-seconds", type=float, default=3.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--batched-cells", type=int, default=1 << 24)
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device three times (a kernel of known traffic "
                         "for calibrating profiler byte counters)")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--no-subcycle", action="store_true")
    ap.add_argument("--no-study", action="store_true")
    ap.add_argument("--study3d-steps", type=int, default=500, help="0 skips the 3D full-vs-reduced study")
    ap.add_argument("--surrogate-steps", type=int, default=40)
    ap.add_argument("--adaptive-steps", type=int, default=20, help="0 skips the adaptive-window leg")
    ap.add_argument("--surrogate-train-iters", type=int, default=24000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the ionization step has no "
              "cross-cell coupling, so a mesh shards into slabs of cells, one per GPU, with no exchange "
              "in the step; the figure measured here is one GPU's share.", file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    from paper_2202_10647_amd import adkion, workloads as wl

    if not os.path.exists(adkion.LIB_PATH):
        from paper_2202_10647_amd import build
        build.build()
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    torch.cuda.set_device(0)

    if args.calibration_copy_mib > 0:
        nfl = args.calibration_copy_mib * (1 << 20) // 4
        src = torch.ones(nfl, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[calibration] copied {args.calibration_copy_mib} MiB device to device 3 times")
        del src, dst

    w, eps = args.window, args.eps
    mesh3 = wl.mesh_3d()
    K = max(1, min(args.steps, mesh3.steps))
    g36 = wl.synthetic_gas(36)
    gas36 = adkion.Gas.from_table(g36)
    spec36 = oracle.GasSpec(g36.U, g36.l, g36.m)
    n3 = mesh3.ncells
    log(f"[setup] 3D mesh {n3} cells, Z=36 m-averaged, w={w}, {K} timed steps, fields resident in HBM")
    head = headline_3d(adkion, oracle, gas36, spec36, mesh3, K, args.warmup, w, eps)
    mid_state = head.pop("_mid_state")

    # the 2D mesh (cache-resident working set), formerly the headline
    mesh2 = wl.mesh_2d()
    g18 = wl.synthetic_gas(18)
    gas = adkion.Gas.from_table(g18)
    spec = oracle.GasSpec(g18.U, g18.l, g18.m)
    mesh2d = None
    if not args.no_mesh2d:
        K2 = min(args.mesh2d_steps, mesh2.steps)
        f64 = torch.empty((K2, mesh2.ncells), dtype=torch.float64, device="cuda")
        for t in range(K2):
            f64[t] = mesh2.field_torch(t, "cuda", torch.float64)
        f32 = f64.to(torch.float32)
        mesh2d = {"workload": f"laser2d_1024x1024_Z18_w{w}", "cells": mesh2.ncells,
                  "note": "state (~25 MB) resident in the 256 MB Infinity Cache: a cache-resident measurement",
                  "timed_steps": f"steps 0..{K2 - 1} of the {mesh2.steps}-step run"}
        mesh2d["mixed"] = measure_path(adkion, gas, mesh2, f32, "mixed", w, eps, 18, args.warmup, "mesh2d")
        mesh2d["f64"] = measure_path(adkion, gas, mesh2, f64, "f64", w, eps, 18, args.warmup, "mesh2d")
        mesh2d["speedup_mixed_vs_f64"] = mesh2d["mixed"]["value"] / mesh2d["f64"]["value"]
        del f64, f32
        torch.cuda.empty_cache()
        if not args.no_parity:
            mesh2d["parity"] = parity_check(adkion, oracle, gas, spec, mesh2, w, eps, 1000, 2024)
    subcycle = None if args.no_subcycle else subcycle_measure(adkion, oracle, gas, spec, mesh2, w, eps, 1000, 2025)
    study = None if args.no_study else window_study(adkion, mesh2, eps)
    study3d = None
    if not args.no_study and args.study3d_steps > 0:
        study3d = window_study_3d(adkion, mesh3, eps, args.study3d_steps)
    head["electron_yield"] = yield_measure(adkion, gas36, w, eps, args.yield_steps)
    adaptive = None
    if args.adaptive_steps > 0:
        adaptive = {}
        for tol in (1e-9, 1e-6):
            r = adaptive_measure(adkion, gas36, mesh3, args.adaptive_steps, eps, tol=tol)
            r["speedup_vs_fixed_w3_mixed"] = r["value"] / head["mixed"]["value"]
            adaptive[f"tol_{tol:g}"] = r
    surrogate = None
    if not args.no_surrogate:
        surrogate = surrogate_measure(adkion, oracle, gas36, spec36, w, eps, args.surrogate_steps,
                                      args.surrogate_train_iters)
        surrogate["speedup_vs_fp64_analytic"] = surrogate["value"] / head["f64"]["value"]
        surrogate["speedup_vs_mixed_analytic"] = surrogate["value"] / head["mixed"]["value"]
    gas36.close()
    batched = None if args.no_batched else batched_measure(adkion, oracle, args.batched_steps, args.batched_cells)
    cpu = cpu_other = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_3d(oracle, spec36, mesh3, mid_state, w, eps, 7, args.cpu_seconds)
        cpu_other = {"chain7_4096": cpu_baseline_chain7(oracle, args.cpu_extra_seconds),
                     "mesh2d": cpu_baseline(oracle, spec, mesh2, w, eps, 1000, 7, args.cpu_extra_seconds),
                     "batched": cpu_baseline_batched(oracle, args.batched_cells, args.cpu_extra_seconds),
                     "nproc": os.cpu_count()}
    del mid_state

    ceil = None if args.no_ceilings else measure_ceilings(adkion)
    if ceil:
        for prec in ("mixed", "f64"):
            head[prec]["frac_of_measured_hbm_copy"] = head[prec]["achieved_gbps"] / ceil["hbm_copy_gbps"]
        if mesh2d:
            for prec in ("mixed", "f64"):
                mesh2d[prec]["frac_of_measured_cache_copy"] = mesh2d[prec]["achieved_gbps"] / ceil["cache_copy_gbps"]

    m = head["mixed"]
    us = m["kernel_avg_us"]
    alg = bytes_per_cell(w, "mixed") * n3
    traffic = measured_traffic("traffic_bytes_per_launch_mixed") if w == 3 else None
    roof = {"bound": "hbm", "achieved": m["achieved_gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": m["achieved_gbps"] / HBM_PEAK_GBPS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, calibrated on a "
                            f"512 MiB copy; profiles/{PROFILE_3D_BYTES})",
            "algorithmic_bytes_per_launch": alg, "bytes_per_cell": bytes_per_cell(w, "mixed"),
            "kernel": f"step_compact_kernel<PolicyMixed,{w}>", "kernel_avg_us": us,
            "timing": "HIP events around one graph replay of the timed steps, divided by the steps",
            "kernel_trace": "profiles/step_compact_mixed_w3_mesh3d_default_bench_trace.md"}
    if traffic:
        roof["counter_bytes_gbps"] = traffic / (us * 1e-6) / 1e9
        roof["frac_counter_bytes"] = roof["counter_bytes_gbps"] / HBM_PEAK_GBPS
    if ceil:
        roof["measured_hbm_copy_gbps"] = ceil["hbm_copy_gbps"]
        roof["frac_of_measured_hbm_copy"] = m["achieved_gbps"] / ceil["hbm_copy_gbps"]
        if traffic:
            roof["frac_counter_bytes_of_measured_hbm_copy"] = roof["counter_bytes_gbps"] / ceil["hbm_copy_gbps"]
    per_level = {"laser3d_Z36_w3": {p: {"run_state": head[p]["parity_run_state"]["per_level_max_abs_err"],
                                        "random_state": head[p]["parity_random_state"]["per_level_max_abs_err"]}
                                    for p in ("mixed", "f64")}}
    if mesh2d and mesh2d.get("parity"):
        per_level["laser2d_Z18_w3"] = {p: mesh2d["parity"][p]["per_level_max_abs_err"] for p in ("mixed", "f64")}
    if batched:
        per_level["batched"] = {p: batched[p]["per_level_max_abs_err"] for p in ("mixed", "f64")}
    if surrogate:
        per_level["surrogate_laser3d_Z36_w3"] = {
            "surrogate": surrogate["error_vs_fp64"]["oracle_sample"]["per_level_max_abs_err"],
            "mixed_analytic_same_cells": surrogate["error_vs_fp64"]["mixed_analytic_same_cells"]["per_level_max_abs_err"]}
    line = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "cell·level updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "cells": n3, "levels": 36, "rates": "m averaged", "window_w": w,
                   "eps": eps, "layout": "compact", "precision": "mixed", "dt_s": mesh3.dt,
                   "timed_steps": head["timed_steps"], "parallelism": "single GPU"},
        "roofline": roof,
        "ceilings": ceil,
        "launch": "timed steps captured in one HIP graph",
        "fp64": {k: head["f64"][k] for k in ("value", "ms_per_step", "kernel_avg_us", "achieved_gbps", "frac_hbm")},
        "speedup_vs_fp64": head["speedup_mixed_vs_f64"],
        "parity": {p: {k: head[p][k] for k in ("parity_run_state", "parity_random_state")} for p in ("mixed", "f64")},
        "per_level_max_abs_err": per_level,
        "mesh3d": head,
        "adaptive_window": adaptive,
        "mesh2d": mesh2d,
        "batched": batched,
        "surrogate": surrogate,
        "subcycled_baseline": subcycle,
        "window_study": study,
        "window_study_3d": study3d,
        "cpu_baseline": cpu,
        "cpu_baseline_other_configs": cpu_other,
    }
    gas.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
