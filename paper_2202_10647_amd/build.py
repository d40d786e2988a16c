"""Build libadkion.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libadkion.so")
ARCH = os.environ.get("ADK_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: plain scalar/FP64 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
PRECS = ("f64", "mixed")
WIDTHS = range(1, 9)
PLAN_WMAX = range(1, 7)


def _jobs(objdir):
    """(command, object) pairs: host table builder, tuner cache file, ABI, batched plan,
    surrogate network and step, one kernel instantiation per (precision,
    window width)."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    obj = os.path.join(objdir, "gas_table.o")
    jobs.append((["hipcc", "-O2", "-std=c++17", "-fPIC", *inc, "-c", os.path.join(CSRC, "gas_table.cpp"),
                  "-o", obj], obj))
    obj = os.path.join(objdir, "tune_cache.o")
    jobs.append((["hipcc", "-O2", "-std=c++17", "-fPIC", *inc, "-c", os.path.join(CSRC, "tune_cache.cpp"),
                  "-o", obj], obj))
    obj = os.path.join(objdir, "abi.o")
    jobs.append((["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, "abi.hip"), "-o", obj], obj))
    for name in ("plan", "mlp", "sur", "subcycle", "wide", "adapt", "ceiling"):
        obj = os.path.join(objdir, f"{name}.o")
        # matrix-core results in ordinary VGPRs (no accumulator-register copies)
        extra = ["-mllvm", "-amdgpu-mfma-vgpr-form"] if name in ("mlp", "sur") else []
        jobs.append((["hipcc", *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, f"{name}.hip"), "-o", obj], obj))
    for prec in PRECS:
        for wmax in PLAN_WMAX:
            obj = os.path.join(objdir, f"plan_{prec}_{wmax}.o")
            jobs.append((["hipcc", *HIP_FLAGS, f"-DADK_PLAN_PREC={prec}", f"-DADK_PLAN_WMAX={wmax}", "-c",
                          os.path.join(CSRC, "plan_inst.hip"), "-o", obj], obj))
    for prec in PRECS:
        for w in WIDTHS:
            obj = os.path.join(objdir, f"inst_{prec}_{w}.o")
            jobs.append((["hipcc", *HIP_FLAGS, f"-DADK_INST_PREC={prec}", f"-DADK_INST_W={w}", "-c",
                          os.path.join(CSRC, "inst.hip"), "-o", obj], obj))
    return jobs


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source (in parallel) and link libadkion.so; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    work = _jobs(objdir)
    # largest instantiations first so the pool stays busy
    work.sort(key=lambda j: (0 if "plan_" in j[1] else 1, -int(j[1].rsplit("_", 1)[-1][:-2])
                             if ("inst_" in j[1] or "plan_" in j[1]) else 0))
    njobs = jobs or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(njobs) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), work))
    objs = [o for _, o in work]
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    if verbose and out.strip():
        print(out)


if __name__ == "__main__":
    print(build(verbose=True))
