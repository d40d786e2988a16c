"""Host-side pieces of the benchmark (no GPU): the algorithmic bytes per cell,
the cell·level unit count, the committed byte-counter summary it reports as
traffic, and the single-GPU contract of the command line."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bytes_per_cell():
    # E read, window index read and written, w + 1 populations read and written
    assert bench.bytes_per_cell(3, "mixed") == 38
    assert bench.bytes_per_cell(3, "f64") == 74
    assert bench.bytes_per_cell(4, "mixed") == 46
    assert bench.bytes_per_cell(4, "f64") == 90


def test_window_units():
    import torch
    lo = torch.tensor([0, 16, 17, 18], dtype=torch.uint8)
    # tops 3, 18, 18, 18: units = populations of each window
    assert bench.window_units(lo, 3, 18) == 4 + 3 + 2 + 1


def test_measured_traffic_is_tied_to_the_kernel_sources():
    """The traffic figure is reported only while the step kernel's sources
    hash to the value recorded with the counters; then it is the measured
    HBM bytes of a launch, below the algorithmic 38 B per cell (wavefronts
    that keep their windows store nothing) and above the read bytes."""
    for profile, n in ((bench.PROFILE_2D_BYTES, 1024 * 1024), (bench.PROFILE_3D_BYTES, 256 * 256 * 512)):
        v = bench.measured_traffic("traffic_bytes_per_launch_mixed", profile)
        if v is None:
            continue  # the step kernel's sources changed since these counters were taken
        assert 21 * n <= v <= 38 * n
        v = bench.measured_traffic("traffic_bytes_per_launch_f64", profile)
        assert 41 * n <= v <= 74 * n
    assert bench.measured_traffic("no_such_key") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
