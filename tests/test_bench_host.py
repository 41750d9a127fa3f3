"""Host-side checks of bench.py's measurement contract (no GPU needed).

The algorithmic byte model is the one the roofline fractions are computed
from: atoms 88 B each (positions and charges read twice, forces written),
the int64 charge grid written and read, the half spectrum across both
corner turns, the potential written and read.  Its totals are checked
against the same model written out independently per workload, and the
multi-GPU request is refused before anything touches a device.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("N,K,fp32,fp64", [
    (4095, 32, 1_703_848, 2_523_048),           # 4,095-atom water box, 32^3
    (65535, 64, 16_383_912, 22_806_440),        # 65,535-atom water box, 64^3
    (209715, 128, 102_865_288, 153_721_224),    # 209,715-atom water box, 128^3
])
def test_step_bytes_cubic(N, K, fp32, fp64):
    assert bench.step_bytes(N, K) == fp32
    assert bench.step_bytes(N, K, fp64=True) == fp64


def test_step_bytes_non_cubic_and_per_kernel_split():
    N, (K1, K2, K3) = 131070, (64, 64, 128)
    pts, half = K1 * K2 * K3, K2 * K3 * (K1 // 2 + 1)
    assert bench.step_bytes(N, (K1, K2, K3)) == 88 * N + 24 * pts + 32 * half
    # a cubic grid given as three sizes is the same grid
    assert bench.step_bytes(1000, (48, 48, 48)) == bench.step_bytes(1000, 48)
    parts = {k: bench.algorithmic_bytes(N, (K1, K2, K3), k)
             for k in ("bin", "spread_x", "convolve_yz", "interpolate")}
    assert parts["bin"] == 32 * N
    assert parts["convolve_yz"] == 16 * half
    assert sum(parts.values()) == bench.step_bytes(N, (K1, K2, K3))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
