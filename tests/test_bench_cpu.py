"""Host-side pieces of bench.py: the algorithmic bytes per packet-step that the roofline
divides by, and the refusal of more than one GPU (no GPU needed)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("precision,ppc,want", [
    # forward: state read + written once (FP64 x, u: 96 B; FP32 cell, off, u: 56 B), plus per
    # cell the fields read once (6 components) and the FP64 exchange (4 components) read and
    # written once, shared by the cell's ppc packets
    ("fp64", 64, 96 + (48 + 64) / 64),   # workload 2: 97.75
    ("fp64", 32, 96 + (48 + 64) / 32),   # workload 4 in FP64: 99.5
    ("fp32", 32, 56 + (24 + 64) / 32),   # workload 4: 58.75
    ("fp32", 8, 56 + (24 + 64) / 8),     # workload 3: 67
])
def test_forward_algorithmic_bytes(precision, ppc, want):
    assert bench.algorithmic_bytes_per_packet_step(precision, ppc) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("precision,want", [
    # recompute: state read, written and stored; reverse: stored state read, adjoint read and
    # written; per cell the fields read by both passes and dL/dE, dL/dB read and written (FP64)
    ("fp64", 3 * 48 + 3 * 48 + (2 * 48 + 2 * 48) / 32),                 # 294
    ("fp32", 3 * 28 + (28 + 24 + 24) + (2 * 24 + 2 * 48) / 32),         # 164.5
])
def test_backward_algorithmic_bytes(precision, want):
    assert bench.algorithmic_bytes_backward(precision, 32) == pytest.approx(want, rel=1e-15)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""
