"""Host-side checks of bench.py's bookkeeping (no GPU): the algorithmic-byte
model of the step kernels and of the sampled timing, and the single-GPU
contract of the command line."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N = 512 * 256 * 64


def test_alg_bytes_per_pass():
    """One cycle of k = 4 steps plus the converging step: column pass 4 s N
    per step; dots (nu + 2) s N and direction pass (2 nu + 6) s N (+ the
    iterate, 2 * 8 N, at nu = k - 1) on every step but the last."""
    steps, k, s = 5, 4, 8
    assert bench.alg_bytes("update_thomas", steps, k, N, s) == 5 * 4 * s * N
    assert bench.alg_bytes("stencil_dots", steps, k, N, s) == (2 + 3 + 4 + 5) * s * N
    assert bench.alg_bytes("dir_update", steps, k, N, s) == (6 + 8 + 10 + 12) * s * N + 16 * N
    # binary32 vectors with the FP64 iterate
    assert bench.alg_bytes("dir_update", steps, k, N, 4) == (6 + 8 + 10 + 12) * 4 * N + 16 * N


def test_alg_bytes_sampled_steps():
    """With a stride the bytes are those of the sampled steps only; a stride
    coprime with k samples every pass index alike, so the per-launch average
    stays within a launch's spread of the full average."""
    steps, k, s = 357, 4, 8
    full = bench.alg_bytes("dir_update", steps, k, N, s)
    samp = bench.alg_bytes("dir_update", steps, k, N, s, stride=5)
    n_samp = len([t for t in range(1, steps) if t % 5 == 0])
    assert samp == sum((2 * ((t - 1) % k) + 6) * s * N + (16 * N if (t - 1) % k == k - 1 else 0)
                       for t in range(5, steps, 5))
    assert abs(samp / n_samp - full / (steps - 1)) < 0.01 * full / (steps - 1)
    assert bench.TIMED_STRIDE % 2 and bench.TIMED_STRIDE % bench.K


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
