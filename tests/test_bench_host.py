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
    """One cycle of k = 4 steps plus the converging step.  Algorithmic bytes
    of the direction pass: the direction phase (2 nu + 5) s N plus the
    iterate (2 * 8 N) at nu = k - 1; the design's own kernels: column pass
    4 s N, dots (nu + 2) s N, direction pass (2 nu + 6) s N (+ the iterate),
    the last step running the column pass only."""
    steps, k, s = 5, 4, 8
    assert bench.alg_bytes("dir_update", steps, k, N, s) == (5 + 7 + 9 + 11) * s * N + 16 * N
    assert bench.alg_bytes("update_thomas", steps, k, N, s, design=True) == 5 * 4 * s * N
    assert bench.alg_bytes("stencil_dots", steps, k, N, s, design=True) == (2 + 3 + 4 + 5) * s * N
    assert bench.alg_bytes("dir_update", steps, k, N, s, design=True) == (6 + 8 + 10 + 12) * s * N + 16 * N
    # binary32 vectors with the FP64 iterate
    assert bench.alg_bytes("dir_update", steps, k, N, 4) == (5 + 7 + 9 + 11) * 4 * N + 16 * N


def test_solve_bytes_model():
    """A whole solve: W(nu) = (3 nu + 11) s N per step (the converging step
    only its update phase, nu + 6), 4 s N of backup per cycle, 6 s N for the
    start of each round and 3 * 8 N per FP64 true-residual pass; at k = 4 a
    step averages 16.5 sweeps and the design moves 17 (e stored and re-read,
    the iterate once per cycle)."""
    k, s = 4, 8
    steps = 4 * 100 + 1
    alg = bench.solve_bytes(steps, k, N, s)
    per_cycle = sum(3 * nu + 11 for nu in range(4)) + 4
    expect = 100 * per_cycle * s * N + (6 + 4) * s * N + 6 * s * N + 24 * N
    assert alg == expect
    des = bench.solve_bytes(steps, k, N, s, design=True)
    assert des == 100 * (4 * 4 + (2 + 3 + 4 + 5) + (6 + 8 + 10 + 12)) * s * N + 100 * 16 * N + 4 * s * N \
        + 6 * s * N + 24 * N
    fr = bench.step_frac(steps, k, N, s, ms=100.0)
    assert abs(fr["alg_gbs"] - alg / 0.1 / 1e9) < 1e-6 and abs(fr["frac"] - fr["alg_gbs"] / 8000.0) < 1e-12
    assert 0.02 < fr["design_overhead"] < 0.04


def test_alg_bytes_sampled_steps():
    """With a stride the bytes are those of the sampled steps only; a stride
    coprime with k samples every pass index alike, so the per-launch average
    stays within a launch's spread of the full average."""
    steps, k, s = 357, 4, 8
    full = bench.alg_bytes("dir_update", steps, k, N, s)
    samp = bench.alg_bytes("dir_update", steps, k, N, s, stride=5)
    n_samp = len([t for t in range(1, steps) if t % 5 == 0])
    assert samp == sum((2 * ((t - 1) % k) + 5) * s * N + (16 * N if (t - 1) % k == k - 1 else 0)
                       for t in range(5, steps, 5))
    assert abs(samp / n_samp - full / (steps - 1)) < 0.01 * full / (steps - 1)
    assert bench.TIMED_STRIDE % 2 and bench.TIMED_STRIDE % bench.K


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_gmres_bytes_model():
    """FT-GMRES(k): 2j + 8 sweeps for step j of a cycle, plus m + 5 per cycle
    of m steps: k^2 + 8k + 5 sweeps for a full cycle."""
    import bench
    assert bench.gmres_solve_bytes(16, 1, 16, 1, 1) == 16 * 16 + 8 * 16 + 5
    assert bench.gmres_solve_bytes(4, 1, 4, 1, 1) == 8 + 10 + 12 + 14 + 4 + 5
    # two full cycles and a cut one of 3 steps, FP64 on 100 points
    full = 16 * 16 + 8 * 16 + 5
    cut = (8 + 10 + 12) + 3 + 5
    assert bench.gmres_solve_bytes(35, 3, 16, 100) == (2 * full + cut) * 8 * 100
