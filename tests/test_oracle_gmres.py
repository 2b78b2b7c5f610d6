"""Pins of the oracle's FT-GMRES(k): the fault layer of Algorithm 1 (the
monotone residual-norm test, the backup after each complete Krylov cycle,
the rollback and the stagnation rule) on right-preconditioned restarted
GMRES(k), the other Krylov solver the paper's method is meant to extend to
(abstract; Section 1).

* restarted GMRES computed a different way: a dense, power-basis,
  QR-and-least-squares solve of every cycle's minimisation on tiny grids
  (no Arnoldi, no Givens rotations), with the same restart points -- the
  per-step residual norms and the iterate after several cycles agree;
* one long cycle (k above the step count) minimises over the same Krylov
  space as GCR(k) without restart: the residual norms equal the GCR
  oracle's;
* dense LU solutions;
* predicted fault outcomes: a flip of x (never read inside a cycle) shows in
  the explicit residual at the cycle's end and is rolled back there; a flip
  that overflows v_j or A z_j makes the step's residual norm NaN and is
  caught at that step; both recover the fault-free iterate bit for bit
  (Section 3: if all faults are detected, convergence matches the
  baseline); a flip of z_j is carried consistently into A z_j and into the
  correction (as in flexible GMRES), so the residual norm stays exact and
  nothing is detected.
"""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, Problem

TINY = [Problem(8, 4, 3, hill_amp=0.8), Problem(16, 8, 4, hill_lat=-0.4)]


def _dense_pinv(o):
    n = o.n
    return np.stack([o.apply_pinv(np.eye(n)[c]).reshape(-1) for c in range(n)], 1)


def _dense_restarted_gmres(m, pinv, rhs, k, cycles):
    """Per-step residual norms and the iterate of restarted right-
    preconditioned GMRES(k), each cycle's minimisation solved directly:
    min over c of |s - (A P^-1) Q c| with Q an orthonormal basis (QR) of the
    power Krylov basis [s, B s, ..., B^{j-1} s], B = A P^-1."""
    b = m @ pinv
    x = np.zeros(rhs.size)
    norms = []
    for _ in range(cycles):
        s = rhs - m @ x
        kb = [s / np.linalg.norm(s)]
        for _ in range(k - 1):
            v = b @ kb[-1]
            kb.append(v / np.linalg.norm(v))
        kb = np.stack(kb, 1)
        for j in range(1, k + 1):
            q, _ = np.linalg.qr(kb[:, :j])
            c, *_ = np.linalg.lstsq(b @ q, s, rcond=None)
            norms.append(np.linalg.norm(s - b @ q @ c))
        x = x + pinv @ (q @ c)
    return np.array(norms), x


@pytest.mark.parametrize("pb,k", [(TINY[0], 4), (TINY[1], 3)])
def test_matches_dense_restarted_gmres(oracle_mod, pb, k):
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 21).reshape(-1)
    cycles = 5
    x, st, log, hist = o.solve(rhs, tol=1e-30, k=k, max_steps=cycles * k, ft=False, method="gmres")
    assert st["steps_executed"] == cycles * k and st["status"] == oracle_mod.MAX_STEPS
    assert st["cycles"] == cycles
    ref_norms, ref_x = _dense_restarted_gmres(o.dense_matrix(), _dense_pinv(o), rhs, k, cycles)
    np.testing.assert_allclose(np.sqrt(hist), ref_norms, rtol=1e-8)
    np.testing.assert_allclose(x.reshape(-1), ref_x, rtol=0, atol=1e-9 * np.abs(ref_x).max())


def test_one_long_cycle_equals_gcr(oracle_mod):
    pb = TINY[0]
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 12).reshape(-1)
    steps = 40
    _, sg, _, hg = o.solve(rhs, tol=1e-30, k=steps + 5, max_steps=steps, ft=False, method="gmres")
    _, sc, _, hc = o.solve(rhs, tol=1e-30, k=steps + 5, max_steps=steps, ft=False)
    assert sg["steps_executed"] == sc["steps_executed"] == steps
    keep = np.sqrt(hc / sc["rhs_norm2"]) > 1e-9
    assert keep.sum() >= 15
    np.testing.assert_allclose(hg[keep], hc[keep], rtol=1e-6)


@pytest.mark.parametrize("pb", TINY)
def test_solution_matches_dense_lu(oracle_mod, pb):
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 11).reshape(-1)
    m = o.dense_matrix()
    ref = np.linalg.solve(m, rhs)
    tol = 1e-12
    x, st, log, hist = o.solve(rhs, tol=tol, k=4, method="gmres")
    assert st["status"] == oracle_mod.CONVERGED and st["detections"] == 0
    err = np.linalg.norm(x.reshape(-1) - ref) / np.linalg.norm(ref)
    assert err <= 2 * np.linalg.cond(m) * tol
    assert np.linalg.norm(m @ x.reshape(-1) - rhs) / np.linalg.norm(rhs) <= tol
    # fault-free: the step norms never increase inside a cycle
    assert st["steps_wasted"] == 0


def _clean(o, rhs, k):
    return o.solve(rhs, tol=1e-10, k=k, method="gmres", hist_cap=4096)


def test_x_flip_caught_at_cycle_end_and_recovered_exactly(oracle_mod):
    pb = Problem(32, 16, 8, hill_amp=0.7)
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 5)
    xc, sc, _, _ = _clean(o, rhs, 4)
    # step 6 is the second step of the second cycle; the cycle ends at step 8
    plan = [FaultEvent(6, "x", 62, idx=np.array([1234]))]
    x, st, log, _ = o.solve(rhs, tol=1e-10, k=4, method="gmres", plan=plan)
    assert [(d["step"], d["nu"], d["action"]) for d in log] == [(8, -1, 0)]
    assert st["events_applied"] == 1 and st["steps_wasted"] == 4
    assert st["steps_executed"] == sc["steps_executed"] + 4
    assert np.array_equal(x, xc)


@pytest.mark.parametrize("vec,step,nu", [("r", 7, 2), ("ap", 3, 2), ("r", 9, 0)])
def test_overflowing_flip_caught_at_its_step(oracle_mod, vec, step, nu):
    """Bit 62 of entries below 1 in magnitude multiplies them by 2^1024: the
    squared norms overflow, the step's residual norm is NaN, and the
    detector (which treats NaN as a fault) fires at that step; the cycle is
    redone from the backup."""
    pb = Problem(32, 16, 8, hill_amp=0.7)
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 5)
    xc, sc, _, _ = _clean(o, rhs, 4)
    plan = [FaultEvent(step, vec, 62, idx=np.array([100, 2000, 3000]))]
    x, st, log, _ = o.solve(rhs, tol=1e-10, k=4, method="gmres", plan=plan)
    assert [(d["step"], d["nu"], d["action"]) for d in log] == [(step, nu, 0)]
    assert st["steps_wasted"] == nu + 1
    assert np.array_equal(x, xc)


def test_z_flip_stays_consistent_and_undetected(oracle_mod):
    pb = Problem(32, 16, 8, hill_amp=0.7)
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 5)
    plan = [FaultEvent(5, "e", 40, idx=np.arange(0, pb.n, 17))]
    x, st, log, _ = o.solve(rhs, tol=1e-10, k=4, method="gmres", plan=plan)
    assert st["events_applied"] == 1 and st["detections"] == 0
    assert st["status"] == oracle_mod.CONVERGED
    assert o.true_residual(x, rhs) <= 1e-10


def test_ft_off_takes_no_decisions(oracle_mod):
    pb = Problem(32, 16, 8, hill_amp=0.7)
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, 5)
    plan = [FaultEvent(6, "x", 40, idx=np.array([1234]))]
    x, st, log, _ = o.solve(rhs, tol=1e-10, k=4, method="gmres", plan=plan, ft=False)
    assert st["detections"] == 0 and log == []
    # a restart recomputes the residual of the corrupted x, so restarted
    # GMRES corrects a finite flip of x by itself
    assert st["status"] == oracle_mod.CONVERGED and o.true_residual(x, rhs) <= 1e-10


def test_stagnation_is_accepted(oracle_mod):
    """<v0, A P^-1 v0> = 0 up to round-off: the first step cannot lower the
    residual (the Givens sine is 1 to rounding); if that reads as a fault the
    rerun detects it again at the same place and it is accepted."""
    pb = Problem(8, 4, 3)
    o = oracle_mod.Oracle(pb)
    m = o.dense_matrix()
    b = m @ _dense_pinv(o)
    w, v = np.linalg.eigh(0.5 * (b + b.T))
    for j in (1, 2, 3):
        rhs = v[:, 0] + np.sqrt(-w[0] / w[j]) * v[:, j]
        x, st, log, _ = o.solve(rhs, tol=1e-10, k=3, method="gmres")
        assert [(d["step"], d["nu"], d["action"]) for d in log] in ([], [(1, 0, 0), (2, 0, 1)])
        assert st["status"] == oracle_mod.CONVERGED
