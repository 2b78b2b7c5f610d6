"""Pins of the oracle's faults in e = P^-1(r), the paper's injection site
(Section 3: right after the preconditioner), against what the mathematics of
GCR fixes independently of any implementation:

* e feeds both the new direction p^{nu+1} = e + sum alpha p^l and its image
  L(p^{nu+1}) = L(e) + sum alpha L(p^l), so a finite flip keeps the pair
  consistent: the next steps are exact minimal-residual steps along a worse
  direction.  The residual still decreases monotonically (nothing to detect)
  and the recursive residual stays equal to A x - R -- a flip placed anywhere
  else (only into p, or only into L(e)) would break that equality.
* A flip that overflows makes <L p, L p> infinite one step later: the
  detector fires at step s + 1 and the rollback returns to the fault-free
  trajectory bit for bit, at the cost bound of Section 2 (at most a cycle).
* A step that exits or rolls back never computes e; its e events do not apply.
"""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent

K = 3


@pytest.fixture(scope="module")
def c1(oracle_mod):
    pb = I.C1
    o = oracle_mod.Oracle(pb)
    rhs = I.rhs(pb, I.SEEDS["c1_rhs"])
    x, st, log, hist = o.solve(rhs, tol=1e-10, k=K)
    return o, rhs, x, st, hist


def _true_rel(o, x, rhs):
    return o.true_residual(x, rhs)


@pytest.mark.parametrize("step,bits", [(4, (40, 51)), (9, (30, 45)), (20, (0, 51))])
def test_finite_e_flip_keeps_directions_consistent(oracle_mod, c1, step, bits):
    o, rhs, xc, sc, hc = c1
    rng = np.random.default_rng(step)
    idx = np.sort(rng.choice(I.C1.n, 300, replace=False))
    plan = [FaultEvent(step=step, vec="e", bit=0, idx=idx,
                       bits=rng.integers(bits[0], bits[1] + 1, idx.size).astype(np.uint8))]
    # stop a few steps after the event: the recursive residual of that state
    # against the operator applied to its x
    x, st, log, hist = o.solve(rhs, tol=1e-14, k=K, plan=plan, max_steps=step + 6)
    assert st["events_applied"] == 1 and st["detections"] == 0
    assert np.all(np.diff(hist) < 0), "the residual must keep decreasing"
    rec = np.sqrt(hist[-1] / np.dot(rhs.ravel(), rhs.ravel()))
    true = _true_rel(o, x, rhs)
    assert abs(true - rec) <= 1e-9 * max(true, 1e-12) + 1e-13
    # the direction changed, so the iterates differ from the fault-free run
    x0, _, _, _ = o.solve(rhs, tol=1e-14, k=K, max_steps=step + 6)
    assert not np.array_equal(x, x0)
    # and the full solve still converges with nothing detected
    xf, sf, lf, _ = o.solve(rhs, tol=1e-10, k=K, plan=plan)
    assert sf["status"] == oracle_mod.CONVERGED and sf["detections"] == 0


@pytest.mark.parametrize("step", [2, 3, 4, 7, 12])
def test_overflowing_e_flip_detected_next_step(oracle_mod, c1, step):
    """Bit 62 of every entry of e at step s: entries below 2 in magnitude
    become spikes beyond 1e300, Inf or NaN, so <L p^{nu+1}, L p^{nu+1}> is
    not finite and step s + 1 fails the test.  The rollback goes to the start
    of the cycle holding step s + 1 (or to the previous cycle's start when
    s + 1 opens a cycle), and the run then equals the fault-free one."""
    o, rhs, xc, sc, hc = c1
    plan = [FaultEvent(step=step, vec="e", bit=62, start=0, count=I.C1.n)]
    x, st, log, hist = o.solve(rhs, tol=1e-10, k=K, plan=plan)
    assert st["events_applied"] == 1
    nu_next = step % K           # pass index of step s + 1
    assert [(d["step"], d["nu"], d["action"]) for d in log] == [(step + 1, nu_next, 0)]
    assert st["steps_wasted"] == (K + 1 if nu_next == 0 else nu_next + 1)
    assert st["steps_executed"] == sc["steps_executed"] + st["steps_wasted"]
    np.testing.assert_array_equal(x, xc)


def test_e_events_of_rejected_or_final_steps_do_not_apply(oracle_mod, c1):
    o, rhs, xc, sc, hc = c1
    # step 5 rolls back (bit 62 of all of r): its e is never computed
    plan = [FaultEvent(step=5, vec="r", bit=62, start=0, count=I.C1.n),
            FaultEvent(step=5, vec="e", bit=62, start=0, count=I.C1.n)]
    x, st, log, _ = o.solve(rhs, tol=1e-10, k=K, plan=plan)
    assert st["events_applied"] == 1
    assert [(d["step"], d["action"]) for d in log] == [(5, 0)]
    np.testing.assert_array_equal(x, xc)
    # the converging step exits before its preconditioner
    last = sc["steps_executed"]
    plan = [FaultEvent(step=last, vec="e", bit=62, start=0, count=I.C1.n)]
    x, st, _, _ = o.solve(rhs, tol=1e-10, k=K, plan=plan)
    assert st["events_applied"] == 0
    np.testing.assert_array_equal(x, xc)


def test_paper_plans_shape():
    """The paper-model generator: Bernoulli steps (at most 10), each event a
    set of distinct entries of e inside one process' share, one bit each."""
    pb = I.Problem(64, 32, 8)
    plans = I.paper_plans(pb, 50, prob=0.05, data_loss=0.01, procs=8, horizon=200)
    counts = [len(p) for p in plans]
    assert max(counts) <= 10 and sum(counts) > 0
    share = pb.n // 8
    for plan in plans:
        steps = [e.step for e in plan]
        assert steps == sorted(set(steps)) and all(1 <= s <= 200 for s in steps)
        for ev in plan:
            assert ev.vec == I.VEC_E and ev.bits is not None and ev.bits.max() <= 63
            assert ev.count == int(np.ceil(0.01 * pb.n))
            assert np.unique(ev.idx).size == ev.idx.size
            cols = np.unique(ev.idx % (pb.nx * pb.ny))
            assert cols.max() - cols.min() < share // pb.nz + 1
    big = I.paper_plans(pb, 5, prob=0.5, data_loss=0.2, procs=8, horizon=20)
    assert all(ev.count == share for plan in big for ev in plan)
    # the readings of the flipped bit: "uniform" is the U{0..63} stream
    # itself; "finite" draws the same steps and entries and never bit 62
    uni = I.paper_plans(pb, 20, prob=0.05, data_loss=0.01, procs=8, horizon=200, bits="uniform")
    fin = I.paper_plans(pb, 20, prob=0.05, data_loss=0.01, procs=8, horizon=200, bits="finite")
    ref = I.paper_plans(pb, 20, prob=0.05, data_loss=0.01, procs=8, horizon=200)
    seen = np.zeros(64, dtype=bool)
    for pu, pf, pr in zip(uni, fin, ref):
        assert [e.step for e in pu] == [e.step for e in pf] == [e.step for e in pr]
        for eu, ef, er in zip(pu, pf, pr):
            assert np.array_equal(eu.bits, er.bits)
            assert np.array_equal(eu.idx, ef.idx)
            assert not np.any(ef.bits == 62)
            seen[ef.bits] = True
    assert seen.sum() == 63 and not seen[62]
