"""GPU parity for faults in e = P^-1(r), the paper's injection site (Section
3): the HIP path injects into the stored e between the step's decision and
its stencil pass, so both of e's readers (L(e) and the new direction) see the
flip, as in the oracle.  Bars as for the other faults: identical decisions
and applied-event counts, x within 1e-10 at equal step counts."""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, Problem

pytestmark = pytest.mark.gpu

K = 3


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def ft(torch_dev):
    from paper_2103_07210_amd import ftgcr
    ftgcr.load()
    return ftgcr


def _decisions(log):
    return [(d["step"], d["nu"], d["action"]) for d in log]


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert np.isfinite(a).all() and np.isfinite(b).all()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = ["finite@4", "finite@3+overflow@9", "overflow@2", "overflow@3", "overflow@7", "r+e@5", "late"]


def _plan(case, n):
    rng = np.random.default_rng(CASES.index(case) + 1)
    idx = np.sort(rng.choice(n, 300, replace=False))
    finite = rng.integers(40, 52, idx.size).astype(np.uint8)
    return {
        "finite@4": [FaultEvent(4, "e", 0, idx=idx, bits=finite)],
        "finite@3+overflow@9": [FaultEvent(3, "e", 0, idx=idx, bits=finite),
                                FaultEvent(9, "e", 62, start=0, count=n)],
        "overflow@2": [FaultEvent(2, "e", 62, start=0, count=n)],
        "overflow@3": [FaultEvent(3, "e", 62, start=0, count=n)],
        "overflow@7": [FaultEvent(7, "e", 62, start=0, count=n)],
        "r+e@5": [FaultEvent(5, "r", 62, start=0, count=n), FaultEvent(5, "e", 62, start=0, count=n)],
        "late": [FaultEvent(10 ** 6, "e", 62, start=0, count=n)],
    }[case]


@pytest.mark.parametrize("case", CASES)
def test_e_faults_match_oracle(ft, oracle_mod, case):
    _say("e fault", case)
    pb = I.C1
    rhs = I.rhs(pb, I.SEEDS["c1_rhs"])
    plan = _plan(case, pb.n)
    s = ft.Solver(pb, kmax=K)
    x, st = s.solve(rhs, tol=1e-10, k=K, plan=plan)
    s.close()
    o = oracle_mod.Oracle(pb)
    xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=K, plan=plan)
    assert _decisions(st["log"]) == _decisions(logo), (st["log"], logo)
    assert st["events_applied"] == so["events_applied"]
    assert st["status"] == so["status"] == ft.CONVERGED
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
    xe, _, _, _ = o.solve(rhs, tol=1e-13, k=K, plan=plan, max_steps=st["steps_executed"])
    assert _rel(x.cpu().numpy(), xe) <= 1e-10


def test_e_event_at_the_last_allowed_step(ft, oracle_mod):
    """A step that ends the solve by the step cap still passed its tests:
    its e event applies on both sides (and changes nothing returned)."""
    pb = Problem(32, 16, 8)
    rhs = I.rhs(pb, 9)
    plan = [FaultEvent(6, "e", 62, start=0, count=pb.n)]
    s = ft.Solver(pb, kmax=K, max_steps=6)
    x, st = s.solve(rhs, tol=1e-10, k=K, plan=plan)
    s.close()
    xo, so, _, _ = oracle_mod.Oracle(pb).solve(rhs, tol=1e-10, k=K, plan=plan, max_steps=6)
    assert st["status"] == so["status"] == ft.MAX_STEPS
    assert st["events_applied"] == so["events_applied"] == 1
    assert _rel(x.cpu().numpy(), xo) <= 1e-12


@pytest.mark.parametrize("bits", ["uniform", "finite"])
def test_paper_campaign_slice_matches_oracle(ft, oracle_mod, bits):
    """The paper's fault model (Bernoulli per step, several events per run,
    random bits in a process' share of e) on a small grid, under both
    readings of the flipped bit (any of 64, or all but the top exponent
    bit): per run the same decisions and applied events as the oracle."""
    pb = Problem(64, 32, 8, hill_amp=0.7)
    rhs = I.rhs(pb, 2)
    o = oracle_mod.Oracle(pb)
    s = ft.Solver(pb, kmax=4)
    plans = I.paper_plans(pb, 10, prob=0.08, data_loss=0.01, procs=8, horizon=120, seed0=7000, bits=bits)
    assert sum(len(p) for p in plans) > 10
    for m, plan in enumerate(plans):
        _say("paper plan", bits, m, [(e.step, e.count) for e in plan])
        x, st = s.solve(rhs, tol=1e-10, k=4, plan=plan)
        xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=4, plan=plan)
        assert _decisions(st["log"]) == _decisions(logo), (m, st["log"], logo)
        assert st["events_applied"] == so["events_applied"], m
        assert st["status"] == so["status"]
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
        xe, _, _, _ = o.solve(rhs, tol=1e-13, k=4, plan=plan, max_steps=st["steps_executed"])
        if np.all(np.isfinite(xe)):
            assert _rel(x.cpu().numpy(), xe) <= 1e-10
    s.close()


def test_mixed_e_fault_still_converges(ft):
    """Mixed form: bit 30 (binary32 exponent MSB) of every 7th entry of e at
    step 6.  Entries below 1 in magnitude grow by 2^128 but stay finite, and
    the FP64 inner products of such spikes cannot overflow, so the step is an
    exact minimal-residual step along a poor direction and usually passes
    the test (as binary32 faults in L(p) do); the FP64 refinement still takes
    the true residual to the tolerance.  (Flipping every entry below 1 would
    only rescale e by 2^128, which GCR does not see at all.)"""
    pb = I.C1
    rhs = I.rhs(pb, 1)
    s = ft.Solver(pb, "mixed", kmax=K)
    plan = [FaultEvent(6, "e", 30, idx=np.arange(0, pb.n, 7))]
    x, st = s.solve(rhs, tol=1e-8, k=K, plan=plan)
    x0, st0 = s.solve(rhs, tol=1e-8, k=K)
    s.close()
    assert st["events_applied"] == 1
    assert st["status"] == ft.CONVERGED and st["rel_res_true"] <= 1e-8
    assert st["steps_executed"] != st0["steps_executed"] or not np.array_equal(x.cpu().numpy(), x0.cpu().numpy())


def test_batch_member_e_fault(ft, oracle_mod):
    """e events inside a batched launch sequence land on their member only,
    between the combined decision and the combined stencil pass."""
    pbs = [Problem(64, 32, 8), Problem(48, 24, 6, hill_lon=1.0), Problem(64, 32, 8, hill_amp=0.3)]
    rhs = [I.rhs(pb, 60 + m) for m, pb in enumerate(pbs)]
    plans = [[], [FaultEvent(5, "e", 62, start=0, count=pbs[1].n)],
             [FaultEvent(4, "e", 45, idx=np.arange(0, pbs[2].n, 7))]]
    solvers = [ft.Solver(pb, kmax=K) for pb in pbs]
    xs, sts = ft.solve_batch(solvers, rhs, tols=[1e-10] * 3, k=K, plans=plans)
    for m, pb in enumerate(pbs):
        o = oracle_mod.Oracle(pb)
        xo, so, logo, _ = o.solve(rhs[m], tol=1e-10, k=K, plan=plans[m])
        assert _decisions(sts[m]["log"]) == _decisions(logo), m
        assert sts[m]["events_applied"] == so["events_applied"], m
        assert abs(sts[m]["steps_executed"] - so["steps_executed"]) <= 1, m
        xe, _, _, _ = o.solve(rhs[m], tol=1e-13, k=K, plan=plans[m], max_steps=sts[m]["steps_executed"])
        assert _rel(xs[m].cpu().numpy(), xe) <= 1e-10, m
    for s in solvers:
        s.close()
