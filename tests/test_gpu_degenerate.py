"""Degenerate problems through the C ABI, against the oracle: grids of one
level or one latitude row and the minimum three longitudes (columns of a
single cell make P the diagonal of A), and a zero right-hand side, for which
every solver family must return x = 0 after no step (the exit test of
Algorithm 1 holds at the start: <r, r> = 0 <= tol^2 <R, R> = 0)."""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, OctProblem, Problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2103_07210_amd import ftgcr
    ftgcr.load()
    return ftgcr


def _decisions(log):
    return [(d["step"], d["nu"], d["action"]) for d in log]


@pytest.mark.parametrize("shape", [(3, 1, 1), (5, 2, 1), (4, 3, 2), (3, 1, 9), (7, 1, 5)])
def test_tiny_grids_match_oracle(ft, oracle_mod, shape):
    _say("tiny grid", shape)
    pb = Problem(*shape, hill_amp=0.6)
    rhs = I.rhs(pb, 7)
    o = oracle_mod.Oracle(pb)
    plan = [FaultEvent(2, "r", 62, idx=np.array([pb.n - 1]))]
    for p in (None, plan):
        s = ft.Solver(pb, kmax=3)
        x, st = s.solve(rhs, tol=1e-10, k=3, plan=p)
        s.close()
        xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=3, plan=p)
        assert st["status"] == so["status"] == ft.CONVERGED
        assert _decisions(st["log"]) == _decisions(logo)
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
        xe, _, _, _ = o.solve(rhs, tol=1e-13, k=3, plan=p, max_steps=st["steps_executed"])
        err = np.linalg.norm(x.cpu().numpy().ravel() - xe.ravel()) / np.linalg.norm(xe)
        assert err <= 1e-10, err


def test_zero_rhs_every_family(ft):
    """FT-GCR (column preconditioner and P = I), the mixed form, FT-GMRES,
    the octahedral mesh, a batch and the allocation-free entry point."""
    pb = Problem(32, 16, 8)
    z = np.zeros(pb.shape)
    cases = [
        ("gcr", dict()),
        ("gcr P=I", dict(precond="none")),
        ("gmres", dict(method=ft.METHOD_GMRES)),
        ("gmres P=I", dict(method=ft.METHOD_GMRES, precond="none")),
    ]
    for name, kw in cases:
        _say("zero rhs", name)
        s = ft.Solver(pb, kmax=4, max_steps=500, **kw)
        x, st = s.solve(z, tol=1e-10, k=4)
        s.close()
        assert st["status"] == ft.CONVERGED and st["steps_executed"] == 0, (name, st["status"])
        assert not np.any(x.cpu().numpy()), name
    _say("zero rhs mixed")
    s = ft.Solver(pb, "mixed", kmax=4, max_steps=500)
    x, st = s.solve(z, tol=1e-8, k=4)
    s.close()
    assert st["status"] == ft.CONVERGED and st["steps_executed"] == 0 and st["refinements"] == 0
    assert not np.any(x.cpu().numpy())
    _say("zero rhs octahedral")
    po = OctProblem(4, 5)
    s = ft.Solver(po, kmax=3, max_steps=500)
    x, st = s.solve(np.zeros(po.shape), tol=1e-10, k=3)
    s.close()
    assert st["status"] == ft.CONVERGED and st["steps_executed"] == 0
    assert not np.any(x.cpu().numpy())
    _say("zero rhs batch and no-alloc")
    solvers = [ft.Solver(pb, kmax=3, max_steps=500), ft.Solver(Problem(16, 8, 4), kmax=3, max_steps=500)]
    rhs = [z, I.rhs(solvers[1].problem, 3)]
    xs, sts = ft.solve_batch(solvers, rhs, k=3)
    assert sts[0]["status"] == ft.CONVERGED and sts[0]["steps_executed"] == 0
    assert not np.any(xs[0].cpu().numpy())
    assert sts[1]["status"] == ft.CONVERGED and sts[1]["steps_executed"] > 0
    x, st = solvers[0].solve(z, tol=1e-10, k=3, noalloc=True)
    assert st["status"] == ft.CONVERGED and st["steps_executed"] == 0
    for sv in solvers:
        sv.close()
