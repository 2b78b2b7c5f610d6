"""GPU parity of FT-GMRES(k) (options.method = GMRES: the fault layer of
Algorithm 1 on right-preconditioned restarted GMRES) against the oracle's
FT-GMRES on the same seeded inputs and fault plans, through the C ABI.

Bars as for FT-GCR: identical decision lists (step, nu, action; nu = -1 for
a cycle-end check), natural executed-step counts within +-1, x within 1e-10
relative at equal executed-step counts.  Restarted GMRES with a small k
converges slowly on this operator and its step count moves by up to +-20
when a coefficient is perturbed by 2e-16 (measured on the oracle), so the
cases here use Krylov sizes at which the oracle's own count, decisions and
iterate do not move under such perturbations (measured: count spread 0, x
drift <= 5e-12, drift of the per-step squared residual norms <= 9e-4); the
per-step norms are compared within 1e-2 relative while above 1e-24 |R|^2."""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, Problem

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


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert np.array_equal(np.isfinite(a), np.isfinite(b))
    f = np.isfinite(b)
    return float(np.linalg.norm(a[f] - b[f]) / np.linalg.norm(b[f]))


def _parity(ft, oracle_mod, pb, k, tol=1e-10, plan=None, rhs_seed=1, **opts):
    rhs = I.rhs(pb, rhs_seed)
    s = ft.Solver(pb, kmax=max(k, 2), method=ft.METHOD_GMRES, **opts)
    x, st = s.solve(rhs, tol=tol, k=k, plan=plan, hist_cap=100000)
    o = oracle_mod.Oracle(pb)
    xo, so, logo, ho = o.solve(rhs, tol=tol, k=k, plan=plan, method="gmres")
    assert _decisions(st["log"]) == _decisions(logo), (st["log"], logo)
    assert st["status"] == so["status"], (st["status"], so["status"])
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, (st["steps_executed"], so["steps_executed"])
    assert st["events_applied"] == so["events_applied"]
    xe, se, _, he = o.solve(rhs, tol=tol * 1e-3, k=k, plan=plan, method="gmres",
                            max_steps=st["steps_executed"])
    err = _rel(x.cpu().numpy(), xe)
    assert err <= 1e-10, err
    n = min(len(he), len(st["hist"]))
    keep = he[:n] > 1e-24 * so["rhs_norm2"]
    np.testing.assert_allclose(st["hist"][:n][keep], he[:n][keep], rtol=1e-2)
    s.close()
    _say(f"steps {st['steps_executed']} (oracle {so['steps_executed']}), decisions {_decisions(st['log'])}, "
         f"x error {err:.1e}")
    return x, st, so


@pytest.mark.parametrize("shape,k", [((64, 32, 8), 16), ((100, 7, 5), 16), ((70, 9, 33), 12), ((64, 8, 96), 8),
                                     ((96, 48, 12), 16), ((64, 32, 8), 12)])
def test_gmres_matches_oracle(ft, oracle_mod, shape, k):
    _say("gmres", shape, k)
    _parity(ft, oracle_mod, Problem(*shape, hill_amp=0.7, hill_lon=1.1), k, rhs_seed=3)


@pytest.mark.parametrize("case", range(6))
def test_gmres_fault_decisions_match_oracle(ft, oracle_mod, case):
    """x flips (caught at the cycle's end), overflowing flips of v_j and of
    A z_j (caught at their step), flips of z_j (consistent, undetected),
    several events in one run and a range of entries."""
    pb = Problem(64, 32, 8, hill_amp=0.7, hill_lon=np.pi / 2)
    n = pb.n
    plans = [
        [FaultEvent(6, "x", 62, idx=np.array([1234]))],
        [FaultEvent(7, "r", 62, idx=np.array([100, 2000, 3000]))],
        [FaultEvent(3, "ap", 62, idx=np.array([5]))],
        [FaultEvent(5, "e", 40, idx=np.arange(0, n, 17))],
        [FaultEvent(1, "r", 62, idx=np.array([9])), FaultEvent(10, "x", 61, idx=np.array([3, 4000])),
         FaultEvent(11, "p", 62, idx=np.array([77]))],
        [FaultEvent(9, "ap", 52, start=100, count=n // 10), FaultEvent(20, "r", 30, start=0, count=n // 3)],
    ]
    _say("gmres faults", case)
    x, st, so = _parity(ft, oracle_mod, pb, 16, plan=plans[case], rhs_seed=5)
    if case in (1, 2):   # the overflowing flips are caught at their step
        assert st["detections"] >= 1


def test_gmres_recovers_fault_free_iterate(ft):
    """A detected transient fault (an x flip caught at the cycle end) is
    rolled back and the run replays the fault-free one bit for bit."""
    pb = Problem(64, 32, 8, hill_amp=0.7)
    rhs = I.rhs(pb, 5)
    s = ft.Solver(pb, kmax=4, method=ft.METHOD_GMRES)
    xc, sc = s.solve(rhs, tol=1e-10, k=4)
    x, st = s.solve(rhs, tol=1e-10, k=4, plan=[FaultEvent(6, "x", 62, idx=np.array([1234]))])
    s.close()
    assert _decisions(st["log"]) == [(8, -1, 0)] and st["steps_wasted"] == 4
    assert np.array_equal(x.cpu().numpy(), xc.cpu().numpy())
    assert st["steps_executed"] == sc["steps_executed"] + 4


def test_gmres_step_cap_and_edge_cases(ft, oracle_mod):
    pb = Problem(16, 8, 4)
    rhs = I.rhs(pb, 5)
    o = oracle_mod.Oracle(pb)
    s = ft.Solver(pb, kmax=4, method=ft.METHOD_GMRES, max_steps=7)
    # the cap cuts the second cycle after its third step
    x, st = s.solve(rhs, tol=1e-10, k=4)
    xo, so, _, _ = o.solve(rhs, tol=1e-10, k=4, max_steps=7, method="gmres")
    assert st["status"] == so["status"] == ft.MAX_STEPS and st["steps_executed"] == 7
    assert _rel(x.cpu().numpy(), xo) <= 1e-12
    s.set_options(max_steps=100000)
    # exact initial guess: no step
    xs = np.linalg.solve(o.dense_matrix(), rhs.ravel()).reshape(pb.shape)
    x, st = s.solve(rhs, x=xs, tol=1e-10, k=4)
    assert st["status"] == ft.CONVERGED and st["steps_executed"] == 0
    s.close()
    # GMRES is built for FP64 single solves
    sm = ft.Solver(pb, "mixed", kmax=4)
    with pytest.raises(ft.FtgcrError):
        sm.set_options(method=ft.METHOD_GMRES)
    sm.close()


def test_gmres_stagnation(ft, oracle_mod):
    pb = Problem(8, 4, 3)
    o = oracle_mod.Oracle(pb)
    n = pb.n
    m = o.dense_matrix()
    pinv = np.stack([o.apply_pinv(np.eye(n)[c]).reshape(-1) for c in range(n)], 1)
    b = m @ pinv
    w, v = np.linalg.eigh(0.5 * (b + b.T))
    s = ft.Solver(pb, kmax=3, method=ft.METHOD_GMRES)
    for j in (1, 2, 3):
        rhs = v[:, 0] + np.sqrt(-w[0] / w[j]) * v[:, j]
        _say("gmres stagnation", j)
        x, st = s.solve(rhs, tol=1e-10, k=3)
        _, so, logo, _ = o.solve(rhs, tol=1e-10, k=3, method="gmres")
        for log in (st["log"], logo):
            assert _decisions(log) in ([], [(1, 0, 0), (2, 0, 1)])
        assert st["status"] == so["status"] == ft.CONVERGED
    s.close()


def test_gmres_campaign_slice(ft, oracle_mod):
    """Single-event campaign plans (step 1..20, vector x / r / p / A z,
    1 entry, 1% or a 10% block, bit 0..63) on 64x32x8, k = 16."""
    pb = Problem(64, 32, 8)
    rhs = I.rhs(pb, 2)
    o = oracle_mod.Oracle(pb)
    s = ft.Solver(pb, kmax=16, method=ft.METHOD_GMRES)
    for m, plan in enumerate(I.campaign_plans(pb, count=8, seed0=1000)):
        _say("gmres campaign", m, plan[0].step, plan[0].vec, plan[0].count, plan[0].bit)
        x, st = s.solve(rhs, tol=1e-10, k=16, plan=plan)
        xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=16, plan=plan, method="gmres")
        assert _decisions(st["log"]) == _decisions(logo), (m, st["log"], logo)
        assert st["status"] == so["status"]
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
        xe, _, _, _ = o.solve(rhs, tol=1e-13, k=16, plan=plan, method="gmres", max_steps=st["steps_executed"])
        if np.all(np.isfinite(xe)):
            assert _rel(x.cpu().numpy(), xe) <= 1e-10
    s.close()
