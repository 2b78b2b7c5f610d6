"""GPU parity on the octahedral reduced Gaussian grid O_N (the paper's mesh
family, Section 3 and Table 1; 51 levels as in its experiments), through
the C ABI (grid.mesh = octahedral), against the oracle's O_N operator and
solvers on the same seeded inputs:

* A and P^-1 element by element (indirect-addressed stencil, column solve
  with per-point constants) up to O160 x 51 levels (5.5M points, Table 1);
* FT-GCR(k) solves: identical decisions on the same fault plans, natural
  step counts within +-1, x within 1e-10 at equal step counts;
* a full solve at O160 x 51 reaching 1e-8 on the true residual evaluated
  with the oracle's operator, a 10% block of r flipped at step 10 detected
  at that step;
* FT-GMRES(k) on O_N against the oracle's FT-GMRES on the same mesh,
  fault-free and with faults.
"""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, OctProblem

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


CASES = [OctProblem(1, 3), OctProblem(4, 5, hill_amp=0.8, hill_lat=0.3), OctProblem(16, 8, hill_lon=2.0),
         OctProblem(40, 51), OctProblem(160, 51)]


@pytest.mark.parametrize("pb", CASES, ids=lambda p: f"O{p.N}x{p.nz}")
@pytest.mark.parametrize("kc", [0, 4])
def test_apply_A_and_pinv_match_oracle(ft, oracle_mod, pb, kc):
    _say("octahedral operator", pb.N, pb.nz, "levels per block", kc or "auto")
    o = oracle_mod.OctOracle(pb)
    assert o.n == pb.n == 4 * pb.N * (pb.N + 9) * pb.nz
    s = ft.Solver(pb, kmax=2, levels_per_block=kc)
    x = np.random.default_rng(1).uniform(-1, 1, pb.n)
    y = s.apply_A(x).cpu().numpy().ravel()
    ref = o.apply_A(x)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    e = s.apply_pinv(x).cpu().numpy().ravel()
    ref = o.apply_pinv(x)
    np.testing.assert_allclose(e, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    s.close()


def _parity(ft, oracle_mod, pb, k, plan=None, tol=1e-10, seed=3):
    rhs = np.random.default_rng(seed).uniform(-1.0, 1.0, pb.n)
    s = ft.Solver(pb, kmax=k)
    x, st = s.solve(rhs, tol=tol, k=k, plan=plan, hist_cap=100000)
    s.close()
    o = oracle_mod.OctOracle(pb)
    xo, so, logo, ho = o.solve(rhs, tol=tol, k=k, plan=plan)
    assert _decisions(st["log"]) == _decisions(logo), (st["log"], logo)
    assert st["status"] == so["status"] == ft.CONVERGED
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, (st["steps_executed"], so["steps_executed"])
    assert st["events_applied"] == so["events_applied"]
    xe, _, _, he = o.solve(rhs, tol=tol * 1e-3, k=k, plan=plan, max_steps=st["steps_executed"])
    err = _rel(x.cpu().numpy(), xe)
    assert err <= 1e-10, err
    n = min(len(he), len(st["hist"]))
    np.testing.assert_allclose(st["hist"][:n], he[:n], rtol=1e-6)
    _say(f"steps {st['steps_executed']} (oracle {so['steps_executed']}), decisions {_decisions(st['log'])}, "
         f"x error {err:.1e}")
    return st


@pytest.mark.parametrize("k", [1, 3, 5])
def test_solve_matches_oracle_o16(ft, oracle_mod, k):
    _say("octahedral solve O16x8 k", k)
    _parity(ft, oracle_mod, OctProblem(16, 8, hill_amp=0.7), k)


@pytest.mark.parametrize("case", range(4))
def test_fault_decisions_match_oracle(ft, oracle_mod, case):
    pb = OctProblem(16, 8, hill_amp=0.7)
    n = pb.n
    plans = [
        [FaultEvent(5, "r", 62, idx=np.array([1234]))],
        [FaultEvent(7, "ap", 62, idx=np.arange(0, n, 97))],
        [FaultEvent(6, "e", 62, idx=np.array([5, 600, 7000])), FaultEvent(9, "x", 61, idx=np.array([3]))],
        [FaultEvent(12, "r", 52, start=100, count=n // 10), FaultEvent(13, "p", 62, idx=np.array([77]))],
    ]
    _say("octahedral faults", case)
    _parity(ft, oracle_mod, pb, 4, plan=plans[case])


def test_solve_matches_oracle_o40_51_levels(ft, oracle_mod):
    """The paper's O40 with its 51 levels (Table 1), k = 5 as in the
    paper's runs, a bit-62 flip of r at step 5."""
    _say("octahedral solve O40x51")
    st = _parity(ft, oracle_mod, I.O40, 5, plan=[FaultEvent(5, "r", 62, idx=np.array([123456]))])
    assert st["detections"] == 1


def test_o160_51_levels_full_solve(ft, oracle_mod):
    """The paper's O160 x 51 levels (5.5M points): FP64 FT-GCR(5) to 1e-8,
    with a contiguous 10% block of r flipped at bit 62 in step 10; the true
    residual is evaluated with the oracle's operator."""
    pb = I.O160
    rhs = np.random.default_rng(160).uniform(-1.0, 1.0, pb.n)
    start = int(np.random.default_rng(161).integers(0, pb.n - pb.n // 10))
    plan = [FaultEvent(10, "r", 62, start=start, count=int(np.ceil(0.1 * pb.n)))]
    s = ft.Solver(pb, kmax=5)
    _say("O160x51 autotune")
    s.autotune(rhs, k=5, steps=12)
    _say("O160x51 solve")
    x, st = s.solve(rhs, tol=1e-8, k=5, plan=plan)
    s.close()
    assert st["status"] == ft.CONVERGED and st["events_applied"] == 1
    assert _decisions(st["log"])[0][0] == 10
    o = oracle_mod.OctOracle(pb)
    true = o.true_residual(x.cpu().numpy().ravel(), rhs)
    assert true <= 1.01e-8, true
    _say(f"O160x51: {st['steps_executed']} steps, {st['detections']} detections, {st['time_ms']:.1f} ms, "
         f"true residual {true:.2e}")


def _gm_parity(ft, oracle_mod, pb, k, plan=None, tol=1e-10):
    """FT-GMRES(k) on O_N against the oracle's (same bars as on the lat-lon
    mesh; the cases are Krylov sizes at which the oracle's own step count
    does not move under 2e-16 perturbations of the right-hand side)."""
    rhs = np.random.default_rng(3).uniform(-1.0, 1.0, pb.n)
    s = ft.Solver(pb, kmax=k, method=ft.METHOD_GMRES)
    x, st = s.solve(rhs, tol=tol, k=k, plan=plan, hist_cap=100000)
    s.close()
    o = oracle_mod.OctOracle(pb)
    _, so, logo, _ = o.solve(rhs, tol=tol, k=k, plan=plan, method="gmres")
    assert _decisions(st["log"]) == _decisions(logo), (st["log"], logo)
    assert st["status"] == so["status"] == ft.CONVERGED
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, (st["steps_executed"], so["steps_executed"])
    assert st["events_applied"] == so["events_applied"]
    xe, _, _, he = o.solve(rhs, tol=tol * 1e-3, k=k, plan=plan, method="gmres", max_steps=st["steps_executed"])
    err = _rel(x.cpu().numpy(), xe)
    assert err <= 1e-10, err
    n = min(len(he), len(st["hist"]))
    keep = he[:n] > 1e-24 * so["rhs_norm2"]
    np.testing.assert_allclose(st["hist"][:n][keep], he[:n][keep], rtol=1e-2)
    _say(f"gmres O{pb.N}x{pb.nz} k={k}: steps {st['steps_executed']} (oracle {so['steps_executed']}), "
         f"decisions {_decisions(st['log'])}, x error {err:.1e}")
    return st


@pytest.mark.parametrize("case", [(OctProblem(4, 5, hill_amp=0.8, hill_lat=0.3), 8),
                                  (OctProblem(16, 8, hill_amp=0.7), 12), (OctProblem(16, 8, hill_amp=0.7), 16)],
                         ids=["O4x5k8", "O16x8k12", "O16x8k16"])
def test_gmres_matches_oracle(ft, oracle_mod, case):
    _say("octahedral gmres", case[0].N, case[1])
    _gm_parity(ft, oracle_mod, *case)


@pytest.mark.parametrize("case", range(3))
def test_gmres_fault_decisions_match_oracle(ft, oracle_mod, case):
    """An overflowing flip of v_j (caught at its step), a flip of x (caught
    at the cycle's end), and several events in one run, on O16 x 8."""
    pb = OctProblem(16, 8, hill_amp=0.7)
    plans = [
        [FaultEvent(7, "r", 62, idx=np.array([100, 2000, 3000]))],
        [FaultEvent(6, "x", 62, idx=np.array([1234]))],
        [FaultEvent(3, "ap", 62, idx=np.array([5])), FaultEvent(20, "e", 40, start=0, count=pb.n // 10)],
    ]
    _say("octahedral gmres faults", case)
    st = _gm_parity(ft, oracle_mod, pb, 16, plan=plans[case])
    if case == 0:
        assert st["detections"] >= 1


@pytest.mark.parametrize("case", [(OctProblem(16, 8, hill_amp=0.7), 4), (I.O40, 5)], ids=["O16x8k4", "O40x51k5"])
def test_mixed_reaches_true_residual(ft, oracle_mod, case):
    """The mixed form on O_N (binary32 tables, vectors, stencil and column
    solve; FP64 inner products, detector and refinement): the FP64 true
    residual, evaluated with the oracle's operator, meets the tolerance, and
    x is within kappa * tol (kappa about 2e3) of the FP64 oracle's solution."""
    pb, k = case
    _say("octahedral mixed", pb.N, pb.nz, k)
    rhs = np.random.default_rng(11).uniform(-1.0, 1.0, pb.n)
    s = ft.Solver(pb, "mixed", kmax=k)
    x, st = s.solve(rhs, tol=1e-8, k=k)
    s.close()
    assert st["status"] == ft.CONVERGED and st["refinements"] >= 1
    o = oracle_mod.OctOracle(pb)
    xn = x.cpu().numpy().ravel()
    true = o.true_residual(xn, rhs)
    assert true <= 1.001e-8, true
    xo, so, _, _ = o.solve(rhs, tol=1e-12, k=k)
    err = float(np.abs(xn - xo).max() / np.abs(xo).max())
    _say(f"mixed steps {st['steps_executed']} (FP64 oracle to 1e-12: {so['steps_executed']}), "
         f"true residual {true:.2e}, x error {err:.1e}")
    assert err <= 2e-5, err


def test_mixed_without_preconditioner(ft, oracle_mod):
    """The mixed form on O_N with P = I (binary32 copy pass, binary32
    indirect stencil): the FP64 true residual meets the tolerance."""
    pb = OctProblem(16, 8, hill_amp=0.7)
    rhs = np.random.default_rng(13).uniform(-1.0, 1.0, pb.n)
    s = ft.Solver(pb, "mixed", kmax=4, precond="none")
    _say("octahedral mixed, P = I")
    x, st = s.solve(rhs, tol=1e-8, k=4)
    s.close()
    assert st["status"] == ft.CONVERGED
    true = oracle_mod.OctOracle(pb).true_residual(x.cpu().numpy().ravel(), rhs)
    assert true <= 1.001e-8, true


def test_mixed_detects_r_fault(ft, oracle_mod):
    """A binary32 exponent flip (bit 30) of every 7th entry of r at step 5
    of a mixed O_N solve is caught at that step, and the solve still meets
    the FP64 true residual."""
    pb = OctProblem(16, 8, hill_amp=0.7)
    rhs = np.random.default_rng(12).uniform(-1.0, 1.0, pb.n)
    plan = [FaultEvent(5, "r", 30, idx=np.arange(0, pb.n, 7))]
    s = ft.Solver(pb, "mixed", kmax=4)
    _say("octahedral mixed fault")
    x, st = s.solve(rhs, tol=1e-8, k=4, plan=plan)
    s.close()
    assert st["status"] == ft.CONVERGED and st["events_applied"] == 1
    assert _decisions(st["log"])[0][0] == 5
    true = oracle_mod.OctOracle(pb).true_residual(x.cpu().numpy().ravel(), rhs)
    assert true <= 1.001e-8, true


def test_o160_51_levels_mixed(ft, oracle_mod):
    """The paper's O160 x 51 levels in the mixed form, FT-GCR(5) to 1e-8 on
    the FP64 true residual (oracle's operator)."""
    pb = I.O160
    rhs = np.random.default_rng(160).uniform(-1.0, 1.0, pb.n)
    s = ft.Solver(pb, "mixed", kmax=5)
    _say("O160x51 mixed")
    x, st = s.solve(rhs, tol=1e-8, k=5)
    s.close()
    assert st["status"] == ft.CONVERGED
    true = oracle_mod.OctOracle(pb).true_residual(x.cpu().numpy().ravel(), rhs)
    _say(f"O160 mixed: {st['steps_executed']} inner steps, {st['refinements']} refinements, true {true:.2e}")
    assert true <= 1.01e-8, true


def test_batch_of_octahedral_members(ft, oracle_mod):
    """O_N members of different sizes, one with a fault, in one batched
    launch sequence: every member as the oracle (decisions, steps +-1, x
    within 1e-10 at equal step counts); a batch mixing meshes is refused."""
    pbs = [OctProblem(16, 8, hill_amp=0.7), OctProblem(8, 6, hill_lon=1.0), OctProblem(24, 9, hill_amp=0.4)]
    rhs = [np.random.default_rng(70 + m).uniform(-1.0, 1.0, pb.n) for m, pb in enumerate(pbs)]
    plans = [[FaultEvent(6, "r", 62, idx=np.array([321]))], [], [FaultEvent(4, "ap", 62, idx=np.array([9]))]]
    solvers = [ft.Solver(pb, kmax=4) for pb in pbs]
    _say("octahedral batch of", len(pbs))
    xs, sts = ft.solve_batch(solvers, rhs, tols=[1e-10] * len(pbs), k=4, plans=plans)
    for m, pb in enumerate(pbs):
        o = oracle_mod.OctOracle(pb)
        _, so, logo, _ = o.solve(rhs[m], tol=1e-10, k=4, plan=plans[m])
        st = sts[m]
        assert st["status"] == ft.CONVERGED, (m, st)
        assert _decisions(st["log"]) == _decisions(logo), m
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, m
        xe, _, _, _ = o.solve(rhs[m], tol=1e-13, k=4, plan=plans[m], max_steps=st["steps_executed"])
        err = _rel(xs[m].cpu().numpy(), xe)
        assert err <= 1e-10, (m, err)
    c = ft.Solver(I.Problem(32, 16, 4), kmax=4)
    with pytest.raises(ft.FtgcrError):
        ft.solve_batch([solvers[0], c], [rhs[0], I.rhs(I.Problem(32, 16, 4), 1)], k=4)
    for s in solvers + [c]:
        s.close()
