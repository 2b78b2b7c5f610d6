"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars: operator and preconditioner element by element to a few ulps of FP64;
solves: x within 1e-10 relative at equal executed-step counts, natural step
counts within +-1, identical detect / rollback / stagnation decisions
(step, nu, action) on the same fault plans (Algorithm 1, red part).
"""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, Problem

pytestmark = pytest.mark.gpu


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


def _rel(a, b):
    """Relative difference of two solutions.  A fault can drive entries to
    Inf / NaN (the same entries with the same class on both sides) or to huge
    finite values (|v| > 1e150, compared entry by entry); the ordinary
    entries are compared by relative 2-norm."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    fa, fb = np.isfinite(a), np.isfinite(b)
    assert np.array_equal(fa, fb), "different entries became non-finite"
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(a[~fa & ~np.isnan(a)], b[~fb & ~np.isnan(b)])
    huge = fb & (np.abs(b) > 1e150)
    ordinary = fb & ~huge
    err = 0.0
    if huge.any():
        err = float(np.max(np.abs(a[huge] / b[huge] - 1.0)))
    if ordinary.any():
        nb = np.linalg.norm(b[ordinary])
        err = max(err, float(np.linalg.norm(a[ordinary] - b[ordinary]) / max(nb, 1e-300)))
    return err


def _decisions(log):
    return [(d["step"], d["nu"], d["action"]) for d in log]


SHAPES = [(64, 32, 8), (100, 7, 5), (3, 1, 1), (70, 9, 33), (128, 64, 16), (64, 8, 96), (200, 30, 2),
          (66, 6, 55), (64, 8, 56)]


@pytest.mark.parametrize("shape", SHAPES)
def test_apply_A_matches_oracle(ft, oracle_mod, shape):
    _say("apply_A", shape)
    pb = Problem(*shape, hill_amp=0.7, hill_lat=0.2)
    s = ft.Solver(pb, kmax=2)
    x = np.random.default_rng(1).uniform(-1, 1, pb.shape)
    y = s.apply_A(x).cpu().numpy()
    ref = oracle_mod.Oracle(pb).apply_A(x)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * scale)
    s.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_apply_pinv_matches_oracle(ft, oracle_mod, shape):
    _say("apply_pinv", shape)
    pb = Problem(*shape, hill_amp=0.9, hill_lon=0.3)
    s = ft.Solver(pb, kmax=2)
    r = np.random.default_rng(2).uniform(-1, 1, pb.shape)
    e = s.apply_pinv(r).cpu().numpy()
    ref = oracle_mod.Oracle(pb).apply_pinv(r)
    np.testing.assert_allclose(e, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    s.close()


def _solve_parity(ft, oracle_mod, pb, k, tol=1e-10, plan=None, rhs_seed=1, steps_tol=1):
    rhs = I.rhs(pb, rhs_seed)
    s = ft.Solver(pb, kmax=k)
    x, st = s.solve(rhs, tol=tol, k=k, plan=plan, hist_cap=100000)
    o = oracle_mod.Oracle(pb)
    xo, so, logo, ho = o.solve(rhs, tol=tol, k=k, plan=plan)
    assert st["status"] == so["status"] == ft.CONVERGED, (st, so)
    assert abs(st["steps_executed"] - so["steps_executed"]) <= steps_tol
    assert _decisions(st["log"]) == _decisions(logo)
    # the state after exactly the GPU's step count (a lower tol keeps the
    # oracle from exiting one step earlier)
    xe, se, _, he = o.solve(rhs, tol=tol * 1e-3, k=k, plan=plan, max_steps=st["steps_executed"])
    err = _rel(x.cpu().numpy(), xe)
    assert err <= 1e-10, err
    n = min(len(he), len(st["hist"]))
    np.testing.assert_allclose(st["hist"][:n], he[:n], rtol=1e-6)
    s.close()
    return x, st, so


@pytest.mark.parametrize("k", [1, 3, 4])
def test_solve_matches_oracle_c1(ft, oracle_mod, k):
    _say("solve C1 k", k)
    _solve_parity(ft, oracle_mod, I.C1, k)


def test_solve_matches_oracle_ragged(ft, oracle_mod):
    _say("solve ragged 100x7x5")
    _solve_parity(ft, oracle_mod, Problem(100, 7, 5, hill_lat=-0.3, hill_amp=0.9), 3, rhs_seed=7)


def test_solve_deterministic(ft):
    _say("determinism C1")
    rhs = I.rhs(I.C1, 3)
    s = ft.Solver(I.C1, kmax=3)
    x1, s1 = s.solve(rhs, tol=1e-10, k=3, hist_cap=100000)
    x2, s2 = s.solve(rhs, tol=1e-10, k=3, hist_cap=100000)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert np.array_equal(s1["hist"], s2["hist"])
    assert s1["steps_executed"] == s2["steps_executed"]
    s.close()


def test_graph_replay_matches_direct_launches(ft):
    """Steps replayed from a captured graph (several replays, with the
    solver's own synchronising status reads between them) give bit-identical
    results to directly launched steps, fault events included."""
    _say("graphs vs direct")
    pb = Problem(96, 40, 12, hill_amp=0.8)
    rhs = I.rhs(pb, 9)
    plan = [FaultEvent(37, "r", 62, idx=np.array([123])), FaultEvent(70, "ap", 61, idx=np.array([5, 6]))]
    out = []
    for graphs in (0, 1, 1):
        s = ft.Solver(pb, kmax=4, use_graphs=graphs, poll_steps=8)
        x, st = s.solve(rhs, tol=1e-10, k=4, plan=plan, hist_cap=10000)
        out.append((x.cpu().numpy(), st))
        s.close()
    for x, st in out[1:]:
        assert np.array_equal(x, out[0][0])
        assert np.array_equal(st["hist"], out[0][1]["hist"])
        assert _decisions(st["log"]) == _decisions(out[0][1]["log"])


def test_c1_fault_plan(ft, oracle_mod):
    """Bit 62 of one residual entry at step 5: detected at step 5, rolled
    back, and the run then replays the fault-free one exactly."""
    _say("C1 plan")
    pb = I.C1
    plan = I.single_flip_plan(pb, I.SEEDS["c1_plan"], step=5, vec="r", bit=62)
    x, st, so = _solve_parity(ft, oracle_mod, pb, 3, plan=plan)
    assert _decisions(st["log"]) == [(5, 1, 0)]
    assert st["steps_wasted"] == 2 and st["events_applied"] == 1
    s = ft.Solver(pb, kmax=3)
    xc, sc = s.solve(I.rhs(pb, 1), tol=1e-10, k=3)
    assert np.array_equal(x.cpu().numpy(), xc.cpu().numpy())
    assert st["steps_executed"] == sc["steps_executed"] + 2
    s.close()


@pytest.mark.parametrize("vec", ["x", "p"])
def test_x_p_faults_leave_residual_history(ft, vec):
    _say("x/p fault", vec)
    pb = I.C1
    rhs = I.rhs(pb, 1)
    s = ft.Solver(pb, kmax=3)
    xc, sc = s.solve(rhs, tol=1e-10, k=3, hist_cap=10000)
    at = 777
    plan = [FaultEvent(step=7, vec=vec, bit=62, idx=np.array([at]))]
    x, st = s.solve(rhs, tol=1e-10, k=3, plan=plan, hist_cap=10000)
    assert st["detections"] == 0 and st["events_applied"] == 1
    assert np.array_equal(st["hist"], sc["hist"])
    diff = np.flatnonzero(x.cpu().numpy().ravel() != xc.cpu().numpy().ravel())
    assert diff.tolist() == [at]
    s.close()


@pytest.mark.parametrize("step", [1, 4, 6, 8, 30])
def test_ap_faults_match_oracle(ft, oracle_mod, step):
    _say("Ap fault step", step)
    plan = [FaultEvent(step=step, vec="ap", bit=62, idx=np.arange(100, 4000, 37))]
    _solve_parity(ft, oracle_mod, I.C1, 3, plan=plan)


@pytest.mark.parametrize("case", range(6))
def test_assorted_faults_match_oracle(ft, oracle_mod, case):
    """Faults at cycle starts after a rollback (the copy-on-write paths),
    repeated events, ranges and per-entry bits."""
    _say("assorted faults", case)
    pb = I.C1
    n = pb.n
    plans = [
        [FaultEvent(4, "ap", 62, idx=np.array([5])), FaultEvent(5, "r", 62, idx=np.array([9]))],
        [FaultEvent(6, "ap", 62, idx=np.array([11])), FaultEvent(7, "x", 61, idx=np.array([3, 4000]))],
        [FaultEvent(6, "r", 62, idx=np.array([11])), FaultEvent(7, "p", 62, idx=np.array([12]))],
        [FaultEvent(10, "r", 52, start=100, count=n // 10)],
        [FaultEvent(3, "ap", 63, idx=np.arange(0, n, 97), bits=np.full(len(range(0, n, 97)), 62, np.uint8)),
         FaultEvent(9, "ap", 62, idx=np.array([1]))],
        [FaultEvent(20, "r", 40, idx=np.arange(0, n, 11)), FaultEvent(20, "ap", 62, idx=np.array([2]))],
    ]
    _solve_parity(ft, oracle_mod, pb, 3, plan=plans[case])


def test_stagnation_decisions_match_oracle(ft, oracle_mod):
    """Right-hand sides with <r0, A P^-1 r0> = 0 up to round-off (the first
    step cannot lower the residual): the detection recurs at the same place
    after the rollback and is accepted as stagnation.  Such a start is
    chaotic for GCR -- the oracle's own executed-step count moves over a wide
    range when the right-hand side or the coefficients are perturbed by
    1e-15 relative, a perturbation of the size of the GPU's different
    rounding (measured over 300 + 300 perturbations per case by
    tests/golden/make_goldens.py, oracle only) -- so the GPU's count must lie
    inside that measured spread; the decision pattern and the outcome must
    be the oracle's."""
    import json
    import os
    _say("stagnation")
    with open(os.path.join(os.path.dirname(__file__), "golden", "stagnation_spread.json")) as f:
        spread = json.load(f)
    pb = Problem(*spread["grid"])
    o = oracle_mod.Oracle(pb)
    n = pb.n
    m = o.dense_matrix()
    pinv = np.stack([o.apply_pinv(np.eye(n)[c]).reshape(-1) for c in range(n)], 1)
    b = m @ pinv
    w, v = np.linalg.eigh(0.5 * (b + b.T))
    s = ft.Solver(pb, kmax=3)
    for case in spread["cases"]:
        j = case["j"]
        rhs = v[:, 0] + np.sqrt(-w[0] / w[j]) * v[:, j]
        xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=3)
        assert so["steps_executed"] == case["steps_unperturbed"]
        x, st = s.solve(rhs, tol=1e-10, k=3)
        # the first step changes the norm by less than an ulp, so whether it
        # reads as "equal" depends on the summation order -- a tie inside
        # the logged band; whatever either side decides must be the
        # stagnation pattern
        for log in (st["log"], logo):
            assert _decisions(log) in ([], [(1, 0, 0), (2, 0, 1)])
        if st["log"]:
            assert st["stagnation_accepts"] == 1
            assert st["log"][0]["rr_new"] == st["log"][1]["rr_new"]
            assert abs(st["log"][0]["rr_new"] / st["log"][0]["rr_old"] - 1) <= 1e-10
        assert st["status"] == so["status"] == ft.CONVERGED
        assert case["steps_min"] <= st["steps_executed"] <= case["steps_max"], (j, st["steps_executed"], case)
        _say(f"stagnation j={j}: GPU {st['steps_executed']} steps, oracle {so['steps_executed']}, "
             f"oracle spread {case['steps_min']}..{case['steps_max']}")
    s.close()


def test_campaign_decisions_match_oracle(ft, oracle_mod):
    """A slice of the fault campaign (one event per solve: step 1..20, vector
    x / r / p / Ap, 1 entry, 1% or a 10% block, bit 0..63) on a mid-size grid:
    identical decisions, x at equal step counts within 1e-10."""
    pb = Problem(128, 64, 16)
    rhs = I.rhs(pb, 2)
    o = oracle_mod.Oracle(pb)
    s = ft.Solver(pb, kmax=4)
    plans = I.campaign_plans(pb, count=12, seed0=1000)
    for m, plan in enumerate(plans):
        _say("campaign", m, plan[0].step, plan[0].vec, plan[0].count, plan[0].bit)
        x, st = s.solve(rhs, tol=1e-10, k=4, plan=plan)
        xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=4, plan=plan)
        assert _decisions(st["log"]) == _decisions(logo), (m, st["log"], logo)
        assert st["status"] == so["status"]
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
        xe, _, _, _ = o.solve(rhs, tol=1e-13, k=4, plan=plan, max_steps=st["steps_executed"])
        if np.all(np.isfinite(xe)):
            assert _rel(x.cpu().numpy(), xe) <= 1e-10
    s.close()


def test_edge_cases(ft, oracle_mod, torch_dev):
    _say("edge cases")
    pb = Problem(16, 8, 4)
    rhs = I.rhs(pb, 5)
    s = ft.Solver(pb, kmax=16)
    o = oracle_mod.Oracle(pb)
    # exact initial guess: zero steps
    xs = np.linalg.solve(o.dense_matrix(), rhs.ravel()).reshape(pb.shape)
    x, st = s.solve(rhs, x=xs, tol=1e-10, k=3)
    assert st["status"] == ft.CONVERGED and st["steps_executed"] == 0
    assert np.array_equal(x.cpu().numpy(), xs)
    # max steps
    s.set_options(max_steps=7)
    x, st = s.solve(rhs, tol=1e-10, k=3)
    assert st["status"] == ft.MAX_STEPS and st["steps_executed"] == 7
    xo, so, _, _ = o.solve(rhs, tol=1e-10, k=3, max_steps=7)
    assert _rel(x.cpu().numpy(), xo) <= 1e-12
    s.set_options(max_steps=100000)
    # k = kmax = 16
    x, st = s.solve(rhs, tol=1e-10, k=16)
    xo, so, _, _ = o.solve(rhs, tol=1e-10, k=16)
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
    # events scheduled after convergence never fire
    x, st = s.solve(rhs, tol=1e-10, k=3, plan=[FaultEvent(10 ** 6, "r", 62, idx=np.array([0]))])
    assert st["events_applied"] == 0
    # invalid calls are errors, not crashes
    with pytest.raises(ft.FtgcrError):
        s.solve(rhs, tol=1e-10, k=17)
    with pytest.raises(ft.FtgcrError):
        s.solve(rhs, tol=-1.0, k=3)
    with pytest.raises(ft.FtgcrError):
        s.solve(rhs, tol=1e-10, k=3, plan=[FaultEvent(1, "r", 62, idx=np.array([pb.n]))])
    with pytest.raises(ft.FtgcrError):
        s.solve(rhs, tol=1e-10, k=3, plan=[FaultEvent(1, "r", 64, idx=np.array([0]))])
    s.close()


def test_ft_off_matches_plain_gcr(ft, oracle_mod):
    _say("ft off with fault")
    pb = I.C1
    rhs = I.rhs(pb, 1)
    plan = [FaultEvent(5, "r", 62, idx=np.array([100]))]
    s = ft.Solver(pb, kmax=3, ft=0, max_steps=600)
    x, st = s.solve(rhs, tol=1e-10, k=3, plan=plan)
    xo, so, _, _ = oracle_mod.Oracle(pb).solve(rhs, tol=1e-10, k=3, plan=plan, ft=False, max_steps=600)
    assert st["detections"] == 0 and so["detections"] == 0
    assert st["status"] == so["status"]
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
    s.close()


def test_batch_matches_oracle_per_member(ft, oracle_mod):
    """Several problems of different sizes and hills solved by one batched
    launch sequence: every member converges as the oracle does (steps +-1,
    the same decisions, x within 1e-10 at equal step counts)."""
    shapes = [(64, 32, 8), (96, 48, 12), (64, 32, 8), (128, 64, 16), (70, 9, 5), (96, 48, 12)]
    pbs = [Problem(*sh, hill_lon=0.4 * m, hill_lat=0.3 - 0.1 * m, hill_amp=0.2 + 0.15 * m)
           for m, sh in enumerate(shapes)]
    rhs = [I.rhs(pb, 40 + m) for m, pb in enumerate(pbs)]
    plans = [[], [FaultEvent(6, "r", 62, idx=np.array([17]))], [], [FaultEvent(9, "ap", 62, idx=np.array([3]))],
             [FaultEvent(2, "x", 50, idx=np.array([4]))], []]
    tols = [1e-10, 1e-10, 1e-9, 1e-10, 1e-10, 1e-8]
    solvers = [ft.Solver(pb, kmax=3) for pb in pbs]
    _say("batch of", len(pbs))
    xs, sts = ft.solve_batch(solvers, rhs, tols=tols, k=3, plans=plans)
    for m, pb in enumerate(pbs):
        o = oracle_mod.Oracle(pb)
        xo, so, logo, _ = o.solve(rhs[m], tol=tols[m], k=3, plan=plans[m])
        st = sts[m]
        assert st["status"] == ft.CONVERGED, (m, st)
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, m
        assert _decisions(st["log"]) == _decisions(logo), m
        xe, _, _, _ = o.solve(rhs[m], tol=tols[m] * 1e-3, k=3, plan=plans[m], max_steps=st["steps_executed"])
        assert _rel(xs[m].cpu().numpy(), xe) <= 1e-10, m
        assert st["rel_res_true"] <= 1.01 * tols[m] or plans[m]
    for s in solvers:
        s.close()


def test_batch_graph_replay_matches_direct_launches(ft):
    """Batched steps replayed from captured graphs (several chunk replays per
    solve, a re-capture whenever finished members are compacted out, and a
    second call reusing the cached graph and tables) give bit-identical
    results to directly launched batched steps, fault events included."""
    shapes = [(64, 32, 8), (96, 48, 12), (48, 24, 6), (128, 64, 16), (70, 9, 5)]
    pbs = [Problem(*sh, hill_lon=0.5 * m, hill_amp=0.3 + 0.1 * m) for m, sh in enumerate(shapes)]
    rhs = [I.rhs(pb, 90 + m) for m, pb in enumerate(pbs)]
    plans = [[], [FaultEvent(6, "r", 62, idx=np.array([17]))], [FaultEvent(40, "e", 62, idx=np.arange(0, 6912, 7))],
             [], [FaultEvent(3, "ap", 62, idx=np.array([3]))]]
    tols = [1e-10, 1e-10, 1e-8, 1e-10, 1e-9]
    out = []
    for graphs in (0, 1, 1):
        solvers = [ft.Solver(pb, kmax=4, poll_steps=8) for pb in pbs]
        solvers[0].set_options(use_graphs=graphs)
        _say("batch graphs", graphs)
        for rep in range(2 if graphs else 1):
            xs, sts = ft.solve_batch(solvers, rhs, tols=tols, k=4, plans=plans)
            out.append(([x.cpu().numpy() for x in xs], sts))
        for sv in solvers:
            sv.close()
    ref_x, ref_st = out[0]
    assert all(st["status"] == ft.CONVERGED for st in ref_st)
    for xs, sts in out[1:]:
        for m in range(len(pbs)):
            assert np.array_equal(xs[m], ref_x[m]), m
            assert sts[m]["steps_executed"] == ref_st[m]["steps_executed"], m
            assert _decisions(sts[m]["log"]) == _decisions(ref_st[m]["log"]), m


def test_batch_autotune_keeps_results(ft, oracle_mod):
    """The batch tiling autotuner picks 2, 4 or 8 levels per block for the
    combined launches, records it on the first member only, leaves every
    member's other options as they were, and a batch at the chosen tiling
    (with a fault in one member) still takes the oracle's decisions with x
    within 1e-10 at equal step counts."""
    pbs = [Problem(64, 32, 8), Problem(48, 24, 6, hill_lon=1.0), Problem(100, 7, 5), Problem(96, 48, 12)]
    rhs = [I.rhs(pb, 70 + m) for m, pb in enumerate(pbs)]
    plans = [[], [FaultEvent(5, "r", 62, idx=np.array([11]))], [], []]
    solvers = [ft.Solver(pb, kmax=3) for pb in pbs]
    before = [s.options() for s in solvers]
    _say("batch autotune")
    kc = ft.autotune_batch(solvers, rhs, k=3, steps=8)
    assert kc in (2, 4, 8)
    after = [s.options() for s in solvers]
    assert after[0]["batch_levels_per_block"] == kc
    for m, (b, a) in enumerate(zip(before, after)):
        for key in b:
            if not (m == 0 and key == "batch_levels_per_block"):
                assert a[key] == b[key], (m, key)
    xs, sts = ft.solve_batch(solvers, rhs, tols=[1e-10] * 4, k=3, plans=plans)
    for m, pb in enumerate(pbs):
        o = oracle_mod.Oracle(pb)
        xo, so, logo, _ = o.solve(rhs[m], tol=1e-10, k=3, plan=plans[m])
        assert sts[m]["status"] == ft.CONVERGED, m
        assert _decisions(sts[m]["log"]) == _decisions(logo), m
        assert abs(sts[m]["steps_executed"] - so["steps_executed"]) <= 1, m
        xe, _, _, _ = o.solve(rhs[m], tol=1e-13, k=3, plan=plans[m], max_steps=sts[m]["steps_executed"])
        assert _rel(xs[m].cpu().numpy(), xe) <= 1e-10, m
    for s in solvers:
        s.close()


def test_batch_ensemble_workload(ft, oracle_mod):
    """The 64-member ensemble (sizes drawn from 64x32x8 .. 256x128x32, hill
    centre and amplitude per member, 6 members with one bit-62 flip in r):
    every member converges to the true residual tolerance; the faulty small
    members take the oracle's decisions."""
    members = I.ensemble(64, seed=I.SEEDS["c4_table"])
    solvers = [ft.Solver(mb.problem, kmax=3) for mb in members]
    rhs = [I.rhs(mb.problem, mb.rhs_seed) for mb in members]
    _say("ensemble 64")
    xs, sts = ft.solve_batch(solvers, rhs, tols=[1e-10] * 64, k=3, plans=[mb.plan for mb in members])
    for m, mb in enumerate(members):
        assert sts[m]["status"] == ft.CONVERGED, m
        assert sts[m]["rel_res_true"] <= 2e-10, (m, sts[m]["rel_res_true"])
        if mb.plan and mb.problem.n <= 131072:
            o = oracle_mod.Oracle(mb.problem)
            _, so, logo, _ = o.solve(rhs[m], tol=1e-10, k=3, plan=mb.plan)
            assert _decisions(sts[m]["log"]) == _decisions(logo), m
            assert abs(sts[m]["steps_executed"] - so["steps_executed"]) <= 1
    assert sum(st["events_applied"] for st in sts) >= 1
    for s in solvers:
        s.close()


@pytest.mark.parametrize("shape,k", [((64, 32, 8), 3), ((128, 64, 16), 4), ((100, 7, 5), 4)])
def test_mixed_precision_reaches_true_residual(ft, oracle_mod, shape, k):
    """Mixed form: binary32 vectors inside, FP64 true residual outside.  The
    returned x meets the tolerance on the FP64 true residual (checked with
    the oracle's operator), and is as close to the oracle's FP64 solution as
    that residual allows (kappa ~ 2e3 for this shift)."""
    _say("mixed", shape, k)
    pb = Problem(*shape, hill_amp=0.6)
    rhs = I.rhs(pb, 21)
    tol = 1e-8
    s = ft.Solver(pb, "mixed", kmax=k)
    x, st = s.solve(rhs, tol=tol, k=k)
    assert st["status"] == ft.CONVERGED and st["refinements"] >= 1
    o = oracle_mod.Oracle(pb)
    xg = x.cpu().numpy()
    true = o.true_residual(xg, rhs)
    assert true <= tol * 1.001, true
    assert abs(true - st["rel_res_true"]) <= 1e-3 * tol
    xo, so, _, _ = o.solve(rhs, tol=1e-12, k=k)
    assert _rel(xg, xo) <= 2.1e3 * tol
    s.close()


def test_mixed_precision_detects_r_fault(ft):
    """A bit-30 flip (binary32 exponent MSB) of a residual entry below 1 in
    magnitude is a spike near 1e38 whose FP64 square does not overflow: the
    norm jumps and the detector fires; the solve still meets the tolerance."""
    _say("mixed fault")
    pb = I.C1
    rhs = I.rhs(pb, 1)
    s = ft.Solver(pb, "mixed", kmax=3)
    x, st = s.solve(rhs, tol=1e-8, k=3, plan=[FaultEvent(12, "r", 30, idx=np.array([200]))])
    assert st["events_applied"] == 1 and st["detections"] >= 1
    assert st["log"][0]["step"] == 12
    assert st["status"] == ft.CONVERGED and st["rel_res_true"] <= 1e-8
    s.close()


def test_autotune_keeps_results(ft, oracle_mod):
    """The tiling autotuner only changes how the stencil passes are tiled:
    after tuning, the solve still matches the oracle."""
    _say("autotune")
    pb = Problem(128, 64, 16, hill_amp=0.7)
    s = ft.Solver(pb, kmax=3)
    rhs = I.rhs(pb, 8)
    kc = s.autotune(rhs, k=3, steps=12)
    assert kc in (2, 4, 8)
    assert s.options()["levels_per_block"] == 0
    s.close()
    _solve_parity(ft, oracle_mod, pb, 3, rhs_seed=8)


@pytest.mark.parametrize("shape,kc", [((70, 9, 33), 1), ((70, 9, 33), 16), ((64, 8, 96), 2), ((64, 8, 96), 8),
                                      ((130, 5, 7), 4), ((66, 6, 55), 8), ((64, 8, 56), 4)])
def test_solve_parity_across_tilings(ft, oracle_mod, shape, kc):
    """Odd and maximal column heights (nz 33, 55 and 96: half columns of 17,
    28 and 48 levels; nz 56 fills 28-level halves exactly, on whole
    128-column blocks), ragged tiles in x and y, and every level tiling (the dots
    pass at kc levels per block, the direction pass at min(kc, 4)), with a
    fault in the run: the same decisions, x within 1e-10 at equal steps."""
    _say("tiling", shape, kc)
    pb = Problem(*shape, hill_lon=2.0, hill_amp=0.8)
    rhs = I.rhs(pb, 31)
    plan = [FaultEvent(7, "ap", 62, idx=np.arange(0, pb.n, 13))]
    s = ft.Solver(pb, kmax=4, levels_per_block=kc)
    x, st = s.solve(rhs, tol=1e-10, k=4, plan=plan)
    s.close()
    o = oracle_mod.Oracle(pb)
    xo, so, logo, _ = o.solve(rhs, tol=1e-10, k=4, plan=plan)
    assert _decisions(st["log"]) == _decisions(logo)
    assert st["status"] == so["status"] == ft.CONVERGED
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
    xe, _, _, _ = o.solve(rhs, tol=1e-13, k=4, plan=plan, max_steps=st["steps_executed"])
    assert _rel(x.cpu().numpy(), xe) <= 1e-10


@pytest.mark.parametrize("shape,kc", [((70, 9, 33), 16), ((64, 8, 96), 4), ((64, 8, 56), 8)])
def test_mixed_across_tilings(ft, oracle_mod, shape, kc):
    """The mixed form on odd and maximal column heights (binary32 column
    solve with 17- and 48-level half columns) and other tilings: the FP64
    true residual meets the tolerance (oracle's operator)."""
    _say("mixed tiling", shape, kc)
    pb = Problem(*shape, hill_amp=0.5)
    rhs = I.rhs(pb, 32)
    s = ft.Solver(pb, "mixed", kmax=4, levels_per_block=kc)
    x, st = s.solve(rhs, tol=1e-8, k=4)
    s.close()
    assert st["status"] == ft.CONVERGED
    true = oracle_mod.Oracle(pb).true_residual(x.cpu().numpy(), rhs)
    assert true <= 1.001e-8, true


@pytest.mark.parametrize("shape", [(128, 64, 16), (70, 9, 30), (64, 32, 8), (64, 8, 96)])
def test_mixed_preconditioner_matches_fp64_step_counts(ft, shape):
    """The binary32 column solve (one lane per column up to 64 levels, two
    lanes beyond) applies the same P as the FP64 one up to binary32
    rounding: the mixed form's inner step count stays within 10% of the FP64
    solve's (a wrong P would still converge, but in many more steps)."""
    _say("mixed step counts", shape)
    pb = Problem(*shape, hill_amp=0.7)
    rhs = I.rhs(pb, 33)
    s64 = ft.Solver(pb, kmax=4)
    _, st64 = s64.solve(rhs, tol=1e-8, k=4)
    s64.close()
    sm = ft.Solver(pb, "mixed", kmax=4)
    _, stm = sm.solve(rhs, tol=1e-8, k=4)
    sm.close()
    assert st64["status"] == stm["status"] == ft.CONVERGED
    assert stm["rel_res_true"] <= 1.001e-8
    assert stm["steps_executed"] <= 1.10 * st64["steps_executed"] + 8, (stm["steps_executed"], st64["steps_executed"])


def test_kernel_times_and_sampled_timing(ft):
    """profile_kernels: timing every step kernel counts one launch per
    executed step; a mask with a step stride times only the chosen kernel on
    every stride-th step; timing changes no result."""
    _say("kernel timing")
    pb = Problem(64, 32, 8, hill_amp=0.6)
    rhs = I.rhs(pb, 5)
    s = ft.Solver(pb, kmax=4)
    x0, st0 = s.solve(rhs, tol=1e-10, k=4)
    steps = st0["steps_executed"]
    s.set_options(profile_kernels=1)
    s.reset_kernel_times()
    x1, st1 = s.solve(rhs, tol=1e-10, k=4)
    kt = s.kernel_times()
    assert kt["update_thomas"][0] == steps
    assert kt["stencil_dots"][0] in (steps - 1, steps) and kt["dir_update"][0] in (steps - 1, steps)
    assert all(v[1] > 0 for v in kt.values())
    s.set_options(profile_kernels=(5 << 8) | (2 << 2))
    s.reset_kernel_times()
    x2, st2 = s.solve(rhs, tol=1e-10, k=4)
    kt2 = s.kernel_times()
    assert kt2["update_thomas"][0] == 0 and kt2["stencil_dots"][0] == 0
    assert kt2["dir_update"][0] in (steps // 5 - 1, steps // 5) and kt2["dir_update"][1] > 0
    s.close()
    for x, st in ((x1, st1), (x2, st2)):
        assert st["steps_executed"] == steps
        assert np.array_equal(x.cpu().numpy(), x0.cpu().numpy())
