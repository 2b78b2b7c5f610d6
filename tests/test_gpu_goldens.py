"""GPU parity at the full sizes of the workload configurations, against the
oracle's expected values stored under tests/golden/ (written by
tests/golden/make_goldens.py, which runs only the CPU oracle).

Bars (Algorithm 1; readings of the comparison points in the design notes):
  * identical decision lists (step, nu, action) on the same seeded plans;
  * natural executed-step counts within +-1;
  * x compared at equal executed-step counts (the GPU solve stopped at the
    oracle's natural count): every sampled entry within 1e-10 of the largest
    ordinary |x| (element-wise), entries made huge / infinite / NaN by a
    flipped bit of x in the same class (huge ones within 1e-10 relative),
    and the whole-vector 2-norm and largest |x| within 1e-10 relative;
  * residual histories <r, r> per executed step within 1e-6 relative (they
    fall by 16 orders of magnitude; the bar is on the decisions and x).
The mixed form (binary32 vectors) is checked with the oracle's operator on
the FP64 true residual and against the FP64 oracle solution, with the error
printed.
"""
import json
import os

import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
REL = 1e-10
HUGE = 1e150


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        meta = json.load(f)
    arr = np.load(os.path.join(GOLDEN, name + ".npz"))
    return meta, arr


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


def _gold_decisions(rec):
    return [tuple(d[:3]) for d in rec["decisions"]]


def _summary(x):
    x = x.reshape(-1)
    fin = np.isfinite(x)
    ordinary = fin & (np.abs(np.where(fin, x, 0.0)) <= HUGE)
    xo = x[ordinary]
    return {"max_abs_ordinary": float(np.max(np.abs(xo))) if xo.size else 0.0,
            "norm2_ordinary": float(np.linalg.norm(xo)),
            "n_huge": int((fin & ~ordinary).sum()), "n_nan": int(np.isnan(x).sum()),
            "n_inf": int(np.isinf(x).sum())}


def check_x(xg, idx, xo, rec, rel=REL):
    """x of the GPU (whole vector, host) against the oracle's sampled
    entries and whole-vector figures; returns the element-wise error
    relative to the largest ordinary |x|."""
    xg = np.asarray(xg, dtype=np.float64).reshape(-1)
    xs = xg[idx]
    assert np.array_equal(np.isnan(xs), np.isnan(xo)), "NaN entries differ"
    inf = np.isinf(xo)
    assert np.array_equal(np.isinf(xs), inf) and np.array_equal(xs[inf], xo[inf]), "infinite entries differ"
    fin = np.isfinite(xo)
    huge = fin & (np.abs(np.where(fin, xo, 0.0)) > HUGE)
    if huge.any():
        assert np.max(np.abs(xs[huge] / xo[huge] - 1.0)) <= rel, "huge entries differ"
    ordinary = fin & ~huge
    scale = rec["max_abs_ordinary"]
    err = float(np.max(np.abs(xs[ordinary] - xo[ordinary]))) / scale if ordinary.any() else 0.0
    assert err <= rel, f"element-wise error {err:.3e} of max |x|"
    g = _summary(xg)
    for key in ("n_huge", "n_nan", "n_inf"):
        assert g[key] == rec[key], (key, g[key], rec[key])
    assert abs(g["norm2_ordinary"] - rec["norm2_ordinary"]) <= rel * rec["norm2_ordinary"]
    assert abs(g["max_abs_ordinary"] - rec["max_abs_ordinary"]) <= rel * rec["max_abs_ordinary"]
    return err


def _solve_and_compare(ft, solver, rhs, tol, k, plan, rec, idx, xo, hist=None):
    """Natural solve (decisions, status, steps +-1, history), then x at the
    oracle's natural step count."""
    x, st = solver.solve(rhs, tol=tol, k=k, plan=plan, hist_cap=100000 if hist is not None else 0)
    assert _decisions(st["log"]) == _gold_decisions(rec), (st["log"], rec["decisions"])
    assert st["status"] == rec["status"], (st["status"], rec["status"])
    assert abs(st["steps_executed"] - rec["steps_executed"]) <= 1, (st["steps_executed"], rec["steps_executed"])
    assert st["events_applied"] == rec["events_applied"]
    if hist is not None:
        m = min(len(hist), len(st["hist"]))
        np.testing.assert_allclose(st["hist"][:m], hist[:m], rtol=1e-6)
    n_o = rec["steps_executed"]
    if st["steps_executed"] != n_o:
        opts = solver.options()
        solver.set_options(max_steps=n_o)
        x, st2 = solver.solve(rhs, tol=tol * 1e-3, k=k, plan=plan)
        solver.set_options(max_steps=opts["max_steps"])
        assert st2["steps_executed"] == n_o
    return check_x(x.cpu().numpy(), idx, xo, rec), st


# --- 256x128x32 --------------------------------------------------------------

def test_c2_clean_matches_golden(ft):
    meta, arr = _load("c2_campaign")
    pb = I.C2
    rhs = I.rhs(pb, meta["rhs_seed"])
    s = ft.Solver(pb, kmax=meta["k"])
    _say("256x128x32 clean")
    err, st = _solve_and_compare(ft, s, rhs, meta["tol"], meta["k"], None, meta["clean"], arr["idx_clean"],
                                 arr["x_clean"], hist=arr["hist_clean"])
    s.close()
    _say(f"steps {st['steps_executed']} (oracle {meta['clean']['steps_executed']}), x error {err:.2e}")


def test_c2_campaign_200_plans_match_golden(ft):
    """The 200-plan single-event campaign: every plan's decisions, outcome
    and x at equal step counts."""
    meta, arr = _load("c2_campaign")
    pb = I.C2
    rhs = I.rhs(pb, meta["rhs_seed"])
    s = ft.Solver(pb, kmax=meta["k"])
    idx = arr["idx_plan"]
    worst = 0.0
    detected = 0
    for m, rec in enumerate(meta["plans"]):
        plan = I.campaign_plans(pb, count=1, seed0=rec["seed"])[0]
        ev = plan[0]
        _say("campaign", m, "step", ev.step, "vec", ev.vec, "count", ev.count, "bit", ev.bit)
        err, st = _solve_and_compare(ft, s, rhs, meta["tol"], meta["k"], plan, rec, idx, arr["x_plan"][m])
        worst = max(worst, err)
        detected += st["detections"] > 0
    s.close()
    _say(f"200 plans: decisions identical, {detected} with detections, worst x error {worst:.2e}")


# --- 512x256x64 and 1024x512x96, FP64 -----------------------------------------

PROBLEMS = {"c3": I.C3, "c5": I.C5, "o160": I.O160}


@pytest.mark.parametrize("name,tag", [("c3", "clean"), ("c5", "clean"), ("c5", "fault"), ("o160", "clean"),
                                      ("o160", "fault")])
def test_fp64_full_solve_matches_golden(ft, name, tag):
    """Whole FP64 solves to 1e-8 in the benchmark's launch configuration
    (autotuned tiling; k = 4 on the lat-lon grids, k = 5 on the paper's
    O160 x 51 levels): natural step count, decisions (the 10% block of r
    flipped at bit 62 in step 10 for 1024x512x96 and O160), residual history
    and x at equal step counts."""
    meta, arr = _load(f"{name}_fp64")
    pb = PROBLEMS[name]
    rec = meta[tag]
    rhs = I.rhs(pb, meta["rhs_seed"])
    plan = I.block_plan(pb, step=10, vec="r", fraction=0.1, bit=62, seed=I.SEEDS["c5_plan"]) if tag == "fault" else None
    s = ft.Solver(pb, kmax=meta["k"])
    _say(f"{name} fp64 {tag}: autotune")
    s.autotune(rhs, k=meta["k"], steps=12)
    _say(f"{name} fp64 {tag}: solve")
    err, st = _solve_and_compare(ft, s, rhs, meta["tol"], meta["k"], plan, rec, arr["idx"], arr[f"x_{tag}"],
                                 hist=arr[f"hist_{tag}"])
    s.close()
    _say(f"{name} {tag}: steps {st['steps_executed']} (oracle {rec['steps_executed']}), x error {err:.2e}")


# --- mixed form against the FP64 oracle ------------------------------------

@pytest.mark.parametrize("name,fault", [("c3", False), ("c5", False), ("c5", True), ("o160", False)])
def test_mixed_full_solve_against_fp64_golden(ft, oracle_mod, name, fault):
    """The mixed form (binary32 vectors, FP64 inner products, detector and
    refinement) on the full-size problems, with the 10% block of r flipped
    at binary32 bit 30 (the exponent's most significant bit) in step 10 for
    the faulty case: the FP64 true residual computed with the oracle's
    operator meets 1e-8, and x agrees with the FP64 oracle solution within
    what that residual allows (condition number of the Jacobi-scaled
    operator <= (2 + sigma) / sigma ~ 2e3: within 2.1e3 * tol of max |x|)."""
    meta, arr = _load(f"{name}_fp64")
    pb = PROBLEMS[name]
    tol = meta["tol"]
    rhs = I.rhs(pb, meta["rhs_seed"])
    plan = I.block_plan(pb, step=10, vec="r", fraction=0.1, bit=30, seed=I.SEEDS["c5_plan"]) if fault else None
    s = ft.Solver(pb, "mixed", kmax=meta["k"])
    _say(f"{name} mixed fault={fault}: autotune")
    s.autotune(rhs, k=meta["k"], steps=12)
    _say(f"{name} mixed fault={fault}: solve")
    x, st = s.solve(rhs, tol=tol, k=meta["k"], plan=plan)
    s.close()
    assert st["status"] == ft.CONVERGED and st["refinements"] >= 1
    if fault:
        assert st["events_applied"] == 1 and st["detections"] >= 1 and st["log"][0]["step"] == 10
    xg = x.cpu().numpy()
    _say(f"{name} mixed: oracle true residual")
    orc = oracle_mod.OctOracle(pb) if name == "o160" else oracle_mod.Oracle(pb)
    true = orc.true_residual(xg.reshape(-1) if name == "o160" else xg, rhs)
    assert true <= tol * 1.001, true
    assert abs(true - st["rel_res_true"]) <= 1e-3 * tol
    rec = meta["clean"]
    xs = xg.reshape(-1)[arr["idx"]]
    err = float(np.max(np.abs(xs - arr["x_clean"]))) / rec["max_abs_ordinary"]
    g = _summary(xg)
    nerr = abs(g["norm2_ordinary"] - rec["norm2_ordinary"]) / rec["norm2_ordinary"]
    assert err <= 2.1e3 * tol and nerr <= 2.1e3 * tol, (err, nerr)
    _say(f"{name} mixed fault={fault}: {st['steps_executed']} inner steps, {st['refinements']} rounds, "
         f"true residual {true:.3e}, x vs FP64 oracle: max-entry {err:.2e}, norm {nerr:.2e}")
