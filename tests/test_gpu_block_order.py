"""GPU parity under every block order of the stencil-grid passes (which
workgroup takes which column tile and chunk of levels: tiles in a row, a
tile's level chunks in a row, or the latter spread over the GPU's dies in
contiguous ranges), through the C ABI, against the oracle.

An order is a permutation of the blocks: the operator and the
preconditioner are unchanged, and only the order of the block partial sums
of the inner products moves, so every order must give what the default
gives: A element by element, the same fault decisions, step counts within
+-1 and x within 1e-10 at equal step counts, on ragged tiles and level
chunks of both meshes.
"""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, OctProblem, Problem

pytestmark = pytest.mark.gpu

ORDERS = (1, 2, 3)   # FTGCR_ORDER_X, _Z, _XCD
PAIRS = [(1, 1), (2, 2), (3, 3), (1, 3), (3, 2), (2, 1)]


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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ragged in every direction: 130 = 2 * 64 + 2 longitudes, 9 = 2 * 4 + 1
# latitudes, 21 levels in chunks of 4 (the last one of 1 level); O16 has
# 1600 points per level (6.25 blocks of 256) and 7 levels in chunks of 2
LATLON = Problem(130, 9, 21, hill_lon=2.0, hill_amp=0.8)
OCT = OctProblem(16, 7, hill_amp=0.7)


def _oracle(oracle_mod, pb):
    return oracle_mod.OctOracle(pb) if isinstance(pb, OctProblem) else oracle_mod.Oracle(pb)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("mesh", ["latlon", "octahedral"])
def test_apply_A_every_order(ft, oracle_mod, mesh, order):
    pb = LATLON if mesh == "latlon" else OCT
    kc = 4 if mesh == "latlon" else 2
    _say("apply_A", mesh, "order", order, "levels per block", kc)
    s = ft.Solver(pb, kmax=2, levels_per_block=kc, order_stencil=order, order_dir=order)
    x = np.random.default_rng(5).uniform(-1, 1, pb.n)
    if mesh == "latlon":
        x = x.reshape(pb.shape)
    y = s.apply_A(x).cpu().numpy().ravel()
    s.close()
    ref = _oracle(oracle_mod, pb).apply_A(x).ravel()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def _parity(ft, oracle_mod, pb, k, kc, pair, plan, rhs_seed):
    rhs = I.rhs(pb, rhs_seed)
    s = ft.Solver(pb, kmax=k, levels_per_block=kc, order_stencil=pair[0], order_dir=pair[1])
    x, st = s.solve(rhs, tol=1e-10, k=k, plan=plan)
    s.close()
    o = _oracle(oracle_mod, pb)
    _, so, logo, _ = o.solve(rhs, tol=1e-10, k=k, plan=plan)
    assert _decisions(st["log"]) == _decisions(logo)
    assert st["status"] == so["status"] == ft.CONVERGED
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, (st["steps_executed"], so["steps_executed"])
    xe, _, _, _ = o.solve(rhs, tol=1e-13, k=k, plan=plan, max_steps=st["steps_executed"])
    err = _rel(x.cpu().numpy(), xe)
    assert err <= 1e-10, err
    _say(f"steps {st['steps_executed']} (oracle {so['steps_executed']}), x error {err:.1e}")


@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: f"dots{p[0]}-dir{p[1]}")
def test_solve_parity_every_order_pair_latlon(ft, oracle_mod, pair):
    _say("lat-lon solve, orders", pair)
    plan = [FaultEvent(7, "ap", 62, idx=np.arange(0, LATLON.n, 13))]
    _parity(ft, oracle_mod, LATLON, 4, 4, pair, plan, 31)


@pytest.mark.parametrize("pair", [(1, 1), (2, 2), (3, 3), (2, 3)], ids=lambda p: f"dots{p[0]}-dir{p[1]}")
def test_solve_parity_every_order_pair_octahedral(ft, oracle_mod, pair):
    _say("octahedral solve, orders", pair)
    plan = [FaultEvent(5, "r", 62, idx=np.array([1234]))]
    _parity(ft, oracle_mod, OCT, 4, 2, pair, plan, 9)


def test_mixed_every_order(ft, oracle_mod):
    """The binary32 passes under the two cached orders: the FP64 true
    residual (oracle's operator) meets the tolerance."""
    pb = Problem(70, 9, 33, hill_amp=0.5)
    rhs = I.rhs(pb, 32)
    for pair in [(3, 2), (2, 3)]:
        _say("mixed, orders", pair)
        s = ft.Solver(pb, "mixed", kmax=4, levels_per_block=8, order_stencil=pair[0], order_dir=pair[1])
        x, st = s.solve(rhs, tol=1e-8, k=4)
        s.close()
        assert st["status"] == ft.CONVERGED
        true = oracle_mod.Oracle(pb).true_residual(x.cpu().numpy(), rhs)
        assert true <= 1.001e-8, true


def test_batch_members_with_orders(ft, oracle_mod):
    """Batched members carry their handles' block orders."""
    pbs = [Problem(96, 48, 12, hill_amp=0.4), Problem(70, 9, 5, hill_lat=0.2, hill_amp=0.6)]
    rhs = [I.rhs(pb, 50 + m) for m, pb in enumerate(pbs)]
    plans = [[FaultEvent(6, "r", 62, idx=np.array([17]))], []]
    solvers = [ft.Solver(pbs[0], kmax=3, order_stencil=3, order_dir=2),
               ft.Solver(pbs[1], kmax=3, order_stencil=2, order_dir=3)]
    _say("batch with orders")
    xs, sts = ft.solve_batch(solvers, rhs, tols=[1e-10, 1e-10], k=3, plans=plans)
    for s in solvers:
        s.close()
    for m, pb in enumerate(pbs):
        o = oracle_mod.Oracle(pb)
        _, so, logo, _ = o.solve(rhs[m], tol=1e-10, k=3, plan=plans[m])
        st = sts[m]
        assert st["status"] == ft.CONVERGED, (m, st)
        assert abs(st["steps_executed"] - so["steps_executed"]) <= 1, m
        assert _decisions(st["log"]) == _decisions(logo), m
        xe, _, _, _ = o.solve(rhs[m], tol=1e-13, k=3, plan=plans[m], max_steps=st["steps_executed"])
        assert _rel(xs[m].cpu().numpy(), xe) <= 1e-10, m


@pytest.mark.parametrize("mesh", ["latlon", "octahedral"])
def test_autotune_orders_keep_results(ft, oracle_mod, mesh):
    """The autotuner's search over levels per block and block orders leaves
    the options on auto and the solve at parity with the oracle."""
    pb = Problem(128, 40, 12, hill_amp=0.6) if mesh == "latlon" else OctProblem(24, 9, hill_amp=0.5)
    rhs = I.rhs(pb, 12)
    s = ft.Solver(pb, kmax=3)
    _say("autotune", mesh)
    kc = s.autotune(rhs, k=3, steps=8)
    assert kc in (2, 4, 8)
    o = s.options()
    assert o["levels_per_block"] == 0 and o["order_stencil"] == 0 and o["order_dir"] == 0
    t = s.tiling()
    _say("tuned", t)
    assert t["levels_per_block"] == kc and t["order_stencil"] in ORDERS and t["order_dir"] in ORDERS
    x, st = s.solve(rhs, tol=1e-10, k=3)
    s.close()
    orc = _oracle(oracle_mod, pb)
    _, so, logo, _ = orc.solve(rhs, tol=1e-10, k=3)
    assert st["status"] == so["status"] == ft.CONVERGED
    assert abs(st["steps_executed"] - so["steps_executed"]) <= 1
    xe, _, _, _ = orc.solve(rhs, tol=1e-13, k=3, max_steps=st["steps_executed"])
    assert _rel(x.cpu().numpy(), xe) <= 1e-10


def test_invalid_order_rejected(ft):
    s = ft.Solver(Problem(64, 8, 4), kmax=2)
    with pytest.raises(ft.FtgcrError):
        s.set_options(order_stencil=4)
    with pytest.raises(ft.FtgcrError):
        s.set_options(order_dir=-1)
    s.close()


def test_tiling_reports_defaults_and_options(ft):
    s = ft.Solver(LATLON, kmax=2, levels_per_block=4)
    assert s.tiling() == {"levels_per_block": 4, "levels_per_block_dir": 4, "order_stencil": 1, "order_dir": 1}
    s.set_options(levels_per_block=8, order_stencil=3, order_dir=2)
    assert s.tiling() == {"levels_per_block": 8, "levels_per_block_dir": 4, "order_stencil": 3, "order_dir": 2}
    s.close()
    s = ft.Solver(OCT, kmax=2, levels_per_block=2)
    assert s.tiling() == {"levels_per_block": 2, "levels_per_block_dir": 2, "order_stencil": 3, "order_dir": 3}
    s.close()
