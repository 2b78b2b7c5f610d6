"""The oracle's threaded mode splits only the operator and preconditioner
applications, by planes or columns with disjoint outputs: every result --
the face weights, A x, P^-1 r, the solvers' iterates, step counts, decisions and residual
histories, on both meshes -- is bitwise the serial one."""
import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I
from paper_2103_07210_amd.inputs import FaultEvent, OctProblem, Problem


@pytest.fixture()
def threaded(oracle_mod):
    before = oracle_mod.threads()
    yield oracle_mod
    oracle_mod.set_threads(before)


def _run_latlon(om, pb, rhs):
    o = om.Oracle(pb)
    plan = [FaultEvent(4, "r", 62, idx=np.array([5, pb.n - 1])), FaultEvent(9, "e", 40, start=0, count=pb.n // 5)]
    out = [o.apply_A(rhs), o.apply_pinv(rhs), *o.face_weights()]
    for method in ("gcr", "gmres"):
        x, st, log, h = o.solve(rhs, tol=1e-9, k=4, plan=plan, method=method, max_steps=300)
        out += [x, h, np.array([st["steps_executed"], st["detections"]]),
                np.array([(d["step"], d["nu"], d["action"]) for d in log]).reshape(-1)]
    return out


def test_threads_give_bitwise_serial_results(threaded):
    om = threaded
    pb = Problem(64, 32, 40, hill_amp=0.7)   # 81920 cells: above the split threshold
    rhs = I.rhs(pb, 9).reshape(-1)
    om.set_threads(1)
    ref = _run_latlon(om, pb, rhs)
    opb = OctProblem(40, 16, hill_amp=0.6)    # 7840 points per level x 16: split
    orhs = np.random.default_rng(3).uniform(-1, 1, opb.n)
    oo = om.OctOracle(opb)
    oref = [oo.apply_A(orhs), oo.apply_pinv(orhs), oo.solve(orhs, tol=1e-8, k=3, max_steps=80)[0]]
    for t in (2, 5):
        om.set_threads(t)
        assert om.threads() == t
        for a, b in zip(_run_latlon(om, pb, rhs), ref):
            assert a.tobytes() == b.tobytes()
        got = [oo.apply_A(orhs), oo.apply_pinv(orhs), oo.solve(orhs, tol=1e-8, k=3, max_steps=80)[0]]
        for a, b in zip(got, oref):
            assert a.tobytes() == b.tobytes()
    with pytest.raises(ValueError):
        om.set_threads(0)
