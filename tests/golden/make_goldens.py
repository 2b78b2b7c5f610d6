"""Write the oracle's expected values for the full-size parity tests.

Everything stored here comes from the CPU oracle (oracle/, the plain FP64
rendering of Algorithm 1) run on the seeded inputs of
paper_2103_07210_amd/inputs.py; nothing comes from the GPU library.  The GPU
tests (tests/test_gpu_goldens.py) compare the HIP path against these files.

  python tests/golden/make_goldens.py [c2] [c3] [c5] [o160] [stag] [--jobs 7]

Targets (each writes <name>.json with the solve outcomes and decision logs,
and <name>.npz with float arrays: residual histories, the sampled entries of
x and their flat indices):

  c2    256x128x32, k = 4, tol 1e-10: the fault-free solve and the 200-plan
        single-event campaign (plan seeds 1000..1199: step U{1..20}, vector
        x / r / p / L(p), one entry, 1% of entries or a 10% contiguous block,
        bit U{0..63}).
  c3    512x256x64, k = 4, tol 1e-8, FP64, fault-free.
  c5    1024x512x96, k = 4, tol 1e-8, FP64, fault-free and with the 10%
        contiguous block of r flipped at bit 62 in step 10.
  o160  the paper's O160 with 51 levels (Section 3, Table 1), k = 5 as in
        the paper's runs, tol 1e-8, FP64, fault-free and with the same 10%
        block fault (x sampled uniformly).
  stag  the stagnating right-hand sides of the 8x4x3 test (<r, A P^-1 r> = 0
        up to round-off): the oracle's own spread of executed steps when the
        right-hand side (1e-15 relative) or the coefficients (1e-15 relative
        hill amplitude and shift) are perturbed -- the GPU's arithmetic is a
        perturbation of that size.

For every solve: status, executed / accepted / wasted steps, cycles,
detections, events applied, the decision log (step, nu, action, rr_old,
rr_new), the residual history <r, r> per executed step, and x after the
natural stopping step: sampled entries (a seeded uniform sample plus the
entries of the pole rows, the periodic seam and a stencil-tile boundary at
the bottom, middle and top levels), the largest |x| and the 2-norm over the
ordinary entries (finite, at most 1e150), and the counts of the entries a
flipped exponent bit made huge, infinite or NaN.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.oracle import OctOracle, Oracle  # noqa: E402
from paper_2103_07210_amd import inputs as I  # noqa: E402


def sample_indices(pb, n_random: int, seed: int, structured: bool = True) -> np.ndarray:
    """Flat indices of the sampled entries of x: n_random drawn uniformly
    without replacement, plus (structured) every entry of the two pole rows,
    of the longitudes 0, 1, 63, 64 and nlon-1 (periodic seam, a 64-wide
    tile boundary) at levels 0, nz/2 and nz-1."""
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(pb.n, min(n_random, pb.n), replace=False).tolist())
    if structured:
        plane = pb.nx * pb.ny
        for k in sorted({0, pb.nz // 2, pb.nz - 1}):
            for j in (0, pb.ny - 1):
                idx.update(range(k * plane + j * pb.nx, k * plane + (j + 1) * pb.nx))
            for i in sorted({0, 1, 63, 64, pb.nx - 1}):
                if i < pb.nx:
                    idx.update(k * plane + j2 * pb.nx + i for j2 in range(pb.ny))
    return np.array(sorted(idx), dtype=np.int64)


HUGE = 1e150   # entries beyond this were made by a flipped exponent bit


def x_summary(x: np.ndarray) -> dict:
    """Whole-vector figures of x: ordinary entries (finite, |x| <= HUGE) and
    the counts of the others a flipped exponent bit can leave in x (the
    recurrence never reads x, so such entries stay where the flip put them)."""
    x = x.reshape(-1)
    fin = np.isfinite(x)
    ordinary = fin & (np.abs(np.where(fin, x, 0.0)) <= HUGE)
    xo = x[ordinary]
    return {"max_abs_ordinary": float(np.max(np.abs(xo))) if xo.size else 0.0,
            "norm2_ordinary": float(np.linalg.norm(xo)),
            "n_huge": int((fin & ~ordinary).sum()),
            "n_nan": int(np.isnan(x).sum()),
            "n_inf": int(np.isinf(x).sum())}


def outcome(st: dict, log: list) -> dict:
    keys = ("status", "steps_executed", "steps_accepted", "steps_wasted", "cycles", "detections",
            "stagnation_accepts", "events_applied", "rel_res_recursive")
    out = {k: st[k] for k in keys}
    out["decisions"] = [[d["step"], d["nu"], d["action"], d["rr_old"], d["rr_new"]] for d in log]
    return out


def plan_json(plan) -> list:
    out = []
    for ev in plan:
        out.append({"step": int(ev.step), "vec": int(ev.vec), "bit": int(ev.bit), "count": int(ev.count),
                    "range": ev.idx is None, "start": int(ev.start)})
    return out


# --- 256x128x32 campaign ----------------------------------------------------

C2_TOL, C2_K = 1e-10, 4


def _c2_plan(args):
    m, idx = args
    pb = I.C2
    rhs = I.rhs(pb, I.SEEDS["c2_rhs"])
    plan = I.campaign_plans(pb, count=1, seed0=I.SEEDS["c2_plan0"] + m)[0]
    x, st, log, _ = Oracle(pb).solve(rhs, tol=C2_TOL, k=C2_K, plan=plan)
    rec = outcome(st, log)
    rec.update(x_summary(x))
    rec["plan"] = plan_json(plan)
    rec["seed"] = I.SEEDS["c2_plan0"] + m
    return m, rec, x.reshape(-1)[idx]


def make_c2(jobs: int):
    pb = I.C2
    rhs = I.rhs(pb, I.SEEDS["c2_rhs"])
    idx_clean = sample_indices(pb, 4096, 2001)
    idx_plan = sample_indices(pb, 768, 2002, structured=False)
    t0 = time.time()
    x, st, log, hist = Oracle(pb).solve(rhs, tol=C2_TOL, k=C2_K)
    clean = outcome(st, log)
    clean.update(x_summary(x))
    x_clean = x.reshape(-1)[idx_clean]
    print(f"c2 clean: {st['steps_executed']} steps, {time.time() - t0:.0f} s", flush=True)
    recs = [None] * 200
    xs = np.zeros((200, idx_plan.size))
    with mp.Pool(jobs, maxtasksperchild=8) as pool:
        for m, rec, xv in pool.imap_unordered(_c2_plan, [(m, idx_plan) for m in range(200)]):
            recs[m] = rec
            xs[m] = xv
            print(f"c2 plan {m}: {rec['steps_executed']} steps, {len(rec['decisions'])} decisions", flush=True)
    meta = {"grid": [pb.nx, pb.ny, pb.nz], "k": C2_K, "tol": C2_TOL, "rhs_seed": I.SEEDS["c2_rhs"],
            "clean": clean, "plans": recs}
    _write("c2_campaign", meta, hist_clean=hist, idx_clean=idx_clean, x_clean=x_clean,
           idx_plan=idx_plan, x_plan=xs)


# --- 512x256x64 and 1024x512x96 -------------------------------------------

BIG_TOL, BIG_K = 1e-8, 4


def _big(args):
    name, with_fault = args
    pb = I.C3 if name == "c3" else I.C5
    rhs = I.rhs(pb, I.SEEDS[f"{name}_rhs"])
    plan = I.block_plan(pb, step=10, vec="r", fraction=0.1, bit=62, seed=I.SEEDS["c5_plan"]) if with_fault else []
    t0 = time.time()
    x, st, log, hist = Oracle(pb).solve(rhs, tol=BIG_TOL, k=BIG_K, plan=plan)
    idx = sample_indices(pb, 8192, 3001 if name == "c3" else 5001)
    rec = outcome(st, log)
    rec.update(x_summary(x))
    rec["plan"] = plan_json(plan)
    rec["oracle_seconds"] = time.time() - t0
    print(f"{name} fault={with_fault}: {st['steps_executed']} steps, {time.time() - t0:.0f} s", flush=True)
    return name, with_fault, rec, hist, idx, x.reshape(-1)[idx]


def make_big(names, jobs: int):
    work = []
    for name in names:
        work.append((name, False))
        if name == "c5":
            work.append((name, True))
    with mp.Pool(min(jobs, len(work))) as pool:
        res = pool.map(_big, work)
    for name in names:
        pb = I.C3 if name == "c3" else I.C5
        meta = {"grid": [pb.nx, pb.ny, pb.nz], "k": BIG_K, "tol": BIG_TOL, "rhs_seed": I.SEEDS[f"{name}_rhs"]}
        arrays = {}
        for nm, wf, rec, hist, idx, xv in res:
            if nm != name:
                continue
            tag = "fault" if wf else "clean"
            meta[tag] = rec
            arrays[f"hist_{tag}"] = hist
            arrays["idx"] = idx
            arrays[f"x_{tag}"] = xv
        _write(f"{name}_fp64", meta, **arrays)


# --- O160 x 51 levels ---------------------------------------------------------

O160_K = 5


def _o160(with_fault):
    pb = I.O160
    rhs = I.rhs(pb, I.SEEDS["c3_rhs"])
    plan = I.block_plan(pb, step=10, vec="r", fraction=0.1, bit=62, seed=I.SEEDS["c5_plan"]) if with_fault else []
    t0 = time.time()
    x, st, log, hist = OctOracle(pb).solve(rhs, tol=BIG_TOL, k=O160_K, plan=plan)
    idx = sample_indices(pb, 16384, 16001, structured=False)
    rec = outcome(st, log)
    rec.update(x_summary(x))
    rec["plan"] = plan_json(plan)
    rec["oracle_seconds"] = time.time() - t0
    print(f"o160 fault={with_fault}: {st['steps_executed']} steps, {time.time() - t0:.0f} s", flush=True)
    return with_fault, rec, hist, idx, x.reshape(-1)[idx]


def make_o160(jobs: int):
    pb = I.O160
    with mp.Pool(min(jobs, 2)) as pool:
        res = pool.map(_o160, [False, True])
    meta = {"mesh": "octahedral", "N": pb.N, "nz": pb.nz, "k": O160_K, "tol": BIG_TOL,
            "rhs_seed": I.SEEDS["c3_rhs"]}
    arrays = {}
    for wf, rec, hist, idx, xv in res:
        tag = "fault" if wf else "clean"
        meta[tag] = rec
        arrays[f"hist_{tag}"] = hist
        arrays["idx"] = idx
        arrays[f"x_{tag}"] = xv
    _write("o160_fp64", meta, **arrays)


# --- stagnation spread -------------------------------------------------------

STAG_TRIALS = 300


def stagnation_rhs(o: Oracle) -> list:
    """Right-hand sides with <r0, A P^-1 r0> = 0 up to round-off: a
    combination of the eigenvectors of the symmetric part of A P^-1 for its
    lowest (negative) and j-th eigenvalues, j = 1, 2, 3."""
    n = o.n
    m = o.dense_matrix()
    pinv = np.stack([o.apply_pinv(np.eye(n)[c]).reshape(-1) for c in range(n)], 1)
    b = m @ pinv
    w, v = np.linalg.eigh(0.5 * (b + b.T))
    return [v[:, 0] + np.sqrt(-w[0] / w[j]) * v[:, j] for j in (1, 2, 3)]


def make_stag():
    pb = I.Problem(8, 4, 3)
    o = Oracle(pb)
    rng = np.random.default_rng(7001)
    out = {"grid": [pb.nx, pb.ny, pb.nz], "k": 3, "tol": 1e-10, "trials": STAG_TRIALS, "cases": []}
    for j, rhs in enumerate(stagnation_rhs(o), start=1):
        _, so, logo, _ = o.solve(rhs, tol=1e-10, k=3)
        by_rhs, by_coef, statuses = [], [], {}
        # the spread is over the perturbed runs that converge (an exact tie
        # can instead end in a breakdown, <L p, L p> = 0); the outcomes are
        # counted
        for _ in range(STAG_TRIALS):
            pert = rhs * (1.0 + 1e-15 * rng.uniform(-1.0, 1.0, rhs.size))
            _, s2, _, _ = o.solve(pert, tol=1e-10, k=3)
            statuses[str(s2["status"])] = statuses.get(str(s2["status"]), 0) + 1
            if s2["status"] == 0:
                by_rhs.append(int(s2["steps_executed"]))
        for _ in range(STAG_TRIALS):
            pb2 = dataclasses.replace(pb, hill_amp=pb.hill_amp * (1.0 + 1e-15 * rng.uniform(-1.0, 1.0)),
                                      helmholtz=pb.helmholtz * (1.0 + 1e-15 * rng.uniform(-1.0, 1.0)))
            _, s2, _, _ = Oracle(pb2).solve(rhs, tol=1e-10, k=3)
            statuses[str(s2["status"])] = statuses.get(str(s2["status"]), 0) + 1
            if s2["status"] == 0:
                by_coef.append(int(s2["steps_executed"]))
        allc = by_rhs + by_coef
        out["cases"].append({"j": j, "steps_unperturbed": int(so["steps_executed"]),
                             "decisions_unperturbed": [[d["step"], d["nu"], d["action"]] for d in logo],
                             "status_unperturbed": int(so["status"]),
                             "steps_min": int(min(allc)), "steps_max": int(max(allc)),
                             "outcomes": statuses,
                             "rhs_perturbed": {"min": int(min(by_rhs)), "max": int(max(by_rhs)),
                                               "median": float(np.median(by_rhs))},
                             "coef_perturbed": {"min": int(min(by_coef)), "max": int(max(by_coef)),
                                                "median": float(np.median(by_coef))}})
        print(f"stag j={j}: unperturbed {so['steps_executed']}, spread {min(allc)}..{max(allc)}", flush=True)
    path = os.path.join(HERE, "stagnation_spread.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


def _write(name: str, meta: dict, **arrays):
    meta = dict(meta)
    meta["generator"] = "tests/golden/make_goldens.py (CPU oracle only)"
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    np.savez(os.path.join(HERE, name + ".npz"), **arrays)
    print("wrote", name, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("targets", nargs="*", default=["stag", "c2", "c3", "c5", "o160"])
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    if "stag" in args.targets:
        make_stag()
    big = [t for t in ("c3", "c5") if t in args.targets]
    if big:
        make_big(big, args.jobs)
    if "o160" in args.targets:
        make_o160(args.jobs)
    if "c2" in args.targets:
        make_c2(args.jobs)


if __name__ == "__main__":
    main()
