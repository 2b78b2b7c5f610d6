"""Fault campaigns on the GPU solver: per-run outcome records and the
summaries the paper reports (Section 3, Tables 2-3).

  python -m paper_2103_07210_amd.campaign [--count 200] [--grid 256,128,32] [--k 4]

runs the seeded campaign (one event per solve: step U{1..20}, vector
x / r / p / A p, one entry, 1% of entries or a 10% contiguous block, bit
U{0..63}) with fault tolerance on and off, and prints a JSON summary:
detection rate, extra executed steps and final error against the fault-free
solve, and the return on fault tolerance.

RoFT (Section 3, the equation after Fig. 1) = (GCR - FT-GCR) / baseline,
with GCR and FT-GCR the mean iteration counts of unprotected and protected
runs and baseline the fault-free count.
"""
from __future__ import annotations

import argparse
import json
from typing import Dict, List, Sequence

import numpy as np


def roft(mean_unprotected: float, mean_protected: float, baseline: float) -> float:
    """Return on fault tolerance in percent."""
    return 100.0 * (mean_unprotected - mean_protected) / baseline


def summarize(records: Sequence[Dict], clean_steps: int) -> Dict:
    """records: one dict per run with events_applied, detections, steps (FT
    on), steps_off (FT off, optional), err (FT on, relative to the fault-free
    solution), err_off."""
    applied = [r for r in records if r["events_applied"] > 0]
    out = {"runs": len(records), "runs_with_fault": len(applied), "baseline_steps": clean_steps}
    if not applied:
        return out
    det = [r["detections"] > 0 for r in applied]
    out["detection_rate"] = float(np.mean(det))
    out["extra_steps_mean"] = float(np.mean([r["steps"] - clean_steps for r in applied]))
    out["extra_steps_max"] = int(max(r["steps"] - clean_steps for r in applied))
    out["final_error_median"] = float(np.median([r["err"] for r in applied]))
    out["final_error_max"] = float(np.max([r["err"] for r in applied]))
    out["bitwise_equal_to_fault_free"] = int(sum(r["err"] == 0.0 for r in applied))
    if all("steps_off" in r for r in applied):
        on = float(np.mean([r["steps"] for r in applied]))
        off = float(np.mean([r["steps_off"] for r in applied]))
        out["mean_steps_ft"] = on
        out["mean_steps_noft"] = off
        out["roft_percent"] = roft(off, on, clean_steps)
        out["final_error_noft_median"] = float(np.median([r["err_off"] for r in applied]))
    by_vec: Dict[str, List[bool]] = {}
    for r, d in zip(applied, det):
        by_vec.setdefault(r["vec"], []).append(d)
    out["detection_rate_by_vector"] = {v: float(np.mean(ds)) for v, ds in by_vec.items()}
    return out


def run(problem, plans, k: int = 4, tol: float = 1e-10, with_unprotected: bool = True, rhs_seed: int = 2):
    import torch
    from . import ftgcr
    from . import inputs as I
    rhs = torch.from_numpy(I.rhs(problem, rhs_seed)).cuda()
    on = ftgcr.Solver(problem, "fp64", kmax=k)
    off = ftgcr.Solver(problem, "fp64", kmax=k, ft=0) if with_unprotected else None
    x_clean, st_clean = on.solve(rhs, tol=tol, k=k)
    x_clean = x_clean.clone()
    nrm = float(torch.linalg.norm(x_clean))
    names = {0: "x", 1: "r", 2: "p", 3: "ap"}
    records = []
    for m, plan in enumerate(plans):
        x, st = on.solve(rhs, tol=tol, k=k, plan=plan)
        rec = {"run": m, "vec": names[plan[0].vec], "count": int(plan[0].count), "bit": int(plan[0].bit),
               "step": int(plan[0].step), "events_applied": st["events_applied"], "detections": st["detections"],
               "steps": st["steps_executed"], "status": st["status"]}
        d = torch.nan_to_num(x - x_clean, nan=np.inf, posinf=np.inf, neginf=np.inf)
        rec["err"] = float(torch.linalg.norm(d)) / nrm
        if off is not None:
            xo, so = off.solve(rhs, tol=tol, k=k, plan=plan)
            d = torch.nan_to_num(xo - x_clean, nan=np.inf, posinf=np.inf, neginf=np.inf)
            rec["steps_off"] = so["steps_executed"]
            rec["err_off"] = float(torch.linalg.norm(d)) / nrm
        records.append(rec)
    return records, summarize(records, st_clean["steps_executed"])


def main():
    from . import inputs as I
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--grid", default="256,128,32")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-10)
    args = ap.parse_args()
    pb = I.Problem(*[int(v) for v in args.grid.split(",")])
    plans = I.campaign_plans(pb, count=args.count, seed0=I.SEEDS["c2_plan0"])
    import torch
    torch.cuda.set_device(0)
    records, summary = run(pb, plans, k=args.k, tol=args.tol)
    summary["grid"] = [pb.nx, pb.ny, pb.nz]
    summary["k"] = args.k
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
