"""Fault campaigns on the GPU solver: per-run outcome records and the
summaries the paper reports (Section 3, Tables 2-3).

  python -m paper_2103_07210_amd.campaign [--count 200] [--grid 256,128,32 | O40x51] [--k 4]
  python -m paper_2103_07210_amd.campaign --model paper [--prob 0.02]
         [--loss 4e-6,4e-4,2e-3,0.01,0.05,0.2] [--procs 36] [--count 100] [--k 5]
         [--bits uniform|finite]

The default model runs the seeded single-event campaign (one event per
solve: step U{1..20}, vector x / r / p / A p, one entry, 1% of entries or a
10% contiguous block, bit U{0..63}) with fault tolerance on and off.  The
paper model is the paper's own (Section 3): after the preconditioner of
every step a fault event with probability `prob` (at most 10 per run) flips
one random bit in each of a fraction `loss` of the entries of e = P^-1(r),
inside one randomly chosen process' share of the grid.  Both print a JSON
summary: detection rate, extra executed steps and final error against the
fault-free solve, and the return on fault tolerance.

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


def run(problem, plans, k: int = 4, tol: float = 1e-10, with_unprotected: bool = True, rhs_seed: int = 2,
        precision: str = "fp64", cap_factor: float = 0.0):
    """One protected (and optionally one unprotected) solve per plan.  With
    cap_factor > 0 every faulty solve stops after cap_factor times the
    fault-free step count (an unprotected run that took an Inf or NaN never
    converges); such runs count at the cap and are reported."""
    import torch
    from . import ftgcr
    from . import inputs as I
    rhs = torch.from_numpy(I.rhs(problem, rhs_seed)).cuda()
    on = ftgcr.Solver(problem, precision, kmax=k)
    off = ftgcr.Solver(problem, precision, kmax=k, ft=0) if with_unprotected else None
    x_clean, st_clean = on.solve(rhs, tol=tol, k=k)
    if cap_factor > 0:
        cap = int(cap_factor * max(st_clean["steps_executed"], 1))
        on.set_options(max_steps=cap)
        if off is not None:
            off.set_options(max_steps=cap)
    x_clean = x_clean.clone()
    nrm = float(torch.linalg.norm(x_clean))
    names = {0: "x", 1: "r", 2: "p", 3: "ap", 4: "e"}
    records = []
    for m, plan in enumerate(plans):
        x, st = on.solve(rhs, tol=tol, k=k, plan=plan)
        first = plan[0] if plan else None
        rec = {"run": m, "vec": names[first.vec] if first else "none",
               "count": int(first.count) if first else 0, "bit": int(first.bit) if first else -1,
               "step": int(first.step) if first else 0, "events_planned": len(plan),
               "events_applied": st["events_applied"], "detections": st["detections"],
               "steps": st["steps_executed"], "cycles": st["cycles"], "status": st["status"],
               "converged": st["status"] == ftgcr.CONVERGED}
        d = torch.nan_to_num(x - x_clean, nan=np.inf, posinf=np.inf, neginf=np.inf)
        rec["err"] = float(torch.linalg.norm(d)) / nrm
        if off is not None:
            xo, so = off.solve(rhs, tol=tol, k=k, plan=plan)
            d = torch.nan_to_num(xo - x_clean, nan=np.inf, posinf=np.inf, neginf=np.inf)
            rec["steps_off"] = so["steps_executed"]
            rec["converged_off"] = so["status"] == ftgcr.CONVERGED
            rec["cycles_off"] = so["cycles"]
            rec["events_applied_off"] = so["events_applied"]
            rec["err_off"] = float(torch.linalg.norm(d)) / nrm
        records.append(rec)
    on.close()
    if off is not None:
        off.close()
    return records, summarize(records, st_clean["steps_executed"]), st_clean


def summarize_paper(records: Sequence[Dict], clean_steps: int, clean_cycles: int) -> Dict:
    """The columns of the paper's Tables 2-3 over runs that had at least one
    fault applied (the paper disregards fault-free runs): faults per run,
    faults detected per run, detection rate (the per-run mean of detected /
    applied, in percent), mean iterations with and without fault tolerance
    and RoFT, in executed steps and in outer cycles (the paper's unit).
    Runs stopped by the step cap count at the cap and are reported."""
    faulty = [r for r in records if r["events_applied"] > 0]
    out = {"runs": len(records), "runs_with_fault": len(faulty), "baseline_steps": clean_steps,
           "baseline_cycles": clean_cycles}
    if not faulty:
        return out
    out["faults_per_run"] = float(np.mean([r["events_applied"] for r in faulty]))
    out["detected_per_run"] = float(np.mean([r["detections"] for r in faulty]))
    out["detection_rate_percent"] = 100.0 * float(np.mean([r["detections"] / r["events_applied"] for r in faulty]))
    out["not_converged_ft"] = int(sum(not r.get("converged", True) for r in faulty))
    out["mean_steps_ft"] = float(np.mean([r["steps"] for r in faulty]))
    out["mean_cycles_ft"] = float(np.mean([r["cycles"] for r in faulty]))
    out["final_error_ft_max"] = float(np.max([r["err"] for r in faulty]))
    if all("steps_off" in r for r in faulty):
        out["not_converged_noft"] = int(sum(not r.get("converged_off", True) for r in faulty))
        out["mean_steps_noft"] = float(np.mean([r["steps_off"] for r in faulty]))
        out["mean_cycles_noft"] = float(np.mean([r["cycles_off"] for r in faulty]))
        out["roft_percent_steps"] = roft(out["mean_steps_noft"], out["mean_steps_ft"], clean_steps)
        out["roft_percent_cycles"] = roft(out["mean_cycles_noft"], out["mean_cycles_ft"], clean_cycles)
        out["final_error_noft_max"] = float(np.max([r["err_off"] for r in faulty]))
    return out


def parse_grid(text: str):
    """'nlon,nlat,nz' (lat-lon) or 'O<N>' / 'O<N>x<nz>' (octahedral, 51
    levels unless given, as in the paper's Table 1)."""
    from . import inputs as I
    if text[:1] in ("O", "o"):
        n, _, nz = text[1:].partition("x")
        return I.OctProblem(int(n), int(nz) if nz else 51)
    return I.Problem(*[int(v) for v in text.split(",")])


def grid_label(pb) -> list:
    return [f"O{pb.N}", pb.nz] if hasattr(pb, "N") else [pb.nx, pb.ny, pb.nz]


def main():
    from . import inputs as I
    ap = argparse.ArgumentParser()
    ap.add_argument("--model", choices=("config", "paper"), default="config")
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--grid", default="256,128,32")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--prob", type=float, default=0.02)
    ap.add_argument("--loss", default="4e-6,4e-4,2e-3,0.01,0.05,0.2")
    ap.add_argument("--procs", type=int, default=36)
    ap.add_argument("--cap", type=float, default=4.0, help="paper model: step cap as a multiple of the fault-free count")
    ap.add_argument("--bits", choices=("uniform", "finite"), default="uniform",
                    help="paper model: which bits a flip may hit (all 64, or all but the top exponent bit)")
    args = ap.parse_args()
    pb = parse_grid(args.grid)
    import torch
    torch.cuda.set_device(0)
    if args.model == "config":
        plans = I.campaign_plans(pb, count=args.count, seed0=I.SEEDS["c2_plan0"])
        records, summary, _ = run(pb, plans, k=args.k, tol=args.tol)
        summary["grid"] = grid_label(pb)
        summary["k"] = args.k
        print(json.dumps(summary), flush=True)
        return
    for loss in [float(v) for v in args.loss.split(",")]:
        plans = I.paper_plans(pb, args.count, prob=args.prob, data_loss=loss, procs=args.procs, bits=args.bits)
        records, _, st_clean = run(pb, plans, k=args.k, tol=args.tol, rhs_seed=I.SEEDS["c2_rhs"],
                                   cap_factor=args.cap)
        summary = summarize_paper(records, st_clean["steps_executed"], st_clean["cycles"])
        summary.update({"grid": grid_label(pb), "k": args.k, "prob": args.prob,
                        "data_loss_percent": 100.0 * loss, "procs": args.procs, "bits": args.bits})
        print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
