"""Benchmark: FT-GCR(4) on the 512 x 256 x 64 hill-on-sphere problem.

A step of this benchmark is one whole solve (every row of the hot path:
initial residual, preconditioned GCR(4) steps with the monotone-norm fault
test and per-cycle backups, the deferred iterate update and the final FP64
true residual) to a relative residual of 1e-8, inputs resident in HBM.
`value` is executed GCR inner steps per second of the FP64 solve.  The same
run times the mixed-precision solve (binary32 vectors, FP64 inner products,
detector and refinement) to the same 1e-8 true residual, the per-kernel
device time of the dominant kernel against the HBM roofline, and the CPU
oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
GRID = (512, 256, 64)
K = 4
TOL = 1e-8
TIMED_STRIDE = 5   # timed region: dominant-kernel events on every 5th step (coprime with K)


# Algorithmic bytes: the method's own HBM traffic when every operand is read
# once per phase between two global reductions and e, L(e) are recomputed
# rather than stored (s = bytes per stored value, N cells):
#   update phase U(nu): read r, L(p^nu), x, p^nu, L(p^0..nu-1); write r, x
#                       (nu + 6) s N
#   direction phase O(nu): read r, p^0..nu, L(p^0..nu); write p^{nu+1},
#                       L(p^{nu+1})                            (2 nu + 5) s N
#   backup: [x, r, p^0, L(p^0)] written once per cycle          4 s N
# so a step moves W(nu) = (3 nu + 11) s N plus 4 s N per cycle (16.5 sweeps
# per step at k = 4).  The converging step runs U only.  Once per solve (or
# refinement round) the initial residual, P^{-1} r0 and A p0 move 6 s N, and
# every FP64 true-residual pass (x, R read, r_t written) 3 * 8 N.
# The design's own kernels move more: the column pass stores e (4 s N: r,
# L(p^nu) read, r+, e written), the dots pass re-reads it ((nu + 2) s N), the
# direction pass re-reads it with r ((2 nu + 6) s N) and the iterate is read
# and written once per cycle (2 * 8 N at nu = k - 1); that excess is reported
# as design overhead, not as work.


def pass_bytes(kernel, nu, k, n, s, xs=8, design=False):
    """Bytes of one launch of a step kernel at pass index nu: the method's
    algorithmic bytes of the phase it implements (dir_update: the direction
    phase plus the once-per-cycle iterate update it carries), or with
    design=True what the kernel moves by design."""
    x_upd = 2 * xs * n if nu == k - 1 else 0
    if kernel == "dir_update":
        return ((2 * nu + 6) if design else (2 * nu + 5)) * s * n + x_upd
    if kernel == "update_thomas":
        return 4 * s * n
    if kernel == "stencil_dots":
        return (nu + 2) * s * n
    raise KeyError(kernel)


def alg_bytes(kernel, steps, k, n, s, xs=8, stride=1, design=False):
    """Bytes of one fault-free solve's launches of `kernel` (of the steps
    whose number is a multiple of `stride`: the ones the timed region times).
    Executed step t (1-based) has pass index nu = (t-1) mod k; the
    converging step does not run the direction kernels."""
    total = 0
    for t in range(1, steps + 1):
        if t % stride:
            continue
        nu = (t - 1) % k
        if kernel != "update_thomas" and t == steps:
            continue
        total += pass_bytes(kernel, nu, k, n, s, xs, design)
    return total


def solve_bytes(steps, k, n, s, rounds=1, residual_passes=1, design=False):
    """Bytes of a whole fault-free solve of `steps` executed steps in
    `rounds` refinement rounds (FP64: one round) with `residual_passes` FP64
    true-residual passes.  The pass index runs over the executed steps as
    one sequence (a round boundary shifts it by less than k steps: under
    0.5% of a solve).  design=True: what the design's kernels move."""
    total = 0
    for t in range(1, steps + 1):
        nu = (t - 1) % k
        last = t == steps
        if design:
            total += sum(pass_bytes(q, nu, k, n, s, design=True) for q in
                         (("update_thomas",) if last else ("update_thomas", "stencil_dots", "dir_update")))
        else:
            total += (nu + 6) * s * n + (0 if last else (2 * nu + 5) * s * n)
    if not design:
        total += 4 * s * n * ((steps + k - 1) // k)
    total += 6 * s * n * rounds + 3 * 8 * n * residual_passes
    return total


def gmres_solve_bytes(steps, cycles, k, n, s=8):
    """Algorithmic bytes of a fault-free FT-GMRES(k) solve (classical
    Gram-Schmidt, each phase's operands read once): step j of a cycle reads
    v_j and writes z_j = P^-1 v_j (2 sweeps), forms w = A z_j with the
    <w, v_i>, i <= j (reads z_j and v_0..v_j, writes w: j + 3), and
    orthogonalises and normalises (reads w and v_0..v_j, writes v_{j+1}:
    j + 3): 2j + 8 sweeps; a cycle of m steps adds the correction (reads x and
    z_0..z_{m-1}, writes x: m + 2) and the explicit residual (reads x and R,
    writes s: 3)."""
    total = 0
    left = steps
    for _ in range(cycles):
        m = min(k, left)
        total += sum(2 * j + 8 for j in range(m)) + m + 5
        left -= m
    return total * s * n


def step_frac(steps, k, n, s, ms, rounds=1, residual_passes=1):
    """Whole-solve rate on the algorithmic bytes against the HBM peak, and
    the design's bytes over them."""
    alg = solve_bytes(steps, k, n, s, rounds, residual_passes)
    des = solve_bytes(steps, k, n, s, rounds, residual_passes, design=True)
    gbs = alg / (ms * 1e-3) / 1e9
    return {"ms": ms, "steps": steps, "alg_bytes": alg, "alg_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "design_bytes": des, "design_overhead": des / alg - 1.0}


def cpu_cores() -> int:
    """Host cores this process may use: its affinity set, capped by
    OMP_NUM_THREADS where that is set."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(env))) if env.isdigit() else n


def cpu_baseline(pb, rhs, steps=24):
    """The oracle on the first `steps` steps of the same solve, on all the
    cores (its threaded mode, bitwise the serial results) and on one."""
    from oracle import oracle as om
    o = om.Oracle(pb)
    cores = cpu_cores()
    before = om.threads()
    out = {}
    try:
        for t in (cores, 1):
            om.set_threads(t)
            t0 = time.perf_counter()
            _, st, _, _ = o.solve(rhs, tol=TOL, k=K, max_steps=steps)
            out[t] = (st["steps_executed"], time.perf_counter() - t0)
    finally:
        om.set_threads(before)
    n, dt = out[cores]
    n1, dt1 = out[1]
    return {"value": n / dt, "unit": "GCR iter/s", "cores": cores, "kind": "oracle",
            "value_1core": n1 / dt1,
            "sample": f"first {n} steps of the FP64 FT-GCR({K}) solve on {GRID[0]}x{GRID[1]}x{GRID[2]} "
                      f"(face weights included), C oracle: {dt:.1f} s on {cores} threads (operator, "
                      f"preconditioner and face weights split, results bitwise serial), {dt1:.1f} s on 1"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for counter passes: one FP64 solve and the 1 GiB copy probe only")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-member batched ensemble timing")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024x512x96 solves")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the octahedral O160 x 51 and FT-GMRES(16) timings")
    ap.add_argument("--grid", default="512,256,64",
                    help="with --profile-run: the grid of the profiled FP64 solve (nlon,nlat,nz)")
    args = ap.parse_args()
    grid = tuple(int(v) for v in args.grid.split(","))
    if grid != GRID and not args.profile_run:
        ap.error("--grid is for --profile-run only; the benchmark workload is 512x256x64")
    if args.profile_run:
        args.steps, args.warmup, args.no_cpu, args.mixed_steps, args.no_ensemble, args.no_large = 1, 0, True, 0, True, True
        args.no_extra = True
    if args.gpus != 1:
        print(json.dumps({"error": "the FT-GCR library runs on one GPU; sharding across GPUs (horizontal "
                                   "blocks of whole columns) is not implemented; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2103_07210_amd import ftgcr
    from paper_2103_07210_amd import inputs as I

    torch.cuda.set_device(0)
    pb = I.Problem(*grid)
    n = pb.n
    grid_tag = "x".join(str(v) for v in grid)
    rhs_np = I.rhs(pb, I.SEEDS["c3_rhs" if grid == GRID else "c5_rhs"])
    rhs = torch.from_numpy(rhs_np).cuda()
    x = torch.zeros_like(rhs)
    print(f"[bench] grid {grid} N={n} k={K} tol={TOL}", flush=True)

    s64 = ftgcr.Solver(pb, "fp64", kmax=K, poll_steps=32)
    kc64 = s64.autotune(rhs, k=K, steps=24) if not args.profile_run else s64.options()["levels_per_block"]
    til64 = s64.tiling()
    print(f"[bench] fp64 stencil tiling: {til64}", flush=True)
    for _ in range(args.warmup):
        x.zero_()
        s64.solve(rhs, x, tol=TOL, k=K)
    torch.cuda.synchronize()
    print("[bench] fp64 warmup done", flush=True)

    # per-kernel breakdown (one solve, every step kernel's launch stamped
    # with HIP start/stop events by its own dispatch), which also names the
    # dominant kernel
    names = ("update_thomas", "stencil_dots", "dir_update")
    s64.set_options(profile_kernels=1)
    s64.reset_kernel_times()
    x.zero_()
    s64.solve(rhs, x, tol=TOL, k=K)
    torch.cuda.synchronize()
    kt_all = s64.kernel_times()
    kernels = {q: {"launches": int(v[0]), "avg_us": (v[1] / v[0] * 1e3) if v[0] else 0.0} for q, v in kt_all.items()}
    dom = max(names, key=lambda q: kt_all[q][1])

    # timed region: K whole solves; only the dominant kernel's launches of
    # every TIMED_STRIDE-th step carry HIP start/stop events (stamped by the
    # dispatch, on the solve stream), so the timing costs the whole-solve rate
    # as little as possible
    s64.set_options(profile_kernels=(TIMED_STRIDE << 8) | (2 << names.index(dom)))
    s64.reset_kernel_times()
    torch.cuda.synchronize()
    steps_total, stats = 0, None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        _, stats = s64.solve(rhs, x, tol=TOL, k=K)
        steps_total += stats["steps_executed"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = s64.kernel_times()
    s64.set_options(profile_kernels=0)
    iters_per_s = steps_total / wall
    steps_per_solve = stats["steps_executed"]
    print(f"[bench] fp64: {steps_per_solve} steps/solve, {wall / args.steps * 1e3:.2f} ms/solve, "
          f"true residual {stats['rel_res_true']:.3e}", flush=True)

    # roofline of the dominant kernel, timed inside the timed region (the
    # launches of every TIMED_STRIDE-th step, which for a stride coprime with
    # k sample every pass index alike)
    launches, ms = kt[dom]
    bytes_dom = alg_bytes(dom, steps_per_solve, K, n, 8, stride=TIMED_STRIDE) * args.steps
    design_dom = alg_bytes(dom, steps_per_solve, K, n, 8, stride=TIMED_STRIDE, design=True) * args.steps
    achieved = bytes_dom / (ms * 1e-3) / 1e9
    whole_gbs = solve_bytes(steps_per_solve, K, n, 8) * args.steps / wall / 1e9
    for q in names:
        v = kernels[q]
        if v["launches"]:
            b = alg_bytes(q, steps_per_solve, K, n, 8, design=True) / v["launches"]
            v["design_bytes_per_launch"] = b
            v["design_gbs"] = b / (v["avg_us"] * 1e-6) / 1e9
    from paper_2103_07210_amd.profsum import read_traffic
    traffic = read_traffic(os.path.join(ROOT, "profiles", f"traffic_dir_update_fp64_{grid_tag}.md"))

    # HBM copy probe: the library's streaming copy kernel, 1 GiB read and
    # 1 GiB written per copy
    copy_gbs = ftgcr.bw_probe(1 << 30, reps=5)

    # mixed precision, same problem, time to the same 1e-8 true residual,
    # against FP64 solves timed the same way (no per-kernel events)
    fp64_runs = []
    for _ in range(5 if args.mixed_steps > 0 else 0):
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s64.solve(rhs, x, tol=TOL, k=K)
        torch.cuda.synchronize()
        fp64_runs.append((time.perf_counter() - t1) * 1e3)
    fp64_ms = float(np.median(fp64_runs)) if fp64_runs else wall / args.steps * 1e3

    # fault-tolerance overhead on a fault-free solve: the same solve with the
    # detector, backups and rollbacks switched off
    ft_overhead = None
    if args.mixed_steps > 0:
        s_off = ftgcr.Solver(pb, "fp64", kmax=K, poll_steps=32, ft=0, levels_per_block=kc64)
        x.zero_()
        s_off.solve(rhs, x, tol=TOL, k=K)
        off_runs = []
        for _ in range(5):
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, st_off = s_off.solve(rhs, x, tol=TOL, k=K)
            torch.cuda.synchronize()
            off_runs.append((time.perf_counter() - t1) * 1e3)
        off_ms = float(np.median(off_runs))
        ft_overhead = {"ft_on_ms": fp64_ms, "ft_off_ms": off_ms, "overhead": fp64_ms / off_ms - 1.0,
                       "steps_on": steps_per_solve, "steps_off": st_off["steps_executed"]}
        print(f"[bench] FT on {fp64_ms:.2f} ms, FT off {off_ms:.2f} ms", flush=True)
        s_off.close()
    fracs = {f"{grid_tag}_fp64": step_frac(steps_per_solve, K, n, 8, fp64_ms)}
    mixed = None
    if args.mixed_steps > 0:
        sm = ftgcr.Solver(pb, "mixed", kmax=K, poll_steps=32)
        kcm = sm.autotune(rhs, k=K, steps=24)
        xm = torch.zeros_like(rhs)
        sm.solve(rhs, xm, tol=TOL, k=K)
        torch.cuda.synchronize()
        mixed_ms, mstats = [], None
        for _ in range(args.mixed_steps):
            xm.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, mstats = sm.solve(rhs, xm, tol=TOL, k=K)
            torch.cuda.synchronize()
            mixed_ms.append((time.perf_counter() - t1) * 1e3)
        mixed_med = float(np.median(mixed_ms))
        xd = x.double()
        mixed_err = float(torch.linalg.norm(xm - xd) / torch.linalg.norm(xd))
        print(f"[bench] mixed: {mixed_med:.2f} ms, {mstats['steps_executed']} inner steps, "
              f"{mstats['refinements']} refinements, true residual {mstats['rel_res_true']:.3e}", flush=True)
        mixed = {"fp64": fp64_ms, "mixed": mixed_med, "speedup": fp64_ms / mixed_med,
                 "fp64_true_residual": stats["rel_res_true"], "mixed_true_residual": mstats["rel_res_true"],
                 "mixed_inner_steps": mstats["steps_executed"], "mixed_refinements": mstats["refinements"],
                 "mixed_vs_fp64_solution_rel_diff": mixed_err, "mixed_levels_per_block": kcm,
                 "mixed_tiling": sm.tiling()}
        fracs["512x256x64_mixed"] = step_frac(mstats["steps_executed"], K, n, 4, mixed_med,
                                              rounds=mstats["refinements"],
                                              residual_passes=mstats["refinements"] + 1)

    # 64-member ensemble (sizes 64x32x8 .. 256x128x32, 6 members with a
    # fault): one batched launch sequence against the members one by one
    ensemble = None
    if not args.no_ensemble:
        members = I.ensemble(64, seed=I.SEEDS["c4_table"])
        solvers = [ftgcr.Solver(mb.problem, "fp64", kmax=3, poll_steps=32) for mb in members]
        erhs = [torch.from_numpy(I.rhs(mb.problem, mb.rhs_seed)).cuda() for mb in members]
        plans = [mb.plan for mb in members]
        batch_kc = ftgcr.autotune_batch(solvers, erhs, k=3, steps=24)
        print(f"[bench] ensemble tiling: {batch_kc} levels per block", flush=True)
        ftgcr.solve_batch(solvers, erhs, tols=[1e-10] * 64, k=3, plans=plans)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, bst = ftgcr.solve_batch(solvers, erhs, tols=[1e-10] * 64, k=3, plans=plans)
        torch.cuda.synchronize()
        batched_ms = (time.perf_counter() - t1) * 1e3
        # the same batch with every chunk of steps launched directly (no
        # graph replay), for the graph's share
        solvers[0].set_options(use_graphs=0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, bst_d = ftgcr.solve_batch(solvers, erhs, tols=[1e-10] * 64, k=3, plans=plans)
        torch.cuda.synchronize()
        direct_ms = (time.perf_counter() - t1) * 1e3
        solvers[0].set_options(use_graphs=1)
        same_steps = [b["steps_executed"] for b in bst] == [b["steps_executed"] for b in bst_d]
        t1 = time.perf_counter()
        for sv, r, pl in zip(solvers, erhs, plans):
            sv.solve(r, tol=1e-10, k=3, plan=pl)
        torch.cuda.synchronize()
        seq_ms = (time.perf_counter() - t1) * 1e3
        steps_all = sum(b["steps_executed"] for b in bst)
        points = sum(mb.problem.n for mb in members)
        # aggregate algorithmic bytes of the members' solves (rolled-back
        # steps of the faulty members counted as executed) over the batched time
        ens_bytes = sum(solve_bytes(b["steps_executed"], 3, mb.problem.n, 8) for b, mb in zip(bst, members))
        ensemble = {"members": 64, "points": points, "k": 3, "tol": 1e-10, "levels_per_block": batch_kc,
                    "batched_ms": batched_ms, "batched_direct_ms": direct_ms,
                    "graph_speedup": direct_ms / batched_ms, "graph_same_steps": same_steps,
                    "sequential_ms": seq_ms,
                    "member_steps_total": steps_all, "member_steps_per_s_batched": steps_all / batched_ms * 1e3,
                    "all_converged": all(b["status"] == 0 for b in bst),
                    "alg_bytes": ens_bytes, "alg_gbs": ens_bytes / (batched_ms * 1e-3) / 1e9,
                    "frac": ens_bytes / (batched_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "detections": sum(b["detections"] for b in bst)}
        print(f"[bench] ensemble: batched {batched_ms:.1f} ms (direct launches {direct_ms:.1f} ms), "
              f"one by one {seq_ms:.1f} ms", flush=True)
        for sv in solvers:
            sv.close()

    # the two small configurations (cache-resident, launch- and
    # latency-bound: timed, not priced against the HBM roofline)
    small = None
    if not args.no_large:
        small = {}
        for name, pbs, kk, rs in (("64x32x8", I.C1, 3, I.SEEDS["c1_rhs"]), ("256x128x32", I.C2, 4, I.SEEDS["c2_rhs"])):
            rhs_s = torch.from_numpy(I.rhs(pbs, rs)).cuda()
            ss = ftgcr.Solver(pbs, "fp64", kmax=kk, poll_steps=32)
            ss.autotune(rhs_s, k=kk, steps=12)
            xs_ = torch.zeros_like(rhs_s)
            ss.solve(rhs_s, xs_, tol=1e-10, k=kk)
            runs_s = []
            for _ in range(5):
                xs_.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, sts = ss.solve(rhs_s, xs_, tol=1e-10, k=kk)
                torch.cuda.synchronize()
                runs_s.append((time.perf_counter() - t1) * 1e3)
            ms_s = float(np.median(runs_s))
            small[name] = {"k": kk, "tol": 1e-10, "ms": ms_s, "steps": sts["steps_executed"],
                           "steps_per_s": sts["steps_executed"] / ms_s * 1e3}
            print(f"[bench] {name}: {ms_s:.2f} ms, {sts['steps_executed']} steps", flush=True)
            ss.close()

    # the paper's octahedral mesh O160 with 51 levels (Table 1; 5.5 M points):
    # FT-GCR(5) as in the paper's runs, FP64 to 1e-8, fault-free and with a
    # 10% block of r flipped at step 10; and FT-GMRES(16) on 512 x 256 x 64
    extra = None
    if not args.no_extra:
        extra = {}
        po = I.O160
        rhs_o = torch.from_numpy(I.rhs(po, I.SEEDS["c3_rhs"])).cuda()
        so = ftgcr.Solver(po, "fp64", kmax=5, poll_steps=32)
        kco = so.autotune(rhs_o, k=5, steps=12)
        x_o = torch.zeros_like(rhs_o)
        so.solve(rhs_o, x_o, tol=TOL, k=5)
        runs_o = []
        for _ in range(3):
            x_o.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, sto = so.solve(rhs_o, x_o, tol=TOL, k=5)
            torch.cuda.synchronize()
            runs_o.append((time.perf_counter() - t1) * 1e3)
        ms_o = float(np.median(runs_o))
        so.set_options(profile_kernels=1)
        so.reset_kernel_times()
        x_o.zero_()
        so.solve(rhs_o, x_o, tol=TOL, k=5)
        kto = so.kernel_times()
        so.set_options(profile_kernels=0)
        plan_o = I.block_plan(po, step=10, vec="r", fraction=0.1, bit=62, seed=I.SEEDS["c5_plan"])
        x_o.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sfo = so.solve(rhs_o, x_o, tol=TOL, k=5, plan=plan_o)
        torch.cuda.synchronize()
        ms_fo = (time.perf_counter() - t1) * 1e3
        til_o = so.tiling()
        so.close()
        fr = step_frac(sto["steps_executed"], 5, po.n, 8, ms_o)
        # the mixed form on the same mesh and right-hand side
        som = ftgcr.Solver(po, "mixed", kmax=5, poll_steps=32)
        som.autotune(rhs_o, k=5, steps=12)
        x_om = torch.zeros_like(rhs_o)
        som.solve(rhs_o, x_om, tol=TOL, k=5)
        runs_om = []
        for _ in range(3):
            x_om.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, stom = som.solve(rhs_o, x_om, tol=TOL, k=5)
            torch.cuda.synchronize()
            runs_om.append((time.perf_counter() - t1) * 1e3)
        ms_om = float(np.median(runs_om))
        til_om = som.tiling()
        som.close()
        fr_m = step_frac(stom["steps_executed"], 5, po.n, 4, ms_om, rounds=stom["refinements"],
                         residual_passes=stom["refinements"] + 1)
        print(f"[bench] O160x51 mixed: {ms_om:.1f} ms, {stom['steps_executed']} inner steps, "
              f"{stom['refinements']} refinements, {ms_o / ms_om:.2f}x FP64", flush=True)
        extra["octahedral_O160x51"] = {
            "points": po.n, "k": 5, "tol": TOL, "levels_per_block": kco, "tiling": til_o, "ms": ms_o,
            "steps": sto["steps_executed"], "us_per_step": ms_o * 1e3 / sto["steps_executed"],
            "rel_res_true": sto["rel_res_true"], "alg_gbs": fr["alg_gbs"], "frac": fr["frac"],
            "kernels_us": {q: v[1] / v[0] * 1e3 for q, v in kto.items() if v[0]},
            "fault_10pct_r_bit62": {"ms": ms_fo, "steps": sfo["steps_executed"], "detections": sfo["detections"],
                                    "steps_wasted": sfo["steps_wasted"], "rel_res_true": sfo["rel_res_true"]},
            "mixed": {"ms": ms_om, "inner_steps": stom["steps_executed"], "refinements": stom["refinements"],
                      "rel_res_true": stom["rel_res_true"], "speedup": ms_o / ms_om, "tiling": til_om,
                      "alg_gbs": fr_m["alg_gbs"], "frac": fr_m["frac"]}}
        print(f"[bench] O160x51 FT-GCR(5): {ms_o:.1f} ms, {sto['steps_executed']} steps, frac {fr['frac']:.3f}; "
              f"10% r block: {ms_fo:.1f} ms, {sfo['detections']} detections", flush=True)
        kg = 16
        sg = ftgcr.Solver(pb, "fp64", kmax=kg, poll_steps=32, method=ftgcr.METHOD_GMRES, levels_per_block=kc64)
        xg = torch.zeros_like(rhs)
        sg.solve(rhs, xg, tol=TOL, k=kg)
        runs_g = []
        for _ in range(3):
            xg.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, stg = sg.solve(rhs, xg, tol=TOL, k=kg)
            torch.cuda.synchronize()
            runs_g.append((time.perf_counter() - t1) * 1e3)
        sg.close()
        ms_g = float(np.median(runs_g))
        gb = gmres_solve_bytes(stg["steps_executed"], stg["cycles"], kg, n)
        extra["gmres_512x256x64"] = {
            "k": kg, "tol": TOL, "ms": ms_g, "steps": stg["steps_executed"], "cycles": stg["cycles"],
            "us_per_step": ms_g * 1e3 / stg["steps_executed"], "rel_res_true": stg["rel_res_true"],
            "alg_bytes": gb, "alg_gbs": gb / (ms_g * 1e-3) / 1e9, "frac": gb / (ms_g * 1e-3) / 1e9 / HBM_PEAK_GBS}
        print(f"[bench] FT-GMRES(16) 512x256x64: {ms_g:.1f} ms, {stg['steps_executed']} steps, "
              f"{stg['cycles']} cycles", flush=True)

    # the 1024 x 512 x 96 problem (one GPU's share of an 8-GPU run at
    # 8x the columns): FP64 and mixed, fault-free and with a 10% contiguous
    # block of r flipped (exponent MSB) at step 10
    large = None
    if not args.no_large:
        s64.close()
        torch.cuda.empty_cache()
        pl = I.C5
        rhs_l = torch.from_numpy(I.rhs(pl, I.SEEDS["c5_rhs"])).cuda()
        x_l = torch.zeros_like(rhs_l)
        large = {"grid": [pl.nx, pl.ny, pl.nz], "k": K, "tol": TOL}
        for prec, bit in (("fp64", 62), ("mixed", 30)):
            plan = I.block_plan(pl, step=10, vec="r", fraction=0.1, bit=bit, seed=I.SEEDS["c5_plan"])
            sl = ftgcr.Solver(pl, prec, kmax=K, poll_steps=32)
            kcl = sl.autotune(rhs_l, k=K, steps=12)
            x_l.zero_()
            sl.solve(rhs_l, x_l, tol=TOL, k=K)
            rec = {"levels_per_block": kcl, "tiling": sl.tiling()}
            for name, pln, reps in (("clean", [], 3), ("fault", plan, 1)):
                runs = []
                for _ in range(reps):
                    x_l.zero_()
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    _, stl = sl.solve(rhs_l, x_l, tol=TOL, k=K, plan=pln)
                    torch.cuda.synchronize()
                    runs.append((time.perf_counter() - t1) * 1e3)
                rec[name] = {"ms": float(np.median(runs)), "steps_executed": stl["steps_executed"],
                             "steps_wasted": stl["steps_wasted"], "detections": stl["detections"],
                             "refinements": stl["refinements"], "rel_res_true": stl["rel_res_true"]}
            large[prec] = rec
            cl = rec["clean"]
            fracs[f"{pl.nx}x{pl.ny}x{pl.nz}_{prec}"] = step_frac(
                cl["steps_executed"], K, pl.n, 8 if prec == "fp64" else 4, cl["ms"],
                rounds=max(1, cl["refinements"]), residual_passes=cl["refinements"] + 1)
            print(f"[bench] {pl.nx}x{pl.ny}x{pl.nz} {prec}: clean {rec['clean']['ms']:.1f} ms "
                  f"({rec['clean']['steps_executed']} steps), 10% r block fault {rec['fault']['ms']:.1f} ms "
                  f"({rec['fault']['detections']} detections, {rec['fault']['steps_wasted']} wasted)", flush=True)
            sl.close()
        del rhs_l, x_l
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu oracle sample ...", flush=True)
        cpu = cpu_baseline(pb, rhs_np)

    out = {
        "metric": "GCR iter/s + HBM GB/s at 512x256x64; time-to-1e-8 residual FP64 vs mixed",
        "value": iters_per_s,
        "unit": "GCR iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FT-GCR(4) FP64 solve to 1e-8, 512x256x64 hill-on-sphere, RHS U[-1,1] seed 3",
                   "grid": list(GRID), "k": K, "tol": TOL, "steps_per_solve": steps_per_solve,
                   "levels_per_block": kc64, "tiling": til64},
        "hbm_gbs_algorithmic": whole_gbs,
        "step_frac": fracs,
        "time_to_1e-8_ms": mixed,
        "ft_overhead_fault_free": ft_overhead,
        "kernels": kernels,
        "ensemble_64": ensemble,
        "large_1024x512x96": large,
        "extra": extra,
        "small_configs": small,
        "copy_probe_gbs": copy_gbs,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic if dom == "dir_update" else None,
                     "avg_launch_us": ms / launches * 1e3 if launches else None,
                     "alg_bytes_per_launch": bytes_dom / (launches or 1),
                     "design_bytes_per_launch": design_dom / (launches or 1),
                     "frac_of_copy_probe": achieved / copy_gbs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
