"""Summarise rocprofv3 output of the benchmark into the short text records
kept under profiles/.

  python -m paper_2103_07210_amd.profsum stats  <rocprof out dir> <cmd> > profiles/<name>.md
  python -m paper_2103_07210_amd.profsum pmc    <fetch out dir> <write out dir> <grid> <cmd> > profiles/<name>.md

`stats` reads the kernel-trace CSV (or the rocpd SQLite database) and lists,
per kernel, dispatches, total and average duration, and the average over
dispatches longer than 20 us (launches enqueued after a solve converged
return at once and would bias the average).  `pmc` reads two counter runs
(FETCH_SIZE, WRITE_SIZE, KiB per dispatch) and reports the per-launch average
for the FP64 dir_update kernel and the library's bandwidth-probe copy kernel
(k_bw_copy) of the 1 GiB calibration copy, whose known size gives the scale
factor.
"""
import csv
import glob
import hashlib
import os
import sqlite3
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS_SRC = os.path.join(ROOT, "paper_2103_07210_amd", "csrc", "kernels.hip")


def source_sha256() -> str:
    return hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest()


def _dispatches(outdir):
    """Yield (kernel name, duration ns) of every dispatch."""
    files = glob.glob(os.path.join(outdir, "**", "*kernel_trace.csv"), recursive=True)
    if files:
        for f in files:
            for row in csv.DictReader(open(f)):
                yield row["Kernel_Name"], int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
        return
    for db in glob.glob(os.path.join(outdir, "**", "*.db"), recursive=True):
        con = sqlite3.connect(db)
        for name, dur in con.execute("select name, duration from kernels"):
            yield name, int(dur)


def stats(outdir, cmd):
    agg = defaultdict(list)
    for name, dur in _dispatches(outdir):
        agg[name].append(dur)
    rows = sorted(agg.items(), key=lambda kv: -sum(kv[1]))
    print("# rocprofv3 kernel trace summary\n")
    print(f"command: `{cmd}`\n")
    print(f"kernels.hip sha256: {source_sha256()}\n")
    print("| kernel | dispatches | total ms | avg us | dispatches > 20 us | avg us (> 20 us) |")
    print("|---|---|---|---|---|---|")
    for name, durs in rows[:24]:
        big = [d for d in durs if d > 20000]
        avg_big = sum(big) / len(big) / 1e3 if big else 0.0
        print(f"| `{name[:90]}` | {len(durs)} | {sum(durs) / 1e6:.2f} | {sum(durs) / len(durs) / 1e3:.2f} | "
              f"{len(big)} | {avg_big:.2f} |")


def _counters(outdir, counter):
    per = defaultdict(list)
    for f in glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name") == counter:
                per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return per


def pmc(fetch_dir, write_dir, grid, cmd):
    fetch = _counters(fetch_dir, "FETCH_SIZE")
    write = _counters(write_dir, "WRITE_SIZE")
    copy_bytes = float(1 << 30)

    def pick(d, key):
        vals = [v for name, vs in d.items() if key in name for v in vs]
        return vals

    def avg_big(vals):
        # launches after convergence return at once: keep dispatches that moved > 1 MiB
        big = [v for v in vals if v > 1024.0]
        return (sum(big) / len(big), len(big)) if big else (0.0, 0)

    f_dir, nf = avg_big(pick(fetch, "k_dir_update<double"))
    w_dir, nw = avg_big(pick(write, "k_dir_update<double"))
    f_cp, _ = avg_big(pick(fetch, "k_bw_copy"))
    w_cp, _ = avg_big(pick(write, "k_bw_copy"))
    sf = copy_bytes / (f_cp * 1024.0) if f_cp else 0.0
    sw = copy_bytes / (w_cp * 1024.0) if w_cp else 0.0
    print(f"# rocprofv3 HBM traffic counters, FP64 dir_update on {grid}\n")
    print(f"command (two passes, FETCH_SIZE then WRITE_SIZE): `{cmd}`\n")
    print(f"kernels_hip_sha256: {source_sha256()}")
    print(f"dir_update_fetch_kib_per_launch: {f_dir:.1f}")
    print(f"dir_update_write_kib_per_launch: {w_dir:.1f}")
    print(f"dir_update_launches_counted: {min(nf, nw)}")
    print(f"copy_1gib_fetch_kib: {f_cp:.1f}")
    print(f"copy_1gib_write_kib: {w_cp:.1f}")
    print(f"copy_scale_fetch: {sf:.4f}")
    print(f"copy_scale_write: {sw:.4f}")
    traffic = (f_dir * sf + w_dir * sw) * 1024.0
    print(f"traffic_bytes_per_launch: {traffic:.0f}")
    print("\nThe copy of 1 GiB reads and writes 1 GiB; its counters give the scale from counter KiB to bytes.")
    print("\nEvery FP64 step kernel, scaled bytes per launch (launches that moved more than 1 MiB):\n")
    print("| kernel | launches | fetch MB | write MB | total MB |")
    print("|---|---|---|---|---|")
    for key in ("k_update_thomas_full<double", "k_update_thomas<double", "k_stencil_dots<double",
                "k_dir_update<double"):
        fk, n1 = avg_big(pick(fetch, key))
        wk, n2 = avg_big(pick(write, key))
        if n1 and not n2:   # a pass that writes only its block partials
            wv = pick(write, key)
            wk, n2 = (sum(wv) / len(wv), n1) if wv else (0.0, 0)
        if n1 and n2:
            fb, wb = fk * sf * 1024.0, wk * sw * 1024.0
            print(f"| `{key}` | {min(n1, n2)} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")


def read_traffic(path):
    """traffic bytes per launch from a pmc summary, or None if missing or
    taken on a different kernels.hip."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "command")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernels_hip_sha256") != source_sha256():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
