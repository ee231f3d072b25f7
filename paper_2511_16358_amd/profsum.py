"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_2511_16358_amd.profsum stats <run_kernel_stats.csv>
    python -m paper_2511_16358_amd.profsum traffic <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes>
    python -m paper_2511_16358_amd.profsum counters <run_counter_collection.csv>
    python -m paper_2511_16358_amd.profsum grids <run_kernel_trace.csv> <kernel name part>

`stats` prints the per-kernel call count and durations of a
``rocprofv3 --kernel-trace --stats --output-format csv`` run.  `traffic` turns
two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs (KiB per dispatch) into
bytes per launch, each counter scaled by what it reads for a plain device copy
of ``copy_bytes`` bytes each way, and prints the per-launch HBM bytes of the
contraction kernels in a line that bench.py reads back (valid only for the
kernel sources whose digest it carries).  `counters` prints the per-dispatch
mean of every counter of a ``--pmc`` run, per kernel; `grids` splits the
launches of one kernel of a kernel trace by workgroup count.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_digest() -> str:
    """sha256 over the HIP sources of the library."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("ifctn::", "")
    return name if len(name) <= 80 else name[:77] + "..."


def stats(path: str) -> None:
    rows = list(csv.DictReader(open(path)))
    print("%-80s %6s %11s %9s %9s %9s %6s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us", "pct"))
    for r in rows:
        print("%-80s %6d %11.1f %9.2f %9.2f %9.2f %6.2f" % (
            _short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))


def _counters(path: str, counter: str):
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def traffic(fetch: str, write: str, cfetch: str, cwrite: str, copy_bytes: str) -> None:
    known_kib = float(copy_bytes) / 1024.0

    def scale(path, counter):
        vals = [v for n, vs in _counters(path, counter).items() if "copyBuffer" in n for v in vs]
        if not vals:
            raise SystemExit(f"no copy dispatch in {path}")
        return known_kib / (sum(vals) / len(vals)), vals

    fs, fv = scale(cfetch, "FETCH_SIZE")
    ws, wv = scale(cwrite, "WRITE_SIZE")
    print(f"copy of {copy_bytes} B each way: FETCH_SIZE reads {sum(fv) / len(fv):.1f} KiB "
          f"-> scale {fs:.4f}; WRITE_SIZE reads {sum(wv) / len(wv):.1f} KiB -> scale {ws:.4f}")
    F, Wr = _counters(fetch, "FETCH_SIZE"), _counters(write, "WRITE_SIZE")
    print("%-80s %4s %12s %12s" % ("kernel", "n", "read_MB", "write_MB"))
    tot_f = tot_w = 0.0
    n_con = 0
    for name in sorted(F, key=lambda n: -sum(F[n]) / len(F[n])):
        f = sum(F[name]) / len(F[name]) * fs * 1024
        w_list = Wr.get(name, [0.0])
        w = sum(w_list) / len(w_list) * ws * 1024
        print("%-80s %4d %12.3f %12.3f" % (_short(name), len(F[name]), f / 1e6, w / 1e6))
        if "k_contract" in name:
            tot_f += sum(F[name]) * fs * 1024
            tot_w += sum(w_list) / len(w_list) * len(F[name]) * ws * 1024
            n_con += len(F[name])
    if n_con:
        print(f"contraction kernels (all layouts, fused X step included): {n_con} launches, "
              f"{tot_f / n_con / 1e6:.3f} MB read + {tot_w / n_con / 1e6:.3f} MB written per launch")
        print(f"bench: kernel_sources_sha256={kernel_source_digest()} "
              f"hbm_bytes_per_launch={(tot_f + tot_w) / n_con:.0f} launches={n_con}")


def grids(path: str, kernel: str) -> None:
    """Launches of one kernel (name contains `kernel`) in a --kernel-trace run,
    split by grid size: count and mean / min / max duration."""
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if kernel in r["Kernel_Name"]:
            per[int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print("%-40s %10s %6s %9s %9s %9s" % ("kernel", "workgroups", "calls", "avg_us", "min_us", "max_us"))
    for wg in sorted(per):
        v = per[wg]
        print("%-40s %10d %6d %9.2f %9.2f %9.2f" % (kernel[:40], wg, len(v), sum(v) / len(v), min(v), max(v)))


def counters(path: str) -> None:
    """Per kernel: dispatch count and the mean of every counter of the run."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    names = []
    for r in csv.DictReader(open(path)):
        c = r["Counter_Name"]
        if c not in names:
            names.append(c)
        per[r["Kernel_Name"]][c].append(float(r["Counter_Value"]))
    print("%-64s %5s " % ("kernel", "n") + " ".join("%14s" % c.replace("SQ_", "")[:14] for c in names))
    order = sorted(per, key=lambda n: -sum(per[n][names[0]]) if per[n][names[0]] else 0)
    for n in order:
        cnt = max(len(v) for v in per[n].values())
        vals = ["%14.0f" % (sum(per[n][c]) / len(per[n][c])) if per[n][c] else "%14s" % "-" for c in names]
        short = _short(n)
        print("%-64s %5d " % (short[:64], cnt) + " ".join(vals))


if __name__ == "__main__":
    if len(sys.argv) < 2 or sys.argv[1] not in ("stats", "traffic", "counters", "grids"):
        raise SystemExit(__doc__)
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "grids":
        grids(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2])
    else:
        traffic(*sys.argv[2:7])
