"""Summarize rocprofv3 CSV output per kernel (a profiling helper, not the path).

    python -m paper_2003_01282_amd.profsum stats <dir>      # --kernel-trace --stats
    python -m paper_2003_01282_amd.profsum pmc <dir>        # --pmc runs

`stats` prints calls and average/total duration per kernel from
*_kernel_stats.csv; `pmc` averages every counter column of
*_counter_collection.csv per kernel (values per dispatch, as rocprofv3
reports them: FETCH_SIZE / WRITE_SIZE in KiB).
"""
import csv
import glob
import os
import sys
from collections import defaultdict


def short(name, width=60):
    name = name.split("(")[0]
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(d):
    f = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    print(f"# {f}")
    print(f"{'kernel':62s} {'calls':>6s} {'avg_us':>12s} {'total_ms':>10s} {'pct':>6s}")
    for r in rows:
        print(f"{short(r['Name']):62s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:12.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.2f} {float(r['Percentage']):6.2f}")


def pmc(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    for f in files:
        rows = list(csv.DictReader(open(f)))
        acc = defaultdict(lambda: defaultdict(list))
        for r in rows:
            k = short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        print(f"# {f}")
        for k, cs in acc.items():
            for c, v in cs.items():
                print(f"{k:62s} {c:16s} dispatches {len(v):4d} avg {sum(v) / len(v):16.1f}")


if __name__ == "__main__":
    {"stats": stats, "pmc": pmc}[sys.argv[1]](sys.argv[2])
