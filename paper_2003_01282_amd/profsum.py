"""Summaries of rocprofv3 CSV output (a profiling helper, not the path).

    python -m paper_2003_01282_amd.profsum stats <dir>      # --kernel-trace --stats
    python -m paper_2003_01282_amd.profsum pmc <dir>        # --pmc runs
    python -m paper_2003_01282_amd.profsum calls <dir> <name>   # every launch of a kernel (--kernel-trace)
    python -m paper_2003_01282_amd.profsum traffic <fetch_dir> <write_dir> <copy_bytes> <out.json> [settings]

`stats` prints calls and average/total duration per kernel from
*_kernel_stats.csv; `pmc` averages every counter column of
*_counter_collection.csv per kernel (values per dispatch, as rocprofv3
reports them: FETCH_SIZE / WRITE_SIZE in KiB).  `traffic` turns a FETCH_SIZE
run and a WRITE_SIZE run of bench.py (with --copy-probe-mb) into HBM bytes
per launch of the SpMM stage: each counter is scaled by the ratio of the
known bytes of the device-to-device copy dispatches (copy_bytes in total) to
what the same counter read for them, and the record is stamped with a digest
of the kernel sources, so a later source change voids it.
"""
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict
from pathlib import Path

SPMM_STAGE = ("spmm_pieces", "spmm_rows", "spmm_heavy")
UPDATE_KERNEL = "update"
COPY_KERNEL = "__amd_rocclr_copyBuffer"
KERNEL_SOURCES = ("common.hpp", "graph.hip", "relabel.hip", "lanczos.hip")


def kernel_sources_digest():
    """sha256 over the sources the SpMM stage and its data layout come from."""
    h = hashlib.sha256()
    csrc = Path(__file__).resolve().parent / "csrc"
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        h.update((csrc / name).read_bytes())
    return h.hexdigest()


def short(name, width=60):
    name = name.split("(")[0]
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(d, out=sys.stdout):
    f = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    print(f"{'kernel':62s} {'calls':>6s} {'avg_us':>12s} {'total_ms':>10s} {'pct':>6s}", file=out)
    for r in rows:
        print(f"{short(r['Name']):62s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:12.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.2f} {float(r['Percentage']):6.2f}", file=out)


def calls(d, stem, out=sys.stdout):
    """Every launch of the kernels whose name contains `stem`, in trace order:
    grid, workgroup size and duration (from the kernel trace)."""
    f = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    print(f"{'#':>5s} {'kernel':48s} {'grid':>10s} {'wg':>5s} {'ms':>10s}", file=out)
    k = 0
    for r in csv.DictReader(open(f)):
        if stem not in r["Kernel_Name"]:
            continue
        ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        print(f"{k:5d} {short(r['Kernel_Name'])[:48]:48s} {int(r['Grid_Size_X']):10d} "
              f"{int(r['Workgroup_Size_X']):5d} {ms:10.3f}", file=out)
        k += 1


def pmc_table(d):
    """{kernel: {counter: [per-dispatch values in dispatch order]}} over every
    counter file under d."""
    acc = defaultdict(lambda: defaultdict(list))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows = list(csv.DictReader(open(f)))
        if rows and "Dispatch_Id" in rows[0]:
            rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        for r in rows:
            k = short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return acc


def pmc(d, out=sys.stdout):
    for k, cs in pmc_table(d).items():
        for c, v in cs.items():
            print(f"{k:62s} {c:16s} dispatches {len(v):4d} avg {sum(v) / len(v):16.1f}", file=out)


def _find(table, stem, pool=True):
    """Counters of the kernels whose names contain stem: every match pooled
    (template variants of one kernel), or only the first match (dispatch
    order kept, as the calibration copy needs)."""
    out = defaultdict(list)
    for k, cs in table.items():
        if stem in k:
            for c, v in cs.items():
                out[c].extend(v)
            if not pool:
                break
    if not out:
        raise KeyError(stem)
    return out


def calibration_dispatch(values, copy_bytes):
    """The counter value (KiB) of the calibration copy among the run's copy
    dispatches in dispatch order: the first one that reads between 0.4 and 1.1
    times the copy's known size (bench.py makes that copy before anything
    else it copies)."""
    for v in values:
        if 0.4 <= v * 1024.0 / copy_bytes <= 1.1:
            return v
    raise SystemExit(f"no calibration copy of {copy_bytes} bytes among {len(values)} copy dispatches")


def traffic(fetch_dir, write_dir, copy_bytes, out_json, settings=None):
    """settings: the graph's schedule settings during the runs (as bench.py
    reports them in config.tuned / slaq_graph_settings); a bench run under
    other settings does not use the record."""
    rec = {"kernels": {}, "digest": kernel_sources_digest(), "settings": settings}
    per_launch = 0.0
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        t = pmc_table(d)
        copy = calibration_dispatch(_find(t, COPY_KERNEL, pool=False)[counter], copy_bytes)
        scale = copy_bytes / (copy * 1024.0)  # true bytes per counted byte
        rec[f"{counter}_scale"] = scale
        for k in SPMM_STAGE + (UPDATE_KERNEL,):
            v = _find(t, f"slaq::{k}")[counter]
            kib = sum(v) / len(v)
            rec["kernels"].setdefault(k, {})[counter + "_KiB"] = kib
            rec["kernels"][k][counter + "_bytes"] = kib * 1024.0 * scale
            if k in SPMM_STAGE:
                per_launch += kib * 1024.0 * scale
    rec["bytes_per_launch"] = per_launch  # the SpMM stage
    rec["update_bytes_per_launch"] = sum(rec["kernels"][UPDATE_KERNEL].get(c + "_bytes", 0.0)
                                         for c in ("FETCH_SIZE", "WRITE_SIZE"))
    Path(out_json).write_text(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "stats":
        stats(sys.argv[2])
    elif cmd == "pmc":
        pmc(sys.argv[2])
    elif cmd == "calls":
        calls(sys.argv[2], sys.argv[3])
    elif cmd == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5],
                json.loads(sys.argv[6]) if len(sys.argv) > 6 else None)
    else:
        raise SystemExit(f"unknown command {cmd}")
