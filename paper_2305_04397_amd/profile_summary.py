"""Reduce rocprofv3 CSV output to short per-kernel tables.

    python -m paper_2305_04397_amd.profile_summary <rocprofv3 output dir> [--delete-raw]
    python -m paper_2305_04397_amd.profile_summary traffic <fetch dir> <write dir> <bench json> <out>

Kernel traces: per-kernel calls, total and average duration (from
*_kernel_stats.csv).  Counter runs: per-kernel dispatch count, the mean of
every counter per dispatch and its total (from *_counter_collection.csv).
With --delete-raw the per-dispatch CSV files are removed afterwards.

``traffic`` turns a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch)
into HBM bytes per launch of the sweep kernels.  Each counter is scaled by
what it reads for the model upload's FP64 -> FP32 conversion kernel, a plain
stream whose bytes are known from the workload's sizes (8 bytes read and 4
written per converted value: N probabilities and 2R rewards; the few
thousand agent-block values are left out, < 0.1 %).  The output records a
hash of the sweep kernels' sources so a later run can tell whether the
counters still describe the code.
"""
from __future__ import annotations

import csv
import glob
import os
import sys
from collections import defaultdict


def short(name: str) -> str:
    n = name.split("(")[0]
    return n[:160]


def summarize(d: str, delete_raw: bool) -> str:
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*_kernel_stats.csv"), recursive=True)):
        out.append(f"# kernel statistics ({os.path.basename(f)})")
        out.append("calls,total_ms,avg_us,percent,kernel")
        with open(f) as fh:
            for row in csv.DictReader(fh):
                out.append(f"{row['Calls']},{float(row['TotalDurationNs']) / 1e6:.3f},"
                           f"{float(row['AverageNs']) / 1e3:.2f},{float(row['Percentage']):.2f},"
                           f"{short(row['Name'])}")
    for f in sorted(glob.glob(os.path.join(d, "**", "*_counter_collection.csv"), recursive=True)):
        acc = defaultdict(lambda: defaultdict(float))
        disp = defaultdict(set)
        with open(f) as fh:
            reader = csv.DictReader(fh)
            if "Counter_Name" not in (reader.fieldnames or []):
                out.append(f"# unrecognised columns in {os.path.basename(f)}: {reader.fieldnames}")
                delete_raw = False
                continue
            for row in reader:
                k = short(row.get("Kernel_Name", row.get("Kernel-Name", "?")))
                acc[k][row["Counter_Name"]] += float(row["Counter_Value"])
                disp[k].add(row.get("Dispatch_Id", row.get("Dispatch-Id")))
        counters = sorted({c for v in acc.values() for c in v})
        out.append(f"# counters per dispatch: mean, then total over dispatches ({os.path.basename(f)})")
        out.append("dispatches," + ",".join(counters) + "," + ",".join(f"{c}_total" for c in counters) + ",kernel")
        for k in sorted(acc, key=lambda k: -len(disp[k])):
            n = len(disp[k])
            out.append(f"{n}," + ",".join(f"{acc[k][c] / n:.6g}" for c in counters) + "," +
                       ",".join(f"{acc[k][c]:.9g}" for c in counters) + f",{k}")
    text = "\n".join(out) + "\n"
    if delete_raw:
        for pat in ("*_kernel_trace.csv", "*_counter_collection.csv", "*_results.db", "*.rocpd"):
            for f in glob.glob(os.path.join(d, "**", pat), recursive=True):
                os.remove(f)
    return text


SWEEP_SOURCES = ("csrc/block.hip", "csrc/halo.hip", "csrc/vi.hip", "csrc/kern.h")


def sources_hash() -> str:
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_table(summary: str, counter: str) -> dict:
    """kernel -> (dispatches, total) from a summary.txt counter table."""
    out = {}
    lines = open(summary).read().splitlines()
    for i, line in enumerate(lines):
        if not line.startswith("dispatches,"):
            continue
        cols = line.split(",")
        ti = cols.index(f"{counter}_total")
        for row in lines[i + 1:]:
            if not row or row.startswith("#"):
                break
            parts = row.split(",", len(cols) - 1)
            out[parts[-1]] = (int(parts[0]), float(parts[ti]))
    return out


def traffic(fetch_dir: str, write_dir: str, bench_json: str, out_path: str) -> str:
    import json
    fetch = _counter_table(os.path.join(fetch_dir, "summary.txt"), "FETCH_SIZE")
    write = _counter_table(os.path.join(write_dir, "summary.txt"), "WRITE_SIZE")
    line = [l for l in open(bench_json).read().splitlines() if l.startswith("{")][-1]
    cfg = json.loads(line)["config"]
    N, R = cfg["nnz"], cfg["rows"]
    cal = "morap::k::to_f32_kernel"
    values = N + 2 * R
    f_scale = 8.0 * values / (fetch[cal][1] * 1024.0)
    w_scale = 4.0 * values / (write[cal][1] * 1024.0)
    rel = lambda q: os.path.relpath(q)   # paths as seen from the repository root
    rows = [f"# HBM traffic of the sweep kernels: {cfg['workload']}",
            f"# command: bash paper_2305_04397_amd/profile.sh {rel(os.path.dirname(os.path.abspath(fetch_dir)))}, then",
            f"#   python3 -m paper_2305_04397_amd.profile_summary traffic {rel(fetch_dir)} {rel(write_dir)} "
            f"{rel(bench_json)} <this file>",
            f"calibration_kernel: {cal} (values converted: N + 2R = {values})",
            f"fetch_scale: {f_scale:.4f}",
            f"write_scale: {w_scale:.4f}",
            f"kernel_source_sha256: {sources_hash()}",
            "dispatches,fetch_bytes_per_dispatch,write_bytes_per_dispatch,traffic_bytes_per_dispatch,kernel"]
    for k in sorted(fetch, key=lambda k: -fetch[k][1]):
        if "bellman" not in k or k not in write:
            continue
        n = fetch[k][0]
        fb = fetch[k][1] * 1024.0 * f_scale / n
        wb = write[k][1] * 1024.0 * w_scale / write[k][0]
        rows.append(f"{n},{fb:.6g},{wb:.6g},{fb + wb:.6g},{k}")
    text = "\n".join(rows) + "\n"
    with open(out_path, "w") as fh:
        fh.write(text)
    return text


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        print(traffic(*sys.argv[2:6]))
        sys.exit(0)
    d = sys.argv[1]
    text = summarize(d, "--delete-raw" in sys.argv)
    with open(os.path.join(d, "summary.txt"), "w") as fh:
        fh.write(text)
    print(text)
