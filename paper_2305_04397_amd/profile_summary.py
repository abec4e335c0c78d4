"""Reduce rocprofv3 CSV output to short per-kernel tables.

    python -m paper_2305_04397_amd.profile_summary <rocprofv3 output dir> [--delete-raw]

Kernel traces: per-kernel calls, total and average duration (from
*_kernel_stats.csv).  Counter runs: per-kernel dispatch count and the mean of
every counter per dispatch (from *_counter_collection.csv).  With
--delete-raw the per-dispatch CSV files are removed afterwards.
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
        out.append(f"# counters per dispatch, mean ({os.path.basename(f)})")
        out.append("dispatches," + ",".join(counters) + ",kernel")
        for k in sorted(acc, key=lambda k: -len(disp[k])):
            n = len(disp[k])
            out.append(f"{n}," + ",".join(f"{acc[k][c] / n:.6g}" for c in counters) + f",{k}")
    text = "\n".join(out) + "\n"
    if delete_raw:
        for pat in ("*_kernel_trace.csv", "*_counter_collection.csv", "*_results.db", "*.rocpd"):
            for f in glob.glob(os.path.join(d, "**", pat), recursive=True):
                os.remove(f)
    return text


if __name__ == "__main__":
    d = sys.argv[1]
    text = summarize(d, "--delete-raw" in sys.argv)
    with open(os.path.join(d, "summary.txt"), "w") as fh:
        fh.write(text)
    print(text)
