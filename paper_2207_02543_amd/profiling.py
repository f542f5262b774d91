"""Summaries of rocprofv3 output for the regions that ``pod2g_mark`` brackets.

``python -m paper_2207_02543_amd.profiling trace <kernel_trace.csv>`` prints,
for the dispatches between the last ``k_mark_begin`` and the next
``k_mark_end``, each kernel's launch count and mean/min/max duration.
``python -m paper_2207_02543_amd.profiling counters <counter_collection.csv>``
prints the mean per-dispatch value of every counter for each kernel in the
same region (rocprofv3 ``--pmc`` output).
``python -m paper_2207_02543_amd.profiling calib`` runs, between markers,
three plain device copies of 256 MiB (torch ``copy_``): the reference that
scales the FETCH_SIZE / WRITE_SIZE counters to bytes.
"""
from __future__ import annotations

import collections
import csv
import sys


def _region(rows, key="Dispatch_Id"):
    rows = sorted(rows, key=lambda r: int(r[key]))
    begins = [i for i, r in enumerate(rows) if "k_mark_begin" in r["Kernel_Name"]]
    if not begins:
        return rows
    b = begins[-1]
    ends = [i for i, r in enumerate(rows) if i > b and "k_mark_end" in r["Kernel_Name"]]
    e = ends[0] if ends else len(rows)
    return rows[b + 1:e]


def trace_summary(path):
    rows = _region(list(csv.DictReader(open(path))))
    agg = collections.defaultdict(list)
    for r in rows:
        agg[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["calls  mean_us  min_us  max_us  total_us  kernel"]
    for name, d in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{len(d):5d} {sum(d) / len(d):8.2f} {min(d):7.2f} {max(d):7.2f} "
                   f"{sum(d):9.0f}  {name}")
    return "\n".join(out)


def counter_summary(path):
    rows = list(csv.DictReader(open(path)))
    ids = _region([{"Dispatch_Id": r["Dispatch_Id"], "Kernel_Name": r["Kernel_Name"]}
                   for r in rows])
    keep = {r["Dispatch_Id"] for r in ids}
    agg = collections.defaultdict(list)
    for r in rows:
        if r["Dispatch_Id"] in keep:
            agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    out = ["dispatches  mean_per_dispatch  counter  kernel"]
    for (name, cn), v in sorted(agg.items()):
        out.append(f"{len(v):5d} {sum(v) / len(v):16.1f}  {cn}  {name}")
    return "\n".join(out)


def calib(mib=256, reps=3):
    import torch
    from . import capi
    src = torch.ones(mib * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    capi.check(capi.pod2g_mark(0), "pod2g_mark")
    for _ in range(reps):
        dst.copy_(src)
    capi.check(capi.pod2g_mark(1), "pod2g_mark")
    torch.cuda.synchronize()
    print(f"copied {reps} x {mib} MiB")


if __name__ == "__main__":
    kind = sys.argv[1]
    if kind == "calib":
        calib()
    else:
        path = sys.argv[2]
        print(trace_summary(path) if kind == "trace" else counter_summary(path))
