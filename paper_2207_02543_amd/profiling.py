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
``python -m paper_2207_02543_amd.profiling run --workload W --kernel K
--out DIR`` drives rocprofv3 (as child processes) over ``bench.py`` for
that workload: one kernel trace, one FETCH_SIZE pass, one WRITE_SIZE pass
and the two calibration passes, and prints a report with the commands, the
trace summary, the kernel's counters, the calibration and a line
``traffic <workload> <kernel> <bytes per launch> source <digest>`` that
bench.py reads back while the library sources are unchanged.
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


# kernel name patterns of the timed kernels (bench.py --kernel)
KERNEL_PATTERNS = {
    "sweep": r"k_sweep<\d, \w+, false>",
    "sweep_final": r"k_sweep<\d, \w+, true>",
    "spmv_pq": r"k_spmv_pq<",
    "restrict": r"k_resid32<|k_restrict<",
    "prolong": r"k_prolong",
    "update": r"k_update<",
}
CALIB_BYTES = 256 * 2 ** 20   # one calibration copy reads and writes this much


def source_digest():
    """Digest of the sources of the iteration kernels (the ones the
    counters measure: solver.hip, the shared device helpers and the ABI
    header); assembly, setup and POD sources do not enter it."""
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    files = [os.path.join(here, "csrc", "solver.hip"), os.path.join(here, "csrc", "common.hpp"),
             os.path.join(os.path.dirname(here), "include", "pod2g.h")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def per_dispatch(path, pattern, counter):
    """Mean per-dispatch value of `counter` over the marked region's
    dispatches whose kernel name matches `pattern`."""
    import re
    rows = list(csv.DictReader(open(path)))
    ids = {r["Dispatch_Id"] for r in _region([{"Dispatch_Id": r["Dispatch_Id"],
                                               "Kernel_Name": r["Kernel_Name"]} for r in rows])}
    v = [float(r["Counter_Value"]) for r in rows
         if r["Dispatch_Id"] in ids and r["Counter_Name"] == counter
         and re.search(pattern, r["Kernel_Name"])]
    return (sum(v) / len(v), len(v)) if v else (float("nan"), 0)


def run(workload, kernel, out, steps, extra, trace_only=False):
    """Profile bench.py on one workload (see the module docstring)."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    bench = [sys.executable, os.path.join(root, "bench.py"), "--workload", workload,
             "--steps", str(steps), "--warmup", "1", "--no-cpu-baseline", "--markers",
             "--kernel", kernel] + extra
    calib_cmd = [sys.executable, "-m", "paper_2207_02543_amd.profiling", "calib"]
    env = dict(os.environ, TMPDIR="/tmp", PYTHONPATH=root)
    out = os.path.abspath(out)   # the profiler runs from /tmp
    os.makedirs(out, exist_ok=True)
    cmds = []

    def prof(args, prog, sub, limit):
        d = os.path.join(out, sub)
        cmd = ["rocprofv3"] + args + ["--output-format", "csv", "-d", d, "-o", "p", "--"] + prog
        cmds.append(" ".join(cmd))
        print(f"[profiling] {sub}", file=sys.stderr, flush=True)
        subprocess.run(cmd, check=True, env=env, cwd="/tmp", timeout=limit)
        return d

    pat = KERNEL_PATTERNS[kernel]
    t = prof(["--kernel-trace"], bench, "trace", 900)
    if trace_only:
        lines = [f"# rocprofv3 kernel trace: workload {workload}",
                 "# commands (run from /tmp with TMPDIR=/tmp, PYTHONPATH=<repo>):"]
        lines += [f"#   {c}" for c in cmds]
        lines += ["", "## kernel trace of the timed region (between the markers)",
                  trace_summary(os.path.join(t, "p_kernel_trace.csv"))]
        return "\n".join(lines)
    f = prof(["--pmc", "FETCH_SIZE", "--kernel-include-regex", f"{pat}|k_mark"], bench, "fetch", 900)
    w = prof(["--pmc", "WRITE_SIZE", "--kernel-include-regex", f"{pat}|k_mark"], bench, "write", 900)
    cf = prof(["--pmc", "FETCH_SIZE"], calib_cmd, "calib_fetch", 120)
    cw = prof(["--pmc", "WRITE_SIZE"], calib_cmd, "calib_write", 120)
    fetch, nf = per_dispatch(os.path.join(f, "p_counter_collection.csv"), pat, "FETCH_SIZE")
    write, nw = per_dispatch(os.path.join(w, "p_counter_collection.csv"), pat, "WRITE_SIZE")
    cfe, _ = per_dispatch(os.path.join(cf, "p_counter_collection.csv"), ".", "FETCH_SIZE")
    cwr, _ = per_dispatch(os.path.join(cw, "p_counter_collection.csv"), ".", "WRITE_SIZE")
    kf, kw = CALIB_BYTES / (cfe * 1024), CALIB_BYTES / (cwr * 1024)
    traffic = fetch * 1024 * kf + write * 1024 * kw
    lines = [f"# rocprofv3 summary: kernel {kernel} ({pat}), workload {workload}",
             "# commands (run from /tmp with TMPDIR=/tmp, PYTHONPATH=<repo>):"]
    lines += [f"#   {c}" for c in cmds]
    lines += ["", "## kernel trace of the timed steps (between the markers)",
              trace_summary(os.path.join(t, "p_kernel_trace.csv")), "",
              "## counters of the timed steps, mean per dispatch (KiB)",
              f"FETCH_SIZE {fetch:.1f} over {nf} dispatches",
              f"WRITE_SIZE {write:.1f} over {nw} dispatches", "",
              f"## calibration: {CALIB_BYTES} B copies read FETCH_SIZE {cfe:.1f} KiB and write "
              f"WRITE_SIZE {cwr:.1f} KiB per dispatch",
              f"bytes per FETCH_SIZE KiB {kf * 1024:.1f}; bytes per WRITE_SIZE KiB {kw * 1024:.1f}", "",
              f"traffic {workload} {kernel} {traffic:.0f} source {source_digest()}"]
    return "\n".join(lines)


def traffic_lookup(profiles_dir, workload, kernel):
    """HBM bytes per launch from a committed report, if the library sources
    are the ones the counters were taken with; else None."""
    import glob
    import os
    digest = source_digest()
    for path in sorted(glob.glob(os.path.join(profiles_dir, "*.txt"))):
        for line in open(path):
            p = line.split()
            if len(p) == 6 and p[0] == "traffic" and p[1] == workload and p[2] == kernel \
                    and p[4] == "source" and p[5] == digest:
                return float(p[3])
    return None


if __name__ == "__main__":
    kind = sys.argv[1]
    if kind == "calib":
        calib()
    elif kind == "run":
        import argparse
        ap = argparse.ArgumentParser()
        ap.add_argument("run")
        ap.add_argument("--workload", required=True)
        ap.add_argument("--kernel", default="sweep")
        ap.add_argument("--out", required=True)
        ap.add_argument("--steps", type=int, default=2)
        ap.add_argument("--trace-only", action="store_true")
        a, extra = ap.parse_known_args()
        print(run(a.workload, a.kernel, a.out, a.steps, extra, a.trace_only))
    else:
        path = sys.argv[2]
        print(trace_summary(path) if kind == "trace" else counter_summary(path))
