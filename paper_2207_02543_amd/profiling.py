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
``python -m paper_2207_02543_amd.profiling run --workload W --out DIR``
drives rocprofv3 (as child processes) over ``bench.py`` for that workload:
one kernel trace, one FETCH_SIZE pass and one WRITE_SIZE pass over every
iteration and setup kernel, one pass of MFMA counters over the batched
products (batched FP32 workloads) and the two calibration passes.  The
offline basis is computed once, outside the profiler, and loaded by every
pass; the counter passes run the launch parameters the traced run tuned.
It prints a report with the commands, the trace summary, per kernel the
counter traffic against the algorithmic bytes (``roofline``), the MFMA
counters, and one line ``traffic <workload> <kernel> <bytes per launch>
source <digest>`` per kernel that bench.py reads back while the library
sources are unchanged.
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
    out.append(idle_summary(rows))
    return "\n".join(out)


def idle_summary(rows):
    """Where the device had no kernel running inside the region: wall time
    from the first start to the last end, busy time (union of the kernels'
    intervals) and the idle gaps between them; gaps above 20 us are counted
    apart (the host's turn between captured chunks)."""
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    if not iv:
        return "## idle: no dispatches in the region"
    busy, gaps, cur_s, cur_e = 0, [], iv[0][0], iv[0][1]
    for s, e in iv[1:]:
        if s > cur_e:
            busy += cur_e - cur_s
            gaps.append((s - cur_e) / 1e3)
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    busy += cur_e - cur_s
    wall = (cur_e - iv[0][0]) / 1e3
    gaps.sort()
    big = [g for g in gaps if g > 20.0]
    small = [g for g in gaps if g <= 20.0]
    med = small[len(small) // 2] if small else 0.0
    return (f"## idle: wall {wall / 1e3:.2f} ms, kernels busy {busy / 1e6:.2f} ms "
            f"({busy / 1e3 / wall:.1%}); {len(small)} gaps <= 20 us total "
            f"{sum(small) / 1e3:.2f} ms (median {med:.2f} us); {len(big)} gaps > 20 us "
            f"total {sum(big) / 1e3:.2f} ms")


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


from .roofline import KERNEL_PATTERNS  # noqa: E402  (kernel key -> name pattern)

CALIB_BYTES = 256 * 2 ** 20   # one calibration copy reads and writes this much
# counters of the batched MFMA products' pass (rocprofv3 --pmc; one pass
# holds at most 8 SQ counters)
MFMA_COUNTERS = ["SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_F32",
                 "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAVES", "GRBM_GUI_ACTIVE"]


def available(names):
    """The counters of `names` that this GPU's profiler lists (rocprofv3 -L)."""
    import subprocess
    try:
        txt = subprocess.run(["rocprofv3", "-L"], capture_output=True, text=True,
                             timeout=120).stdout
    except (subprocess.SubprocessError, OSError):
        return list(names)
    import re
    have = set(re.findall(r"\b[A-Z][A-Z0-9_]+\b", txt))
    return [c for c in names if c in have] or list(names)


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


def trace_means(path):
    """Mean duration (us) and count per kernel key over the marked region."""
    import re
    rows = _region(list(csv.DictReader(open(path))))
    out = {}
    for key, pat in KERNEL_PATTERNS.items():
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
             if re.search(pat, r["Kernel_Name"])]
        if d:
            out[key] = (sum(d) / len(d), len(d))
    return out


def run(workload, out, steps, extra, trace_only=False, mfma=True):
    """Profile bench.py on one workload (see the module docstring): a kernel
    trace, FETCH_SIZE and WRITE_SIZE passes over every iteration and setup
    kernel, a pass of MFMA counters (batched workloads) and the two
    calibration copies; returns the report text."""
    import os
    import shlex
    import subprocess
    from . import inputs as I, roofline as R
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = os.path.abspath(out)   # the profiler runs from /tmp
    os.makedirs(out, exist_ok=True)
    # raw profiler output (large) under /tmp; progress logs under `out`
    raw = os.path.join("/tmp", "pod2g_prof_" + os.path.basename(out))
    basis = os.path.join("/tmp", f"pod2g_basis_{workload}.pt")
    serving = workload == "c4"     # the served stream: trace only, no basis file
    if serving:
        trace_only = True
        bench = [sys.executable, os.path.join(root, "bench.py"), "--workload", workload,
                 "--markers"] + extra
    else:
        bench = [sys.executable, os.path.join(root, "bench.py"), "--workload", workload,
                 "--steps", str(steps), "--warmup", "1", "--no-cpu-baseline", "--markers",
                 "--compare-plain", "0", "--basis-file", basis] + extra
    calib_cmd = [sys.executable, "-m", "paper_2207_02543_amd.profiling", "calib"]
    env = dict(os.environ, TMPDIR="/tmp", PYTHONPATH=root)
    cmds = []

    def prof(args, prog, sub, limit):
        d = os.path.join(raw, sub)
        cmd = ["rocprofv3"] + args + ["--output-format", "csv", "-d", d, "-o", "p", "--"] + prog
        cmds.append(shlex.join(cmd))
        print(f"[profiling] {sub}", file=sys.stderr, flush=True)
        so = os.path.join(out, f"{sub}_stdout.txt")
        with open(os.path.join(out, f"{sub}_stderr.txt"), "w") as err, open(so, "w") as sout:
            rc = subprocess.run(cmd, env=env, cwd="/tmp", timeout=limit, stderr=err,
                                stdout=sout).returncode
        if rc != 0:
            # the profiler can crash in its own teardown after the program
            # has finished: accept the run only when the program's result
            # line was printed and the profiler's tables were written
            with open(so) as fh:
                done = any(ln.startswith('{"metric"') for ln in fh)
            tables = [x for x in (os.listdir(d) if os.path.isdir(d) else [])
                      if x.endswith(".csv") and os.path.getsize(os.path.join(d, x)) > 0]
            if rc not in (-11, 139) or not done or not tables:
                raise subprocess.CalledProcessError(rc, cmd)
            print(f"[profiling] {sub}: profiler ended with status {rc} after the program "
                  f"finished; {len(tables)} result tables written", file=sys.stderr, flush=True)
        return d

    if not serving and not os.path.exists(basis):
        # the offline phase once, outside the profiler
        prep = bench[:2] + ["--workload", workload, "--steps", "1", "--warmup", "0",
                            "--no-cpu-baseline", "--compare-plain", "0", "--basis-file", basis]
        cmds.append(shlex.join(prep))
        print("[profiling] offline basis", file=sys.stderr, flush=True)
        with open(os.path.join(out, "prep_stderr.txt"), "w") as err, \
                open(os.path.join(out, "prep_stdout.txt"), "w") as sout:
            subprocess.run(prep, check=True, env=env, timeout=1200, stderr=err, stdout=sout)
    allpat = "|".join(KERNEL_PATTERNS.values()) + "|k_mark"
    t = prof(["--kernel-trace"], bench, "trace", 900)
    # the counter passes run the launch parameters the traced run tuned
    tuning = _tuning_from(os.path.join(out, "trace_stderr.txt"))
    if tuning is not None:
        import json
        bench = bench + ["--tuning", json.dumps(tuning)]
    tfile = os.path.join(t, "p_kernel_trace.csv")
    head = [f"# rocprofv3 summary: workload {workload}, every iteration and setup kernel",
            "# made by (from the repository root, on the GPU machine): python -m "
            "paper_2207_02543_amd.profiling " + shlex.join(sys.argv[1:]),
            "# commands (run from /tmp with TMPDIR=/tmp, PYTHONPATH=<repo>; the first run",
            "# computes the offline basis and stores it in the --basis-file, the others load it):"]
    if trace_only:
        lines = head + [f"#   {c}" for c in cmds]
        lines += ["", "## kernel trace of the timed region (between the markers)",
                  trace_summary(tfile)]
        return "\n".join(lines)
    f = prof(["--pmc", "FETCH_SIZE", "--kernel-include-regex", allpat], bench, "fetch", 900)
    wr = prof(["--pmc", "WRITE_SIZE", "--kernel-include-regex", allpat], bench, "write", 900)
    w = I.WORKLOADS[workload]
    m, mnote = None, ""
    if mfma and w.precision == "mixed" and w.batch >= 4:
        names = available(MFMA_COUNTERS)
        try:
            m = prof(["--pmc"] + names + ["--kernel-include-regex",
                                          r"k_ptr_b[<(]|k_prolong_b\(|k_mark"],
                     bench, "mfma", 900)
        except (subprocess.SubprocessError, OSError) as e:
            mnote = f"MFMA counter pass failed ({names}): {e}"
    cf = prof(["--pmc", "FETCH_SIZE"], calib_cmd, "calib_fetch", 120)
    cw = prof(["--pmc", "WRITE_SIZE"], calib_cmd, "calib_write", 120)
    cfe, _ = per_dispatch(os.path.join(cf, "p_counter_collection.csv"), ".", "FETCH_SIZE")
    cwr, _ = per_dispatch(os.path.join(cw, "p_counter_collection.csv"), ".", "WRITE_SIZE")
    kf, kw = CALIB_BYTES / (cfe * 1024), CALIB_BYTES / (cwr * 1024)
    tm = trace_means(tfile)
    lines = head + [f"#   {c}" for c in cmds]
    lines += ["", "## kernel trace of the timed steps (between the markers)", trace_summary(tfile), "",
              f"## calibration: {CALIB_BYTES} B copies read FETCH_SIZE {cfe:.1f} KiB and write "
              f"WRITE_SIZE {cwr:.1f} KiB per dispatch",
              f"bytes per FETCH_SIZE KiB {kf * 1024:.1f}; bytes per WRITE_SIZE KiB {kw * 1024:.1f}", "",
              "## per kernel, mean per dispatch: counter traffic (FETCH_SIZE + WRITE_SIZE, "
              "calibrated) against the algorithmic bytes, and the algorithmic rate",
              "kernel        calls   mean_us   algo_MB   fetch_MB   write_MB   traffic/algo   "
              "algo_GB/s   of_8TB/s"]
    traffic_lines = []
    for key, pat in KERNEL_PATTERNS.items():
        fe, nf = per_dispatch(os.path.join(f, "p_counter_collection.csv"), pat, "FETCH_SIZE")
        wb, nw = per_dispatch(os.path.join(wr, "p_counter_collection.csv"), pat, "WRITE_SIZE")
        if key not in tm or not nf:
            continue
        us, cnt = tm[key]
        algo = R.kernel_bytes(w, key, tuning)
        fb, wbb = fe * 1024 * kf, wb * 1024 * kw
        rate = algo / (us * 1e-6) / 1e9
        lines.append(f"{key:12s} {cnt:6d} {us:9.1f} {algo / 1e6:9.1f} {fb / 1e6:10.1f} "
                     f"{wbb / 1e6:10.1f} {(fb + wbb) / algo:14.3f} {rate:11.0f} "
                     f"{rate / R.HBM_PEAK_GBS:10.3f}")
        traffic_lines.append(f"traffic {workload} {key} {fb + wbb:.0f} source {source_digest()}")
    if m is not None:
        lines += ["", "## MFMA counters of the batched products, mean per dispatch",
                  counter_summary(os.path.join(m, "p_counter_collection.csv"))]
    elif mnote:
        lines += ["", "## " + mnote]
    lines += ["", f"## launch parameters of the plan: {tuning}", ""] + traffic_lines
    return "\n".join(lines)


def _tuning_from(path):
    """The plan's launch parameters as bench.py logged them (None if absent)."""
    import ast
    import os
    if not os.path.exists(path):
        return None
    for line in open(path):
        if "[bench] launch parameters:" in line:
            return ast.literal_eval(line.split("launch parameters:", 1)[1].split("  (+")[0].strip())
    return None


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
        ap.add_argument("--out", required=True)
        ap.add_argument("--steps", type=int, default=1)
        ap.add_argument("--trace-only", action="store_true")
        ap.add_argument("--no-mfma", action="store_true")
        a, extra = ap.parse_known_args()
        print(run(a.workload, a.out, a.steps, extra, a.trace_only, not a.no_mfma))
    else:
        path = sys.argv[2]
        print(trace_summary(path) if kind == "trace" else counter_summary(path))
