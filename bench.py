#!/usr/bin/env python3
"""Throughput of the POD-2G preconditioned CG path on one MI355X.

A step is one pass of the online hot path over one batch of query
parameters: assembly of K(theta), f and D^-1; the preconditioner setup
(K P, P^T K P, Cholesky); and the warm-started PCG solve to
||f - K u|| <= tol ||f||.  The offline phase (training solves, POD basis)
and the exact solutions behind the warm starts run before timing; all
inputs are resident on the GPU when the timed region starts.

Prints one JSON line (stdout); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("POD-2G-PCG solves/sec at rel-residual 1e-8 (batched/mixed vs plain); "
          "SpMV HBM GB/s")
# kernels the library can time live (pod2g_timer)
KERNELS = {"spmv_pq": 1, "sweep": 2, "sweep_final": 3, "restrict": 4, "prolong": 5, "update": 6}


T_START = time.perf_counter()


def log(msg):
    print(f"{msg}  (+{time.perf_counter() - T_START:.0f} s)", file=sys.stderr, flush=True)


# the kernel with the largest share of a step's time on each workload
# (rocprofv3 kernel traces of the timed steps)
DOMINANT = {"c1": "restrict", "c2": "restrict", "c4a": "restrict", "c4b": "restrict",
            "c3": "spmv_pq", "c4c": "spmv_pq", "c5": "spmv_pq"}


def plain_baseline(prob, P, xi_d, x0, ustar, count, chunk, sample64=None):
    """The one-solve-at-a-time FP64 path on the same queries: assembly,
    FP64 setup and a captured FP64 PCG per query (batch 1).  With the
    oracle's FP64 iterate of query 0 after m iterations (sample64), the
    same path is stopped after m iterations from the same warm start and
    the two iterates are compared."""
    import numpy as np
    import torch
    from paper_2207_02543_amd import capi as L
    w = prob.w
    sysm = prob.alloc_system(1)
    u = torch.empty(1, w.n, dtype=torch.float64, device=xi_d.device)
    sysm.xi.copy_(xi_d[:1])
    prob.assemble(sysm)
    prec0 = prob.setup(sysm, P, key="setup_plain")
    plan = prob.plan(sysm, prec0, u, chunk=chunk, key="pcg_plain")
    iters, errs = [], []

    def one(j):
        sysm.xi.copy_(xi_d[j:j + 1])
        prob.assemble(sysm)
        prob.setup(sysm, P, key="setup_plain")
        u.copy_(x0[j:j + 1])
        ret, its, rr, st = plan.solve(w.tol, beta=L.BETA_FR)
        if ret != L.OK:
            raise L.Pod2gError(ret, f"plain solve {j}: {st}")
        return its[0]

    one(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(count):
        iters.append(one(j))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for j in [count - 1]:
        errs.append(float(torch.linalg.norm(u[0] - ustar[j]) / torch.linalg.norm(ustar[j])))
    out = {"value": count / dt, "unit": "solves/s", "solves": count,
           "iters_mean": float(np.mean(iters)), "err_vs_fp64_last": errs[0],
           "path": "FP64 cycle and PCG, one query per solve (batch 1), captured chunks"}
    if sample64 is not None:
        m = int(sample64["iters"])
        sysm.xi.copy_(xi_d[:1])
        prob.assemble(sysm)
        prob.setup(sysm, P, key="setup_plain")
        u.copy_(x0[:1])
        ret, its, rr, st = plan.solve(w.tol, maxit=m, beta=L.BETA_FR)
        ug, ur, x00 = u[0].cpu().numpy(), sample64["u"], x0[0].cpu().numpy()
        d = float(np.linalg.norm(ug - ur))
        out["oracle_iterate"] = {"iters_gpu": int(its[0]), "iters_oracle": m,
                                 "rel_diff": d / float(np.linalg.norm(ur)),
                                 "rel_diff_of_correction": d / float(np.linalg.norm(ur - x00))}
    plan.close()
    return out


# ---- CPU baseline: the oracle on the host's cores ------------------------------
# The oracle runs in a child process started before this process touches the
# GPU.  It assembles the first query's K while the GPU runs the offline phase,
# then receives the basis and warm starts, and finishes before the timed GPU
# steps begin, so the two never run at the same time.

def host_cpu():
    """(model name, usable cores) of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    # a host shared by several GPUs gives each a share of its cores, stated
    # in OMP_NUM_THREADS
    share = os.environ.get("OMP_NUM_THREADS", "")
    if share.isdigit() and int(share) > 0:
        cores = min(cores, int(share))
    return model, cores


def _oracle_leg(conn, wname, overrides, nq, seconds, full_max_n, sample_iters):
    """Child process: times the oracle's online phase for the queries of
    workload `wname` on 1 host thread and on every usable core.  Queries are
    solved in full while the time bound allows (n <= full_max_n); larger
    workloads time assembly, setup and `sample_iters` PCG iterations of one
    query, from which the parent extrapolates."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fem, pcg as opcg, problem as oprob, twogrid
    from paper_2207_02543_amd import inputs as I

    w = I.with_(I.WORKLOADS[wname], **overrides)
    _, cores = host_cpu()
    xis = I.query_xis(w, nq)
    mixed = w.precision == "mixed"
    # assembly of the first query on 1 thread and on every core, before the
    # basis arrives (the GPU's offline phase runs meanwhile)
    t_asm0 = {}
    for threads in sorted({1, cores}):
        t = time.perf_counter()
        with threadpool_limits(limits=threads):
            K0 = oprob.stiffness(w, xis[0])
        t_asm0[threads] = time.perf_counter() - t
    f = fem.traction_load(w.dim, w.N)
    msg = conn.recv()
    if msg is None:
        return
    P, x0s = msg["P"], msg["x0"]
    out = {"cores": cores, "runs": {}}

    def setup(K):
        return twogrid.TwoGrid(K, P, w.omega, w.nu_pre, w.nu_post,
                               precision="fp32" if mixed else "fp64")

    beta = "pr" if mixed else "fr"
    for threads in sorted({1, cores}):
        run = {"threads": threads}
        with threadpool_limits(limits=threads):
            if w.n <= full_max_n:
                sols, iters, t_total, j = [], [], 0.0, 0
                while j < len(x0s) and (t_total < seconds or j == 0):
                    t = time.perf_counter()
                    K = K0 if j == 0 else oprob.stiffness(w, xis[j])
                    M = setup(K)
                    r = opcg.pcg(K, f, x0s[j], M, tol=w.tol, maxit=5000, beta=beta)
                    dt = time.perf_counter() - t + (t_asm0[threads] if j == 0 else 0.0)
                    t_total += dt
                    iters.append(r.iters)
                    if threads == 1:
                        sols.append(r.u)
                    j += 1
                    print(f"[bench] oracle ({threads} thread{'s' * (threads > 1)}) solve {j}: "
                          f"{r.iters} iterations, {t_total:.1f} s so far", file=sys.stderr, flush=True)
                run.update(kind="full", solves=j, seconds=t_total, iters=iters)
                if threads == 1:
                    out["solutions"] = np.stack(sols)
            else:
                K, t_asm = K0, t_asm0[threads]
                t = time.perf_counter()
                M = setup(K)
                t_setup = time.perf_counter() - t
                t = time.perf_counter()
                r = opcg.pcg(K, f, x0s[0], M, tol=w.tol, maxit=sample_iters, beta=beta)
                t_iter = (time.perf_counter() - t) / max(1, r.iters)
                run.update(kind="sampled", t_assembly=t_asm, t_setup=t_setup, t_iter=t_iter,
                           iters=r.iters)
                if threads == 1:
                    # the iterate after the sampled iterations, for the parity
                    # checks, and the FP64 method's (the plain path's) beside it
                    out["iterate"] = {"u": r.u, "iters": r.iters}
                    if mixed:
                        M64 = twogrid.TwoGrid(K, P, w.omega, w.nu_pre, w.nu_post, precision="fp64")
                        r64 = opcg.pcg(K, f, x0s[0], M64, tol=w.tol, maxit=sample_iters, beta="fr")
                        out["iterate64"] = {"u": r64.u, "iters": r64.iters}
                    else:
                        out["iterate64"] = out["iterate"]
                print(f"[bench] oracle ({threads} thread{'s' * (threads > 1)}): assembly "
                      f"{t_asm:.1f} s, setup {t_setup:.1f} s, {t_iter:.2f} s per PCG iteration "
                      f"({r.iters} timed)", file=sys.stderr, flush=True)
        out["runs"][threads] = run
    conn.send(out)


class OracleLeg:
    """Parent side of the CPU baseline (see _oracle_leg)."""

    FULL_MAX_N = 1_000_000   # above this one oracle solve takes minutes: sample it

    def __init__(self, w, nq, seconds, sample_iters=4):
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        self.w = w
        self.conn, child = ctx.Pipe()
        overrides = {f: getattr(w, f) for f in ("batch", "precision", "tol")}
        self.proc = ctx.Process(target=_oracle_leg, daemon=True,
                                args=(child, w.name, overrides, nq, seconds, self.FULL_MAX_N,
                                      sample_iters))
        self.proc.start()
        self.sender = None
        self.result = None

    def send(self, P_kn, x0s):
        """Hand the basis ([k, n] device) and warm starts ([Q, n]) to the
        child; a helper thread writes them, since the child reads them only
        once its first assembly is done."""
        import threading
        import numpy as np
        msg = {"P": np.ascontiguousarray(P_kn.cpu().numpy().T), "x0": x0s.cpu().numpy()}
        self.sender = threading.Thread(target=self.conn.send, args=(msg,), daemon=True)
        self.sender.start()

    def wait(self, timeout=1800):
        t = time.perf_counter()
        if self.conn.poll(timeout):
            self.result = self.conn.recv()
        self.proc.join(10)
        self.close()
        return time.perf_counter() - t

    def close(self):
        if self.proc.is_alive():
            if self.sender is None:
                try:
                    self.conn.send(None)
                except OSError:
                    pass
            self.proc.join(5)
            if self.proc.is_alive():
                self.proc.kill()

    def iterate(self, fp64=False):
        """The oracle's iterate of query 0 after the sampled iterations
        (sampled runs; fp64: the FP64 method's), or None."""
        return None if self.result is None else self.result.get("iterate64" if fp64 else "iterate")

    def summary(self, gpu_iters_mean):
        """The cpu_baseline entry: solves/s on every usable core, with the
        one-thread figure beside it; sampled runs are extrapolated to the
        GPU's mean iteration count (labelled as such)."""
        res = self.result
        if res is None:
            return {"value": None, "unit": "solves/s", "cores": None, "kind": "oracle",
                    "sample": "oracle leg did not finish"}
        model, _ = host_cpu()
        vals, desc = {}, []
        for threads, run in sorted(res["runs"].items()):
            if run["kind"] == "full":
                vals[threads] = run["solves"] / run["seconds"]
                desc.append(f"{run['solves']} query solve(s) on {threads} thread(s) in "
                            f"{run['seconds']:.1f} s (oracle iterations {run['iters']})")
            else:
                per = run["t_assembly"] + run["t_setup"] + gpu_iters_mean * run["t_iter"]
                vals[threads] = 1.0 / per
                desc.append(f"{threads} thread(s): assembly {run['t_assembly']:.1f} s + setup "
                            f"{run['t_setup']:.1f} s + {run['t_iter']:.2f} s per PCG iteration "
                            f"(over {run['iters']} iterations) x {gpu_iters_mean:.0f} iterations")
        cores = max(vals)
        sampled = any(r["kind"] == "sampled" for r in res["runs"].values())
        return {"value": vals[cores], "unit": "solves/s", "cores": cores, "kind": "oracle",
                "sample": (f"workload {self.w.name}, assembly + two-grid setup + PCG per query: "
                           + "; ".join(desc)
                           + ("; extrapolated from the timed phases to the GPU's mean iteration "
                              "count (one full oracle solve exceeds the bounded sample)"
                              if sampled else "")),
                "value_1thread": vals.get(1), "threads": cores, "cpu_model": model,
                "extrapolated": sampled}

    def solutions(self):
        return None if self.result is None else self.result.get("solutions")


def serve_bench(args):
    """Serving workload: Poisson arrivals over three problem classes, each
    with its own basis; continuous batching through the library server."""
    import numpy as np
    import torch
    from paper_2207_02543_amd import capi as L, inputs as I, pipeline, serve

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    names = ["c4a", "c4b", "c4c"]
    ws = [I.with_(I.WORKLOADS[nm], precision="mixed") for nm in names]
    free, total = torch.cuda.mem_get_info()
    slots = serve.plan_slots([(w, w.k, "mixed") for w in ws], int(free * args.hbm_fraction),
                             max_slots=args.max_slots)
    log(f"[serve] free HBM {free / 2**30:.1f} GiB of {total / 2**30:.1f}; slots per class {slots}")
    classes, pools = [], []
    for w, m in zip(ws, slots):
        prob = pipeline.Problem(w, dev)
        t0 = time.perf_counter()
        P, lam, U, its = pipeline.offline_basis(prob)
        del U, prob
        c = serve.ServedClass(w, P, m, precision="mixed")
        pools.append(serve.make_pool(c, args.queries))
        classes.append(c)
        torch.cuda.synchronize()
        log(f"[serve] class {w.name}: n {w.n}, k {w.k}, {m} slots, offline + pool "
            f"{time.perf_counter() - t0:.1f} s")
    chunk = args.chunk if args.chunk > 0 else 8
    shares = None
    if args.cu_split and args.cu_split != "none":
        shares = [int(x) for x in args.cu_split.split(",")]
        if len(shares) != len(classes) or sum(shares) > torch.cuda.get_device_properties(dev).multi_processor_count:
            raise ValueError(f"--cu-split {args.cu_split}: one share per class, within the GPU")
    # solo latency of each class on the whole GPU, the reference of the
    # stream's latencies
    srv0 = serve.Server(classes, chunk=chunk)
    solo_whole = serve.solo_latency(srv0, pools, rtol=1e-8)
    srv0.close()
    log(f"[serve] solo latency per class on the whole GPU (ms): "
        f"{dict(zip(names, [round(x, 1) for x in solo_whole]))}")
    srv = serve.Server(classes, chunk=chunk, cu_shares=shares)
    # warm-up: every class, every slot once, queued at t = 0
    nw = sum(slots)
    wc = np.array([i for i, m in enumerate(slots) for _ in range(m)])
    serve.run_stream(srv, pools, np.zeros(nw), wc, np.arange(nw) % args.queries, rtol=1e-8,
                     realtime=False)
    solo = serve.solo_latency(srv, pools, rtol=1e-8)
    log(f"[serve] solo latency per class on its share (ms): "
        f"{dict(zip(names, [round(x, 1) for x in solo]))}")
    times, cls, qidx = I.arrivals(args.rate, args.serve_seconds, len(ws), args.queries)
    log(f"[serve] {len(times)} requests over {args.serve_seconds:.0f} s at {args.rate:.0f}/s")
    if args.markers:
        L.check(L.pod2g_mark(0), "pod2g_mark")
    res = serve.run_stream(srv, pools, times, cls, qidx, rtol=1e-8, check_first=4,
                           max_queue=args.max_queue)
    if args.markers:
        L.check(L.pod2g_mark(1), "pod2g_mark")
        torch.cuda.synchronize()
    s = serve.summarize(res, names, solo, solo_whole)
    srv.close()
    log(f"[serve] {s['completed']} solves in {s['wall_s']:.1f} s ({s['refused']} refused); "
        f"p50 {s['p50_ms']:.1f} ms, p99 {s['p99_ms']:.1f} ms; {s['steps']} steps")
    result = {
        "metric": METRIC, "value": s["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": s["steps"], "warmup": nw, "ms_per_step": s["wall_s"] / max(1, s["steps"]) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "c4 serving: Poisson arrivals over c4a (2D 128x128), c4b (2D "
                               "256x256), c4c (3D 48x48x48), k=20 each, tol 1e-8",
                   "rate_per_s": args.rate, "duration_s": args.serve_seconds,
                   "slots": dict(zip(names, slots)), "graph_chunk": srv.chunk,
                   "cu_split": args.cu_split, "max_queue": args.max_queue,
                   "queries_per_class": args.queries},
        "serving": s,
        "roofline": None,
    }
    print(json.dumps(result), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5",
                    help="c1, c2, c3, c4a, c4b, c4c, c5; c4 = the serving stream")
    ap.add_argument("--queries", type=int, default=8, help="distinct query parameters cycled")
    ap.add_argument("--kernel", default=None, choices=sorted(KERNELS),
                    help="kernel timed live for the roofline entry (default: the workload's "
                         "dominant kernel)")
    ap.add_argument("--compare-plain", type=int, default=None,
                    help="batched workloads: also time this many one-at-a-time FP64 solves "
                         "(default 4 for batched workloads, 0 to skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunk", type=int, default=8,
                    help="PCG iterations per captured graph launch (0: no graph, eager launches)")
    ap.add_argument("--markers", action="store_true",
                    help="launch the k_mark_begin / k_mark_end kernels around the timed steps "
                         "(for cutting a rocprofv3 trace to them)")
    ap.add_argument("--basis-file", default=None,
                    help="load the offline basis from this file if it exists, else compute it "
                         "and save it there (for repeated runs of one workload, e.g. profiling "
                         "passes)")
    ap.add_argument("--tuning", default=None,
                    help="launch parameters as JSON (names as pcg_plan_config) instead of tuning")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch parameters (no timing of candidates)")
    ap.add_argument("--warm", default="noisy", choices=["noisy", "rom", "zero"],
                    help="initial guess: exact + 1%% noise (surrogate stand-in), the reduced-order "
                         "solution P K_c^-1 P^T f formed inside the step, or zero")
    ap.add_argument("--smoother", default="jacobi", choices=["jacobi", "sgs"],
                    help="relaxation of the cycle: damped Jacobi (the configurations') or "
                         "symmetric Gauss-Seidel in multicolour order")
    ap.add_argument("--solver", default="pcg", choices=["pcg", "stationary"],
                    help="PCG preconditioned by the cycle, or the cycle iterated on its own")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="serving: arrival window")
    ap.add_argument("--hbm-fraction", type=float, default=0.5,
                    help="serving: share of the free HBM given to resident queries")
    ap.add_argument("--max-slots", type=int, default=32, help="serving: slots per class at most")
    ap.add_argument("--max-queue", type=int, default=None,
                    help="serving: refuse a request when this many of its class already wait "
                         "for a slot (default: queue without bound)")
    ap.add_argument("--cu-split", default="32,64,160",
                    help="serving: compute units per class, comma-separated (c4a,c4b,c4c), each "
                         "class on its own share of the GPU; 'none': all classes on the whole GPU")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver "
              "shards over independent queries with no collectives; run one process per GPU.",
              file=sys.stderr)
        return 2

    if args.workload == "c4":
        return serve_bench(args)

    from paper_2207_02543_amd import inputs as I
    w = I.WORKLOADS[args.workload]
    # the oracle leg starts before this process touches the GPU
    leg = None if args.no_cpu_baseline else OracleLeg(w, max(args.queries, w.batch),
                                                      args.cpu_seconds)

    import numpy as np
    import torch
    from paper_2207_02543_amd import capi as L, pipeline, profiling, roofline as R

    mixed = w.precision == "mixed"
    if args.kernel is None:
        args.kernel = DOMINANT.get(w.name, "sweep")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] workload {w.name}: dim {w.dim} N {w.N} n {w.n} k {w.k} batch {w.batch} "
        f"{w.precision}")

    # ---- offline phase and query inputs (untimed) -----------------------------
    prob = pipeline.Problem(w, dev)
    t0 = time.perf_counter()
    Q = max(args.queries, w.batch)
    xis = I.query_xis(w, Q)
    if args.basis_file and os.path.exists(args.basis_file):
        saved = torch.load(args.basis_file, weights_only=True)
        P, ustar = saved["P"].to(dev), saved["ustar"].to(dev)
        if tuple(P.shape) != (w.k, w.n) or tuple(ustar.shape) != (Q, w.n):
            raise ValueError(f"{args.basis_file}: basis {tuple(P.shape)} and solutions "
                             f"{tuple(ustar.shape)}, expected {(w.k, w.n)} and {(Q, w.n)}")
        log(f"[bench] offline basis and query solutions loaded from {args.basis_file}")
    else:
        P, lam, U, train_iters = pipeline.offline_basis(prob,
                                                        progress=lambda m: log(f"[bench] {m}"))
        torch.cuda.synchronize()
        log(f"[bench] offline: {w.n_train} training solves ({sum(train_iters)} iterations) + POD "
            f"in {time.perf_counter() - t0:.1f} s; lambda_k/lambda_1 = "
            f"{float(lam[w.k - 1] / lam[0]):.2e}")
        del U
        t0 = time.perf_counter()
        ustar = pipeline.exact_solutions(prob, xis, P, rtol=1e-12)
        torch.cuda.synchronize()
        log(f"[bench] {Q} tight query solutions in {time.perf_counter() - t0:.1f} s")
        if args.basis_file:
            torch.save({"P": P.cpu(), "ustar": ustar.cpu()}, args.basis_file)
    t0 = time.perf_counter()
    g = torch.tensor(np.stack([I.noise(w, j) for j in range(Q)]), device=dev)
    x0 = torch.stack([I.warm_start(ustar[j], g[j], w.noise) for j in range(Q)])
    xi_d = torch.tensor(xis, device=dev)
    torch.cuda.synchronize()
    log(f"[bench] {Q} query warm starts in {time.perf_counter() - t0:.1f} s")
    if leg is not None:
        leg.send(P, x0)

    # ---- timed steps ------------------------------------------------------------
    sysm = prob.alloc_system(w.batch, fp32=mixed)
    u = torch.empty(w.batch, w.n, dtype=torch.float64, device=dev)
    precision = L.MIXED if mixed else L.FP64
    smoother = L.SMOOTHER_SGS if args.smoother == "sgs" else L.SMOOTHER_JACOBI
    timer = L.pod2g_timer_create(KERNELS[args.kernel], 6)
    stats = {"iters": [], "relres": [], "err": []}
    plan = None
    tuning = None
    plan_cfg = None
    if args.chunk > 0 and args.solver == "pcg":
        # capture the PCG iterations once: every step reuses these buffers
        sysm.xi.copy_(xi_d[:w.batch])
        prob.assemble(sysm)
        prec0 = prob.setup(sysm, P, precision=precision, smoother=smoother)
        plan = prob.plan(sysm, prec0, u, chunk=args.chunk, timer=timer)
        if args.tuning:
            plan.configure(**json.loads(args.tuning))
        elif not args.no_tune:
            tuning = plan.tune()
            log(f"[bench] tuned launch parameters: {tuning}")
        plan_cfg = plan.config()
        log(f"[bench] launch parameters: {plan_cfg}")

    def step(i, timed):
        idx = [(i * w.batch + b) % Q for b in range(w.batch)]
        sysm.xi.copy_(xi_d[idx])
        prob.assemble(sysm)
        prec = prob.setup(sysm, P, precision=precision, smoother=smoother)
        if args.warm == "noisy":
            u.copy_(x0[idx])
        elif args.warm == "rom":
            prob.rom_start(sysm, prec, u)
        else:
            u.zero_()
        if args.solver == "stationary":
            ret, its, rr, st = prob.stationary(sysm, prec, u, maxit=20000)
        elif plan is not None:
            ret, its, rr, st = plan.solve(w.tol)
        else:
            ret, its, rr, st = prob.solve(sysm, prec, u, timer=timer if timed else None)
        if ret != L.OK:
            raise L.Pod2gError(ret, f"step {i}: statuses {st}")
        return idx, its, rr

    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    if leg is not None:
        # the oracle leg finishes before the timed region: they never overlap
        waited = leg.wait()
        log(f"[bench] oracle leg done ({waited:.1f} s waited for it)")
    L.pod2g_timer_reset(timer)
    if args.markers:
        L.check(L.pod2g_mark(0), "pod2g_mark")
    t0 = time.perf_counter()
    for i in range(args.steps):
        idx, its, rr = step(args.warmup + i, True)
        stats["iters"] += its
        stats["relres"] += rr
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if args.markers:
        L.check(L.pod2g_mark(1), "pod2g_mark")
        torch.cuda.synchronize()
    # accuracy of the last step against the tight FP64 solutions
    for b, j in enumerate(idx):
        stats["err"].append(float(torch.linalg.norm(u[b] - ustar[j]) / torch.linalg.norm(ustar[j])))
    ms_k, cnt = timer.total_ms, timer.launches
    # the oracle's solutions of the queries it solved in full, against the
    # GPU's for the same queries (solved again after the timed region)
    oracle_check = None
    usol = leg.solutions() if leg is not None else None
    if usol is not None and args.solver == "pcg":
        m = len(usol)
        errs, gpu_its = [], []
        for a in range(0, m, w.batch):
            ids = [(a + b) % Q for b in range(w.batch)]
            sysm.xi.copy_(xi_d[ids])
            prob.assemble(sysm)
            prec = prob.setup(sysm, P, precision=precision, smoother=smoother)
            u.copy_(x0[ids])
            ret, its, rr, st = plan.solve(w.tol) if plan is not None else prob.solve(sysm, prec, u)
            uh = u.cpu().numpy()
            for b in range(min(w.batch, m - a)):
                ref = usol[a + b]
                errs.append(float(np.linalg.norm(uh[b] - ref) / np.linalg.norm(ref)))
                gpu_its.append(its[b])
        o_its = leg.result["runs"][1]["iters"]
        oracle_check = {"queries": m, "err_vs_oracle_max": max(errs),
                        "iters_gpu": gpu_its, "iters_oracle": o_its,
                        "iters_diff_max": int(max(abs(g - o) for g, o in zip(gpu_its, o_its)))}
        log(f"[bench] against the oracle on {m} queries: rel. error <= {max(errs):.2e}, "
            f"iterations GPU {gpu_its} oracle {o_its}")
    sample = leg.iterate() if leg is not None else None
    if sample is not None and args.solver == "pcg":
        # too large for a full oracle solve: the GPU batch holding query 0, in
        # the timed launch configuration, stopped after as many iterations as
        # the oracle ran from the same warm start; query 0's iterates compared
        ids = [b % Q for b in range(w.batch)]
        sysm.xi.copy_(xi_d[ids])
        prob.assemble(sysm)
        prec = prob.setup(sysm, P, precision=precision, smoother=smoother)
        u.copy_(x0[ids])
        m_it = int(sample["iters"])
        ret, its, rr, st = (plan.solve(w.tol, maxit=m_it) if plan is not None
                            else prob.solve(sysm, prec, u, maxit=m_it))
        ug, ur, x00 = u[0].cpu().numpy(), sample["u"], x0[0].cpu().numpy()
        d = float(np.linalg.norm(ug - ur))
        oracle_check = {"queries": 1, "kind": f"iterate after {m_it} iterations from the same "
                        "warm start (a full oracle solve exceeds the bounded sample)",
                        "iters_gpu": [int(its[0])], "iters_oracle": [m_it],
                        "rel_diff": d / float(np.linalg.norm(ur)),
                        "rel_diff_of_correction": d / float(np.linalg.norm(ur - x00))}
        log(f"[bench] against the oracle's iterate after {m_it} iterations (query 0): "
            f"GPU {its[0]} iterations, |u_gpu - u_oracle| / |u_oracle - x0| = "
            f"{oracle_check['rel_diff_of_correction']:.2e}")
    if plan is not None:
        plan.close()
    L.pod2g_timer_destroy(timer)

    solves = args.steps * w.batch
    value = solves / dt
    avg_s = (ms_k / cnt) / 1e3 if cnt else float("nan")
    # the update fused with the second pre-sweep: as tuned, else the library's
    # default (small problems, Jacobi relaxation)
    nbytes = R.kernel_bytes(w, args.kernel, plan_cfg, args.smoother)
    achieved = nbytes / avg_s / 1e9 if cnt else None
    log(f"[bench] {solves} solves in {dt:.3f} s; mean iterations "
        f"{np.mean(stats['iters']):.1f}; {args.kernel}: {cnt} timed launches, "
        f"{avg_s * 1e6:.1f} us avg, {nbytes / 1e6:.2f} MB -> "
        f"{f'{achieved:.0f}' if achieved else '-'} GB/s")

    result = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if mixed else "f64", "data": "synthetic",
        "config": {"workload": w.name,
                   "problem": f"{w.dim}D {'Q4 plane stress' if w.dim == 2 else 'Hex8'} "
                              f"{'x'.join([str(w.N)] * w.dim)}, {w.n_terms} field terms",
                   "n": w.n, "k": w.k, "n_train": w.n_train, "batch": w.batch,
                   "precision": w.precision, "tol": w.tol, "omega": w.omega,
                   "sweeps": [w.nu_pre, w.nu_post], "queries": Q,
                   "graph_chunk": args.chunk if args.solver == "pcg" else 0,
                   "warm_start": args.warm, "solver": args.solver, "smoother": args.smoother,
                   "tuning": tuning,
                   "iters_mean": float(np.mean(stats["iters"])),
                   "relres_max": float(np.max(stats["relres"])),
                   "err_vs_exact_max": float(np.max(stats["err"])),
                   "oracle_check": oracle_check},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": R.HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / R.HBM_PEAK_GBS if achieved else None,
                     "traffic": profiling.traffic_lookup(os.path.join(ROOT, "profiles"), w.name,
                                                         args.kernel),
                     "kernel": args.kernel, "bytes_per_launch": nbytes,
                     "avg_launch_us": avg_s * 1e6, "launches_timed": cnt},
    }
    ncmp = args.compare_plain if args.compare_plain is not None else (4 if w.batch > 1 else 0)
    if ncmp > 0:
        log(f"[bench] timing {ncmp} one-at-a-time FP64 solves of the same queries ...")
        s64 = leg.iterate(fp64=True) if leg is not None else None
        pl = plain_baseline(prob, P, xi_d, x0, ustar, ncmp, args.chunk if args.chunk > 0 else 8,
                            sample64=s64)
        pl["speedup_batched"] = value / pl["value"]
        result["plain_fp64"] = pl
        log(f"[bench] plain FP64: {pl['value']:.2f} solves/s ({pl['iters_mean']:.1f} iterations); "
            f"batched {w.precision}: x{pl['speedup_batched']:.2f}")
        if "oracle_iterate" in pl:
            oi = pl["oracle_iterate"]
            log(f"[bench] plain FP64 path against the oracle's FP64 iterate after "
                f"{oi['iters_oracle']} iterations (query 0): |u_gpu - u_oracle| / |u_oracle - x0| "
                f"= {oi['rel_diff_of_correction']:.2e}")
    if leg is not None:
        result["cpu_baseline"] = leg.summary(float(np.mean(stats["iters"])))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
