"""Served solves: continuous batching of independent queries theta.

The multi-query setting of Sec. 3 (many parametrised solves K(theta) u = f
with one offline basis per problem class) as a request loop.  Each problem
class (mesh size, field terms, basis P) is one slot group of the library's
server (``pod2g_server_*``): its slots hold one query each -- K(theta),
D^-1, the coarse factor and the CG state stay resident on the device.  A
step is one graph launch that advances every live slot of a class (by
default each class on its own stream, at its own pace; optionally all
classes together) by a fixed number of PCG iterations (Alg. 3); requests
that arrive while others run are admitted into free slots between steps,
and finished slots are retired (result copied to the host) and reused.

Every numerical step runs in the HIP library; this module only moves
requests and results and keeps time.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import capi as L
from . import inputs as I
from .pipeline import Problem, _bytes, exact_solutions

SLOT_INFO = np.dtype([("done", "<i4"), ("iter", "<i4"), ("status", "<i4"), ("pad", "<i4"),
                      ("relres", "<f8")])
assert SLOT_INFO.itemsize == 24


def slot_bytes(w: I.Workload, k: int, precision: str) -> int:
    """Device bytes one resident query of class w occupies: its K (FP64 and,
    mixed, FP32), D^-1, K P, the coarse factors and the CG vectors."""
    n, nvals = w.n, (w.n + w.dim) * (3 ** w.dim // 2 + 1) * w.dim   # symmetric half of K
    mixed = precision == "mixed"
    b = nvals * 8 + (nvals * 4 if mixed else 0)        # K
    b += n * 8 + (n * 4 if mixed else 0)               # D^-1
    b += k * n * 8 + 2 * k * k * 8                     # K P, L, L^-1
    b += 9 * n * 8 + (2 * n * 4 if mixed else 0)       # u and the eight solver vectors
    return b


def plan_slots(classes, free_bytes: int, max_slots: int = 32) -> list[int]:
    """Slots per class from the free HBM: an equal share of free_bytes per
    class, at most max_slots (the batched MFMA contraction's width)."""
    share = free_bytes // max(1, len(classes))
    return [int(max(1, min(max_slots, share // slot_bytes(w, k, p)))) for (w, k, p) in classes]


class ServedClass:
    """One problem class: pattern, basis P and `slots` resident queries."""

    def __init__(self, w: I.Workload, P: torch.Tensor, slots: int, precision="mixed",
                 power_iters=0, device="cuda", guard=True):
        """guard: check the damped-Jacobi stability of the class once (on the
        first placeholder instance) and raise on ESMOOTHER; power_iters:
        the per-slot guard of pod2g_setup_slot (0: none)."""
        self.w = w
        self.prob = Problem(w, device)
        if not guard:
            self.prob._guarded.add(w.omega)
        self.P = P
        self.k = P.shape[0]
        self.slots = slots
        self.precision = L.MIXED if precision == "mixed" else L.FP64
        self.power_iters = power_iters
        prob = self.prob
        self.sysm = prob.alloc_system(slots, fp32=self.precision == L.MIXED)
        self.sysm.xi.zero_()
        prob.assemble(self.sysm)          # placeholder instances; also forms f
        self.prec = prob.setup(self.sysm, P, precision=self.precision, key="serve_setup")
        self.u = torch.zeros(slots, prob.n, dtype=torch.float64, device=prob.device)
        self.nbytes = L.pcg_solve_bytes(prob.pat, slots, self.k, self.precision)
        self.work = _bytes(self.nbytes, prob.device)
        self.asm_bytes = L.pod2g_assemble_bytes(prob.pat, 1)
        self.asm_work = _bytes(self.asm_bytes, prob.device)
        self.out = torch.empty(slots, prob.n, dtype=torch.float64).pin_memory()

    def group(self):
        return (self.prob.pat, self.sysm.vals, self.prec, self.sysm.f, self.u, self.work, self.nbytes)

    def load(self, slot: int, xi: torch.Tensor, x0: torch.Tensor, stream=None):
        """Assemble and set up query (xi, x0) in `slot` (both pinned host tensors)."""
        s = self.sysm
        s.xi[slot].copy_(xi, non_blocking=True)
        L.check(L.pod2g_assemble(self.prob.pat, s.xi[slot], 1, s.vals[slot],
                                 s.vals32[slot] if s.vals32 is not None else None, s.dinv[slot],
                                 None, self.asm_work, self.asm_bytes, stream), "pod2g_assemble")
        L.check(L.pod2g_setup_slot(self.prec, slot, self.power_iters, stream), "pod2g_setup_slot")
        self.u[slot].copy_(x0, non_blocking=True)


# Streams restricted to a range of compute units, one per (device, first
# unit, count), created once and kept for the life of the process: torch's
# pinned-memory allocator keeps events of the non-blocking copies issued on
# a stream, so a stream must outlive every pinned buffer ever copied on it.
_CU_STREAMS: dict = {}


def cu_stream(first: int, count: int) -> torch.cuda.ExternalStream:
    key = (torch.cuda.current_device(), first, count)
    if key not in _CU_STREAMS:
        _CU_STREAMS[key] = torch.cuda.ExternalStream(L.pod2g_stream_create_cus(first, count))
    return _CU_STREAMS[key]


class Server:
    """The library server over a list of ServedClass groups.  cu_shares: a
    number of compute units per class (None: every class on the whole GPU);
    each class then steps on a stream restricted to its own units."""

    def __init__(self, classes: list[ServedClass], chunk=8, cu_shares=None):
        self.classes = classes
        self.cu_streams = None
        if cu_shares is not None:
            if len(cu_shares) != len(classes):
                raise ValueError("one compute-unit share per class")
            first, self.cu_streams = 0, []
            for n in cu_shares:
                self.cu_streams.append(cu_stream(first, int(n)))
                first += int(n)
        self.handle = L.pod2g_server_create([c.group() for c in classes], chunk)
        self.chunk = chunk + (chunk & 1)
        self.base = np.cumsum([0] + [c.slots for c in classes])
        self.total = int(self.base[-1])
        assert L.pod2g_server_slots(self.handle) == self.total
        self.info = torch.empty(self.total * SLOT_INFO.itemsize, dtype=torch.uint8).pin_memory()

    def admit(self, ci: int, slot: int, xi, x0, rtol, maxit=5000, beta=None, stream=None):
        c = self.classes[ci]
        if beta is None:
            beta = L.BETA_PR if c.precision == L.MIXED else L.BETA_FR
        c.load(slot, xi, x0, stream)
        L.check(L.pod2g_server_admit(self.handle, ci, slot, rtol, maxit, beta, stream),
                "pod2g_server_admit")

    def step(self, stream=None):
        L.check(L.pod2g_serve_step(self.handle, self.info, stream), "pod2g_serve_step")

    def step_group(self, g: int, nslots=None, stream=None):
        """Step class g; with nslots, only its first nslots slots (the
        smallest captured prefix holding them; the rest must be free)."""
        if nslots is None:
            L.check(L.pod2g_serve_step_group(self.handle, g, self.info, stream),
                    "pod2g_serve_step_group")
        else:
            L.check(L.pod2g_serve_step_prefix(self.handle, g, nslots, self.info, stream),
                    "pod2g_serve_step_prefix")

    def slot_info(self) -> np.ndarray:
        """The info copied by the last step (the caller synchronised)."""
        return np.frombuffer(self.info.numpy().tobytes(), dtype=SLOT_INFO)

    def close(self):
        if self.handle:
            L.pod2g_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Pool:
    """Pre-generated queries of one class: xi, warm start x0 (pinned) and,
    for checking results, the tight solution u* (host)."""
    xi: torch.Tensor
    x0: torch.Tensor
    u_star: np.ndarray


def make_pool(c: ServedClass, count: int, first: int = 0) -> Pool:
    w = c.prob.w
    xis = I.query_xis(w, count, first)
    u = exact_solutions(c.prob, xis, c.P)
    g = torch.tensor(np.stack([I.noise(w, first + j) for j in range(count)]), device=u.device)
    x0 = torch.stack([I.warm_start(u[j], g[j], w.noise) for j in range(count)])
    return Pool(torch.tensor(xis).pin_memory(), x0.cpu().pin_memory(), u.cpu().numpy())


@dataclass
class Request:
    rid: int
    ci: int
    q: int
    t_arrive: float
    t_admit: float = -1.0
    t_done: float = -1.0
    iters: int = -1
    status: int = 1
    relres: float = float("nan")
    err: float = float("nan")
    slot: int = -1


@dataclass
class RunResult:
    requests: list
    occupancy: list = field(default_factory=list)   # (t, live slots per class)
    steps: int = 0
    wall: float = 0.0


REFUSED = 1000    # Request.status of a request the loop turned away (queue full)


def run_stream(server: Server, pools: list[Pool], times, cls, qidx, rtol, maxit=5000,
               check_first=0, realtime=True, independent=True, max_queue=None) -> RunResult:
    """Serve the request stream (arrival times in s from the start, class
    and pool index per request).  With realtime, requests become visible at
    their arrival times; otherwise all are queued at t = 0.  The results of
    the first `check_first` requests of every class are compared with u*
    (relative error); every result is copied to the host.  independent:
    every class is stepped on its own stream at its own pace (otherwise one
    step advances all classes together).  max_queue: a request that arrives
    while its class already has this many requests waiting for a slot is
    refused (status REFUSED, no result) instead of queued (independent
    stepping only)."""
    if independent:
        return _run_groups(server, pools, times, cls, qidx, rtol, maxit, check_first, realtime,
                           max_queue)
    classes = server.classes
    reqs = [Request(i, int(cls[i]), int(qidx[i]), float(times[i]) if realtime else 0.0)
            for i in range(len(times))]
    free = [list(range(c.slots))[::-1] for c in classes]
    live = {}            # global slot -> request
    queue = deque()
    checked = [0] * len(classes)
    pending, ev_ret = [], None
    res = RunResult(reqs)
    nxt = 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt].t_arrive <= now:
            queue.append(reqs[nxt])
            nxt += 1
        # admission in arrival order; a request whose class is full waits
        # without blocking the other classes
        if queue:
            waiting = deque()
            while queue:
                r = queue.popleft()
                if free[r.ci]:
                    slot = free[r.ci].pop()
                    p = pools[r.ci]
                    server.admit(r.ci, slot, p.xi[r.q], p.x0[r.q], rtol, maxit)
                    r.slot, r.t_admit = slot, time.perf_counter() - t0
                    live[int(server.base[r.ci]) + slot] = r
                else:
                    waiting.append(r)
            queue = waiting
        stepped = bool(live)
        if stepped:
            server.step()
            ev = torch.cuda.Event()
            ev.record()
            res.steps += 1
        if pending:
            ev_ret.synchronize()
            t = time.perf_counter() - t0
            for r in pending:
                r.t_done = t
                c = classes[r.ci]
                if checked[r.ci] < check_first:
                    u = c.out[r.slot].numpy()
                    us = pools[r.ci].u_star[r.q]
                    r.err = float(np.linalg.norm(u - us) / np.linalg.norm(us))
                    checked[r.ci] += 1
            pending = []
        if not stepped:
            if nxt >= len(reqs) and not queue:
                break
            if nxt < len(reqs):
                delay = reqs[nxt].t_arrive - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(min(delay, 0.01))
            continue
        ev.synchronize()
        info = server.slot_info()
        res.occupancy.append((time.perf_counter() - t0,
                              [sum(1 for g in live if server.base[i] <= g < server.base[i + 1])
                               for i in range(len(classes))]))
        for g in list(live):
            if info[g]["done"]:
                r = live.pop(g)
                c = classes[r.ci]
                c.out[r.slot].copy_(c.u[r.slot], non_blocking=True)
                r.iters, r.status, r.relres = int(info[g]["iter"]), int(info[g]["status"]), float(info[g]["relres"])
                free[r.ci].append(r.slot)
                pending.append(r)
        if pending:
            ev_ret = torch.cuda.Event()
            ev_ret.record()
    res.wall = time.perf_counter() - t0
    return res


def _run_groups(server, pools, times, cls, qidx, rtol, maxit, check_first, realtime,
                max_queue=None) -> RunResult:
    """run_stream with one stream per class: a class is admitted, stepped
    and retired whenever its previous step has finished.  A request takes
    the lowest free slot, and a step covers only the slots up to the last
    live one (pod2g_serve_step_prefix)."""
    import heapq
    classes = server.classes
    G = len(classes)
    reqs = [Request(i, int(cls[i]), int(qidx[i]), float(times[i]) if realtime else 0.0)
            for i in range(len(times))]
    streams = server.cu_streams or [torch.cuda.Stream() for _ in range(G)]
    free = [list(range(c.slots)) for c in classes]       # min-heaps of free slots
    live = [dict() for _ in range(G)]           # slot -> request
    queues = [deque() for _ in range(G)]
    inflight = [None] * G
    copies = []                                 # (event, requests whose result is being copied)
    checked = [0] * G
    res = RunResult(reqs)
    nxt = 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt].t_arrive <= now:
            r = reqs[nxt]
            if max_queue is not None and len(queues[r.ci]) >= max_queue:
                r.status = REFUSED
            else:
                queues[r.ci].append(r)
            nxt += 1
        for g in range(G):
            c = classes[g]
            if inflight[g] is not None:
                if not inflight[g].query():
                    continue
                inflight[g] = None
                info = server.slot_info()[int(server.base[g]):int(server.base[g + 1])]
                done = []
                with torch.cuda.stream(streams[g]):
                    for slot in list(live[g]):
                        if info[slot]["done"]:
                            r = live[g].pop(slot)
                            c.out[slot].copy_(c.u[slot], non_blocking=True)
                            r.iters, r.status = int(info[slot]["iter"]), int(info[slot]["status"])
                            r.relres = float(info[slot]["relres"])
                            heapq.heappush(free[g], slot)
                            done.append(r)
                    if done:
                        ev = torch.cuda.Event()
                        ev.record(streams[g])
                        copies.append((ev, done))
                res.occupancy.append((time.perf_counter() - t0,
                                      [len(live[i]) for i in range(G)]))
            with torch.cuda.stream(streams[g]):
                while queues[g] and free[g]:
                    r = queues[g].popleft()
                    slot = heapq.heappop(free[g])
                    p = pools[g]
                    server.admit(g, slot, p.xi[r.q], p.x0[r.q], rtol, maxit)
                    r.slot, r.t_admit = slot, time.perf_counter() - t0
                    live[g][slot] = r
                if live[g]:
                    server.step_group(g, nslots=max(live[g]) + 1)
                    ev = torch.cuda.Event()
                    ev.record(streams[g])
                    inflight[g] = ev
                    res.steps += 1
        for item in list(copies):
            ev, done = item
            if ev.query():
                t = time.perf_counter() - t0
                for r in done:
                    r.t_done = t
                    if checked[r.ci] < check_first:
                        u = classes[r.ci].out[r.slot].numpy()
                        us = pools[r.ci].u_star[r.q]
                        r.err = float(np.linalg.norm(u - us) / np.linalg.norm(us))
                        checked[r.ci] += 1
                copies.remove(item)
        busy = any(e is not None for e in inflight) or copies
        if not busy:
            if nxt >= len(reqs) and not any(queues):
                break
            if nxt < len(reqs):
                delay = reqs[nxt].t_arrive - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(min(delay, 0.01))
        else:
            time.sleep(5e-5)
    torch.cuda.synchronize()
    res.wall = time.perf_counter() - t0
    return res


def solo_latency(server: Server, pools: list[Pool], rtol, repeats=3) -> list[float]:
    """Per class, the median latency (ms) of one request served alone on an
    otherwise idle server."""
    out = []
    for g in range(len(server.classes)):
        lat = []
        for rep in range(repeats):
            res = run_stream(server, pools, np.zeros(1), np.array([g]), np.array([rep % len(pools[g].xi)]),
                             rtol=rtol, realtime=False)
            r = res.requests[0]
            lat.append((r.t_done - r.t_arrive) * 1e3)
        out.append(float(np.median(lat)))
    return out


def summarize(res: RunResult, names, solo_ms=None, solo_whole_ms=None) -> dict:
    """Completion, throughput and latency percentiles, overall and per
    class; with solo latencies (on the class's own compute-unit share, and
    on the whole GPU) also the p50 over each."""
    done = [r for r in res.requests if r.t_done >= 0]
    lat = np.array([r.t_done - r.t_arrive for r in done]) * 1e3
    out = {
        "requests": len(res.requests),
        "completed": len(done),
        "refused": sum(1 for r in res.requests if r.status == REFUSED),
        "failed": sum(1 for r in done if r.status != L.OK),
        "wall_s": res.wall,
        "solves_per_s": len(done) / res.wall if res.wall > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "steps": res.steps,
        "per_class": {},
    }
    for i, nm in enumerate(names):
        rs = [r for r in done if r.ci == i]
        if not rs:
            continue
        li = np.array([r.t_done - r.t_arrive for r in rs]) * 1e3
        errs = [r.err for r in rs if r.err == r.err]
        occ = [o[1][i] for o in res.occupancy]
        out["per_class"][nm] = {
            "completed": len(rs),
            "p50_ms": float(np.percentile(li, 50)),
            "p99_ms": float(np.percentile(li, 99)),
            "iters_mean": float(np.mean([r.iters for r in rs])),
            "relres_max": float(max(r.relres for r in rs)),
            "err_vs_exact_max": float(max(errs)) if errs else None,
            "live_slots_mean": float(np.mean(occ)) if occ else 0.0,
            "live_slots_max": int(max(occ)) if occ else 0,
        }
        if solo_ms is not None:
            out["per_class"][nm]["solo_ms"] = solo_ms[i]
            out["per_class"][nm]["p50_over_solo"] = float(np.percentile(li, 50)) / solo_ms[i]
        if solo_whole_ms is not None:
            out["per_class"][nm]["solo_whole_gpu_ms"] = solo_whole_ms[i]
            out["per_class"][nm]["p50_over_solo_whole_gpu"] = (float(np.percentile(li, 50))
                                                               / solo_whole_ms[i])
    return out
