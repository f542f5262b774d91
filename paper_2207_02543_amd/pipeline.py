"""Host-side orchestration of the POD-2G path on one GPU.

Every numerical step runs in the HIP library through ``capi``; this module
only allocates device memory with torch, orders the calls and moves the
small host-side results (iteration counts, statuses).

* ``Problem``      -- one problem class (mesh size, field terms, Poisson ratio):
                      the pattern plus helpers to assemble, set up and solve.
* ``offline_basis``-- the offline phase (Sec. 3.4): training solves at the
                      training parameters, then POD by the method of
                      snapshots (Sec. 3.3) -> P.
* ``exact_solutions`` -- tight solves used to build warm starts
                      (surrogate stand-in) for the queries.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import capi as L
from . import inputs as I


def _bytes(n, device):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def device_view(base: torch.Tensor, ptr: int, count: int, dtype) -> torch.Tensor:
    """A typed view of `count` elements at device address `ptr` inside the
    byte tensor `base` (e.g. a field of a handle living in a workspace)."""
    off = int(ptr) - base.data_ptr()
    nbytes = count * torch.empty(0, dtype=dtype).element_size()
    if off < 0 or off + nbytes > base.numel():
        raise ValueError("pointer outside the buffer")
    return base[off:off + nbytes].view(dtype)


@dataclass
class System:
    """Assembled instances of one problem class (device tensors)."""
    batch: int
    xi: torch.Tensor          # [batch, n_terms] f64
    vals: torch.Tensor        # [batch, nvals] f64
    vals32: torch.Tensor | None
    dinv: torch.Tensor        # [batch, n] f64
    f: torch.Tensor           # [n] f64


class Problem:
    def __init__(self, w: I.Workload, device="cuda"):
        self.w = w
        self.device = torch.device(device)
        self.mesh = L.make_mesh(w.dim, w.N, w.n_terms, w.nu, w.kl_scale)
        nb = L.pod2g_pattern_bytes(self.mesh)
        if nb == 0:
            raise L.Pod2gError(L.EINVAL, "pod2g_pattern_bytes")
        self.pat_buf = _bytes(nb, self.device)
        self.pat = L.Pattern()
        L.check(L.pod2g_pattern_build(self.mesh, self.pat_buf, nb, self.pat), "pod2g_pattern_build")
        self.n = self.pat.n
        self.nvals = self.pat.nvals
        self._work = {}
        self._guarded = set()       # omegas the smoother guard has passed
        self.lambda_max = None

    # -- scratch buffers, reused between calls of the same kind ----------------
    def work(self, key, nbytes):
        t = self._work.get(key)
        if t is None or t.numel() < nbytes:
            t = _bytes(nbytes, self.device)
            self._work[key] = t
        return t

    # -- assembly -----------------------------------------------------------------
    def alloc_system(self, batch, fp32=False) -> System:
        d = self.device
        return System(batch,
                      torch.empty(batch, self.w.n_terms, dtype=torch.float64, device=d),
                      torch.empty(batch, self.nvals, dtype=torch.float64, device=d),
                      torch.empty(batch, self.nvals, dtype=torch.float32, device=d) if fp32 else None,
                      torch.empty(batch, self.n, dtype=torch.float64, device=d),
                      torch.empty(self.n, dtype=torch.float64, device=d))

    def assemble(self, sysm: System, xi=None, stream=None):
        if xi is not None:
            sysm.xi.copy_(torch.as_tensor(np.asarray(xi), dtype=torch.float64).reshape(sysm.batch, -1))
        nb = L.pod2g_assemble_bytes(self.pat, sysm.batch)
        wk = self.work("assemble", nb)
        L.check(L.pod2g_assemble(self.pat, sysm.xi, sysm.batch, sysm.vals, sysm.vals32, sysm.dinv,
                                 sysm.f, wk, nb, stream), "pod2g_assemble")
        return sysm

    # -- preconditioner -----------------------------------------------------------
    # power iterations of the damped-Jacobi stability guard, run on the first
    # setup of each damping weight of a problem class
    GUARD_ITERS = 100

    def setup(self, sysm: System, P, k=None, precision=L.FP64, omega=None, nu_pre=None,
              nu_post=None, power_iters=0, key="setup", smoother=L.SMOOTHER_JACOBI,
              stream=None) -> L.Prec:
        """pod2g_setup on these instances.  The first Jacobi setup with a
        given omega also estimates lambda_max(D^-1 K) of the first instance
        and raises Pod2gError(ESMOOTHER) if omega * lambda_max >= 2 (the
        estimate depends on the mesh and the Poisson ratio, hardly on theta,
        so one check covers the class)."""
        w = self.w
        k = (P.shape[0] if P is not None else 0) if k is None else k
        om = w.omega if omega is None else omega
        if smoother == L.SMOOTHER_JACOBI and om not in self._guarded:
            self.check_smoother(sysm, om)
        nb = L.pod2g_setup_bytes(self.pat, k, sysm.batch, precision)
        wk = self.work(key, nb)
        prec = L.Prec()
        L.check(L.pod2g_setup(self.pat, sysm.vals, sysm.vals32, sysm.dinv, P, k, om,
                              w.nu_pre if nu_pre is None else nu_pre,
                              w.nu_post if nu_post is None else nu_post,
                              precision, sysm.batch, power_iters, wk, nb, prec, stream),
                "pod2g_setup")
        L.check(L.pod2g_set_smoother(prec, smoother), "pod2g_set_smoother")
        prec._keepalive = (wk, P, sysm)
        return prec

    def check_smoother(self, sysm: System, omega: float):
        """The damped-Jacobi guard on instance 0 of sysm (smoother-only setup
        with GUARD_ITERS power iterations); raises on ESMOOTHER."""
        one = System(1, sysm.xi[:1], sysm.vals[:1], None, sysm.dinv[:1], sysm.f)
        nb = L.pod2g_setup_bytes(self.pat, 0, 1, L.FP64)
        wk = _bytes(nb, self.device)
        prec = L.Prec()
        L.check(L.pod2g_setup(self.pat, one.vals, None, one.dinv, None, 0, omega, 1, 1, L.FP64, 1,
                              self.GUARD_ITERS, wk, nb, prec, None), "pod2g_setup (guard)")
        st, lam = L.pod2g_setup_status(prec)
        if st[0] != L.OK:
            raise L.Pod2gError(st[0], f"damped Jacobi with omega = {omega:.4g}: "
                                      f"omega * lambda_max(D^-1 K) ~ {omega * lam[0]:.3f}")
        self._guarded.add(omega)
        self.lambda_max = lam[0]

    # -- solve --------------------------------------------------------------------
    def solve(self, sysm: System, prec, u, rtol=None, maxit=5000, beta=None, key="pcg",
              timer=None, stream=None):
        k = prec.k if prec is not None else 0
        precision = prec.precision if prec is not None else L.FP64
        if beta is None:
            beta = L.BETA_PR if precision == L.MIXED else L.BETA_FR
        nb = L.pcg_solve_bytes(self.pat, sysm.batch, k, precision)
        wk = self.work(key, nb)
        rtol = self.w.tol if rtol is None else rtol
        if timer is not None:
            return L.pcg_solve_timed(self.pat, sysm.vals, sysm.batch, prec, sysm.f, u, rtol, maxit,
                                     beta, wk, nb, timer, stream)
        return L.pcg_solve(self.pat, sysm.vals, sysm.batch, prec, sysm.f, u, rtol, maxit, beta,
                           wk, nb, stream)

    def stationary(self, sysm: System, prec, u, rtol=None, maxit=5000, key="pcg", stream=None):
        """The two-grid scheme iterated on its own: u <- u + B (f - K u)."""
        nb = L.pcg_solve_bytes(self.pat, sysm.batch, prec.k, prec.precision)
        wk = self.work(key, nb)
        rtol = self.w.tol if rtol is None else rtol
        return L.pod2g_stationary_solve(self.pat, sysm.vals, sysm.batch, prec, sysm.f, u, rtol,
                                        maxit, wk, nb, stream)

    def rom_start(self, sysm: System, prec, u, stream=None):
        """u = P (P^T K P)^{-1} P^T f, the reduced-order warm start."""
        nb = L.pod2g_rom_bytes(prec)
        wk = self.work("rom", nb)
        L.check(L.pod2g_rom_start(prec, sysm.f, u, wk, nb, stream), "pod2g_rom_start")
        return u

    def plan(self, sysm: System, prec, u, chunk=8, timer=None, key="pcg"):
        """Capture `chunk` PCG iterations on these buffers (see pcg_plan_create)."""
        k = prec.k if prec is not None else 0
        precision = prec.precision if prec is not None else L.FP64
        nb = L.pcg_solve_bytes(self.pat, sysm.batch, k, precision)
        wk = self.work(key, nb)
        h = L.pcg_plan_create(self.pat, sysm.vals, sysm.batch, prec, sysm.f, u, chunk, wk, nb, timer)
        return Plan(h, sysm.batch, precision, (wk, prec, sysm, u, timer))

    def apply(self, prec, r, s, stream=None):
        nb = L.pod2g_apply_bytes(prec)
        wk = self.work("apply", nb)
        L.check(L.pod2g_apply(prec, r, s, wk, nb, stream), "pod2g_apply")
        return s


# launch parameters of a plan (pod2g_tuning without the timing)
PLAN_PARAMS = ("bgrid", "fuse_dir", "igroup", "xwin", "cons", "fuse_upd", "ptr_grp")


class Plan:
    """Owner of a captured solve plan; keeps its buffers alive."""

    def __init__(self, handle, batch, precision, keep):
        self.handle, self.batch, self.precision, self._keep = handle, batch, precision, keep

    def solve(self, rtol, maxit=5000, beta=None, stream=None):
        if beta is None:
            beta = L.BETA_PR if self.precision == L.MIXED else L.BETA_FR
        return L.pcg_plan_solve(self.handle, rtol, maxit, beta, self.batch, stream)

    def tune(self, trials=8, stream=None) -> dict:
        """Pick the launch parameters by timing (overwrites u: call before
        loading the initial guess)."""
        t = L.pcg_plan_tune(self.handle, trials, stream)
        out = {f: getattr(t, f) for f in PLAN_PARAMS}
        out["ms_per_iteration"] = t.ms_per_iteration
        return out

    def config(self) -> dict:
        t = L.pcg_plan_config(self.handle)
        return {f: getattr(t, f) for f in PLAN_PARAMS}

    def configure(self, **params):
        """Set launch parameters (names as in config()); the rest keep their
        values.  Raises on values the plan cannot take."""
        cur = self.config()
        unknown = set(params) - set(cur)
        if unknown:
            raise ValueError(f"unknown launch parameters {sorted(unknown)}")
        cur.update(params)
        t = L.Tuning(**cur)
        L.check(L.pcg_plan_configure(self.handle, t), "pcg_plan_configure")

    def close(self):
        if self.handle:
            L.pcg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_chunk(prob: Problem, k: int, precision=L.FP64, cap: int = 32, share: float = 0.5) -> int:
    """Instances of one solve batch that fit `share` of the free HBM: per
    instance K and D^-1, K P and the solver vectors (the FP32 cycle adds the
    FP32 copy of K and, in 3D, of K P)."""
    free, _ = torch.cuda.mem_get_info(prob.device)
    per = 8 * (prob.nvals + prob.n * (k + 12))
    if precision == L.MIXED:
        per += 4 * (prob.nvals + prob.n * (k + 2))
    return int(max(1, min(cap, share * free // per)))


fp64_chunk = batch_chunk


def solve_batched(prob: Problem, xis: np.ndarray, P=None, k=0, rtol=1e-12, maxit=20000,
                  chunk=None, u0=None, precision=L.FP64, rom=False):
    """Tight solves at the given parameters (two-grid PCG with the basis P,
    or the smoother-only cycle for k = 0), `chunk` instances at a time
    (default: as many as half the free HBM holds, at most 32).  precision:
    FP64 cycle (Fletcher-Reeves beta) or the FP32 cycle under the FP64 outer
    loop (flexible Polak-Ribiere beta); both stop on the true FP64 residual.
    Initial guess: u0 if given, else the reduced-order solution
    P K_c^-1 P^T f (rom=True, needs P), else zero.  Returns ([len(xis), n],
    iterations)."""
    m = len(xis)
    kk = P.shape[0] if P is not None else k
    if chunk is None:
        chunk = batch_chunk(prob, kk, precision)
    mixed = precision == L.MIXED
    out = torch.empty(m, prob.n, dtype=torch.float64, device=prob.device)
    iters = []
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        sysm = prob.alloc_system(b - a, fp32=mixed)
        prob.assemble(sysm, xis[a:b])
        prec = prob.setup(sysm, P, k=kk, precision=precision, key="setup_train")
        u = out[a:b]
        if u0 is not None:
            u.copy_(u0[a:b])
        elif rom and P is not None:
            prob.rom_start(sysm, prec, u)
        else:
            u.zero_()
        ret, it, rr, st = prob.solve(sysm, prec, u, rtol=rtol, maxit=maxit, key="pcg_train")
        if ret != L.OK:
            raise L.Pod2gError(ret, f"training solve {a}..{b}: statuses {st}")
        iters += it
        del sysm, prec
    # the batch workspaces are sized for this call only: hand them back
    for key in ("setup_train", "pcg_train", "rom"):
        prob._work.pop(key, None)
    torch.cuda.empty_cache()
    return out, iters


def pod_basis(U: torch.Tensor, k: int):
    """P ([k, n]) and all eigenvalues of U^T U (descending) from snapshots U ([N, n])."""
    N, n = U.shape
    P = torch.empty(k, n, dtype=torch.float64, device=U.device)
    lam = torch.empty(N, dtype=torch.float64, device=U.device)
    nb = L.pod2g_pod_basis_bytes(n, N, k)
    wk = _bytes(nb, U.device)
    L.check(L.pod2g_pod_basis(U, n, N, k, P, lam, wk, nb), "pod2g_pod_basis")
    return P, lam


def offline_basis(prob: Problem, n_train=None, k=None, rtol=None, chunk=None, progress=None,
                  precision=None):
    """Offline phase (Sec. 3.4): training solves, then POD of the snapshots
    (Sec. 3.3).  The training solves are incremental: the first one uses
    the smoother-only cycle; every later group (doubling in size up to
    `chunk`) is preconditioned by the POD basis of all snapshots so far and
    starts from that basis's reduced-order solution.  rtol: the workload's
    training tolerance unless given; precision: the workload's cycle
    precision unless given."""
    w = prob.w
    n_train = w.n_train if n_train is None else n_train
    k = w.k if k is None else k
    rtol = w.train_tol if rtol is None else rtol
    if precision is None:
        precision = L.MIXED if w.precision == "mixed" else L.FP64
    xis = np.stack([I.train_xi(w, i) for i in range(n_train)])
    U = torch.empty(n_train, prob.n, dtype=torch.float64, device=prob.device)
    if chunk is None:
        chunk = batch_chunk(prob, k, precision)
    iters = []
    done, size = 0, 1
    while done < n_train:
        b = min(n_train, done + size)
        P_cur = None
        if done > 0:
            kk = min(done, k)
            while P_cur is None:
                try:
                    P_cur, _ = pod_basis(U[:done], kk)
                except L.Pod2gError:
                    if kk == 1:
                        raise
                    kk -= 1
        Ub, its = solve_batched(prob, xis[done:b], P_cur, rtol=rtol, chunk=chunk,
                                precision=precision, rom=True)
        U[done:b] = Ub
        iters += its
        if progress is not None:
            progress(f"training solves {done}..{b - 1}: {max(its)} iterations at most")
        done, size = b, min(chunk, 2 * size)
    P, lam = pod_basis(U, k)
    return P, lam, U, iters


def exact_solutions(prob: Problem, xis, P, rtol=1e-12, chunk=None, precision=None):
    """Tight solves (default 1e-12) at the query parameters, from the
    reduced-order start; precision as the workload's cycle."""
    if precision is None:
        precision = L.MIXED if prob.w.precision == "mixed" else L.FP64
    u, it = solve_batched(prob, xis, P, rtol=rtol, chunk=chunk, precision=precision, rom=True)
    return u
