"""Thin ctypes binding of ``libpod2g.so`` (declared in ``include/pod2g.h``).

Argument marshalling only: every function has the C entry point's name and
argument order, takes torch tensors (or raw ints) for device pointers and
returns the C status (or raises ``Pod2gError`` where noted).  All compute
runs in the library's HIP kernels.  If the library is not built the import
of this module fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpod2g.so")

OK, EINVAL, ESIZE, EHIP, ENOTSPD, ESMOOTHER, EMAXIT, EBREAKDOWN, ENAN = 0, -1, -2, -3, -4, -5, -6, -7, -8
TK_SPMV_PQ, TK_SWEEP, TK_SWEEP_FINAL, TK_RESTRICT, TK_PROLONG, TK_UPDATE = 1, 2, 3, 4, 5, 6
FP64, MIXED = 0, 1
SMOOTHER_JACOBI, SMOOTHER_SGS = 0, 1
BETA_FR, BETA_PR = 0, 1
MAX_K = 64


class Pod2gError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("N", C.c_int), ("n_terms", C.c_int),
                ("nu", C.c_double), ("kl_scale", C.c_double)]


class Pattern(C.Structure):
    _fields_ = [("mesh", Mesh), ("n_nodes", C.c_int), ("n", C.c_int), ("n_slots", C.c_int),
                ("n_elems", C.c_int), ("nvals", C.c_longlong),
                ("colblk", C.c_void_p), ("kref", C.c_void_p)]


class Prec(C.Structure):
    _fields_ = [("pat", Pattern), ("batch", C.c_int), ("k", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("precision", C.c_int), ("omega", C.c_double),
                ("vals", C.c_void_p), ("vals32", C.c_void_p), ("dinv", C.c_void_p),
                ("P", C.c_void_p), ("P32", C.c_void_p), ("dinv32", C.c_void_p),
                ("KP", C.c_void_p), ("KP32", C.c_void_p), ("L", C.c_void_p), ("Linv", C.c_void_p), ("lam", C.c_void_p),
                ("status", C.c_void_p), ("work", C.c_void_p), ("smoother", C.c_int)]


class Tuning(C.Structure):
    _fields_ = [("bgrid", C.c_int), ("fuse_dir", C.c_int), ("igroup", C.c_int), ("xwin", C.c_int),
                ("cons", C.c_int), ("fuse_upd", C.c_int), ("ptr_grp", C.c_int),
                ("ms_per_iteration", C.c_float)]


class SlotInfo(C.Structure):
    _fields_ = [("done", C.c_int), ("iter", C.c_int), ("status", C.c_int), ("pad", C.c_int),
                ("relres", C.c_double)]


class Group(C.Structure):
    _fields_ = [("pat", C.c_void_p), ("vals", C.c_void_p), ("prec", C.c_void_p), ("f", C.c_void_p),
                ("u", C.c_void_p), ("work", C.c_void_p), ("bytes", C.c_size_t)]


class Timer(C.Structure):
    _fields_ = [("kernel", C.c_int), ("per_call", C.c_int), ("start", C.c_void_p),
                ("stop", C.c_void_p), ("total_ms", C.c_double), ("launches", C.c_longlong)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                      "(the HIP library is required; there is no CPU path)")
_lib = C.CDLL(LIB_PATH)

_vp, _i, _d, _sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_PM, _PP, _PR = C.POINTER(Mesh), C.POINTER(Pattern), C.POINTER(Prec)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_f = {
    "pod2g_strerror": _sig("pod2g_strerror", C.c_char_p, [_i]),
    "pod2g_pattern_bytes": _sig("pod2g_pattern_bytes", _sz, [_PM]),
    "pod2g_pattern_build": _sig("pod2g_pattern_build", _i, [_PM, _vp, _sz, _PP, _vp]),
    "pod2g_assemble_bytes": _sig("pod2g_assemble_bytes", _sz, [_PP, _i]),
    "pod2g_assemble": _sig("pod2g_assemble", _i, [_PP, _vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pod2g_setup_bytes": _sig("pod2g_setup_bytes", _sz, [_PP, _i, _i, _i]),
    "pod2g_setup": _sig("pod2g_setup", _i, [_PP, _vp, _vp, _vp, _vp, _i, _d, _i, _i, _i, _i, _i,
                                            _vp, _sz, _PR, _vp]),
    "pod2g_setup_slot": _sig("pod2g_setup_slot", _i, [_PR, _i, _i, _vp]),
    "pod2g_set_smoother": _sig("pod2g_set_smoother", _i, [_PR, _i]),
    "pod2g_gauss_seidel": _sig("pod2g_gauss_seidel", _i, [_PP, _vp, _vp, _i, _i, _i, _vp, _vp, _vp]),
    "pod2g_server_create": _sig("pod2g_server_create", _i, [C.POINTER(Group), _i, _i,
                                                            C.POINTER(_vp), _vp]),
    "pod2g_server_admit": _sig("pod2g_server_admit", _i, [_vp, _i, _i, _d, _i, _i, _vp]),
    "pod2g_serve_step": _sig("pod2g_serve_step", _i, [_vp, _vp, _vp]),
    "pod2g_serve_step_group": _sig("pod2g_serve_step_group", _i, [_vp, _i, _vp, _vp]),
    "pod2g_serve_step_prefix": _sig("pod2g_serve_step_prefix", _i, [_vp, _i, _i, _vp, _vp]),
    "pod2g_server_slots": _sig("pod2g_server_slots", _i, [_vp]),
    "pod2g_stream_create_cus": _sig("pod2g_stream_create_cus", _i, [_i, _i, C.POINTER(_vp)]),
    "pod2g_stream_destroy": _sig("pod2g_stream_destroy", _i, [_vp]),
    "pod2g_server_destroy": _sig("pod2g_server_destroy", _i, [_vp]),
    "pod2g_setup_status": _sig("pod2g_setup_status", _i, [_PR, C.POINTER(_i), C.POINTER(_d), _vp]),
    "pod2g_apply_bytes": _sig("pod2g_apply_bytes", _sz, [_PR]),
    "pod2g_apply": _sig("pod2g_apply", _i, [_PR, _vp, _vp, _vp, _sz, _vp]),
    "pod2g_apply_noalloc": _sig("pod2g_apply_noalloc", _i, [_PR, _vp, _vp, _vp]),
    "pcg_solve_bytes": _sig("pcg_solve_bytes", _sz, [_PP, _i, _i, _i]),
    "pcg_solve": _sig("pcg_solve", _i, [_PP, _vp, _i, _PR, _vp, _vp, _d, _i, _i, C.POINTER(_i),
                                        C.POINTER(_d), C.POINTER(_i), _vp, _sz, _vp]),
    "pod2g_stationary_solve": _sig("pod2g_stationary_solve", _i,
                                   [_PP, _vp, _i, _PR, _vp, _vp, _d, _i, C.POINTER(_i),
                                    C.POINTER(_d), C.POINTER(_i), _vp, _sz, _vp]),
    "pod2g_rom_bytes": _sig("pod2g_rom_bytes", _sz, [_PR]),
    "pod2g_rom_start": _sig("pod2g_rom_start", _i, [_PR, _vp, _vp, _vp, _sz, _vp]),
    "pcg_solve_timed": _sig("pcg_solve_timed", _i, [_PP, _vp, _i, _PR, _vp, _vp, _d, _i, _i,
                                                    C.POINTER(_i), C.POINTER(_d), C.POINTER(_i),
                                                    _vp, _sz, C.POINTER(Timer), _vp]),
    "pod2g_timer_create": _sig("pod2g_timer_create", _i, [_i, _i, C.POINTER(Timer)]),
    "pod2g_timer_reset": _sig("pod2g_timer_reset", _i, [C.POINTER(Timer)]),
    "pod2g_timer_destroy": _sig("pod2g_timer_destroy", _i, [C.POINTER(Timer)]),
    "pcg_plan_create": _sig("pcg_plan_create", _i, [_PP, _vp, _i, _PR, _vp, _vp, _i, _vp, _sz,
                                                    C.POINTER(Timer), C.POINTER(_vp)]),
    "pcg_plan_solve": _sig("pcg_plan_solve", _i, [_vp, _d, _i, _i, C.POINTER(_i), C.POINTER(_d),
                                                  C.POINTER(_i), _vp]),
    "pcg_plan_destroy": _sig("pcg_plan_destroy", _i, [_vp]),
    "pcg_plan_tune": _sig("pcg_plan_tune", _i, [_vp, _i, C.POINTER(Tuning), _vp]),
    "pcg_plan_configure": _sig("pcg_plan_configure", _i, [_vp, C.POINTER(Tuning)]),
    "pcg_plan_config": _sig("pcg_plan_config", _i, [_vp, C.POINTER(Tuning)]),
    "pod2g_mark": _sig("pod2g_mark", _i, [_i, _vp]),
    "pod2g_spmv": _sig("pod2g_spmv", _i, [_PP, _vp, _i, _vp, _vp, _vp]),
    "pod2g_jacobi": _sig("pod2g_jacobi", _i, [_PP, _vp, _vp, _i, _d, _i, _vp, _vp, _vp, _vp]),
    "pod2g_pod_basis_bytes": _sig("pod2g_pod_basis_bytes", _sz, [_i, _i, _i]),
    "pod2g_pod_basis": _sig("pod2g_pod_basis", _i, [_vp, _i, _i, _i, _vp, _vp, _vp, _sz, _vp]),
}


def exported_symbols():
    return sorted(_f)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def strerror(status: int) -> str:
    return _f["pod2g_strerror"](int(status)).decode()


def check(status: int, where: str = ""):
    if status != OK:
        raise Pod2gError(status, where)
    return status


# ---- pattern --------------------------------------------------------------
def make_mesh(dim, N, n_terms, nu=0.3, kl_scale=0.3) -> Mesh:
    return Mesh(dim, N, n_terms, nu, kl_scale)


def pod2g_pattern_bytes(mesh: Mesh) -> int:
    return _f["pod2g_pattern_bytes"](C.byref(mesh))


def pod2g_pattern_build(mesh: Mesh, dbuf, nbytes: int, out: Pattern, stream=None) -> int:
    return _f["pod2g_pattern_build"](C.byref(mesh), _ptr(dbuf), nbytes, C.byref(out), _stream(stream))


# ---- assembly -------------------------------------------------------------
def pod2g_assemble_bytes(pat: Pattern, batch: int) -> int:
    return _f["pod2g_assemble_bytes"](C.byref(pat), batch)


def pod2g_assemble(pat: Pattern, xi, batch, vals, vals32, dinv, f, work, nbytes, stream=None) -> int:
    return _f["pod2g_assemble"](C.byref(pat), _ptr(xi), batch, _ptr(vals), _ptr(vals32), _ptr(dinv),
                                _ptr(f), _ptr(work), nbytes, _stream(stream))


# ---- setup ----------------------------------------------------------------
def pod2g_setup_bytes(pat: Pattern, k: int, batch: int, precision: int) -> int:
    return _f["pod2g_setup_bytes"](C.byref(pat), k, batch, precision)


def pod2g_setup(pat, vals, vals32, dinv, P, k, omega, nu_pre, nu_post, precision, batch,
                power_iters, work, nbytes, out: Prec, stream=None) -> int:
    return _f["pod2g_setup"](C.byref(pat), _ptr(vals), _ptr(vals32), _ptr(dinv), _ptr(P), k,
                             float(omega), nu_pre, nu_post, precision, batch, power_iters,
                             _ptr(work), nbytes, C.byref(out), _stream(stream))


def pod2g_setup_slot(prec: Prec, slot: int, power_iters: int, stream=None) -> int:
    return _f["pod2g_setup_slot"](C.byref(prec), slot, power_iters, _stream(stream))


def pod2g_set_smoother(prec: Prec, smoother: int) -> int:
    return _f["pod2g_set_smoother"](C.byref(prec), smoother)


def pod2g_gauss_seidel(pat, vals, dinv, batch, nsweeps, backward, b, x, stream=None) -> int:
    return _f["pod2g_gauss_seidel"](C.byref(pat), _ptr(vals), _ptr(dinv), batch, nsweeps,
                                    int(backward), _ptr(b), _ptr(x), _stream(stream))


def pod2g_setup_status(prec: Prec, stream=None):
    st = (C.c_int * prec.batch)()
    lam = (C.c_double * prec.batch)()
    check(_f["pod2g_setup_status"](C.byref(prec), st, lam, _stream(stream)), "pod2g_setup_status")
    return list(st), list(lam)


# ---- cycle / solve ----------------------------------------------------------
def pod2g_apply_bytes(prec: Prec) -> int:
    return _f["pod2g_apply_bytes"](C.byref(prec))


def pod2g_apply(prec: Prec, r, s, work, nbytes, stream=None) -> int:
    return _f["pod2g_apply"](C.byref(prec), _ptr(r), _ptr(s), _ptr(work), nbytes, _stream(stream))


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024   # POD2G_NOALLOC_SCRATCH_BYTES


def pod2g_apply_noalloc(prec: Prec, r, s, stream=None) -> int:
    return _f["pod2g_apply_noalloc"](C.byref(prec), _ptr(r), _ptr(s), _stream(stream))


def pcg_solve_bytes(pat: Pattern, batch: int, k: int, precision: int) -> int:
    return _f["pcg_solve_bytes"](C.byref(pat), batch, k, precision)


def pcg_solve(pat, vals, batch, prec, f, u, rtol, maxit, beta, work, nbytes, stream=None):
    """Returns (status, iters[batch], relres[batch], status[batch])."""
    it = (C.c_int * batch)()
    rr = (C.c_double * batch)()
    st = (C.c_int * batch)()
    ret = _f["pcg_solve"](C.byref(pat), _ptr(vals), batch, C.byref(prec) if prec is not None else None,
                          _ptr(f), _ptr(u), float(rtol), int(maxit), int(beta), it, rr, st,
                          _ptr(work), nbytes, _stream(stream))
    return ret, list(it), list(rr), list(st)


def pod2g_stationary_solve(pat, vals, batch, prec, f, u, rtol, maxit, work, nbytes, stream=None):
    """Returns (status, iters[batch], relres[batch], status[batch])."""
    it = (C.c_int * batch)()
    rr = (C.c_double * batch)()
    st = (C.c_int * batch)()
    ret = _f["pod2g_stationary_solve"](C.byref(pat), _ptr(vals), batch, C.byref(prec), _ptr(f),
                                       _ptr(u), float(rtol), int(maxit), it, rr, st, _ptr(work),
                                       nbytes, _stream(stream))
    return ret, list(it), list(rr), list(st)


def pod2g_rom_bytes(prec: Prec) -> int:
    return _f["pod2g_rom_bytes"](C.byref(prec))


def pod2g_rom_start(prec: Prec, f, u, work, nbytes, stream=None) -> int:
    return _f["pod2g_rom_start"](C.byref(prec), _ptr(f), _ptr(u), _ptr(work), nbytes, _stream(stream))


def pcg_solve_timed(pat, vals, batch, prec, f, u, rtol, maxit, beta, work, nbytes, timer,
                    stream=None):
    it = (C.c_int * batch)()
    rr = (C.c_double * batch)()
    st = (C.c_int * batch)()
    ret = _f["pcg_solve_timed"](C.byref(pat), _ptr(vals), batch,
                                C.byref(prec) if prec is not None else None, _ptr(f), _ptr(u),
                                float(rtol), int(maxit), int(beta), it, rr, st, _ptr(work), nbytes,
                                C.byref(timer) if timer is not None else None, _stream(stream))
    return ret, list(it), list(rr), list(st)


def pod2g_timer_create(kernel: int, per_call: int) -> Timer:
    t = Timer()
    check(_f["pod2g_timer_create"](kernel, per_call, C.byref(t)), "pod2g_timer_create")
    return t


def pod2g_timer_reset(t: Timer) -> int:
    return _f["pod2g_timer_reset"](C.byref(t))


def pod2g_timer_destroy(t: Timer) -> int:
    return _f["pod2g_timer_destroy"](C.byref(t))


def pcg_plan_create(pat, vals, batch, prec, f, u, chunk, work, nbytes, timer=None):
    """Returns an opaque plan handle (int) or raises Pod2gError."""
    h = C.c_void_p()
    check(_f["pcg_plan_create"](C.byref(pat), _ptr(vals), batch,
                                C.byref(prec) if prec is not None else None, _ptr(f), _ptr(u),
                                chunk, _ptr(work), nbytes,
                                C.byref(timer) if timer is not None else None, C.byref(h)),
          "pcg_plan_create")
    return h.value


def pcg_plan_solve(plan, rtol, maxit, beta, batch, stream=None):
    it = (C.c_int * batch)()
    rr = (C.c_double * batch)()
    st = (C.c_int * batch)()
    ret = _f["pcg_plan_solve"](plan, float(rtol), int(maxit), int(beta), it, rr, st, _stream(stream))
    return ret, list(it), list(rr), list(st)


def pcg_plan_tune(plan, trials, stream=None) -> Tuning:
    t = Tuning()
    check(_f["pcg_plan_tune"](plan, trials, C.byref(t), _stream(stream)), "pcg_plan_tune")
    return t


def pcg_plan_configure(plan, t: Tuning) -> int:
    return _f["pcg_plan_configure"](plan, C.byref(t))


def pcg_plan_config(plan) -> Tuning:
    t = Tuning()
    check(_f["pcg_plan_config"](plan, C.byref(t)), "pcg_plan_config")
    return t


def pcg_plan_destroy(plan) -> int:
    return _f["pcg_plan_destroy"](plan)


# ---- served solves ----------------------------------------------------------
def pod2g_server_create(groups, chunk, stream=None):
    """groups: list of (pattern, vals, prec, f, u, work, nbytes); the Pattern
    and Prec structures must stay alive while the server does.  Returns the
    opaque server handle (int) or raises Pod2gError."""
    arr = (Group * len(groups))()
    for i, (pat, vals, prec, f, u, work, nbytes) in enumerate(groups):
        arr[i] = Group(C.addressof(pat), _ptr(vals), C.addressof(prec), _ptr(f), _ptr(u), _ptr(work),
                       nbytes)
    h = C.c_void_p()
    check(_f["pod2g_server_create"](arr, len(groups), chunk, C.byref(h), _stream(stream)),
          "pod2g_server_create")
    return h.value


def pod2g_server_admit(server, group, slot, rtol, maxit, beta, stream=None) -> int:
    return _f["pod2g_server_admit"](server, group, slot, float(rtol), int(maxit), int(beta),
                                    _stream(stream))


def pod2g_serve_step(server, info, stream=None) -> int:
    """info: pinned host tensor (uint8) of pod2g_server_slots * sizeof(SlotInfo) bytes."""
    return _f["pod2g_serve_step"](server, _ptr(info), _stream(stream))


def pod2g_serve_step_group(server, group, info, stream=None) -> int:
    return _f["pod2g_serve_step_group"](server, group, _ptr(info), _stream(stream))


def pod2g_serve_step_prefix(server, group, nslots, info, stream=None) -> int:
    return _f["pod2g_serve_step_prefix"](server, group, nslots, _ptr(info), _stream(stream))


def pod2g_stream_create_cus(cu_first: int, cu_count: int) -> int:
    """A stream on compute units [cu_first, cu_first + cu_count) (raw handle)."""
    h = C.c_void_p()
    check(_f["pod2g_stream_create_cus"](cu_first, cu_count, C.byref(h)), "pod2g_stream_create_cus")
    return h.value


def pod2g_stream_destroy(stream: int) -> int:
    return _f["pod2g_stream_destroy"](stream)


def pod2g_server_slots(server) -> int:
    return _f["pod2g_server_slots"](server)


def pod2g_server_destroy(server) -> int:
    return _f["pod2g_server_destroy"](server)


def pod2g_mark(which: int, stream=None) -> int:
    return _f["pod2g_mark"](which, _stream(stream))


def pod2g_spmv(pat, vals, batch, x, y, stream=None) -> int:
    return _f["pod2g_spmv"](C.byref(pat), _ptr(vals), batch, _ptr(x), _ptr(y), _stream(stream))


def pod2g_jacobi(pat, vals, dinv, batch, omega, nsweeps, b, x, tmp, stream=None) -> int:
    return _f["pod2g_jacobi"](C.byref(pat), _ptr(vals), _ptr(dinv), batch, float(omega), nsweeps,
                              _ptr(b), _ptr(x), _ptr(tmp), _stream(stream))


# ---- offline POD ----------------------------------------------------------
def pod2g_pod_basis_bytes(n, N, k) -> int:
    return _f["pod2g_pod_basis_bytes"](n, N, k)


def pod2g_pod_basis(U, n, N, k, P, lam, work, nbytes, stream=None) -> int:
    return _f["pod2g_pod_basis"](_ptr(U), n, N, k, _ptr(P), _ptr(lam), _ptr(work), nbytes,
                                 _stream(stream))
