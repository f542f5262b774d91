"""Preconditioned conjugate gradients with the POD two-grid preconditioner
(Sec. 3.4, Alg. 3; generic PCG Sec. 2.1, Alg. 1), the standalone two-grid
solver (Sec. 2.2 Alg. 2 with P = Phi_r, Sec. 3.3) and the POD-Galerkin
reduced solve (Sec. 3.3, steps 3-4).

Readings of the paper taken here:

* The loop guards print ``while ||r|| < delta``; the loop runs while the
  residual is above the tolerance.
* The tolerance is relative to the load: stop when ||r|| <= tol ||f||.
* The recursively updated residual drives the loop; at exit the true
  residual f - K u is recomputed, and if it is above the tolerance it
  replaces r, the preconditioned residual is recomputed, the search
  direction restarts from it, and iterating continues.
* The iteration count is the number of completed updates of u; an initial
  guess that already meets the tolerance returns 0 iterations.
* beta: "fr" is the ratio of Alg. 1/3 (r_{k+1}^T s_{k+1} / r_k^T s_k);
  "pr" is the flexible Polak-Ribiere form
  (r_{k+1}^T s_{k+1} - r_{k+1}^T s_k) / r_k^T s_k, which equals "fr" in exact
  arithmetic for a fixed SPD preconditioner (r_{k+1}^T s_k = 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

OK = 0
EMAXIT = -6
EBREAKDOWN = -7
ENAN = -8


@dataclass
class Result:
    u: np.ndarray
    iters: int
    relres: float          # true ||f - K u|| / ||f|| at exit
    status: int
    directions: list = field(default_factory=list)   # p_k (when recorded)
    rnorms: list = field(default_factory=list)       # recursive ||r_k||
    replacements: list = field(default_factory=list)  # iterations at which the
                                                      # true residual replaced r


def pcg(K, f, u0, precond=None, tol=1e-8, maxit=5000, beta="fr",
        record=False) -> Result:
    """Alg. 3 (Alg. 1 with T^{-1} = one two-grid cycle); precond=None gives
    plain CG (T = I)."""
    apply = precond if precond is not None else (lambda r: r.copy())
    u = np.array(u0, dtype=np.float64, copy=True)
    f = np.asarray(f, dtype=np.float64)
    fnorm = np.linalg.norm(f)
    thresh = tol * fnorm
    r = f - K @ u
    res = Result(u, 0, 0.0, OK)

    def finish(status):
        res.u = u
        res.relres = float(np.linalg.norm(f - K @ u) / fnorm)
        res.status = status
        return res

    rn = np.linalg.norm(r)
    if not np.isfinite(rn):
        return finish(ENAN)
    if rn <= thresh:
        return finish(OK)
    s = apply(r)
    p = s.copy()
    rho = float(r @ s)
    if not rho > 0.0:
        return finish(EBREAKDOWN)
    k = 0
    while True:
        if k >= maxit:
            return finish(EMAXIT)
        if record:
            res.directions.append(p.copy())
        q = K @ p
        gamma = float(p @ q)
        if not gamma > 0.0:
            return finish(EBREAKDOWN if np.isfinite(gamma) else ENAN)
        alpha = rho / gamma
        u = u + alpha * p
        r = r - alpha * q
        k += 1
        res.iters = k
        rn = np.linalg.norm(r)
        if record:
            res.rnorms.append(rn)
        if not np.isfinite(rn):
            return finish(ENAN)
        restart = False
        if rn <= thresh:
            rt = f - K @ u
            if np.linalg.norm(rt) <= thresh:
                return finish(OK)
            r = rt                       # residual replacement
            restart = True
            res.replacements.append(k)
        s_prev = s
        s = apply(r)
        rho_new = float(r @ s)
        if not rho_new > 0.0:
            return finish(EBREAKDOWN if np.isfinite(rho_new) else ENAN)
        if restart:
            b = 0.0
        elif beta == "fr":
            b = rho_new / rho
        else:
            b = (rho_new - float(r @ s_prev)) / rho
        p = s + b * p
        rho = rho_new


def twogrid_solve(K, f, u0, cycle, tol=1e-8, maxit=5000) -> Result:
    """Standalone POD-2G solver: u <- u + B (f - K u) until
    ||f - K u|| <= tol ||f|| (Alg. 2 with the error operator of Eq. 30)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    f = np.asarray(f, dtype=np.float64)
    fnorm = np.linalg.norm(f)
    k = 0
    res = Result(u, 0, 0.0, OK)
    while True:
        r = f - K @ u
        rn = np.linalg.norm(r)
        res.rnorms.append(rn)
        if not np.isfinite(rn):
            res.status = ENAN
            break
        if rn <= tol * fnorm:
            break
        if k >= maxit:
            res.status = EMAXIT
            break
        u = u + cycle(r)
        k += 1
    res.u = u
    res.iters = k
    res.relres = float(np.linalg.norm(f - K @ u) / fnorm)
    return res


def rom_solve(K, f, P, L):
    """POD-Galerkin reduced solve: K_r u_r = P^T f with K_r = L L^T = P^T K P,
    then u = P u_r (Sec. 3.3, Eqs. 28-29)."""
    from .twogrid import coarse_solve
    return P @ coarse_solve(L, P.T @ np.asarray(f, dtype=np.float64))
