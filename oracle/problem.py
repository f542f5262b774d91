"""Oracle-side construction of a workload from the seeded inputs.

Offline phase (Sec. 3.4, with the snapshot step of Sec. 3.3): training
parameters -> FE solves u_i -> U -> POD basis P = Phi_r.  The training and
reference ("exact") solves are sparse direct solves (a library LU
factorisation), so the snapshots carry no iteration error.  Online phase per
query: assemble K(theta), build the two-grid preconditioner, and run PCG from
the warm start u* + noise (the surrogate stand-in of Sec. 3.2, Eq. 25).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, pod
from .pcg import pcg
from .twogrid import TwoGrid


@dataclass
class Query:
    xi: np.ndarray
    K: object
    f: np.ndarray
    u_exact: np.ndarray
    x0: np.ndarray


def stiffness(w, xi):
    E = fem.young_modulus(w.dim, w.N, xi, w.kl_scale)
    return fem.assemble(w.dim, w.N, w.nu, E)


def direct_solve(K, f):
    return spla.splu(K.tocsc()).solve(f)


def snapshots(w, xis):
    """U = [u_1 ... u_N] from direct solves at the training parameters."""
    f = fem.traction_load(w.dim, w.N)
    return np.stack([direct_solve(stiffness(w, xi), f) for xi in xis], axis=1)


def basis(w, xis, k=None):
    U = snapshots(w, xis)
    P, lam = pod.pod_basis(U, w.k if k is None else k)
    return P, lam, U


def query(w, xi, g):
    """Assemble a query and its warm start exact + noise (g: raw noise)."""
    from paper_2207_02543_amd.inputs import warm_start
    K = stiffness(w, xi)
    f = fem.traction_load(w.dim, w.N)
    u = direct_solve(K, f)
    return Query(np.asarray(xi), K, f, u, warm_start(u, g, w.noise))


def solve_query(w, q: Query, P, precision=None, beta=None, tol=None,
                maxit=5000, record=False):
    prec = precision or ("fp32" if w.precision == "mixed" else "fp64")
    M = TwoGrid(q.K, P, w.omega, w.nu_pre, w.nu_post, precision=prec)
    b = beta or ("pr" if prec == "fp32" else "fr")
    return pcg(q.K, q.f, q.x0, M, tol=w.tol if tol is None else tol,
               maxit=maxit, beta=b, record=record)
