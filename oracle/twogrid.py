"""Damped-Jacobi relaxation and the POD two-grid cycle (Sec. 2.2 Alg. 2,
Sec. 3.3 Eq. 30).

One cycle applied to a right-hand side r from a zero initial guess is the
preconditioner of Alg. 3 (s = AMG(0; K, r, r1, r2)):

1. r1 damped-Jacobi sweeps x <- x + omega D^{-1} (r - K x) from x = 0
   (pre-relaxation);
2. residual r' = r - K x;
3. restriction r_c = P^T r' and the Galerkin coarse solve
   (P^T K P) e_c = r_c, by Cholesky factors L L^T = P^T K P;
4. prolongation and correction x <- x + P e_c;
5. r2 damped-Jacobi sweeps on K x = r (post-relaxation).

The paper analyses Gauss-Seidel relaxation but leaves the smoother of its
experiments open; damped Jacobi keeps the cycle symmetric, so it is a valid
CG preconditioner.  ``smoother="sgs"`` uses Gauss-Seidel instead, forward
sweeps before and backward sweeps after the coarse correction in one fixed
(multicolour) order, which keeps the cycle symmetric as well (in the FP32
mode its sweeps round their result to binary32 after each sweep only).

``precision="fp32"`` emulates an FP32 preconditioner: K, D^{-1}, P and the
residual scaled by ``scale`` are rounded to binary32 and every cycle step
except the coarse Cholesky solve runs in binary32; the coarse solve stays
FP64.  The returned vector is converted back and divided by ``scale``.  The
default scale is the power of two 2^-e with ||r|| = m 2^e, m in [0.5, 1):
scaling by a power of two commutes with binary32 rounding, so it only keeps
the cycle's values inside the binary32 range and changes no result bit.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

ENOTSPD = -4


class NotSPD(ArithmeticError):
    status = ENOTSPD


def jacobi_sweeps(K, dinv, b, x, omega, nsweeps):
    """nsweeps damped-Jacobi iterations x <- x + omega D^{-1} (b - K x)."""
    for _ in range(nsweeps):
        x = x + omega * dinv * (b - K @ x)
    return x


def multicolor_order(dim, N):
    """Free DOFs in multicolour order on the node grid (the Gauss-Seidel
    relaxation of Sec. 2.2 run colour by colour): node (i, j[, l]) has colour
    (i mod 2) + 2 (j mod 2) [+ 4 (l mod 2)]; colours in increasing order,
    nodes by id within a colour, components in order.  Two nodes of one
    colour differ by an even, non-zero step in some coordinate, so they share
    no element and no matrix entry."""
    from .fem import free_dofs
    fd = free_dofs(dim, N)
    nodes = fd[::dim] // dim                  # free nodes in rank order
    i = nodes % (N + 1)
    j = (nodes // (N + 1)) % (N + 1)
    colour = (i % 2) + 2 * (j % 2)
    if dim == 3:
        colour = colour + 4 * ((nodes // (N + 1) ** 2) % 2)
    ranks = np.argsort(colour, kind="stable")
    return (dim * ranks[:, None] + np.arange(dim)[None, :]).reshape(-1)


def gauss_seidel_sweeps(K, b, x, order, nsweeps, backward=False):
    """nsweeps Gauss-Seidel sweeps visiting the unknowns in `order` (reversed
    for backward sweeps): each x_i in turn takes the value that zeroes
    residual i given the current x.  One sweep is x <- x + T^{-1} (b - K x)
    with T the lower (backward: upper) triangle, diagonal included, of K in
    that order."""
    K = sp.csr_matrix(K)
    Kp = K[order][:, order].tocsr()
    T = sp.tril(Kp, format="csr") if not backward else sp.triu(Kp, format="csr")
    from scipy.sparse.linalg import spsolve_triangular
    x = np.array(x, copy=True)
    for _ in range(nsweeps):
        rp = (b - K @ x)[order]
        dx = spsolve_triangular(T, rp, lower=not backward)
        x[order] = x[order] + dx
    return x


def residual(K, b, x):
    """r' = b - K x, recomputed after pre-relaxation (Alg. 2)."""
    return b - K @ x


def restrict(P, rr):
    """r_c = P^T r' (Alg. 2 restriction with P = Phi_r, Sec. 3.3 Eq. 30)."""
    return P.T @ rr


def prolong(x, P, ec):
    """x + P e_c (Alg. 2 prolongation and correction)."""
    return x + P @ ec


def coarse_matrix(K, P):
    """K_c = P^T K P (Alg. 2, restrict-and-solve step; Sec. 3.3 Eq. 28)."""
    return P.T @ (K @ P)


def coarse_factor(K, P):
    """Lower Cholesky factor of K_c; raises NotSPD on a non-positive pivot."""
    Kc = coarse_matrix(K, P)
    try:
        return np.linalg.cholesky(Kc)
    except np.linalg.LinAlgError as e:
        raise NotSPD(str(e)) from e


def coarse_solve(L, rc):
    """e_c with L L^T e_c = r_c (forward then backward substitution)."""
    y = sla.solve_triangular(L, rc, lower=True)
    return sla.solve_triangular(L.T, y, lower=False)


class TwoGrid:
    """The POD two-grid cycle with fixed K, D^{-1}, P and smoother settings."""

    def __init__(self, K, P, omega, nu_pre=2, nu_post=2, precision="fp64", smoother="jacobi",
                 order=None):
        self.smoother = smoother
        self.order = order
        if smoother == "sgs" and order is None:
            raise ValueError("the symmetric Gauss-Seidel smoother needs the sweep order")
        self.K = sp.csr_matrix(K)
        self.dinv = 1.0 / self.K.diagonal()
        self.P = np.asarray(P, dtype=np.float64)
        self.omega = float(omega)
        self.nu_pre = int(nu_pre)
        self.nu_post = int(nu_post)
        self.precision = precision
        self.L = coarse_factor(self.K, self.P) if self.P.shape[1] > 0 else None
        if precision == "fp32":
            self.K32 = self.K.astype(np.float32)
            self.dinv32 = self.dinv.astype(np.float32)
            self.P32 = self.P.astype(np.float32)
            self.omega32 = np.float32(self.omega)

    # -- FP64 cycle ---------------------------------------------------------
    def _relax(self, K, dinv, b, x, w, nsweeps, post):
        if self.smoother == "sgs":
            # symmetric: forward sweeps before, backward sweeps after the
            # coarse correction
            y = gauss_seidel_sweeps(K, b.astype(np.float64), x.astype(np.float64), self.order,
                                    nsweeps, backward=post)
            return y.astype(x.dtype)
        return jacobi_sweeps(K, dinv, b, x, w, nsweeps)

    def _cycle64(self, r):
        K, dinv, P, w = self.K, self.dinv, self.P, self.omega
        x = np.zeros_like(r)
        x = self._relax(K, dinv, r, x, w, self.nu_pre, False)
        if self.L is not None:
            rr = residual(K, r, x)
            rc = restrict(P, rr)
            ec = coarse_solve(self.L, rc)
            x = prolong(x, P, ec)
        x = self._relax(K, dinv, r, x, w, self.nu_post, True)
        return x

    # -- FP32-emulated cycle (coarse solve in FP64) --------------------------
    def _cycle32(self, r, scale):
        # every operand of the relaxation, residual, restriction and
        # prolongation is binary32, so numpy and scipy compute each of these
        # steps in binary32 (no rounding of a wider result afterwards); only
        # the coarse solve widens its input to FP64 and rounds its output
        K, dinv, P, w = self.K32, self.dinv32, self.P32, self.omega32
        b = (r * scale).astype(np.float32)
        x = np.zeros_like(b)
        x = self._relax(K, dinv, b, x, w, self.nu_pre, False)
        if self.L is not None:
            rr = residual(K, b, x)
            rc = restrict(P, rr)
            ec = coarse_solve(self.L, rc.astype(np.float64)).astype(np.float32)
            x = prolong(x, P, ec)
        x = self._relax(K, dinv, b, x, w, self.nu_post, True)
        return x.astype(np.float64) / scale

    def apply(self, r, scale=None):
        """s = B r: one cycle from the zero initial guess."""
        r = np.asarray(r, dtype=np.float64)
        if self.precision == "fp32":
            if scale is None:
                nr = np.linalg.norm(r)
                scale = float(np.ldexp(1.0, -np.frexp(nr)[1])) if nr > 0 else 1.0
            return self._cycle32(r, scale)
        return self._cycle64(r)

    __call__ = apply


def power_lambda_max(K, dinv, iters=50):
    """Power-iteration estimate of lambda_max(D^{-1} K) from the all-ones
    start vector (setup guard: the damped-Jacobi smoother needs
    omega * lambda_max < 2)."""
    x = np.ones(K.shape[0])
    lam = 0.0
    for _ in range(iters):
        y = dinv * (K @ x)
        lam = float(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    return lam
