"""Proper orthogonal decomposition by the method of snapshots (Sec. 3.3).

Given snapshots U = [u_1 ... u_N] (d x N), the correlation matrix is
R = U U^T (no mean centring).  Instead of R's d x d eigenproblem, the
N x N problem U^T U Psi = Psi Lambda is solved and the basis follows from
Phi = U Psi Lambda^{-1/2} (Sec. 3.3, step 1, Eq. 26).  The reduced basis
Phi_r keeps the r columns of the largest eigenvalues (step 2).  Phi_r is the
prolongation P of the two-grid cycle (Sec. 3.3, Eq. 30).
"""
from __future__ import annotations

import numpy as np


def snapshot_gram(U: np.ndarray) -> np.ndarray:
    """G = U^T U."""
    return U.T @ U


def pod_basis(U: np.ndarray, r: int):
    """Return (Phi_r, lam) with lam all eigenvalues of U^T U in descending
    order and Phi_r = U Psi_r Lambda_r^{-1/2} (d x r)."""
    G = snapshot_gram(U)
    lam, Psi = np.linalg.eigh(G)          # ascending
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    Psi = Psi[:, order]
    # numerical rank: eigenvalues below N eps lam_1 are rounding noise
    if r > U.shape[1] or lam[r - 1] <= U.shape[1] * np.finfo(float).eps * lam[0]:
        raise ValueError("snapshot matrix has rank < r")
    Phi_r = U @ Psi[:, :r] / np.sqrt(lam[:r])[None, :]
    return Phi_r, lam
