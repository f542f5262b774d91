"""Shared helpers of the GPU parity tests (test-side only)."""
import numpy as np


def flush(msg):
    print(msg, flush=True)


def block_ell_expected(K, dim, N, colblk, n):
    """The oracle's K laid out in the library's symmetric half block-ELL
    order: vals[((s - H) * dim + b) * (n + dim) + row] for the own slot H
    and the upper slots s > H (zero for an absent neighbour), and zero rows
    n .. n + dim - 1 (the zero node) in every plane."""
    S = 3 ** dim
    H = S // 2
    nn = n // dim
    ns = n + dim
    rows = np.arange(n)
    nodes = rows // dim
    out = np.zeros((H + 1) * dim * ns)
    for s in range(H, S):
        nb = colblk[s * nn + nodes]
        valid = (nb != nodes) | (s == H)
        for b in range(dim):
            cols = dim * nb + b
            v = np.asarray(K[rows[valid], cols[valid]]).ravel()
            blk = np.zeros(n)
            blk[valid] = v
            p = (s - H) * dim + b
            out[p * ns:p * ns + n] = blk
    return out


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    """Element-wise error: max |a - b| over max |b|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
