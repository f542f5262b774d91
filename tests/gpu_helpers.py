"""Shared helpers of the GPU parity tests (test-side only)."""
import numpy as np


def flush(msg):
    print(msg, flush=True)


def block_ell_expected(K, dim, N, colblk, n):
    """The oracle's K laid out in the library's block-ELL order
    vals[(s * dim + b) * n + row] (zero in absent-neighbour slots)."""
    S = 3 ** dim
    nn = n // dim
    rows = np.arange(n)
    nodes = rows // dim
    out = np.zeros(S * dim * n)
    center = S // 2
    for s in range(S):
        nb = colblk[s * nn + nodes]
        valid = (nb != nodes) | (s == center)
        for b in range(dim):
            cols = dim * nb + b
            v = np.asarray(K[rows[valid], cols[valid]]).ravel()
            blk = np.zeros(n)
            blk[valid] = v
            out[(s * dim + b) * n:(s * dim + b + 1) * n] = blk
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
