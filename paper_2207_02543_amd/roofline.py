"""Algorithmic HBM bytes of the library's kernels, per launch.

Each stored matrix value (the symmetric half of K), index and vector entry
a kernel needs is counted once; what all instances of a batch share (block-column indices, the basis
P) is counted once per launch.  Dividing by a launch's duration gives the
rate that is compared with the 8 TB/s HBM3E peak; dividing the profiler's
FETCH_SIZE + WRITE_SIZE bytes by the same count shows how far the kernel's
real traffic is from this minimum (re-reads when above 1, cache hits when
below).

`w` is an ``inputs.Workload``; `tuning` the plan's launch parameters
(``Plan.config()``), or None for the library's size-based defaults.
"""
from __future__ import annotations

HBM_PEAK_GBS = 8000.0

# kernel key -> regular expression on the kernel's name in a rocprofv3 trace
KERNEL_PATTERNS = {
    "spmv_pq": r"k_spmv_pq<",
    "pdir": r"k_pdir\(",
    "sweep": r"k_sweep<\d, \w+, false>",
    "sweep_final": r"k_sweep<\d, \w+, true>",
    "restrict": r"k_resid32<|k_restrict<",
    "ptr_b": r"k_ptr_b[<(]",
    "prolong": r"k_prolong",
    "update": r"k_update<|k_update_sweep<",
    "kp": r"k_kp<",
    "kc": r"k_kc[<(]",
}


def stored_values(w):
    """Values of K stored per instance: the symmetric half of the block-ELL
    layout (own and upper blocks, planes of n + dim rows)."""
    S = 3 ** w.dim
    return (w.n + w.dim) * (S // 2 + 1) * w.dim


def _defaults(w, tuning):
    n, B = w.n, w.batch
    small = n * B <= (1 << 20)
    if tuning is None:
        return small, small
    return bool(tuning.get("fuse_dir", small)), bool(tuning.get("fuse_upd", small))


def kernel_bytes(w, kernel, tuning=None, smoother="jacobi"):
    """Algorithmic bytes of one launch of `kernel` (a KERNEL_PATTERNS key)
    over the batch of workload `w`."""
    mixed = w.precision == "mixed"
    S = 3 ** w.dim
    n, nn, k, B = w.n, w.n_nodes_free, w.k, w.batch
    nvals = stored_values(w)
    batched = mixed and 4 <= B <= 32 and k > 0        # MFMA products over the batch
    fuse_dir, fuse_upd = _defaults(w, tuning)
    fuse_upd = fuse_upd and smoother == "jacobi"
    vb = 4 if mixed else 8                              # cycle precision
    idx = 4 * S * nn                                    # block-column indices
    if kernel == "sweep":        # K, x (gathered), b, D^-1 read; x_out written
        return idx + B * (vb * nvals + 4 * vb * n)
    if kernel == "sweep_final":  # + r (FP64) read, s (FP64) written instead of x_out
        return idx + B * (vb * nvals + 3 * vb * n + 16 * n)
    if kernel == "spmv_pq":      # K, p read (fused: s, p_old read, p written); q written
        return idx + B * (8 * nvals + (32 if fuse_dir else 16) * n)
    if kernel == "pdir":         # p = s + beta p_old: s, p_old read, p written
        return B * 24 * n
    if kernel == "restrict":
        if batched:              # r' = b - K x in FP32: K, x, b read; r' written
            return idx + B * (4 * nvals + 12 * n)
        # K, x, b read, P once; r' also written where the first post-sweep
        # uses it with K P (FP64 path, or FP32 in 3D)
        saved = vb * n if (not mixed or w.dim == 3) else 0
        return idx + vb * k * n + B * (vb * nvals + 2 * vb * n + saved)
    if kernel == "ptr_b":        # P^T R over the batch: P (FP32) once, r' per instance
        return 4 * k * n + B * 4 * n
    if kernel == "prolong":
        # x + P e + omega D^-1 (r' - K P e) where K P is at hand (FP64 path,
        # or FP32 in 3D): P once, K P per instance, x, r', D^-1 read, x written
        if not mixed or w.dim == 3:
            return vb * k * n + B * (vb * k * n + 4 * vb * n)
        return vb * k * n + B * 2 * vb * n
    if kernel == "update" and fuse_upd:
        return idx + B * (vb * nvals + 48 * n + (8 * n if mixed else 0) + (4 * n if mixed else 0)
                          + 2 * vb * n)
    if kernel == "update":       # u, p, r, q (, s) read; u, r written; cycle input and first sweep
        return B * (48 * n + (8 * n if mixed else 0) + (12 * n if mixed else 24 * n))
    if kernel == "kp":           # setup K P: K per instance, P once, K P (FP64) written
        return idx + 8 * k * n + B * (8 * nvals + 8 * k * n)
    if kernel == "kc":           # setup P^T (K P): P once, K P per instance
        return 8 * k * n + B * 8 * k * n
    raise ValueError(kernel)
