"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds no arithmetic of the method itself: it only names the
workloads (mesh size, number of random-field terms, number of POD modes,
smoother settings, tolerance) and draws the random numbers a workload needs
(the standard-normal field coefficients xi and the warm-start noise g).  Both
sides receive the same draws and compute everything else on their own.

The paper's parametrised problems (Sec. 4) need meshes and data that are not
available, so these synthetic elasticity problems stand in for them: a
parametrised SPD stiffness system K(theta) u = f (Sec. 2.1, Eq. 6) with
theta = xi, a POD basis from training solves (Sec. 3.3) and one warm-started
PCG solve per query (Sec. 3.4, Alg. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

TRAIN_SEED0 = 1000   # training parameter i uses seed TRAIN_SEED0 + i
QUERY_SEED0 = 2000   # query parameter j uses seed QUERY_SEED0 + j
NOISE_SEED0 = 3000   # warm-start noise of query j uses seed NOISE_SEED0 + j
ARRIVAL_SEED = 4000  # request stream of the serving workload


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int            # 2: plane-stress Q4 on the unit square; 3: Hex8 on the unit cube
    N: int              # elements per side
    n_terms: int        # random-field terms (length of xi)
    k: int              # POD modes kept (coarse size)
    n_train: int        # training solves for the snapshot matrix
    batch: int = 1      # query instances solved together
    precision: str = "fp64"   # "fp64" or "mixed" (FP32 preconditioner, FP64 outer)
    nu: float = 0.3     # Poisson ratio
    omega: float = 2.0 / 3.0  # damped-Jacobi weight
    nu_pre: int = 2     # pre-smoothing sweeps
    nu_post: int = 2    # post-smoothing sweeps
    tol: float = 1e-8   # relative residual ||f - K u|| / ||f||
    train_tol: float = 1e-12  # relative residual of the training (snapshot) solves
    kl_scale: float = 0.3
    noise: float = 0.01  # warm start = exact + noise * ||exact|| * g / ||g||

    @property
    def n_nodes_free(self) -> int:
        if self.dim == 2:
            return self.N * (self.N + 1)
        return (self.N + 1) ** 2 * self.N

    @property
    def n(self) -> int:
        return self.dim * self.n_nodes_free

    @property
    def n_elems(self) -> int:
        return self.N ** self.dim


# 2D workloads keep omega = 2/3; 3D Hex8 uses omega = 1/2 (omega = 2/3 makes the
# two-grid preconditioner indefinite for Hex8 elasticity at nu = 0.3).
WORKLOADS = {
    "c1": Workload("c1", dim=2, N=32, n_terms=8, k=10, n_train=40),
    "c2": Workload("c2", dim=2, N=256, n_terms=12, k=20, n_train=100),
    "c3": Workload("c3", dim=3, N=64, n_terms=16, k=30, n_train=150, batch=32,
                   precision="mixed", omega=0.5),
    "c4a": Workload("c4a", dim=2, N=128, n_terms=12, k=20, n_train=100),
    "c4b": Workload("c4b", dim=2, N=256, n_terms=12, k=20, n_train=100),
    "c4c": Workload("c4c", dim=3, N=48, n_terms=16, k=20, n_train=100, omega=0.5),
    "c5": Workload("c5", dim=3, N=128, n_terms=16, k=50, n_train=200, batch=8,
                   precision="mixed", omega=0.5, train_tol=1e-8),
}


def small(dim: int, N: int, **kw) -> Workload:
    """A small workload of the same family (for tests)."""
    base = dict(n_terms=8 if dim == 2 else 16, k=6, n_train=12,
                omega=2.0 / 3.0 if dim == 2 else 0.5)
    base.update(kw)
    return Workload(f"d{dim}n{N}", dim=dim, N=N, **base)


def with_(w: Workload, **kw) -> Workload:
    return replace(w, **kw)


def _normal(seed: int, size: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(size)


def train_xi(w: Workload, i: int) -> np.ndarray:
    """Field coefficients of training parameter i (standard normal, FP64)."""
    return _normal(TRAIN_SEED0 + i, w.n_terms)


def query_xi(w: Workload, j: int) -> np.ndarray:
    """Field coefficients of query parameter j (standard normal, FP64)."""
    return _normal(QUERY_SEED0 + j, w.n_terms)


def train_xis(w: Workload) -> np.ndarray:
    return np.stack([train_xi(w, i) for i in range(w.n_train)])


def query_xis(w: Workload, count: int, first: int = 0) -> np.ndarray:
    return np.stack([query_xi(w, first + j) for j in range(count)])


def noise(w: Workload, j: int) -> np.ndarray:
    """Raw standard-normal warm-start noise g of query j, one entry per free DOF."""
    return _normal(NOISE_SEED0 + j, w.n)


def warm_start(u_exact, g, rel: float = 0.01):
    """Surrogate stand-in: u_exact + rel * ||u_exact|| * g / ||g||.

    Works on numpy arrays and torch tensors alike (plain operators only).
    """
    nu = float((u_exact * u_exact).sum()) ** 0.5
    ng = float((g * g).sum()) ** 0.5
    return u_exact + (rel * nu / ng) * g


def arrivals(rate: float, duration: float, n_classes: int, pool: int, seed: int = ARRIVAL_SEED):
    """A Poisson request stream: arrival times (s, from 0) with exponential
    gaps of mean 1/rate up to `duration`, a uniformly drawn class per
    request and, per class, query indices cycling through a pool of `pool`
    pre-generated queries.  Returns (times, classes, query indices)."""
    g = np.random.Generator(np.random.PCG64(seed))
    times = []
    t = g.exponential(1.0 / rate)
    while t < duration:
        times.append(t)
        t += g.exponential(1.0 / rate)
    times = np.asarray(times)
    cls = g.integers(0, n_classes, size=len(times))
    qidx = np.zeros(len(times), dtype=np.int64)
    seen = np.zeros(n_classes, dtype=np.int64)
    for i, c in enumerate(cls):
        qidx[i] = seen[c] % pool
        seen[c] += 1
    return times, cls, qidx
