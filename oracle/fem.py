"""Galerkin FE discretisation of linear elasticity (Sec. 2.1, Eqs. 1-6).

The paper assembles per-element systems (Eq. 5) into the global SPD system
K(theta) u = f (Eq. 6).  The synthetic stand-in problems are:

* 2D: plane stress, thickness 1, unit square, N x N bilinear Q4 elements,
  edge x = 0 clamped, unit traction in +x on edge x = 1.
* 3D: isotropic elasticity with the Lame constants of Sec. 4.1 (Eq. Lame),
  unit cube, N^3 trilinear Hex8 elements, face z = 0 clamped, unit traction
  in +z on face z = 1.

Young's modulus is piecewise constant, evaluated at element centroids from a
truncated cosine expansion driven by the parameter vector xi (theta = xi).
Dirichlet conditions are imposed by elimination: clamped DOFs are removed.
DOF numbering: node (i, j[, l]) has id i + (N+1) j [+ (N+1)^2 l]; its free
DOFs are numbered dim * (free-node rank) + component, in node-id order.

FP64 throughout.  Written for readability, not speed.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# random Young's modulus field
# --------------------------------------------------------------------------
def kl_multi_indices(dim: int, m: int) -> np.ndarray:
    """First m multi-indices of {0..3}^dim without the zero index, in
    lexicographic order with the first (x) coordinate most significant."""
    out = [a for a in itertools.product(range(4), repeat=dim) if any(a)]
    if m > len(out):
        raise ValueError("too many field terms")
    return np.array(out[:m], dtype=np.int64)


def element_centroids(dim: int, N: int) -> np.ndarray:
    """Centroids of the N^dim elements, element (ex, ey[, ez]) at row
    ex + N ey [+ N^2 ez]; columns are the x, y[, z] coordinates."""
    h = 1.0 / N
    c = (np.arange(N) + 0.5) * h
    grids = np.meshgrid(*([c] * dim), indexing="ij")   # axis 0 = x
    # flatten with x fastest
    return np.stack([g.transpose().reshape(-1) for g in grids], axis=1)


def young_modulus(dim: int, N: int, xi, kl_scale: float = 0.3) -> np.ndarray:
    """E_e = exp(kl_scale * sum_t xi_t prod_d cos(pi a_td c_d) / (1 + sum_d a_td))
    at every element centroid c."""
    xi = np.asarray(xi, dtype=np.float64)
    A = kl_multi_indices(dim, xi.size)
    C = element_centroids(dim, N)
    g = np.zeros(C.shape[0])
    for t in range(xi.size):
        term = np.ones(C.shape[0])
        for d in range(dim):
            term = term * np.cos(np.pi * A[t, d] * C[:, d])
        g += xi[t] * term / (1.0 + A[t].sum())
    return np.exp(kl_scale * g)


# --------------------------------------------------------------------------
# element stiffness (unit modulus) by full Gauss quadrature
# --------------------------------------------------------------------------
def _local_nodes(dim: int) -> np.ndarray:
    """Natural coordinates (+-1) of the local nodes; local node
    l = lx + 2 ly [+ 4 lz] sits at (2 lx - 1, 2 ly - 1[, 2 lz - 1])."""
    pts = []
    for l in range(2 ** dim):
        bits = [(l >> d) & 1 for d in range(dim)]
        pts.append([2 * b - 1 for b in bits])
    return np.array(pts, dtype=np.float64)


def _shape_grad(dim: int, s: np.ndarray) -> np.ndarray:
    """dN_l/ds_d of the (bi/tri)linear shape functions at natural point s,
    shape (2^dim, dim)."""
    nodes = _local_nodes(dim)
    G = np.zeros((2 ** dim, dim))
    for l in range(2 ** dim):
        for d in range(dim):
            v = nodes[l, d] / 2.0 ** dim
            for e in range(dim):
                if e != d:
                    v *= 1.0 + nodes[l, e] * s[e]
            G[l, d] = v
    return G


def elasticity_matrix(dim: int, nu: float, E: float = 1.0) -> np.ndarray:
    """Material matrix D with engineering shear strains.
    2D: plane stress.  3D: lambda = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu))."""
    if dim == 2:
        return E / (1.0 - nu * nu) * np.array([[1.0, nu, 0.0],
                                               [nu, 1.0, 0.0],
                                               [0.0, 0.0, (1.0 - nu) / 2.0]])
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def strain_displacement(dim: int, dNdx: np.ndarray) -> np.ndarray:
    """B with strain order (xx, yy, xy) in 2D, (xx, yy, zz, xy, yz, zx) in 3D;
    element DOF order dim * l + component."""
    nn = dNdx.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * nn))
        for l in range(nn):
            dx, dy = dNdx[l]
            B[0, 2 * l] = dx
            B[1, 2 * l + 1] = dy
            B[2, 2 * l] = dy
            B[2, 2 * l + 1] = dx
        return B
    B = np.zeros((6, 3 * nn))
    for l in range(nn):
        dx, dy, dz = dNdx[l]
        B[0, 3 * l] = dx
        B[1, 3 * l + 1] = dy
        B[2, 3 * l + 2] = dz
        B[3, 3 * l] = dy
        B[3, 3 * l + 1] = dx
        B[4, 3 * l + 1] = dz
        B[4, 3 * l + 2] = dy
        B[5, 3 * l] = dz
        B[5, 3 * l + 2] = dx
    return B


def element_stiffness(dim: int, nu: float, h: float) -> np.ndarray:
    """Unit-modulus stiffness of a cubic element of side h (Eq. 5):
    sum over 2^dim Gauss points of B^T D B det(J), weights 1."""
    D = elasticity_matrix(dim, nu)
    g = 1.0 / np.sqrt(3.0)
    detJ = (h / 2.0) ** dim
    Ke = np.zeros((dim * 2 ** dim, dim * 2 ** dim))
    for s in itertools.product((-g, g), repeat=dim):
        dNdx = _shape_grad(dim, np.array(s)) * (2.0 / h)
        B = strain_displacement(dim, dNdx)
        Ke += B.T @ D @ B * detJ
    # B^T D B is symmetric; average out the rounding asymmetry of the products
    return 0.5 * (Ke + Ke.T)


# --------------------------------------------------------------------------
# mesh, DOFs, assembly
# --------------------------------------------------------------------------
def node_id(dim: int, N: int, idx) -> int:
    i = idx[0] + (N + 1) * idx[1]
    if dim == 3:
        i += (N + 1) ** 2 * idx[2]
    return i


def element_connectivity(dim: int, N: int) -> np.ndarray:
    """Global node ids of every element's local nodes, elements in
    ex-fastest order, local node l = lx + 2 ly [+ 4 lz]."""
    conn = []
    for e in itertools.product(range(N), repeat=dim):
        e = e[::-1]          # itertools varies the last entry fastest
        row = []
        for l in range(2 ** dim):
            off = [(l >> d) & 1 for d in range(dim)]
            row.append(node_id(dim, N, [e[d] + off[d] for d in range(dim)]))
        conn.append(row)
    return np.array(conn, dtype=np.int64)


def clamped_nodes(dim: int, N: int) -> np.ndarray:
    """Boolean mask over nodes: x = 0 in 2D, z = 0 in 3D."""
    n_nodes = (N + 1) ** dim
    ids = np.arange(n_nodes)
    if dim == 2:
        return (ids % (N + 1)) == 0
    return ids < (N + 1) ** 2


def free_dofs(dim: int, N: int) -> np.ndarray:
    """Global DOF ids (dim * node + component) that survive elimination,
    in increasing order; position in this array = free DOF id."""
    keep = ~clamped_nodes(dim, N)
    nodes = np.nonzero(keep)[0]
    return (dim * nodes[:, None] + np.arange(dim)[None, :]).reshape(-1)


def assemble_full(dim: int, N: int, nu: float, E: np.ndarray) -> sp.csr_matrix:
    """K_full = sum_e A_e^T (E_e K_ref) A_e over all DOFs (Eqs. 5-6)."""
    Ke = element_stiffness(dim, nu, 1.0 / N)
    conn = element_connectivity(dim, N)
    ndof = dim * (N + 1) ** dim
    edofs = (dim * conn[:, :, None] + np.arange(dim)[None, None, :]).reshape(conn.shape[0], -1)
    m = edofs.shape[1]
    rows = np.repeat(edofs, m, axis=1).reshape(-1)
    cols = np.tile(edofs, (1, m)).reshape(-1)
    vals = (E[:, None, None] * Ke[None, :, :]).reshape(-1)
    return sp.coo_matrix((vals, (rows, cols)), shape=(ndof, ndof)).tocsr()


def assemble(dim: int, N: int, nu: float, E: np.ndarray) -> sp.csr_matrix:
    """Stiffness restricted to the free DOFs (Dirichlet by elimination)."""
    fd = free_dofs(dim, N)
    K = assemble_full(dim, N, nu, E)[fd][:, fd].tocsr()
    K.sort_indices()
    return K


def stiffness_rows(dim: int, N: int, nu: float, E: np.ndarray, rows) -> list:
    """Rows of the free-DOF stiffness (Eqs. 5-6) one by one, without
    assembling K: for free DOF `row`, the sum over the (at most 2^dim)
    elements around its node of E_e times the element-matrix row, on the
    free columns.  Returns one {free column: value} dict per row."""
    Ke = element_stiffness(dim, nu, 1.0 / N)
    fd = free_dofs(dim, N)
    out = []
    for row in rows:
        g = int(fd[row])
        node, comp = divmod(g, dim)
        coord = [(node // (N + 1) ** d) % (N + 1) for d in range(dim)]
        acc = {}
        for eoff in itertools.product((-1, 0), repeat=dim):
            e = [coord[d] + eoff[d] for d in range(dim)]
            if any(v < 0 or v >= N for v in e):
                continue
            eid = sum(e[d] * N ** d for d in range(dim))      # ex-fastest element order
            loc = sum((coord[d] - e[d]) << d for d in range(dim))
            for b in range(2 ** dim):
                nb = node_id(dim, N, [e[d] + ((b >> d) & 1) for d in range(dim)])
                for c in range(dim):
                    col_g = dim * nb + c
                    pos = np.searchsorted(fd, col_g)
                    if pos < len(fd) and fd[pos] == col_g:
                        acc[int(pos)] = acc.get(int(pos), 0.0) + E[eid] * Ke[dim * loc + comp, dim * b + c]
        out.append(acc)
    return out


def traction_load_full(dim: int, N: int) -> np.ndarray:
    """Consistent nodal forces of a unit uniform traction: +x on x = 1 (2D,
    each edge segment gives h/2 to its two nodes), +z on z = 1 (3D, each
    face quad gives h^2/4 to its four nodes)."""
    h = 1.0 / N
    f = np.zeros(dim * (N + 1) ** dim)
    if dim == 2:
        for j in range(N):
            for jj in (j, j + 1):
                f[2 * node_id(2, N, [N, jj]) + 0] += h / 2.0
    else:
        for j in range(N):
            for i in range(N):
                for (di, dj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
                    f[3 * node_id(3, N, [i + di, j + dj, N]) + 2] += h * h / 4.0
    return f


def traction_load(dim: int, N: int) -> np.ndarray:
    return traction_load_full(dim, N)[free_dofs(dim, N)]


def jacobi_inverse_diagonal(K: sp.csr_matrix) -> np.ndarray:
    """D^{-1} = 1 / diag(K)."""
    return 1.0 / K.diagonal()
