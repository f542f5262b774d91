"""Pins of the oracle's POD basis (Sec. 3.3), two-grid cycle (Sec. 2.2 Alg. 2,
Sec. 3.3 Eq. 30) and smoother against textbook routines, the paper's
error-propagation formulas (Eqs. 20-22 and 30) and invariants."""
import numpy as np
import pytest

from oracle import pod, problem, twogrid
from paper_2207_02543_amd import inputs as I


def _tiny(dim, N, k, omega):
    w = I.small(dim, N, k=k, n_train=8, omega=omega)
    P, lam, U = problem.basis(w, I.train_xis(w))
    K = problem.stiffness(w, I.query_xi(w, 0))
    return w, K, P, U


def _dense_B(M, n):
    return np.stack([M(np.eye(n)[:, i]) for i in range(n)], axis=1)


# ---------------------------------------------------------------- POD ------
def test_pod_orthonormal_and_singular_values():
    rng = np.random.default_rng(0)
    U = rng.standard_normal((300, 12)) @ np.diag(np.logspace(0, -3, 12))
    P, lam = pod.pod_basis(U, 7)
    np.testing.assert_allclose(P.T @ P, np.eye(7), atol=1e-12)
    sv = np.linalg.svd(U, compute_uv=False)
    np.testing.assert_allclose(lam, sv ** 2, rtol=1e-10)
    # span equals the top left singular vectors
    Q = np.linalg.svd(U, full_matrices=False)[0][:, :7]
    np.testing.assert_allclose(P @ P.T, Q @ Q.T, atol=1e-10)


def test_pod_of_elasticity_snapshots():
    w, K, P, U = _tiny(2, 6, 5, 2 / 3)
    Q, sv, _ = np.linalg.svd(U, full_matrices=False)
    _, lam = pod.pod_basis(U, 5)
    np.testing.assert_allclose(lam[:5], sv[:5] ** 2, rtol=1e-8)
    # the basis spans the leading left singular subspace
    proj = Q[:, :5].T @ P
    np.testing.assert_allclose(np.linalg.svd(proj, compute_uv=False), 1.0, atol=1e-6)


def test_pod_rank_deficient_raises():
    U = np.ones((10, 3))
    with pytest.raises(ValueError):
        pod.pod_basis(U, 2)


# ------------------------------------------------------------ smoother -----
def test_one_sweep_from_zero_is_scaled_diagonal():
    w, K, P, U = _tiny(2, 5, 3, 2 / 3)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(K.shape[0])
    dinv = 1.0 / K.diagonal()
    x = twogrid.jacobi_sweeps(K, dinv, b, np.zeros_like(b), w.omega, 1)
    assert np.array_equal(x, np.zeros_like(b) + w.omega * dinv * (b - 0.0))


def test_power_iteration_matches_dense_eigenvalue():
    w, K, P, U = _tiny(3, 2, 3, 0.5)
    dinv = 1.0 / K.diagonal()
    exact = np.max(np.linalg.eigvals(dinv[:, None] * K.toarray()).real)
    assert twogrid.power_lambda_max(K, dinv, iters=400) == pytest.approx(exact, rel=1e-6)


# --------------------------------------------------------------- cycle -----
@pytest.mark.parametrize("dim,N,k,omega,nu1,nu2", [
    (2, 4, 4, 2 / 3, 2, 2), (2, 3, 2, 2 / 3, 1, 3), (3, 2, 4, 0.5, 2, 2)])
def test_cycle_error_operator(dim, N, k, omega, nu1, nu2):
    """I - B K = M^{nu2} C M^{nu1} with M = I - omega D^{-1} K and
    C = I - P (P^T K P)^{-1} P^T K (Eqs. 21-22 with the POD prolongation of
    Eq. 30)."""
    w, K, P, U = _tiny(dim, N, k, omega)
    n = K.shape[0]
    Kd = K.toarray()
    M = np.eye(n) - omega * (1.0 / np.diag(Kd))[:, None] * Kd
    C = np.eye(n) - P @ np.linalg.solve(P.T @ Kd @ P, P.T @ Kd)
    E = np.linalg.matrix_power(M, nu2) @ C @ np.linalg.matrix_power(M, nu1)
    B = _dense_B(twogrid.TwoGrid(K, P, omega, nu1, nu2), n)
    np.testing.assert_allclose(np.eye(n) - B @ Kd, E, atol=1e-11)


@pytest.mark.parametrize("dim,N,k,omega,nu", [
    (2, 4, 4, 2 / 3, 2), (2, 6, 3, 2 / 3, 2), (3, 2, 4, 0.5, 2), (3, 3, 5, 0.5, 2),
    (2, 4, 4, 2 / 3, 1), (2, 4, 4, 2 / 3, 3), (3, 2, 4, 0.5, 1), (3, 2, 4, 0.5, 3)])
def test_preconditioner_spd_and_unit_eigenvalues(dim, N, k, omega, nu):
    """Equal pre- and post-relaxation counts give a symmetric positive
    definite B with BK's spectrum in (0, 1] and at least k unit eigenvalues."""
    w, K, P, U = _tiny(dim, N, k, omega)
    n = K.shape[0]
    B = _dense_B(twogrid.TwoGrid(K, P, omega, nu, nu), n)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0
    ev = np.sort(np.linalg.eigvals(B @ K.toarray()).real)
    assert ev[0] > 0.0 and ev[-1] <= 1.0 + 1e-10
    # C annihilates span(P), so I - BK has rank <= n - k: >= k unit eigenvalues
    assert np.sum(np.abs(ev - 1.0) < 1e-8) >= k


def test_3d_two_thirds_damping_is_indefinite():
    """Hex8 elasticity at nu = 0.3 has omega * lambda_max(D^-1 K) > 2 for
    omega = 2/3: the two-grid preconditioner loses definiteness."""
    w, K, P, U = _tiny(3, 2, 4, 2 / 3)
    dinv = 1.0 / K.diagonal()
    assert 2 / 3 * twogrid.power_lambda_max(K, dinv, iters=400) > 2.0
    B = _dense_B(twogrid.TwoGrid(K, P, 2 / 3), K.shape[0])
    assert np.linalg.eigvals(B @ K.toarray()).real.min() < 0.0


def test_full_basis_gives_exact_inverse():
    """k = n: P spans R^n, the coarse correction is exact and B = K^{-1} for
    any smoother."""
    w, K, P, U = _tiny(2, 3, 2, 2 / 3)
    n = K.shape[0]
    Q = np.linalg.qr(np.random.default_rng(2).standard_normal((n, n)))[0]
    B = _dense_B(twogrid.TwoGrid(K, Q, 2 / 3), n)
    np.testing.assert_allclose(B @ K.toarray(), np.eye(n), atol=1e-10)


def test_basis_rotation_invariance():
    """B depends on span(P) only (P -> P Q leaves K_c^{-1}-weighted projector
    unchanged)."""
    w, K, P, U = _tiny(2, 4, 4, 2 / 3)
    Q = np.linalg.qr(np.random.default_rng(3).standard_normal((4, 4)))[0] * 3.0
    r = np.random.default_rng(4).standard_normal(K.shape[0])
    a = twogrid.TwoGrid(K, P, 2 / 3)(r)
    b = twogrid.TwoGrid(K, P @ Q, 2 / 3)(r)
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-14 * np.abs(a).max())


def test_coarse_factor_not_spd():
    w, K, P, U = _tiny(2, 4, 3, 2 / 3)
    Pd = np.concatenate([P, np.zeros((P.shape[0], 1))], axis=1)   # zero pivot
    with pytest.raises(twogrid.NotSPD):
        twogrid.coarse_factor(K, Pd)


def test_fp32_cycle_close_and_scale_exact():
    w, K, P, U = _tiny(2, 8, 4, 2 / 3)
    r = np.random.default_rng(5).standard_normal(K.shape[0])
    s64 = twogrid.TwoGrid(K, P, 2 / 3)(r)
    M32 = twogrid.TwoGrid(K, P, 2 / 3, precision="fp32")
    s32 = M32(r)
    assert np.linalg.norm(s32 - s64) / np.linalg.norm(s64) < 1e-5
    # scaling by powers of two commutes with binary32 rounding
    a = M32.apply(r, scale=1.0)
    b = M32.apply(r, scale=2.0 ** -7)
    c = M32.apply(r, scale=2.0 ** 11)
    assert np.array_equal(a, b) and np.array_equal(a, c)


# -- symmetric Gauss-Seidel in multicolour order --------------------------------
def _gs_loop(Kd, b, x, order, backward):
    """One Gauss-Seidel sweep written as the plain loop of its definition."""
    x = x.copy()
    seq = order[::-1] if backward else order
    for i in seq:
        x[i] += (b[i] - Kd[i] @ x) / Kd[i, i]
    return x


@pytest.mark.parametrize("dim,N", [(2, 3), (3, 2)])
def test_gauss_seidel_sweep_is_the_sequential_update(dim, N):
    w = I.small(dim, N)
    K = problem.stiffness(w, I.query_xi(w, 0))
    Kd = K.toarray()
    order = twogrid.multicolor_order(dim, N)
    assert sorted(order) == list(range(K.shape[0]))
    rng = np.random.default_rng(1)
    b, x = rng.standard_normal(K.shape[0]), rng.standard_normal(K.shape[0])
    for back in (False, True):
        np.testing.assert_allclose(twogrid.gauss_seidel_sweeps(K, b, x, order, 1, back),
                                   _gs_loop(Kd, b, x, order, back), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,N", [(2, 6), (3, 3)])
def test_multicolour_nodes_of_one_colour_are_uncoupled(dim, N):
    """A valid colouring: reversing the node order inside every colour leaves
    a sweep unchanged (same-colour nodes share no matrix entry)."""
    w = I.small(dim, N)
    K = problem.stiffness(w, I.query_xi(w, 1))
    order = twogrid.multicolor_order(dim, N)
    nodes = order[::dim] // dim
    from oracle.fem import free_dofs
    fd = free_dofs(dim, N)
    gnode = fd[::dim][nodes] // dim
    col = (gnode % (N + 1)) % 2 + 2 * ((gnode // (N + 1)) % (N + 1) % 2)
    if dim == 3:
        col = col + 4 * ((gnode // (N + 1) ** 2) % 2)
    assert np.all(np.diff(col) >= 0)
    Kd = K.toarray()
    for c in np.unique(col):
        idx = np.concatenate([np.arange(dim * r, dim * r + dim) for r in nodes[col == c]])
        blk = Kd[np.ix_(idx, idx)]
        # only the nodes' own dim x dim blocks are non-zero
        for a in range(len(idx) // dim):
            blk[dim * a:dim * a + dim, dim * a:dim * a + dim] = 0.0
        assert np.abs(blk).max() == 0.0
    rev = np.concatenate([np.concatenate([np.arange(dim * r, dim * r + dim) for r in nodes[col == c][::-1]])
                          for c in np.unique(col)])
    rng = np.random.default_rng(2)
    b, x = rng.standard_normal(K.shape[0]), rng.standard_normal(K.shape[0])
    np.testing.assert_allclose(twogrid.gauss_seidel_sweeps(K, b, x, order, 2),
                               twogrid.gauss_seidel_sweeps(K, b, x, rev, 2), rtol=1e-12, atol=1e-13)


def test_sgs_cycle_symmetric_pd_and_error_operator():
    """B symmetric positive definite with forward pre- and backward
    post-sweeps; I - B K = S_b^{nu2} C S_f^{nu1} (Eqs. 21-22, 30 with
    Gauss-Seidel relaxation); Gauss-Seidel contracts the energy norm."""
    w = I.small(2, 5, k=4, n_train=8)
    P, lam, U = problem.basis(w, I.train_xis(w))
    K = problem.stiffness(w, I.query_xi(w, 0))
    Kd = K.toarray()
    n = Kd.shape[0]
    order = twogrid.multicolor_order(2, 5)
    M = twogrid.TwoGrid(K, P, w.omega, 2, 2, smoother="sgs", order=order)
    B = np.stack([M(np.eye(n)[:, i]) for i in range(n)], axis=1)
    np.testing.assert_allclose(B, B.T, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    Pm = np.eye(n)[order]                    # row i of Pm selects unknown order[i]
    Kp = Pm @ Kd @ Pm.T
    Sf = np.eye(n) - Pm.T @ np.linalg.solve(np.tril(Kp), Pm @ Kd)
    Sb = np.eye(n) - Pm.T @ np.linalg.solve(np.triu(Kp), Pm @ Kd)
    C = np.eye(n) - P @ np.linalg.solve(P.T @ Kd @ P, P.T @ Kd)
    E = Sb @ Sb @ C @ Sf @ Sf
    np.testing.assert_allclose(np.eye(n) - B @ Kd, E, atol=1e-10)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(n)
    for S in (Sf, Sb):
        assert (S @ e) @ Kd @ (S @ e) < e @ Kd @ e


# -- FP32 mode: every step of the cycle runs in binary32 --------------------------
def test_fp32_cycle_steps_run_in_binary32(monkeypatch):
    """Each relaxation, residual, restriction and prolongation of the FP32
    cycle receives only binary32 operands and returns binary32 (so it is
    computed in binary32, not computed wider and rounded afterwards); the
    coarse solve gets an input that round-trips binary32 and its output is
    rounded to binary32.  A step left in FP64 (an FP64 P, K, D^-1, omega or
    vector) fails here."""
    w, K, P, U = _tiny(2, 8, 4, 2 / 3)
    M32 = twogrid.TwoGrid(K, P, 2 / 3, 2, 2, precision="fp32")
    calls = []

    def spy(name, fn):
        def wrapped(*args, **kw):
            out = fn(*args, **kw)
            calls.append((name, args, out))
            return out
        return wrapped

    for name in ("jacobi_sweeps", "residual", "restrict", "prolong", "coarse_solve"):
        monkeypatch.setattr(twogrid, name, spy(name, getattr(twogrid, name)))
    r = np.random.default_rng(5).standard_normal(K.shape[0])
    M32(r)
    names = [c[0] for c in calls]
    assert names == ["jacobi_sweeps", "residual", "restrict", "coarse_solve", "prolong",
                     "jacobi_sweeps"]
    for name, args, out in calls:
        if name == "coarse_solve":
            rc = args[1]
            assert rc.dtype == np.float64
            assert np.array_equal(rc.astype(np.float32).astype(np.float64), rc)
            continue
        for a in args:
            if isinstance(a, (int,)) and not isinstance(a, np.generic):
                continue                                   # sweep count
            dt = a.dtype
            assert dt == np.float32, (name, dt)
        assert out.dtype == np.float32, name
    # the coarse correction reaches prolong as binary32 values
    ec = [c for c in calls if c[0] == "prolong"][0][1][2]
    assert ec.dtype == np.float32


def _f32_row_loop(K32, x32):
    """(K x)_i as a plain binary32 loop: each product rounded, then added to
    the running sum in column order and rounded."""
    K32 = K32.tocsr()
    K32.sort_indices()
    y = np.zeros(K32.shape[0], dtype=np.float32)
    for i in range(K32.shape[0]):
        acc = np.float32(0.0)
        for jj in range(K32.indptr[i], K32.indptr[i + 1]):
            acc = np.float32(acc + np.float32(K32.data[jj] * x32[K32.indices[jj]]))
        y[i] = acc
    return y


def test_fp32_jacobi_sweep_and_restriction_elementwise():
    """One binary32 damped-Jacobi sweep and the binary32 restriction against
    plain binary32 loops in a fixed summation order, element by element, to
    the rounding bound of binary32 sums (u = 2^-24 per operation)."""
    w, K, P, U = _tiny(2, 6, 4, 2 / 3)
    M32 = twogrid.TwoGrid(K, P, 2 / 3, 1, 1, precision="fp32")
    rng = np.random.default_rng(9)
    n = K.shape[0]
    b = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    u = 2.0 ** -24
    got = twogrid.jacobi_sweeps(M32.K32, M32.dinv32, b, x, M32.omega32, 1)
    assert got.dtype == np.float32
    kx = _f32_row_loop(M32.K32, x)
    wd = (M32.omega32 * M32.dinv32).astype(np.float32)
    ref = np.empty(n, dtype=np.float32)
    for i in range(n):
        ri = np.float32(b[i] - kx[i])
        ref[i] = np.float32(x[i] + np.float32(wd[i] * ri))
    absK = abs(M32.K32).astype(np.float64)
    bound = 8 * u * (np.abs(x) + np.abs(wd) * (np.abs(b) + absK @ np.abs(x).astype(np.float64)))
    assert np.all(np.abs(got.astype(np.float64) - ref) <= bound)
    # restriction r_c = P^T r' with every product and sum rounded to binary32
    rr = twogrid.residual(M32.K32, b, got)
    assert rr.dtype == np.float32
    rc = twogrid.restrict(M32.P32, rr)
    assert rc.dtype == np.float32
    for j in range(P.shape[1]):
        acc = np.float32(0.0)
        for i in range(n):
            acc = np.float32(acc + np.float32(M32.P32[i, j] * rr[i]))
        s_abs = float(np.abs(M32.P32[:, j].astype(np.float64)) @ np.abs(rr.astype(np.float64)))
        assert abs(float(rc[j]) - float(acc)) <= 2 * n * u * s_abs


def test_fp32_cycle_differs_from_fp64_at_binary32_level():
    """The FP32 cycle's departure from the FP64 cycle is of binary32 size:
    above FP64 rounding (so the mode is not secretly FP64) and below a
    binary32 bound."""
    w, K, P, U = _tiny(2, 8, 4, 2 / 3)
    r = np.random.default_rng(6).standard_normal(K.shape[0])
    s64 = twogrid.TwoGrid(K, P, 2 / 3)(r)
    s32 = twogrid.TwoGrid(K, P, 2 / 3, precision="fp32")(r)
    d = np.linalg.norm(s32 - s64) / np.linalg.norm(s64)
    assert 1e-9 < d < 1e-5
