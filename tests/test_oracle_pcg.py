"""Pins of the oracle's POD-2G preconditioned CG (Sec. 3.4 Alg. 3), the
standalone two-grid solver (Alg. 2 with Eq. 30) and the reduced solve
(Sec. 3.3, Eqs. 28-29): dense direct solves, special cases with a known
iteration count, CG invariants (Sec. 2.1: conjugate directions, Eq. 11) and
forced failure statuses."""
import numpy as np
import pytest

from oracle import fem, pcg, problem, twogrid
from paper_2207_02543_amd import inputs as I


def _setup(dim, N, k=4, omega=None, n_train=8):
    w = I.small(dim, N, k=k, n_train=n_train, **({} if omega is None else {"omega": omega}))
    P, lam, U = problem.basis(w, I.train_xis(w))
    q = problem.query(w, I.query_xi(w, 0), I.noise(w, 0))
    return w, P, q


@pytest.mark.parametrize("dim,N", [(2, 4), (2, 8), (3, 2), (3, 3)])
def test_pcg_matches_dense_solve(dim, N):
    w, P, q = _setup(dim, N)
    exact = np.linalg.solve(q.K.toarray(), q.f)
    M = twogrid.TwoGrid(q.K, P, w.omega)
    res = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-14, maxit=500)
    assert res.status == pcg.OK
    np.testing.assert_allclose(res.u, exact, rtol=0, atol=1e-11 * np.abs(exact).max())
    assert res.relres <= 1e-14


def test_plain_cg_matches_dense_solve():
    w, P, q = _setup(2, 6)
    exact = np.linalg.solve(q.K.toarray(), q.f)
    res = pcg.pcg(q.K, q.f, np.zeros_like(q.f), None, tol=1e-13, maxit=2000)
    np.testing.assert_allclose(res.u, exact, rtol=0, atol=1e-10 * np.abs(exact).max())


def test_full_basis_converges_in_one_iteration():
    w, P, q = _setup(2, 3)
    n = q.K.shape[0]
    Q = np.linalg.qr(np.random.default_rng(7).standard_normal((n, n)))[0]
    res = pcg.pcg(q.K, q.f, q.x0, twogrid.TwoGrid(q.K, Q, w.omega), tol=1e-10)
    assert res.iters == 1 and res.status == pcg.OK


def test_coarse_only_with_error_in_span_converges_in_one_step():
    """nu1 = nu2 = 0 and x0 - u* in span(P): s_0 = e_0, alpha_0 = 1."""
    w, P, q = _setup(2, 5, k=4)
    c = np.array([1.0, -2.0, 0.5, 3.0])
    x0 = q.u_exact - P @ c * 1e-3
    res = pcg.pcg(q.K, q.f, x0, twogrid.TwoGrid(q.K, P, w.omega, 0, 0), tol=1e-10)
    assert res.iters == 1 and res.status == pcg.OK
    np.testing.assert_allclose(res.u, q.u_exact, rtol=0, atol=1e-12 * np.abs(q.u_exact).max())


def test_initial_guess_already_converged():
    w, P, q = _setup(2, 4)
    res = pcg.pcg(q.K, q.f, q.u_exact, twogrid.TwoGrid(q.K, P, w.omega), tol=1e-8)
    assert res.iters == 0 and res.status == pcg.OK


def test_conjugate_directions_and_residual_orthogonality():
    w, P, q = _setup(2, 12, k=4)
    M = twogrid.TwoGrid(q.K, P, w.omega)
    res = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-12, maxit=10, record=True)
    ps = res.directions[:10]
    Kp = [q.K @ p for p in ps]
    for i in range(len(ps)):
        for j in range(i):
            bound = 1e-10 * np.sqrt((ps[i] @ Kp[i]) * (ps[j] @ Kp[j]))
            assert abs(ps[i] @ Kp[j]) <= bound


def test_energy_error_monotone_and_fr_equals_pr():
    w, P, q = _setup(2, 12, k=4)
    M = twogrid.TwoGrid(q.K, P, w.omega)
    errs = []
    u = q.x0.copy()
    for it in range(1, 12):
        r = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-30, maxit=it)
        e = r.u - q.u_exact
        errs.append(e @ (q.K @ e))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    fr = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-10, beta="fr")
    pr = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-10, beta="pr")
    assert abs(fr.iters - pr.iters) <= 1
    np.testing.assert_allclose(fr.u, pr.u, rtol=0, atol=1e-9 * np.abs(q.u_exact).max())


def test_failure_statuses():
    w, P, q = _setup(2, 4)
    M = twogrid.TwoGrid(q.K, P, w.omega)
    f = q.f.copy()
    f[3] = np.nan
    assert pcg.pcg(q.K, f, q.x0, M).status == pcg.ENAN
    r = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-14, maxit=1)
    assert r.status == pcg.EMAXIT and r.iters == 1
    # an indefinite "preconditioner" (3D, omega = 2/3) breaks PCG down
    w3, P3, q3 = _setup(3, 2, omega=2 / 3)
    M3 = twogrid.TwoGrid(q3.K, P3, 2 / 3)
    B = np.stack([M3(np.eye(q3.K.shape[0])[:, i]) for i in range(q3.K.shape[0])], axis=1)
    ev, V = np.linalg.eigh(0.5 * (B + B.T))
    assert ev.min() < 0
    # a residual along the negative direction of B gives r^T B r < 0 at once
    Kd = q3.K.toarray()
    x0 = q3.u_exact - np.linalg.solve(Kd, V[:, 0])
    assert pcg.pcg(q3.K, q3.f, x0, M3, tol=1e-14).status == pcg.EBREAKDOWN


def test_standalone_twogrid_energy_error_decreases():
    w, P, q = _setup(2, 10, k=5)
    M = twogrid.TwoGrid(q.K, P, w.omega)
    u = q.x0.copy()
    errs = []
    for _ in range(8):
        e = u - q.u_exact
        errs.append(e @ (q.K @ e))
        u = u + M(q.f - q.K @ u)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    res = pcg.twogrid_solve(q.K, q.f, q.x0, M, tol=1e-8, maxit=2000)
    assert res.status == pcg.OK and res.relres <= 1e-8


def test_rom_solve_exact_when_solution_in_span():
    w, P, q = _setup(2, 6, k=4)
    Pu = np.concatenate([P, q.u_exact[:, None]], axis=1)
    L = twogrid.coarse_factor(q.K, Pu)
    np.testing.assert_allclose(pcg.rom_solve(q.K, q.f, Pu, L), q.u_exact,
                               rtol=0, atol=1e-10 * np.abs(q.u_exact).max())


def test_warm_start_noise_level():
    w, P, q = _setup(2, 6)
    assert np.linalg.norm(q.x0 - q.u_exact) / np.linalg.norm(q.u_exact) == pytest.approx(0.01, rel=1e-12)


def test_mixed_mode_iteration_count_close_to_fp64():
    w = I.WORKLOADS["c1"]
    P, lam, U = problem.basis(w, I.train_xis(w)[:16], k=8)
    q = problem.query(w, I.query_xi(w, 0), I.noise(w, 0))
    a = problem.solve_query(w, q, P, precision="fp64", beta="fr")
    b = problem.solve_query(w, q, P, precision="fp32", beta="pr")
    assert a.status == b.status == pcg.OK
    assert abs(a.iters - b.iters) <= 2
    assert np.linalg.norm(a.u - b.u) / np.linalg.norm(a.u) < 1e-6


def test_rom_solve_galerkin_orthogonality():
    """The reduced solution's residual is orthogonal to the basis (Galerkin
    condition of the reduced system), and the reduced solution minimises the
    energy norm of the error over span(P)."""
    w, P, q = _setup(2, 8, k=5)
    L = twogrid.coarse_factor(q.K, P)
    u = pcg.rom_solve(q.K, q.f, P, L)
    r = q.f - q.K @ u
    assert np.abs(P.T @ r).max() <= 1e-10 * np.abs(P.T @ q.f).max()
    Kd = q.K.toarray()

    def energy(v):
        e = v - q.u_exact
        return e @ (Kd @ e)
    rng = np.random.default_rng(5)
    for _ in range(5):
        assert energy(u) <= energy(u + P @ (1e-3 * rng.standard_normal(P.shape[1])))


def test_standalone_twogrid_one_cycle_with_full_basis():
    """k = n: the coarse correction is exact, so one cycle solves the system."""
    w, P, q = _setup(2, 3, k=4)
    n = q.K.shape[0]
    M = twogrid.TwoGrid(q.K, np.eye(n), w.omega)
    res = pcg.twogrid_solve(q.K, q.f, q.x0, M, tol=1e-10, maxit=5)
    assert res.status == pcg.OK and res.iters == 1


# -- residual replacement (the exit check on the true residual) ------------------
def _replacement_case(precision):
    w = I.small(2, 16, k=6, n_train=12)
    P, lam, U = problem.basis(w, I.train_xis(w))
    q = problem.query(w, I.query_xi(w, 0), I.noise(w, 0))
    M = twogrid.TwoGrid(q.K, P, w.omega, 2, 2, precision=precision)
    return w, q, M, ("pr" if precision == "fp32" else "fr")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_replacement_is_a_restart_from_the_true_residual(precision):
    """At 1e-14 the recursive residual passes the test one iteration before
    the true residual does, so the exit check replaces r by f - K u.  The
    replacement must act as a CG restart: the iterates after it are exactly
    those of a fresh PCG started from the iterate where it happened (r_0 =
    f - K u, s_0 = B r_0, p_0 = s_0, rho = r_0^T s_0), and the solve ends
    when the true residual passes."""
    w, q, M, beta = _replacement_case(precision)
    tol = 1e-14
    full = pcg.pcg(q.K, q.f, q.x0, M, tol=tol, maxit=500, beta=beta, record=True)
    assert full.status == pcg.OK and full.relres <= tol
    assert len(full.replacements) >= 1
    k0 = full.replacements[0]
    thresh = tol * np.linalg.norm(q.f)
    # at k0 the recursive residual had passed, the true one had not
    assert full.rnorms[k0 - 1] <= thresh
    head = pcg.pcg(q.K, q.f, q.x0, M, tol=tol, maxit=k0, beta=beta)
    assert head.iters == k0 and head.status == pcg.EMAXIT
    assert np.linalg.norm(q.f - q.K @ head.u) > thresh
    tail = pcg.pcg(q.K, q.f, head.u, M, tol=tol, maxit=500, beta=beta)
    assert tail.status == pcg.OK
    assert k0 + tail.iters == full.iters
    assert np.array_equal(tail.u, full.u)
    assert tail.relres == full.relres


def test_replacement_below_attainable_accuracy_ends_at_the_limit():
    """A tolerance below what FP64 residuals can show (1e-16): the recursive
    residual keeps passing, every exit check fails, the true residual keeps
    replacing it, and the solve ends with EMAXIT at maxit, reporting the true
    residual of the final iterate (which is near FP64 rounding)."""
    w, q, M, beta = _replacement_case("fp32")
    res = pcg.pcg(q.K, q.f, q.x0, M, tol=1e-16, maxit=120, beta=beta)
    assert res.status == pcg.EMAXIT and res.iters == 120
    assert len(res.replacements) >= 3
    true = np.linalg.norm(q.f - q.K @ res.u) / np.linalg.norm(q.f)
    assert res.relres == true
    assert 1e-16 < true < 1e-13


def test_basis_from_snapshots_solved_to_1e8():
    """Snapshots solved iteratively to a relative residual of 1e-8 (the c5
    training tolerance) instead of exactly: the POD basis (Sec. 3.3) moves
    by far less than its weakest retained direction, and PCG with it takes
    the same number of iterations on the queries."""
    w = I.small(2, 24, k=8, n_train=16)
    xis = I.train_xis(w)
    f = fem.traction_load(w.dim, w.N)
    U_exact = problem.snapshots(w, xis)
    cols = []
    for xi in xis:
        K = problem.stiffness(w, xi)
        r = pcg.pcg(K, f, np.zeros(w.n), None, tol=1e-8, maxit=20000)
        assert r.status == pcg.OK and r.relres <= 1e-8
        cols.append(r.u)
    U_loose = np.stack(cols, axis=1)
    P1, lam1 = problem.pod.pod_basis(U_exact, w.k)
    P2, lam2 = problem.pod.pod_basis(U_loose, w.k)
    # largest sine of the principal angles between the two spans
    sin_max = np.linalg.norm(P2 - P1 @ (P1.T @ P2), axis=0).max()
    # (observed 3e-8; snapshots to 1e-5 already give 3e-5)
    assert sin_max < 1e-6
    assert np.allclose(lam1[:w.k], lam2[:w.k], rtol=1e-7)
    for j in range(3):
        q = problem.query(w, I.query_xi(w, j), I.noise(w, j))
        a = problem.solve_query(w, q, P1)
        b = problem.solve_query(w, q, P2)
        assert abs(a.iters - b.iters) <= 1
        assert np.linalg.norm(a.u - b.u) <= 1e-6 * np.linalg.norm(a.u)
