"""GPU parity: every step of the HIP path against the oracle, element by
element, through the C ABI (small and ragged meshes; see test_gpu_fullsize
for the workload sizes)."""
import numpy as np
import pytest

from gpu_helpers import block_ell_expected, flush, maxrel, relerr
from oracle import fem, pcg as opcg, pod as opod, problem as oprob, twogrid
from paper_2207_02543_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_02543_amd import capi, pipeline
    return torch, capi, pipeline


def _colblk(prob, torch):
    S = prob.pat.n_slots
    nn = prob.pat.n_nodes
    return prob.pat_buf[: S * nn * 4].view(torch.int32).cpu().numpy()


MESHES = [(2, 7), (2, 32), (2, 41), (3, 3), (3, 5), (3, 9)]


@pytest.mark.parametrize("dim,N", MESHES)
def test_assembly_matches_oracle(env, dim, N):
    torch, capi, pipeline = env
    flush(f"assembly dim={dim} N={N}")
    w = I.small(dim, N)
    prob = pipeline.Problem(w)
    xis = I.query_xis(w, 2)
    sysm = prob.alloc_system(2, fp32=True)
    prob.assemble(sysm, xis)
    torch.cuda.synchronize()
    colblk = _colblk(prob, torch)
    f_ref = fem.traction_load(dim, N)
    np.testing.assert_allclose(sysm.f.cpu().numpy(), f_ref, rtol=1e-14, atol=1e-18)
    for b in range(2):
        K = oprob.stiffness(w, xis[b])
        exp = block_ell_expected(K, dim, N, colblk, w.n)
        got = sysm.vals[b].cpu().numpy()
        scale = np.abs(exp).max()
        assert np.abs(got - exp).max() <= 1e-13 * scale
        np.testing.assert_array_equal(sysm.vals32[b].cpu().numpy(), got.astype(np.float32))
        np.testing.assert_allclose(sysm.dinv[b].cpu().numpy(), 1.0 / K.diagonal(), rtol=1e-13)


@pytest.mark.parametrize("dim,N", [(2, 32), (3, 5), (3, 9)])
def test_spmv_and_jacobi_match_oracle(env, dim, N):
    torch, capi, pipeline = env
    flush(f"spmv/jacobi dim={dim} N={N}")
    w = I.small(dim, N)
    prob = pipeline.Problem(w)
    xis = I.query_xis(w, 3)
    sysm = prob.alloc_system(3)
    prob.assemble(sysm, xis)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((3, w.n))
    bb = rng.standard_normal((3, w.n))
    xd = torch.tensor(x, device="cuda")
    yd = torch.empty_like(xd)
    capi.check(capi.pod2g_spmv(prob.pat, sysm.vals, 3, xd, yd), "spmv")
    xj = torch.tensor(x, device="cuda")
    tmp = torch.empty_like(xj)
    capi.check(capi.pod2g_jacobi(prob.pat, sysm.vals, sysm.dinv, 3, w.omega, 3,
                                 torch.tensor(bb, device="cuda"), xj, tmp), "jacobi")
    torch.cuda.synchronize()
    for b in range(3):
        K = oprob.stiffness(w, xis[b])
        ref = K @ x[b]
        # element by element, within the rounding bound of a dot product of
        # at most 81 terms (either side's summation order)
        bound = 2 * 81 * np.finfo(float).eps * (abs(K) @ np.abs(x[b]))
        assert np.all(np.abs(yd[b].cpu().numpy() - ref) <= bound)
        refj = twogrid.jacobi_sweeps(K, 1.0 / K.diagonal(), bb[b], x[b], w.omega, 3)
        assert maxrel(xj[b].cpu().numpy(), refj) < 1e-13


def _basis(w):
    P, lam, U = oprob.basis(w, I.train_xis(w))
    return P, lam, U


@pytest.mark.parametrize("dim,N,k,nu1,nu2,prec", [
    (2, 32, 10, 2, 2, "fp64"), (2, 41, 6, 1, 3, "fp64"), (3, 5, 6, 2, 2, "fp64"),
    (2, 32, 10, 2, 2, "mixed"), (3, 9, 8, 2, 2, "mixed"), (2, 7, 4, 0, 2, "fp64"),
    (2, 7, 4, 2, 0, "fp64"), (2, 7, 4, 0, 0, "mixed")])
def test_cycle_matches_oracle(env, dim, N, k, nu1, nu2, prec):
    torch, capi, pipeline = env
    flush(f"cycle dim={dim} N={N} k={k} nu=({nu1},{nu2}) {prec}")
    w = I.small(dim, N, k=k, n_train=max(12, k + 2))
    P, lam, U = _basis(w)
    prob = pipeline.Problem(w)
    xis = I.query_xis(w, 2)
    sysm = prob.alloc_system(2, fp32=(prec == "mixed"))
    prob.assemble(sysm, xis)
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    precision = capi.MIXED if prec == "mixed" else capi.FP64
    pr = prob.setup(sysm, Pd, precision=precision, nu_pre=nu1, nu_post=nu2)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((2, w.n)) * 1e-3
    rd = torch.tensor(r, device="cuda")
    sd = torch.empty_like(rd)
    prob.apply(pr, rd, sd)
    torch.cuda.synchronize()
    for b in range(2):
        K = oprob.stiffness(w, xis[b])
        M = twogrid.TwoGrid(K, P, w.omega, nu1, nu2, precision="fp32" if prec == "mixed" else "fp64")
        ref = M(r[b])
        # element by element (FP32: 24-bit rounding through four sweeps of
        # up to 81-term rows and the basis products)
        tol = 1e-12 if prec == "fp64" else 5e-6
        got = sd[b].cpu().numpy()
        flush(f"  {b}: max elementwise {maxrel(got, ref):.2e}, norm {relerr(got, ref):.2e}")
        assert maxrel(got, ref) < tol


@pytest.mark.parametrize("dim,N,k", [(2, 32, 10), (3, 5, 6)])
def test_setup_coarse_factor(env, dim, N, k):
    torch, capi, pipeline = env
    flush(f"setup dim={dim} N={N} k={k}")
    w = I.small(dim, N, k=k, n_train=12)
    P, lam, U = _basis(w)
    prob = pipeline.Problem(w)
    xis = I.query_xis(w, 1)
    sysm = prob.alloc_system(1)
    prob.assemble(sysm, xis)
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(P.T), device="cuda"), power_iters=200)
    st, lamh = capi.pod2g_setup_status(pr)
    assert st == [capi.OK]
    Ld = pipeline.device_view(pr._keepalive[0], pr.L, k * k, torch.float64).cpu().numpy().reshape(k, k)
    K = oprob.stiffness(w, xis[0])
    Kc = twogrid.coarse_matrix(K, P)
    np.testing.assert_allclose(Ld @ Ld.T, Kc, rtol=0, atol=1e-12 * np.abs(Kc).max())
    Li = pipeline.device_view(pr._keepalive[0], pr.Linv, k * k, torch.float64).cpu().numpy().reshape(k, k)
    np.testing.assert_allclose(Li @ Ld, np.eye(k), atol=1e-10)
    assert np.all(np.triu(Li, 1) == 0.0)
    lmax = twogrid.power_lambda_max(K, 1.0 / K.diagonal(), iters=200)
    assert lamh[0] == pytest.approx(lmax, rel=1e-10)


def test_setup_errors(env):
    torch, capi, pipeline = env
    flush("setup errors")
    w = I.small(2, 8, k=4, n_train=8)
    P, lam, U = _basis(w)
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(1)
    prob.assemble(sysm, I.query_xis(w, 1))
    Pz = np.concatenate([P, np.zeros((P.shape[0], 1))], axis=1)
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(Pz.T), device="cuda"))
    assert capi.pod2g_setup_status(pr)[0] == [capi.ENOTSPD]
    # the failed setup propagates to the solve
    u = torch.zeros(1, w.n, dtype=torch.float64, device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u)
    assert ret == capi.ENOTSPD and st == [capi.ENOTSPD]
    # 3D Hex8 with omega = 2/3: smoother guard
    w3 = I.small(3, 3, k=4, n_train=8, omega=2 / 3)
    P3, _, _ = _basis(w3)
    prob3 = pipeline.Problem(w3)
    s3 = prob3.alloc_system(1)
    prob3.assemble(s3, I.query_xis(w3, 1))
    P3d = torch.tensor(np.ascontiguousarray(P3.T), device="cuda")
    # the host path checks the smoother once per class and refuses it
    with pytest.raises(capi.Pod2gError) as e:
        prob3.setup(s3, P3d)
    assert e.value.status == capi.ESMOOTHER
    assert prob3.lambda_max is None
    # the library's own per-instance guard
    prob3._guarded.add(w3.omega)
    pr3 = prob3.setup(s3, P3d, power_iters=300)
    st3, lam3 = capi.pod2g_setup_status(pr3)
    assert st3 == [capi.ESMOOTHER] and lam3[0] * 2 / 3 > 2.0
    # argument errors are reported, not crashed on
    assert capi.pod2g_setup(prob.pat, sysm.vals, None, sysm.dinv, None, 65, 0.5, 2, 2, 0, 1, 0,
                            prob.work("x", 16), 16, capi.Prec()) == capi.EINVAL
    assert capi.pod2g_setup(prob.pat, sysm.vals, None, sysm.dinv, None, 0, 0.5, 2, 2, 0, 1, 0,
                            prob.work("x", 16), 16, capi.Prec()) == capi.ESIZE


def _gpu_query_solve(torch, capi, pipeline, w, P, queries, precision, beta):
    prob = pipeline.Problem(w)
    m = len(queries)
    sysm = prob.alloc_system(m, fp32=(precision == capi.MIXED))
    prob.assemble(sysm, np.stack([q.xi for q in queries]))
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(P.T), device="cuda"), precision=precision)
    u = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u, beta=beta)
    return ret, it, rr, st, u.cpu().numpy()


@pytest.mark.parametrize("wname,dim,N,prec", [
    ("c1", 2, 32, "fp64"), ("c1", 2, 32, "mixed"), ("s3", 3, 6, "fp64"), ("s3", 3, 6, "mixed"),
    ("s2", 2, 45, "fp64")])
def test_pcg_matches_oracle(env, wname, dim, N, prec):
    torch, capi, pipeline = env
    flush(f"pcg {wname} dim={dim} N={N} {prec}")
    if wname == "c1":
        w = I.WORKLOADS["c1"]
    else:
        w = I.small(dim, N, k=8, n_train=16)
    P, lam, U = _basis(w)
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(2)]
    precision = capi.MIXED if prec == "mixed" else capi.FP64
    beta = capi.BETA_PR if prec == "mixed" else capi.BETA_FR
    ret, it, rr, st, u = _gpu_query_solve(torch, capi, pipeline, w, P, queries, precision, beta)
    assert ret == capi.OK, st
    for j, q in enumerate(queries):
        ref = oprob.solve_query(w, q, P, precision="fp32" if prec == "mixed" else "fp64",
                                beta="pr" if prec == "mixed" else "fr")
        assert ref.status == opcg.OK
        flush(f"  query {j}: gpu iters {it[j]} relres {rr[j]:.3e}; oracle iters {ref.iters}")
        assert abs(it[j] - ref.iters) <= 2
        assert rr[j] <= w.tol
        assert relerr(u[j], ref.u) <= 1e-6
        # the oracle's own residual of the GPU solution
        assert np.linalg.norm(q.f - q.K @ u[j]) / np.linalg.norm(q.f) <= 1.01 * w.tol


def test_plain_cg_matches_oracle(env):
    torch, capi, pipeline = env
    flush("plain cg")
    w = I.small(2, 12)
    q = oprob.query(w, I.query_xi(w, 0), I.noise(w, 0))
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(1)
    prob.assemble(sysm, q.xi[None])
    u = torch.tensor(q.x0[None], device="cuda")
    ret, it, rr, st = prob.solve(sysm, None, u)
    ref = opcg.pcg(q.K, q.f, q.x0, None, tol=w.tol)
    assert ret == capi.OK and abs(it[0] - ref.iters) <= 2
    assert relerr(u[0].cpu().numpy(), ref.u) <= 1e-6


def test_batch_equals_alone_and_deterministic(env):
    torch, capi, pipeline = env
    flush("batch vs alone")
    w = I.small(2, 20, k=6, n_train=12)
    P, lam, U = _basis(w)
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(3)]
    ret, it, rr, st, u = _gpu_query_solve(torch, capi, pipeline, w, P, queries, capi.FP64, capi.BETA_FR)
    assert ret == capi.OK
    for j in range(3):
        r1, i1, rr1, s1, u1 = _gpu_query_solve(torch, capi, pipeline, w, P, [queries[j]], capi.FP64,
                                               capi.BETA_FR)
        assert i1[0] == it[j]
        np.testing.assert_array_equal(u1[0], u[j])
    ret2, it2, rr2, st2, u2 = _gpu_query_solve(torch, capi, pipeline, w, P, queries, capi.FP64,
                                               capi.BETA_FR)
    np.testing.assert_array_equal(u2, u)


def test_pcg_statuses(env):
    torch, capi, pipeline = env
    flush("pcg statuses")
    w = I.small(2, 10, k=4, n_train=8)
    P, lam, U = _basis(w)
    q = oprob.query(w, I.query_xi(w, 0), I.noise(w, 0))
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(1)
    prob.assemble(sysm, q.xi[None])
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(P.T), device="cuda"))
    # exact initial guess: 0 iterations
    u = torch.tensor(q.u_exact[None], device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u)
    assert ret == capi.OK and it == [0]
    # iteration limit
    u = torch.tensor(q.x0[None], device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u, rtol=1e-14, maxit=1)
    assert ret == capi.EMAXIT and it == [1]
    # non-finite load
    sysm.f[3] = float("nan")
    u = torch.tensor(q.x0[None], device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u)
    assert ret == capi.ENAN


def test_pod_basis_matches_oracle(env):
    torch, capi, pipeline = env
    flush("pod basis")
    w = I.small(2, 16, k=6, n_train=20)
    P, lam, U = _basis(w)
    Ud = torch.tensor(np.ascontiguousarray(U.T), device="cuda")
    Pg, lamg = pipeline.pod_basis(Ud, 6)
    lamg = lamg.cpu().numpy()
    np.testing.assert_allclose(lamg[:6], lam[:6], rtol=1e-9)
    Pg = Pg.cpu().numpy().T
    np.testing.assert_allclose(Pg.T @ Pg, np.eye(6), atol=1e-8)
    np.testing.assert_allclose(Pg @ Pg.T, P @ P.T, atol=1e-8)
    # odd snapshot count and rank-deficient input
    Pg2, _ = pipeline.pod_basis(Ud[:7].contiguous(), 5)
    P2 = Pg2.cpu().numpy().T
    Q = np.linalg.svd(U[:, :7], full_matrices=False)[0][:, :5]
    np.testing.assert_allclose(P2.T @ P2, np.eye(5), atol=1e-6)
    np.testing.assert_allclose(P2 @ P2.T, Q @ Q.T, atol=1e-6)
    Ur = torch.ones(4, w.n, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.Pod2gError):
        pipeline.pod_basis(Ur, 2)


def test_offline_pipeline_matches_direct_solves(env):
    torch, capi, pipeline = env
    flush("offline pipeline")
    w = I.small(2, 16, k=5, n_train=12)
    prob = pipeline.Problem(w)
    Pg, lamg, Ug, iters = pipeline.offline_basis(prob, rtol=1e-12)
    U = oprob.snapshots(w, I.train_xis(w))
    assert relerr(Ug.cpu().numpy().T, U) < 1e-9
    P, lam = opod.pod_basis(U, 5)
    Pg = Pg.cpu().numpy().T
    np.testing.assert_allclose(Pg @ Pg.T, P @ P.T, atol=1e-7)


@pytest.mark.parametrize("dim,N,nu,prec,batch", [
    (2, 24, 1, "fp64", 2), (2, 24, 3, "fp64", 2), (2, 24, 1, "mixed", 4),
    (3, 6, 1, "mixed", 4), (3, 6, 3, "mixed", 4), (3, 6, 3, "fp64", 2)])
def test_pcg_other_sweep_counts_match_oracle(env, dim, N, nu, prec, batch):
    """PCG with nu pre- and nu post-relaxation sweeps (one: the cycle ends in
    the pass that forms s, after the K P form of the first post-sweep; three:
    a plain pre-sweep after the fused update and two post-sweeps), one
    instance at a time (FP64) and batched (FP32 cycle, MFMA products),
    against the oracle with the same sweep counts."""
    torch, capi, pipeline = env
    flush(f"pcg sweeps nu={nu} dim={dim} N={N} {prec} batch={batch}")
    w = I.with_(I.small(dim, N, k=6, n_train=12), nu_pre=nu, nu_post=nu)
    P, lam, U = _basis(w)
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(batch)]
    precision = capi.MIXED if prec == "mixed" else capi.FP64
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=(prec == "mixed"))
    prob.assemble(sysm, np.stack([q.xi for q in queries]))
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(P.T), device="cuda"), precision=precision,
                    nu_pre=nu, nu_post=nu)
    u = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    beta = capi.BETA_PR if prec == "mixed" else capi.BETA_FR
    ret, it, rr, st = prob.solve(sysm, pr, u, beta=beta)
    assert ret == capi.OK, st
    uh = u.cpu().numpy()
    for j, q in enumerate(queries):
        ref = oprob.solve_query(w, q, P, precision="fp32" if prec == "mixed" else "fp64",
                                beta="pr" if prec == "mixed" else "fr")
        assert ref.status == opcg.OK
        flush(f"  query {j}: gpu iters {it[j]}; oracle iters {ref.iters}")
        assert abs(it[j] - ref.iters) <= 2
        assert rr[j] <= w.tol
        assert relerr(uh[j], ref.u) <= 1e-6
