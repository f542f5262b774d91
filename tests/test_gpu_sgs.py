"""Symmetric Gauss-Seidel relaxation in multicolour order: sweeps, the cycle
and PCG through the C ABI against the oracle."""
import numpy as np
import pytest

from gpu_helpers import flush, relerr
from oracle import pcg as opcg, problem as oprob, twogrid
from paper_2207_02543_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,N", [(2, 7), (2, 32), (3, 3), (3, 6)])
def test_gauss_seidel_sweeps_match_oracle(dim, N):
    import torch
    from paper_2207_02543_amd import capi, pipeline
    flush(f"gauss-seidel sweeps dim={dim} N={N}")
    w = I.small(dim, N)
    prob = pipeline.Problem(w)
    xis = I.query_xis(w, 2)
    sysm = prob.alloc_system(2)
    prob.assemble(sysm, xis)
    rng = np.random.default_rng(4)
    b = rng.standard_normal((2, w.n))
    x0 = rng.standard_normal((2, w.n))
    order = twogrid.multicolor_order(dim, N)
    for back in (False, True):
        x = torch.tensor(x0, device="cuda")
        capi.check(capi.pod2g_gauss_seidel(prob.pat, sysm.vals, sysm.dinv, 2, 2, back,
                                           torch.tensor(b, device="cuda"), x), "pod2g_gauss_seidel")
        got = x.cpu().numpy()
        for j in range(2):
            K = oprob.stiffness(w, xis[j])
            ref = twogrid.gauss_seidel_sweeps(K, b[j], x0[j], order, 2, backward=back)
            assert relerr(got[j], ref) <= 1e-12, (back, j)


@pytest.mark.parametrize("dim,N,k,batch,mixed", [(2, 20, 6, 2, False), (3, 5, 8, 1, False),
                                                 (3, 6, 8, 5, True), (2, 14, 6, 4, True)])
def test_sgs_cycle_matches_oracle(dim, N, k, batch, mixed):
    import torch
    from paper_2207_02543_amd import capi, pipeline
    flush(f"sgs cycle dim={dim} N={N} k={k} batch={batch} mixed={mixed}")
    w = I.small(dim, N, k=k, n_train=max(12, k + 2))
    P, lam, U = oprob.basis(w, I.train_xis(w))
    prob = pipeline.Problem(w)
    xis = I.query_xis(w, batch)
    sysm = prob.alloc_system(batch, fp32=mixed)
    prob.assemble(sysm, xis)
    pr = prob.setup(sysm, torch.tensor(np.ascontiguousarray(P.T), device="cuda"),
                    precision=capi.MIXED if mixed else capi.FP64, smoother=capi.SMOOTHER_SGS)
    r = np.random.default_rng(9).standard_normal((batch, w.n))
    rd = torch.tensor(r, device="cuda")
    sd = torch.empty_like(rd)
    prob.apply(pr, rd, sd)
    torch.cuda.synchronize()
    s = sd.cpu().numpy()
    order = twogrid.multicolor_order(dim, N)
    for j in range(batch):
        K = oprob.stiffness(w, xis[j])
        ref = twogrid.TwoGrid(K, P, w.omega, smoother="sgs", order=order)(r[j])
        err = relerr(s[j], ref)
        flush(f"  {j}: vs fp64 sgs cycle {err:.2e}")
        assert err <= (5e-6 if mixed else 1e-11)


@pytest.mark.parametrize("dim,N,k,batch,mixed", [(2, 30, 8, 1, False), (3, 6, 10, 2, False),
                                                 (3, 7, 10, 4, True)])
def test_pcg_with_sgs_matches_oracle(dim, N, k, batch, mixed):
    import torch
    from paper_2207_02543_amd import capi, pipeline
    flush(f"pcg sgs dim={dim} N={N} k={k} batch={batch} mixed={mixed}")
    w = I.small(dim, N, k=k, n_train=max(12, k + 2))
    P, lam, U = oprob.basis(w, I.train_xis(w))
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(batch)]
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=mixed)
    prob.assemble(sysm, np.stack([q.xi for q in queries]))
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    pr = prob.setup(sysm, Pd, precision=capi.MIXED if mixed else capi.FP64,
                    smoother=capi.SMOOTHER_SGS)
    u = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u)
    assert ret == capi.OK, st
    prj = prob.setup(sysm, Pd, precision=capi.MIXED if mixed else capi.FP64, key="setup_j")
    uj = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    _, itj, _, _ = prob.solve(sysm, prj, uj, key="pcg_j")
    order = twogrid.multicolor_order(dim, N)
    u = u.cpu().numpy()
    for j, q in enumerate(queries):
        M = twogrid.TwoGrid(q.K, P, w.omega, smoother="sgs", order=order,
                            precision="fp32" if mixed else "fp64")
        ref = opcg.pcg(q.K, q.f, q.x0, M, tol=w.tol, beta="pr" if mixed else "fr")
        flush(f"  {j}: gpu {it[j]} (jacobi {itj[j]}), oracle {ref.iters}")
        assert abs(it[j] - ref.iters) <= 2
        assert rr[j] <= w.tol
        assert relerr(u[j], q.u_exact) <= 1e-6
