"""The two-grid scheme as a standalone solver and the reduced-order warm
start, through the C ABI, against the oracle."""
import numpy as np
import pytest

from gpu_helpers import flush, relerr
from oracle import pcg as opcg, problem as oprob, twogrid
from paper_2207_02543_amd import inputs as I

pytestmark = pytest.mark.gpu


def _prep(w, batch, mixed=False, extra_col=None):
    import torch
    from paper_2207_02543_amd import capi, pipeline
    P, lam, U = oprob.basis(w, I.train_xis(w))
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(batch)]
    if extra_col is not None:
        P = np.concatenate([P, extra_col[:, None]], axis=1)
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=mixed)
    prob.assemble(sysm, np.stack([q.xi for q in queries]))
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    pr = prob.setup(sysm, Pd, precision=capi.MIXED if mixed else capi.FP64)
    return P, queries, prob, sysm, pr


@pytest.mark.parametrize("dim,N,k,batch,mixed", [(2, 24, 6, 2, False), (3, 5, 8, 1, False),
                                                 (3, 6, 8, 4, True), (2, 17, 6, 5, True)])
def test_stationary_solver_matches_oracle(dim, N, k, batch, mixed):
    import torch
    from paper_2207_02543_amd import capi
    flush(f"stationary dim={dim} N={N} k={k} batch={batch} mixed={mixed}")
    w = I.small(dim, N, k=k, n_train=max(12, k + 2))
    P, queries, prob, sysm, pr = _prep(w, batch, mixed)
    u = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    ret, it, rr, st = prob.stationary(sysm, pr, u, maxit=3000)
    assert ret == capi.OK, st
    u = u.cpu().numpy()
    for j, q in enumerate(queries):
        M = twogrid.TwoGrid(q.K, P, w.omega, w.nu_pre, w.nu_post,
                            precision="fp32" if mixed else "fp64")
        ref = opcg.twogrid_solve(q.K, q.f, q.x0, M, tol=w.tol, maxit=3000)
        flush(f"  {j}: gpu {it[j]} cycles relres {rr[j]:.2e}; oracle {ref.iters}")
        assert ref.status == opcg.OK
        assert abs(it[j] - ref.iters) <= (1 if not mixed else 2)
        assert rr[j] <= w.tol
        # the GPU's reported residual is the true one
        assert abs(np.linalg.norm(q.f - q.K @ u[j]) / np.linalg.norm(q.f) - rr[j]) <= 1e-3 * rr[j]
        assert relerr(u[j], q.u_exact) <= 1e-6


def test_stationary_iteration_limit_and_arguments():
    import torch
    from paper_2207_02543_amd import capi
    w = I.small(2, 16, k=4, n_train=8)
    P, queries, prob, sysm, pr = _prep(w, 1)
    u = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    ret, it, rr, st = prob.stationary(sysm, pr, u, maxit=3)
    assert ret == capi.EMAXIT and it == [3] and rr[0] > w.tol
    ret, it, rr, st = prob.stationary(sysm, pr, u, maxit=0)
    assert ret == capi.EINVAL


@pytest.mark.parametrize("dim,N,k,batch", [(2, 20, 6, 3), (3, 5, 8, 2)])
def test_rom_start_matches_oracle(dim, N, k, batch):
    import torch
    flush(f"rom start dim={dim} N={N} k={k} batch={batch}")
    w = I.small(dim, N, k=k, n_train=max(12, k + 2))
    P, queries, prob, sysm, pr = _prep(w, batch)
    u = torch.empty(batch, w.n, dtype=torch.float64, device="cuda")
    prob.rom_start(sysm, pr, u)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    for j, q in enumerate(queries):
        L = twogrid.coarse_factor(q.K, P)
        ref = opcg.rom_solve(q.K, q.f, P, L)
        assert relerr(u[j], ref) <= 1e-9
        # Galerkin: the residual of the reduced solution is orthogonal to the basis
        r = q.f - q.K @ u[j]
        assert np.abs(P.T @ r).max() <= 1e-8 * np.abs(P.T @ q.f).max()


def test_rom_start_exact_in_span_and_as_pcg_start():
    import torch
    from paper_2207_02543_amd import capi
    w = I.small(2, 16, k=5, n_train=10)
    q0 = oprob.query(w, I.query_xi(w, 0), I.noise(w, 0))
    P, queries, prob, sysm, pr = _prep(w, 1, extra_col=q0.u_exact)
    u = torch.empty(1, w.n, dtype=torch.float64, device="cuda")
    prob.rom_start(sysm, pr, u)
    torch.cuda.synchronize()
    assert relerr(u.cpu().numpy()[0], q0.u_exact) <= 1e-9
    # without the exact column: PCG from the reduced solution
    P, queries, prob, sysm, pr = _prep(w, 1)
    prob.rom_start(sysm, pr, u)
    ret, it, rr, st = prob.solve(sysm, pr, u)
    assert ret == capi.OK and rr[0] <= w.tol
    q = queries[0]
    x0 = opcg.rom_solve(q.K, q.f, P, twogrid.coarse_factor(q.K, P))
    ref = opcg.pcg(q.K, q.f, x0, twogrid.TwoGrid(q.K, P, w.omega), tol=w.tol, beta="fr")
    flush(f"  pcg from the reduced solution: gpu {it[0]}, oracle {ref.iters}")
    assert abs(it[0] - ref.iters) <= 2
    assert relerr(u.cpu().numpy()[0], q.u_exact) <= 1e-6
