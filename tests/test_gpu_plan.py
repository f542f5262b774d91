"""Captured solve plans (HIP graphs of PCG iterations) against the eager
launches: every replay, with eager work and synchronisations between the
replays, must reproduce the eager result bit for bit."""
import numpy as np
import pytest

from gpu_helpers import flush
from oracle import problem as oprob
from paper_2207_02543_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,N,prec,chunk,batch", [
    (2, 24, "fp64", 8, 1), (2, 24, "mixed", 5, 2), (3, 6, "fp64", 8, 3), (2, 17, "fp64", 1, 1)])
def test_plan_replays_match_eager(dim, N, prec, chunk, batch):
    import torch
    from paper_2207_02543_amd import capi, pipeline
    flush(f"plan dim={dim} N={N} {prec} chunk={chunk} batch={batch}")
    w = I.small(dim, N, k=6, n_train=12)
    P, lam, U = oprob.basis(w, I.train_xis(w))
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    precision = capi.MIXED if prec == "mixed" else capi.FP64
    nq = 3 * batch
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(nq)]
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=(prec == "mixed"))
    u = torch.empty(batch, w.n, dtype=torch.float64, device="cuda")

    def load(j0):
        qs = queries[j0:j0 + batch]
        prob.assemble(sysm, np.stack([q.xi for q in qs]))
        pr = prob.setup(sysm, Pd, precision=precision)
        u.copy_(torch.tensor(np.stack([q.x0 for q in qs])))
        return pr

    eager = []
    for j0 in range(0, nq, batch):
        pr = load(j0)
        ret, it, rr, st = prob.solve(sysm, pr, u)
        assert ret == capi.OK
        eager.append((it, u.cpu().numpy().copy()))
    timer = capi.pod2g_timer_create(capi.TK_SWEEP, 4)
    pr = load(0)
    plan = prob.plan(sysm, pr, u, chunk=chunk, timer=timer)
    for rep in range(2):
        for m, j0 in enumerate(range(0, nq, batch)):
            load(j0)
            ret, it, rr, st = plan.solve(w.tol)
            assert ret == capi.OK, (ret, st)
            assert it == eager[m][0]
            np.testing.assert_array_equal(u.cpu().numpy(), eager[m][1])
            # eager work on the same stream between replays
            torch.cuda.synchronize()
            _ = (u * 2.0).sum().item()
    assert timer.launches > 0 and timer.total_ms > 0.0
    plan.close()
    capi.pod2g_timer_destroy(timer)
