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
    timer = capi.pod2g_timer_create(capi.TK_UPDATE, 4)
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


@pytest.mark.parametrize("dim,N,prec,batch", [(2, 24, "fp64", 1), (3, 6, "mixed", 8)])
def test_tuned_plan_solves_like_eager(dim, N, prec, batch):
    """The tuner only changes launch parameters (grid of the batched
    restriction, fused or separate direction update, block order): the tuned
    plan converges like the eager solve (iterations within 2, same accuracy)."""
    import torch
    from paper_2207_02543_amd import capi, pipeline
    flush(f"tuned plan dim={dim} N={N} {prec} batch={batch}")
    w = I.small(dim, N, k=6, n_train=12)
    P, lam, U = oprob.basis(w, I.train_xis(w))
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    precision = capi.MIXED if prec == "mixed" else capi.FP64
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(batch)]
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=(prec == "mixed"))
    prob.assemble(sysm, np.stack([q.xi for q in queries]))
    pr = prob.setup(sysm, Pd, precision=precision)
    x0 = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    u = x0.clone()
    ret, it_e, rr_e, st = prob.solve(sysm, pr, u)
    assert ret == capi.OK
    u_e = u.cpu().numpy().copy()
    plan = prob.plan(sysm, pr, u, chunk=8)
    t = plan.tune(trials=4)
    flush(f"  tuning {t}")
    assert t["bgrid"] in (256, 512, 1024, 2048) or t["bgrid"] <= 512
    assert t["fuse_dir"] in (0, 1) and batch % t["igroup"] == 0 and t["ms_per_iteration"] > 0
    u.copy_(x0)
    ret, it, rr, st = plan.solve(w.tol)
    assert ret == capi.OK
    for b in range(batch):
        assert abs(it[b] - it_e[b]) <= 2 and rr[b] <= w.tol
        assert np.linalg.norm(u[b].cpu().numpy() - u_e[b]) <= 1e-6 * np.linalg.norm(u_e[b])
    plan.close()


@pytest.mark.parametrize("dim,N,prec,batch", [
    (2, 24, "fp64", 1), (2, 24, "fp64", 4), (2, 24, "mixed", 4), (3, 6, "fp64", 2), (3, 6, "mixed", 4)])
def test_launch_parameters_keep_the_result(dim, N, prec, batch):
    """Each launch parameter set explicitly, one at a time, on the same plan:
    the direction update fused or not, sums finished by consumers or
    producers, the LDS-staged neighbourhood (2D), the instance grouping and
    the row groups of the batched restriction loaded together give the
    same bits; the fused vector update (other grouping of the ||r||^2
    and r^T s_old partials) and the batched restriction's grid (other
    partition of its sums) change rounding only.  Invalid values are
    rejected and leave the plan as it was."""
    import torch
    from paper_2207_02543_amd import capi, pipeline
    flush(f"launch parameters dim={dim} N={N} {prec} batch={batch}")
    w = I.small(dim, N, k=6, n_train=12)
    P, lam, U = oprob.basis(w, I.train_xis(w))
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    precision = capi.MIXED if prec == "mixed" else capi.FP64
    queries = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(batch)]
    prob = pipeline.Problem(w)
    sysm = prob.alloc_system(batch, fp32=(prec == "mixed"))
    prob.assemble(sysm, np.stack([q.xi for q in queries]))
    pr = prob.setup(sysm, Pd, precision=precision)
    x0 = torch.tensor(np.stack([q.x0 for q in queries]), device="cuda")
    u = x0.clone()
    plan = prob.plan(sysm, pr, u, chunk=8)
    base = plan.config()
    flush(f"  default {base}")

    def run():
        u.copy_(x0)
        ret, it, rr, st = plan.solve(w.tol)
        assert ret == capi.OK, st
        return list(it), u.cpu().numpy().copy()

    it0, u0 = run()
    variants = [dict(fuse_dir=1 - base["fuse_dir"]), dict(cons=1 - base["cons"])]
    if dim == 2:
        variants.append(dict(xwin=0 if base["xwin"] else 1))
    if batch % 2 == 0:
        variants.append(dict(igroup=2))
    if batch % 4 == 0:
        variants.append(dict(igroup=4))
    # row groups of the batched restriction loaded together: schedule only
    variants += [dict(ptr_grp=g) for g in (1, 2, 4) if g != base["ptr_grp"]]
    for v in variants:
        plan.configure(**{**base, **v})
        it, uv = run()
        flush(f"  {v}: iterations {it}")
        assert it == it0
        np.testing.assert_array_equal(uv, u0)
    # rounding-only changes
    rounding = [dict(fuse_upd=1 - base["fuse_upd"])]
    if base["bgrid"] > 1:
        rounding.append(dict(bgrid=1))
    for v in rounding:
        plan.configure(**{**base, **v})
        it, uv = run()
        flush(f"  {v}: iterations {it}")
        for b in range(batch):
            assert abs(it[b] - it0[b]) <= 1
            assert np.linalg.norm(uv[b] - u0[b]) <= 1e-7 * np.linalg.norm(u0[b])
    # invalid values: rejected, plan unchanged
    plan.configure(**base)
    for bad in [dict(bgrid=0), dict(cons=2), dict(fuse_upd=-1), dict(igroup=3), dict(igroup=16),
                dict(ptr_grp=3), dict(ptr_grp=0)] + \
            ([dict(xwin=1)] if dim == 3 else []):
        t = capi.Tuning(**{**base, **bad})
        assert capi.pcg_plan_configure(plan.handle, t) == capi.EINVAL, bad
        assert plan.config() == base
    it, uv = run()
    assert it == it0
    np.testing.assert_array_equal(uv, u0)
    plan.close()
