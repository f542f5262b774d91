"""Served solves (continuous batching): a query gives the same result alone
and in a mix of other live queries of two problem classes admitted at
different times, the same as the one-shot batched solve, and matches the
oracle; failures and residual replacement behave as in the one-shot solve."""
import numpy as np
import pytest

from gpu_helpers import flush, relerr
from oracle import problem as oprob
from paper_2207_02543_amd import inputs as I

pytestmark = pytest.mark.gpu

SLOTS = 4


def _class(w, precision="mixed", slots=SLOTS, **kw):
    import torch
    from paper_2207_02543_amd import serve
    P, lam, U = oprob.basis(w, I.train_xis(w))
    Pd = torch.tensor(np.ascontiguousarray(P.T), device="cuda")
    return serve.ServedClass(w, Pd, slots, precision=precision, **kw), P


def _pool(w, count):
    import torch
    from paper_2207_02543_amd import serve
    qs = [oprob.query(w, I.query_xi(w, j), I.noise(w, j)) for j in range(count)]
    pool = serve.Pool(torch.tensor(np.stack([q.xi for q in qs])).pin_memory(),
                      torch.tensor(np.stack([q.x0 for q in qs])).pin_memory(),
                      np.stack([q.u_exact for q in qs]))
    return pool, qs


def _drain(srv, want, max_steps=2000):
    """Step until every global slot in `want` reports done."""
    import torch
    for _ in range(max_steps):
        srv.step()
        torch.cuda.synchronize()
        info = srv.slot_info()
        if all(info[g]["done"] for g in want):
            return info
    raise AssertionError("served solves did not finish")


@pytest.fixture(scope="module")
def two_classes():
    w2 = I.small(2, 20, k=6, n_train=12)
    w3 = I.small(3, 6, k=8, n_train=12)
    c2, P2 = _class(w2)
    c3, P3 = _class(w3)
    p2, q2 = _pool(w2, 5)
    p3, q3 = _pool(w3, 4)
    return (w2, c2, P2, p2, q2), (w3, c3, P3, p3, q3)


def test_alone_equals_mix_equals_batched_solve(two_classes):
    import torch
    from paper_2207_02543_amd import capi, serve
    (w2, c2, P2, p2, q2), (w3, c3, P3, p3, q3) = two_classes
    srv = serve.Server([c2, c3], chunk=4)
    A = 3   # query of class 0 followed through both runs
    flush("serve: query alone")
    srv.admit(0, 1, p2.xi[A], p2.x0[A], w2.tol)
    info = _drain(srv, [1])
    alone_u = c2.u[1].cpu().numpy().copy()
    alone = info[1].copy()
    assert alone["status"] == capi.OK and alone["relres"] <= w2.tol

    flush("serve: query in a mix admitted over several steps")
    base3 = SLOTS
    srv.admit(0, 0, p2.xi[0], p2.x0[0], w2.tol)
    srv.admit(1, 2, p3.xi[0], p3.x0[0], w3.tol)
    srv.step()
    srv.admit(0, 3, p2.xi[A], p2.x0[A], w2.tol)       # A, other slot, others live
    srv.admit(1, 0, p3.xi[1], p3.x0[1], w3.tol)
    srv.step()
    srv.step()
    srv.admit(0, 2, p2.xi[1], p2.x0[1], w2.tol)
    srv.admit(1, 3, p3.xi[2], p3.x0[2], w3.tol)
    info = _drain(srv, [0, 2, 3, base3 + 0, base3 + 2, base3 + 3])
    mix_u = c2.u[3].cpu().numpy()
    assert info[3]["iter"] == alone["iter"]
    np.testing.assert_array_equal(mix_u, alone_u)
    for g in [0, 2, 3, base3 + 0, base3 + 2, base3 + 3]:
        assert info[g]["status"] == capi.OK
        assert info[g]["relres"] <= (w2.tol if g < base3 else w3.tol)

    flush("serve: one-shot batched solve of the same queries")
    prob = c2.prob
    sysm = prob.alloc_system(SLOTS, fp32=True)
    order = [A, 0, 1, 2]
    prob.assemble(sysm, np.stack([q2[j].xi for j in order]))
    pr = prob.setup(sysm, c2.P, precision=capi.MIXED)
    u = torch.tensor(np.stack([q2[j].x0 for j in order]), device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u, key="pcg_ref")
    assert ret == capi.OK
    assert it[0] == alone["iter"]
    np.testing.assert_array_equal(u[0].cpu().numpy(), alone_u)
    np.testing.assert_array_equal(u[1].cpu().numpy(), c2.u[0].cpu().numpy())

    flush("serve: against the oracle")
    for slot, j, c, w, qs, P in [(3, A, c2, w2, q2, P2), (2, 0, c3, w3, q3, P3),
                                 (0, 1, c3, w3, q3, P3)]:
        g = slot + (base3 if c is c3 else 0)
        ref64 = oprob.solve_query(w, qs[j], P, precision="fp64", beta="fr")
        ref32 = oprob.solve_query(w, qs[j], P, precision="fp32", beta="pr")
        got = c.u[slot].cpu().numpy()
        flush(f"  slot {g}: gpu {info[g]['iter']} oracle fp32 {ref32.iters} fp64 {ref64.iters}")
        assert abs(int(info[g]["iter"]) - ref32.iters) <= 2
        assert relerr(got, ref64.u) <= 1e-6
    srv.close()


@pytest.mark.parametrize("independent", [True, False])
def test_stream_completes_every_request(two_classes, independent):
    from paper_2207_02543_amd import capi, serve
    (w2, c2, P2, p2, q2), (w3, c3, P3, p3, q3) = two_classes
    srv = serve.Server([c2, c3], chunk=2)
    n_req = 19
    times = np.zeros(n_req)
    cls = np.array([j % 2 for j in range(n_req)])
    qidx = np.array([(j // 2) % 4 for j in range(n_req)])
    flush(f"serve: stream of {n_req} queued requests over {2 * SLOTS} slots, "
          f"{'one stream per class' if independent else 'classes stepped together'}")
    res = serve.run_stream(srv, [p2, p3], times, cls, qidx, rtol=1e-8, check_first=n_req,
                           realtime=False, independent=independent)
    s = serve.summarize(res, ["2d", "3d"])
    flush(f"  {s['completed']} done in {res.steps} steps")
    assert s["completed"] == n_req and s["failed"] == 0
    for r in res.requests:
        assert r.status == capi.OK and r.relres <= 1e-8
        assert r.err <= 1e-6, (r.rid, r.err)
    # the same pool query gives the same iteration count wherever it ran
    by_q = {}
    for r in res.requests:
        by_q.setdefault((r.ci, r.q), set()).add(r.iters)
    assert all(len(v) == 1 for v in by_q.values())
    srv.close()


def test_setup_failure_is_reported_per_slot():
    from paper_2207_02543_amd import capi, serve
    w = I.small(2, 12, k=4, n_train=8, omega=1.95)
    # the class-level guard refuses the class outright
    with pytest.raises(capi.Pod2gError) as e:
        _class(w)
    assert e.value.status == capi.ESMOOTHER
    # without it, the per-slot guard fails the slot
    c, P = _class(w, power_iters=30, guard=False)
    pool, qs = _pool(w, 1)
    srv = serve.Server([c], chunk=2)
    flush("serve: slot whose smoother guard fails")
    srv.admit(0, 2, pool.xi[0], pool.x0[0], w.tol)
    info = _drain(srv, [2])
    assert info[2]["status"] == capi.ESMOOTHER
    srv.close()


def test_replacement_and_limit_match_one_shot():
    """A tolerance below what the FP32 cycle reaches drives residual
    replacement and the iteration limit: same outcome as pcg_solve."""
    import torch
    from paper_2207_02543_amd import capi, serve
    w = I.small(2, 16, k=6, n_train=12)
    c, P = _class(w)
    pool, qs = _pool(w, 1)
    srv = serve.Server([c], chunk=2)
    flush("serve: rtol 1e-16 with maxit 120")
    srv.admit(0, 1, pool.xi[0], pool.x0[0], 1e-16, maxit=120)
    info = _drain(srv, [1])
    prob = c.prob
    sysm = prob.alloc_system(SLOTS, fp32=True)
    prob.assemble(sysm, np.stack([qs[0].xi] * SLOTS))
    pr = prob.setup(sysm, c.P, precision=capi.MIXED)
    u = torch.tensor(np.stack([qs[0].x0] * SLOTS), device="cuda")
    ret, it, rr, st = prob.solve(sysm, pr, u, rtol=1e-16, maxit=120, key="pcg_ref")
    flush(f"  served {info[1]['iter']} {info[1]['status']}; one-shot {it[0]} {st[0]}")
    assert info[1]["status"] == st[0] == capi.EMAXIT
    assert info[1]["iter"] == it[0]
    assert info[1]["relres"] == rr[0]
    np.testing.assert_array_equal(c.u[1].cpu().numpy(), u[0].cpu().numpy())
    # the oracle (FP32-emulated cycle, flexible PR) on the same input: its
    # exit checks replace the recursive residual, it ends at the limit, and
    # the served result agrees with it at the attainable accuracy
    ref = oprob.solve_query(w, qs[0], P, precision="fp32", beta="pr", tol=1e-16, maxit=120)
    uh = c.u[1].cpu().numpy()
    flush(f"  oracle {ref.iters} {ref.status}, replacements at {ref.replacements}; "
          f"true residual served {info[1]['relres']:.2e} oracle {ref.relres:.2e}; "
          f"difference {relerr(uh, ref.u):.1e}")
    assert ref.status == capi.EMAXIT and ref.iters == info[1]["iter"] == 120
    assert ref.replacements
    assert info[1]["relres"] < 1e-10 and ref.relres < 1e-10
    assert relerr(uh, ref.u) < 1e-9
    srv.close()


def test_prefix_steps_give_the_same_bits():
    """A slot stepped through the graph of a slot prefix (the first four of
    eight slots) and through the whole group's graph: same iterations, same
    bits."""
    import torch
    from paper_2207_02543_amd import serve
    w = I.small(2, 20, k=6, n_train=12)
    c, P = _class(w, slots=8)
    pool, qs = _pool(w, 1)
    srv = serve.Server([c], chunk=4)
    flush("serve: prefix of 4 of 8 slots against the whole group")
    results = []
    for nslots in (2, None):
        srv.admit(0, 1, pool.xi[0], pool.x0[0], w.tol)
        for _ in range(2000):
            srv.step_group(0, nslots=nslots)
            torch.cuda.synchronize()
            info = srv.slot_info()
            if info[1]["done"]:
                break
        assert info[1]["done"] and info[1]["status"] == 0
        results.append((int(info[1]["iter"]), float(info[1]["relres"]), c.u[1].cpu().numpy().copy()))
    flush(f"  prefix {results[0][0]} iterations, whole group {results[1][0]}")
    assert results[0][0] == results[1][0] and results[0][1] == results[1][1]
    np.testing.assert_array_equal(results[0][2], results[1][2])
    srv.close()


def test_compute_unit_shares_keep_the_bits():
    """A class stepped on a stream restricted to a share of the compute
    units gives the same bits as on the whole GPU."""
    import torch
    from paper_2207_02543_amd import serve
    w = I.small(2, 20, k=6, n_train=12)
    c, P = _class(w)
    pool, qs = _pool(w, 2)
    out = []
    for shares in (None, [64]):
        srv = serve.Server([c], chunk=4, cu_shares=shares)
        res = serve.run_stream(srv, [pool], np.zeros(2), np.zeros(2, dtype=int), np.arange(2),
                               rtol=w.tol, realtime=False)
        torch.cuda.synchronize()
        out.append(([r.iters for r in res.requests], [c.out[r.slot].numpy().copy() for r in res.requests]))
        srv.close()
    flush(f"serve: iterations whole GPU {out[0][0]}, 64 compute units {out[1][0]}")
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        np.testing.assert_array_equal(a, b)
    # ranges outside the GPU's compute units are refused (no stream made)
    from paper_2207_02543_amd import capi
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    for first, count in ((0, ncu + 1), (-1, 4), (ncu - 2, 3), (0, 0)):
        with pytest.raises(capi.Pod2gError) as e:
            capi.pod2g_stream_create_cus(first, count)
        assert e.value.status == capi.EINVAL


def test_full_queue_refuses_requests():
    """With a bound on the requests waiting for a slot, arrivals beyond it
    are refused and the admitted ones complete."""
    import torch
    from paper_2207_02543_amd import serve
    w = I.small(2, 16, k=6, n_train=12)
    c, P = _class(w)
    pool, qs = _pool(w, 2)
    srv = serve.Server([c], chunk=4)
    res = serve.run_stream(srv, [pool], np.zeros(10), np.zeros(10, dtype=int), np.arange(10) % 2,
                           rtol=w.tol, realtime=False, max_queue=3)
    torch.cuda.synchronize()
    s = serve.summarize(res, ["a"])
    flush(f"serve: {s['completed']} completed, {s['refused']} refused")
    assert s["completed"] == 3 and s["refused"] == 7 and s["failed"] == 0
    srv.close()
