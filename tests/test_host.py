"""Host-side logic on the CPU: the request-stream generator, slot planning
from free HBM, the serving summary, the rocprofv3 summaries and the
counter-traffic lookup, and the benchmark's algorithmic byte counts."""
import importlib.util
import os

import numpy as np
import pytest

from paper_2207_02543_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_arrivals_are_a_seeded_poisson_stream():
    rate, dur = 200.0, 60.0
    t, cls, q = I.arrivals(rate, dur, 3, 8)
    # count of a Poisson process: mean rate * duration, sd sqrt(mean)
    mean = rate * dur
    assert abs(len(t) - mean) <= 5 * mean ** 0.5
    assert np.all(np.diff(t) > 0) and t[0] > 0 and t[-1] < dur
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() * rate - 1.0) < 0.03
    # exponential gaps: P(gap > 1/rate) = e^-1
    assert abs(np.mean(gaps > 1.0 / rate) - np.exp(-1.0)) < 0.02
    for c in range(3):
        sel = q[cls == c]
        assert abs(len(sel) / len(t) - 1.0 / 3.0) < 0.02
        np.testing.assert_array_equal(sel, np.arange(len(sel)) % 8)   # cycles through the pool
    t2, cls2, q2 = I.arrivals(rate, dur, 3, 8)
    np.testing.assert_array_equal(t, t2)
    np.testing.assert_array_equal(cls, cls2)
    t3, _, _ = I.arrivals(rate, dur, 3, 8, seed=I.ARRIVAL_SEED + 1)
    assert len(t3) != len(t) or not np.array_equal(t3, t)


def test_slot_planning_shares_free_memory():
    from paper_2207_02543_amd import serve
    classes = [(I.WORKLOADS[nm], 20, "mixed") for nm in ("c4a", "c4b", "c4c")]
    sizes = [serve.slot_bytes(w, k, p) for (w, k, p) in classes]
    # a c4c slot (3D 48^3, mixed) holds its FP64 and FP32 matrices (the
    # symmetric half: 14 of 27 blocks per node)
    w = I.WORKLOADS["c4c"]
    assert sizes[2] > (w.n + 3) * 42 * 12
    assert serve.plan_slots(classes, 10 ** 15) == [32, 32, 32]
    assert serve.plan_slots(classes, 10 ** 15, max_slots=7) == [7, 7, 7]
    assert serve.plan_slots(classes, 1) == [1, 1, 1]
    free = 3 * 10 * sizes[2]
    got = serve.plan_slots(classes, free)
    assert got[2] == 10
    for g, s in zip(got, sizes):
        assert g == min(32, (free // 3) // s)


def test_serving_summary():
    from paper_2207_02543_amd import capi, serve
    reqs = []
    lat = {0: [10, 20, 30, 40], 1: [100, 200]}
    rid = 0
    for ci, ls in lat.items():
        for j, l in enumerate(ls):
            r = serve.Request(rid=rid, ci=ci, q=j, t_arrive=1.0 + j)
            r.t_done = r.t_arrive + l / 1e3
            r.iters, r.status, r.relres, r.err = 10 + ci, capi.OK, 1e-9 * (j + 1), 1e-10
            reqs.append(r)
            rid += 1
    pending = serve.Request(rid=rid, ci=1, q=9, t_arrive=5.0)
    reqs.append(pending)
    res = serve.RunResult(requests=reqs, occupancy=[(0.0, [2, 1]), (1.0, [4, 3])], steps=7, wall=2.0)
    s = serve.summarize(res, ["a", "b"])
    all_lat = [10, 20, 30, 40, 100, 200]
    assert s["requests"] == 7 and s["completed"] == 6 and s["failed"] == 0 and s["refused"] == 0
    assert s["solves_per_s"] == pytest.approx(3.0)
    assert s["p50_ms"] == pytest.approx(np.percentile(all_lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(all_lat, 99))
    a, b = s["per_class"]["a"], s["per_class"]["b"]
    assert a["completed"] == 4 and a["p50_ms"] == pytest.approx(25.0) and a["iters_mean"] == 10
    assert b["relres_max"] == pytest.approx(2e-9)
    assert a["live_slots_mean"] == pytest.approx(3.0) and b["live_slots_max"] == 3
    # against solo latencies (on the class's share and on the whole GPU)
    s = serve.summarize(res, ["a", "b"], [12.5, 100.0], [10.0, 50.0])
    a, b = s["per_class"]["a"], s["per_class"]["b"]
    assert a["p50_over_solo"] == pytest.approx(2.0) and b["p50_over_solo"] == pytest.approx(1.5)
    assert a["p50_over_solo_whole_gpu"] == pytest.approx(2.5)
    assert b["solo_whole_gpu_ms"] == 50.0 and b["p50_over_solo_whole_gpu"] == pytest.approx(3.0)


def _write_csv(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for r in rows:
            f.write(",".join(str(x) for x in r) + "\n")


def test_trace_and_counter_summaries_keep_the_marked_region(tmp_path):
    from paper_2207_02543_amd import profiling
    tr = tmp_path / "t.csv"
    # dispatch id, kernel, start, end (ns); only 3..5 lie between the markers
    rows = [(1, "k_warm", 0, 5000), (2, "k_mark_begin", 6000, 6100),
            (3, "k_spmv_pq<3>", 7000, 9000), (4, "k_spmv_pq<3>", 9000, 13000),
            (5, "k_sweep<3>", 13000, 14000), (6, "k_mark_end", 15000, 15100),
            (7, "k_spmv_pq<3>", 16000, 99000)]
    _write_csv(tr, ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = profiling.trace_summary(str(tr)).splitlines()
    assert len(out) == 4
    # the three region dispatches run back to back: busy all of the 7 us
    assert out[3].startswith("## idle: wall 0.01 ms") and "(100.0%)" in out[3]
    assert "0 gaps <= 20 us" in out[3] and "0 gaps > 20 us" in out[3]
    calls, mean, mn, mx, tot, name = out[1].split()
    assert name == "k_spmv_pq<3>" and int(calls) == 2
    assert float(mean) == pytest.approx(3.0) and float(mn) == 2.0 and float(mx) == 4.0
    assert out[2].split()[-1] == "k_sweep<3>"
    pc = tmp_path / "c.csv"
    crow = [(1, "k_spmv_pq<3>", "FETCH_SIZE", 999.0), (2, "k_mark_begin", "FETCH_SIZE", 0.0),
            (3, "k_spmv_pq<3>", "FETCH_SIZE", 10.0), (4, "k_spmv_pq<3>", "FETCH_SIZE", 30.0),
            (5, "k_sweep<3>", "FETCH_SIZE", 7.0), (6, "k_mark_end", "FETCH_SIZE", 0.0)]
    _write_csv(pc, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], crow)
    mean, cnt = profiling.per_dispatch(str(pc), r"k_spmv_pq<", "FETCH_SIZE")
    assert cnt == 2 and mean == pytest.approx(20.0)


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path):
    from paper_2207_02543_amd import profiling
    d = profiling.source_digest()
    assert len(d) == 16 and profiling.source_digest() == d
    (tmp_path / "a.txt").write_text(f"header\ntraffic c9 spmv_pq 12345 source {d}\n")
    (tmp_path / "b.txt").write_text("traffic c9 sweep 777 source 0000000000000000\n")
    assert profiling.traffic_lookup(str(tmp_path), "c9", "spmv_pq") == 12345.0
    assert profiling.traffic_lookup(str(tmp_path), "c9", "sweep") is None
    assert profiling.traffic_lookup(str(tmp_path), "c8", "spmv_pq") is None


def test_algorithmic_bytes():
    from paper_2207_02543_amd import roofline as R
    w = I.WORKLOADS["c2"]
    n, nn, k = w.n, w.n_nodes_free, w.k
    assert (n, nn, k) == (131584, 65792, 20)
    # FP64 values: the own and 4 upper 2x2 blocks per node (symmetric half),
    # planes of n + 2 rows
    K = (n + 2) * 5 * 2 * 8
    idx = 9 * nn * 4           # block-column indices
    # restriction: K, x, b read, r' written (for the first post-sweep with
    # K P), P read once
    assert R.kernel_bytes(w, "restrict") == idx + K + 3 * n * 8 + k * n * 8
    assert R.kernel_bytes(w, "restrict") == 37106848
    # FP32 cycle in 2D keeps the plain post-sweep: no r' to save
    wm = I.with_(w, precision="mixed")
    assert R.kernel_bytes(wm, "restrict") == idx + k * n * 4 + (n + 2) * 5 * 2 * 4 + 2 * n * 4
    # outer SpMV with the direction update folded in: K, s, p_old read, p, q written
    assert R.kernel_bytes(w, "spmv_pq") == idx + K + 4 * n * 8
    assert R.kernel_bytes(w, "spmv_pq", {"fuse_dir": 0}) == idx + K + 2 * n * 8
    w3 = I.WORKLOADS["c3"]
    n3, nn3, B, k3 = w3.n, w3.n_nodes_free, w3.batch, w3.k
    K3 = (n3 + 3) * 14 * 3 * 8
    # large batch: the direction update is its own pass; p read, q written
    assert R.kernel_bytes(w3, "spmv_pq") == 27 * nn3 * 4 + B * (K3 + 2 * n3 * 8)
    assert R.kernel_bytes(w3, "pdir") == B * 3 * n3 * 8
    # batched restriction products: the FP32 basis once, r' per instance
    assert R.kernel_bytes(w3, "ptr_b") == k3 * n3 * 4 + B * n3 * 4
    # setup: K per instance, P once, K P written per instance
    assert R.kernel_bytes(w3, "kp") == 27 * nn3 * 4 + k3 * n3 * 8 + B * (K3 + k3 * n3 * 8)
    # the fused update costs the second sweep's matrix pass on top of the update
    assert R.kernel_bytes(w, "update", {"fuse_upd": 1}) > R.kernel_bytes(w, "update", {"fuse_upd": 0}) + K
    # Gauss-Seidel relaxation never fuses the update with a Jacobi sweep
    assert R.kernel_bytes(w, "update", {"fuse_upd": 1}, "sgs") == R.kernel_bytes(w, "update", {"fuse_upd": 0})
    for key in R.KERNEL_PATTERNS:
        assert R.kernel_bytes(w3, key) > 0


def test_idle_summary_counts_gaps_and_overlaps():
    from paper_2207_02543_amd import profiling
    # two overlapping kernels (one busy stretch), a 0.5 us gap, a 56 us host turn
    rows = [{"Start_Timestamp": str(a), "End_Timestamp": str(b)}
            for a, b in [(0, 1000), (1500, 3000), (2500, 4000), (60000, 61000)]]
    line = profiling.idle_summary(rows)
    assert "wall 0.06 ms" in line and "(7.4%)" in line
    assert "1 gaps <= 20 us total 0.00 ms (median 0.50 us)" in line
    assert "1 gaps > 20 us total 0.06 ms" in line


def test_oracle_leg_samples_and_returns_the_iterates():
    """The CPU-baseline leg run in this process on c1 with the sampled
    branch forced (full_max_n = 0): it returns query 0's iterates after the
    sampled iterations, in the workload's precision and in FP64, equal to
    the oracle's own runs from the same start; the summary extrapolates
    assembly + setup + iterations to the given iteration count."""
    import multiprocessing as mp
    import threading
    import bench
    from oracle import fem, pcg as opcg, problem as oprob, twogrid
    from paper_2207_02543_amd import inputs as I
    w = I.with_(I.WORKLOADS["c1"], precision="mixed")
    P, lam, U = oprob.basis(w, I.train_xis(w))
    q = oprob.query(w, I.query_xis(w, 1)[0], I.noise(w, 0))
    a, b = mp.Pipe()
    t = threading.Thread(target=a.send, args=({"P": P, "x0": q.x0[None]},), daemon=True)
    t.start()
    bench._oracle_leg(b, "c1", {"precision": "mixed"}, 1, 1.0, 0, 4)
    out = a.recv()
    t.join(5)
    assert all(r["kind"] == "sampled" and r["iters"] == 4 for r in out["runs"].values())
    f = fem.traction_load(w.dim, w.N)
    want = opcg.pcg(q.K, f, q.x0, twogrid.TwoGrid(q.K, P, w.omega, w.nu_pre, w.nu_post,
                                                  precision="fp32"), tol=w.tol, maxit=4, beta="pr")
    want64 = opcg.pcg(q.K, f, q.x0, twogrid.TwoGrid(q.K, P, w.omega, w.nu_pre, w.nu_post,
                                                    precision="fp64"), tol=w.tol, maxit=4, beta="fr")
    assert out["iterate"]["iters"] == out["iterate64"]["iters"] == 4
    np.testing.assert_array_equal(out["iterate"]["u"], want.u)
    np.testing.assert_array_equal(out["iterate64"]["u"], want64.u)
    assert np.linalg.norm(want.u - want64.u) > 0.0    # the two precisions differ
    leg = object.__new__(bench.OracleLeg)
    leg.w, leg.result = w, out
    assert leg.iterate() is out["iterate"] and leg.iterate(fp64=True) is out["iterate64"]
    s = leg.summary(100.0)
    run = out["runs"][s["cores"]]
    assert s["value"] == pytest.approx(1.0 / (run["t_assembly"] + run["t_setup"] + 100.0 * run["t_iter"]))
    assert s["kind"] == "oracle" and "extrapolated" in s["sample"]
