"""Host-side logic of the sweep, serving loop and benchmark that runs without a
GPU: request and sweep generation, the arena allocator, the latency report,
the serving summary and the host LAPACK comparator."""
import json
import os
import sys

import numpy as np
import pytest

from paper_2207_03803_amd import gap, serve, sweep

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sweep_recipe_ranges_and_determinism():
    r = sweep.SWEEP_RECIPE
    a = sweep.make_sweep(seed=3)
    b = sweep.make_sweep(seed=3)
    assert a == b and len(a) == r["n_fits"]
    for s in a:
        assert r["n_configs"][0] <= s.n_configs <= r["n_configs"][1]
        assert r["M"][0] <= s.M <= r["M"][1]
        assert s.d in r["ds"] and s.zeta in r["zetas"] and s.sigma_per_atom in r["sigmas"]
    assert sweep.make_sweep(seed=4) != a
    # the tuning-table bucket of the committed table is the recipe's
    assert sweep.bucket(sweep.make_sweep(seed=0)) in sweep.load_table()


def test_requests_follow_the_mix_and_arrive_in_order():
    reqs = serve.make_requests(2000, rate=10.0, seed=1)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    kinds = [r.kind for r in reqs]
    big = sum(1 for r in reqs if r.kind == "fit" and r.spec.n_configs == 100_000)
    small = sum(1 for r in reqs if r.kind == "fit") - big
    assert abs(small / len(reqs) - 0.70) < 0.04
    assert abs(big / len(reqs) - 0.05) < 0.02
    assert abs(kinds.count("predict") / len(reqs) - 0.25) < 0.04
    assert all(1 <= r.n_configs <= 4096 for r in reqs if r.kind == "predict")
    # mean inter-arrival time of a Poisson process at rate 10/s
    assert abs(np.mean(np.diff(t)) - 0.1) < 0.01
    again = serve.make_requests(2000, rate=10.0, seed=1)
    assert [(r.kind, r.arrival) for r in again] == [(r.kind, r.arrival) for r in reqs]


def _host_arena(nbytes):
    """An Arena whose bookkeeping runs on the host (no device buffer)."""
    a = object.__new__(serve.Arena)
    a.size = nbytes
    a.free = [(0, nbytes)]
    a.used = 0
    return a


def test_arena_first_fit_alignment_and_coalescing():
    a = _host_arena(1 << 20)
    x = a.alloc(1)
    y = a.alloc(300)
    assert x == (0, 256) and y == (256, 512)
    a.release(x)
    z = a.alloc(200)  # first fit reuses the hole at 0
    assert z == (0, 256)
    a.release(z)
    a.release(y)
    assert a.free == [(0, 1 << 20)] and a.used == 0
    assert a.alloc((1 << 20) + 1) is None


def test_arena_random_sequences_never_overlap():
    rng = np.random.default_rng(11)
    a = _host_arena(64 << 20)
    live = []
    for _ in range(4000):
        if live and rng.random() < 0.45:
            a.release(live.pop(int(rng.integers(len(live)))))
        else:
            blk = a.alloc(int(rng.integers(1, 2 << 20)))
            if blk is not None:
                live.append(blk)
        spans = sorted(live)
        for (o1, n1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + n1 <= o2
        assert all(o % 256 == 0 and n % 256 == 0 for o, n in live)
        assert a.used == sum(n for _, n in live)
        assert a.used + sum(n for _, n in a.free) == a.size
    for blk in live:
        a.release(blk)
    assert a.free == [(0, 64 << 20)]


def test_latency_report_counts_and_nearest_rank_percentiles():
    reqs = []
    for i in range(100):
        spec = sweep.FitSpec(i, 400, 1000, 500, 2, 1e-3, i)
        r = serve.Request(i, "fit", arrival=float(i), spec=spec)
        r.admitted = r.arrival + 0.01
        r.done = r.arrival + 0.001 * (i + 1)  # latencies 1 .. 100 ms
        r.meta = {"status": gap.GAP_OK}
        if i % 10 == 0:
            r.meta["fallback"] = True
        reqs.append(r)
    bad = serve.Request(100, "fit", arrival=100.0, spec=sweep.FitSpec(100, 128, 10, 20, 3, 1e-4, 0))
    bad.admitted, bad.done, bad.meta = 100.0, 100.5, {"status": gap.GAP_ENOCONV}
    reqs.append(bad)
    for i in range(10):
        p = serve.Request(200 + i, "predict", arrival=float(i), n_configs=7)
        p.admitted, p.done = p.arrival, p.arrival + 0.002
        reqs.append(p)
    rep = serve.latency_report(reqs)
    assert rep["fit"]["n"] == 101 and rep["predict"]["n"] == 10
    assert rep["fit"]["p50_ms"] == pytest.approx(51.0)
    assert rep["fit"]["p99_ms"] == pytest.approx(100.0)
    assert rep["predict"]["p50_ms"] == pytest.approx(2.0)
    assert rep["fit_status"] == {"ok": 100, gap.status_string(gap.GAP_ENOCONV): 1}
    assert rep["fp64_fallbacks"] == 10
    assert rep["failed_fits"] == [dict(rid=100, n_configs=10, M=20, d=128, zeta=3, sigma_per_atom=1e-4,
                                       status=gap.status_string(gap.GAP_ENOCONV))]


def _bench():
    sys.path.insert(0, ROOT)
    import bench

    return bench


def test_serving_summary_renders_every_point():
    bench = _bench()
    pt = lambda load, rate: {"load": load, "arrival_rate_per_s": rate, "fit": {"p50_ms": 10, "p99_ms": 90},
                             "predict": {"p50_ms": 2, "p99_ms": 20}, "fits_per_s": 3.0,
                             "fit_status": {"ok": 5}, "fp64_fallbacks": 1, "all_fits_ok": True}
    out = {"n_requests_per_point": 1000, "mix": "m", "points": [pt(0.5, 5.0), pt(1.0, 10.0)],
           "saturation": {"requests_per_s": 10.0, "fits_per_s": 7.0, "fit_status": {"ok": 9},
                          "fp64_fallbacks": 0, "all_fits_ok": True}}
    md = bench.serve_sweep_md(out, None)
    assert "--serve-requests 1000" in md
    assert "| 0.5 | 5.00 | 10 | 90 | 2 | 20 | 3.00 | - |" in md
    assert "| load 1.0 | ok: 5 | 1 |" in md and "| saturation | ok: 9 | 0 |" in md
    assert md.rstrip().endswith("True.")


def test_lapack_comparator_on_the_tiny_workload():
    bench = _bench()
    r = bench.lapack_baseline("tiny_fp64")
    assert r["kind"] == "lapack" and r["unit"] == "s" and r["cores"] >= 1
    assert np.isfinite(r["value"]) and r["value"] > 0
    json.dumps(r)


def test_bench_refuses_more_than_one_gpu_before_touching_a_device():
    import subprocess

    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT, capture_output=True,
                           text=True, timeout=60, env={**os.environ, **env})
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def _counter_csv(path, rows):
    import csv

    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, counter, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": 256, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_record_scales_the_knm_launch_by_the_copy_calibration(tmp_path):
    import argparse

    from paper_2207_03803_amd import profiling

    knm = "void gap::knm_kernel<64>(gap::KnmArgs)"
    copy = "__amd_rocclr_copyBuffer"
    paths = {}
    for key, counter, rows in (
            ("fit_fetch", "FETCH_SIZE",
             [(knm, "FETCH_SIZE", 100.0), (knm, "FETCH_SIZE", 3.0e8), ("other", "FETCH_SIZE", 9e9)]),
            ("fit_write", "WRITE_SIZE", [(knm, "WRITE_SIZE", 2.0), (knm, "WRITE_SIZE", 3.0e7)]),
            ("copy_fetch", "FETCH_SIZE", [(copy, "FETCH_SIZE", v) for v in (5.0e5, 5.2e5, 5.4e5)]),
            ("copy_write", "WRITE_SIZE", [(copy, "WRITE_SIZE", v) for v in (1.0e6, 1.1e6, 1.2e6)])):
        d = tmp_path / key
        d.mkdir()
        paths[key] = str(d / "counter_collection.csv")
        _counter_csv(paths[key], rows)
    out = str(tmp_path / "rec")
    profiling.traffic(argparse.Namespace(out=out, bench_args="--steps 1 --forms none", **paths))
    rec = json.load(open(out + ".json"))
    ff = profiling.COPY_BYTES / (5.2e5 * 1024)  # the median copy launch, the largest K_NM dispatch
    wf = profiling.COPY_BYTES / (1.1e6 * 1024)
    assert rec["fetch_size_kib_per_launch"] == 3.0e8 and rec["write_size_kib_per_launch"] == 3.0e7
    assert rec["hbm_read_bytes_per_launch"] == pytest.approx(3.0e8 * 1024 * ff, rel=1e-12)
    assert rec["hbm_write_bytes_per_launch"] == pytest.approx(3.0e7 * 1024 * wf, rel=1e-12)
    assert rec["traffic_bytes_per_launch"] == pytest.approx(
        rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"], rel=1e-15)
    assert rec["source_sha256"] == profiling.source_hash()
    md = open(out + ".md").read()
    assert f"-d {tmp_path / 'fit_fetch'} -o fit" in md and f"-d {tmp_path / 'copy_write'} -o copy" in md
    assert "python3 bench.py --steps 1 --forms none" in md


def test_committed_traffic_record_is_consistent():
    from paper_2207_03803_amd import profiling

    rec = json.load(open(os.path.join(ROOT, "profiles", "knm_kernel_realistic_fp64_traffic.json")))
    cal = rec["copy_calibration"]
    assert cal["fetch_factor"] == pytest.approx(profiling.COPY_BYTES / (cal["fetch_size_kib"] * 1024), rel=1e-12)
    assert rec["hbm_read_bytes_per_launch"] == pytest.approx(
        rec["fetch_size_kib_per_launch"] * 1024 * cal["fetch_factor"], rel=1e-12)
    assert rec["traffic_bytes_per_launch"] == pytest.approx(
        rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"], rel=1e-12)
    # the K_NM launch moves at least its algorithmic bytes: descriptors once, the N x M output once
    assert rec["traffic_bytes_per_launch"] > 20.8e9
    bench = _bench()
    expect = rec["traffic_bytes_per_launch"] if rec["source_sha256"] == profiling.source_hash() else None
    assert bench.knm_traffic() == expect


def test_trace_table_aggregates_kernels_by_name(tmp_path):
    import sqlite3

    from paper_2207_03803_amd import profiling

    db = str(tmp_path / "t.db")
    con = sqlite3.connect(db)
    con.execute("create table kernels (kernel_name text, start integer, end integer)")
    con.executemany("insert into kernels values (?, ?, ?)",
                    [("void gap::a(int)", 0, 2_000_000), ("void gap::a(int)", 5_000_000, 9_000_000),
                     ("gap::b", 0, 500_000)])  # timestamps in ns
    con.commit()
    con.close()
    t = profiling.trace_table(db).splitlines()
    assert t[2] == "| `gap::a` | 2 | 6.00 | 3000.0 | 2000.0 | 4000.0 |"
    assert t[3] == "| `gap::b` | 1 | 0.50 | 500.0 | 500.0 | 500.0 |"
