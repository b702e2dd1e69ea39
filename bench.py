"""Benchmark: one GAP fit (K_NM build + Cholesky + Householder QR + solve) at
the realistic workload, N = 1e5 configurations of 16..64 atoms, d = 400,
M = 1e4 sparse points, zeta = 4, FP64, beside the three forms around it:

  mixed  the same fit with an FP32 Householder QR and FP64 refinement of c
  bf16   mixed, with the factored K_NM block from BF16 descriptor dot products
  fp16   mixed, with FP16 descriptor dot products
  int8   the FP64 fit with its K_NM dot products emulated on INT8 MFMA, and the mixed fit on that K_NM
         (Ozaki scheme: 7 slices per value, 28 exact slice products)
  cur    CUR sparse-point selection of M rows from the descriptor rows
         (leverages on FP64 MFMA, sampling by exponential keys)
  forces a fit with energies, forces and virials (2e4 atoms, 6.2e4
         derivative observations, d = 400, M = 4000), FP64 and mixed
  sweep  64 uneven fits of a hyperparameter sweep, one HIP graph per fit
         replayed on several streams (FP32 QR + FP64 refinement), against the
         same fits run one after another in plain FP64
  serve  Poisson fit/predict requests through the continuous-batching loop:
         p50/p99 latency and fits/s, mixed precision and plain FP64

Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms mixed,bf16,fp16,int8,cur,forces,sweep,serve | none]
                  [--workload realistic_fp64|tiny_fp64] [--no-cpu-baseline]

A step is one whole fit on inputs already resident in HBM; `value` is the FP64
fit's seconds per step.  Inputs are synthetic (seeded), shaped like a GAP
training set: see paper_2207_03803_amd/synth.py and sweep.py.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
# The sweep and the serving loop run fits on up to 16 streams at once: give the
# process as many hardware queues (HIP's default is 4), before HIP starts.
os.environ["GPU_MAX_HW_QUEUES"] = "16"
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12   # MI355X dense FP64 matrix peak, FLOP/s
PEAK_FP32_MFMA = 157.3e12  # MI355X dense FP32 matrix peak, FLOP/s
PEAK_BF16_MFMA = 2.5e15    # MI355X dense BF16 / FP16 matrix peak, FLOP/s
PEAK_INT8_MFMA = 5.0e15    # MI355X dense INT8 matrix peak, OP/s
PEAK_HBM = 8.0e12          # MI355X HBM3E, B/s
GOLDEN = os.path.join(ROOT, "tests", "golden", "realistic_fp64_seed0.npz")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def knm_traffic():
    """HBM bytes per knm_kernel launch from the committed counter runs, or None when
    the kernel's source has changed since those counters were taken."""
    from paper_2207_03803_amd.profiling import source_hash

    path = os.path.join(ROOT, "profiles", "knm_kernel_realistic_fp64_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if source_hash() != rec.get("source_sha256"):
        return None
    return rec["traffic_bytes_per_launch"]


def load_reference(workload, seed):
    """The oracle's full-size reference fit (y, c, loss) for this workload and seed,
    or None (written by tests/golden/make_reference_fits.py from the oracle alone)."""
    import numpy as np

    if workload != "realistic_fp64" or seed != 0 or not os.path.exists(GOLDEN):
        return None
    z = np.load(GOLDEN, allow_pickle=False)
    ref = {k: z[k] for k in z.files if k != "meta"}
    ref["meta"] = json.loads(str(z["meta"]))
    return ref


def bench_cur(args, X, n, d, M, host_inputs):
    """CUR sparse-point selection over the workload's descriptor rows: M rows
    sampled in proportion to their leverage (gap_cur_select), timed with HIP events
    on the current stream over --steps calls after --warmup; with the host-drawn
    inputs the selection is compared with the oracle's
    (tests/golden/cur_realistic_seed0.npz)."""
    import numpy as np
    import torch

    from paper_2207_03803_amd import gap, synth

    draws = torch.from_numpy(synth.cur_draws(n, args.seed)).cuda()
    ws = torch.empty(gap.cur_workspace_bytes(n, d), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        gap.cur_select(X, M, draws=draws, workspace=ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        idx, lev = gap.cur_select(X, M, draws=draws, leverage=True, workspace=ws, wait=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    flops = 2.0 * n * d * d  # Gram (symmetric) and the triangular projection: n d^2 each
    out = {"ms": ms, "n_rows": n, "d": d, "M": M, "tflops": flops / (ms / 1e3) / 1e12,
           "sum_leverage": float(lev.sum().item()),
           "note": "leverages x_i^T (X^T X)^-1 x_i (Gram and projection on FP64 MFMA, Cholesky, triangular "
                   "inverse), M rows sampled in proportion to leverage by exponential keys (radix select)"}
    golden = os.path.join(ROOT, "tests", "golden", "cur_realistic_seed0.npz")
    if host_inputs and args.seed == 0 and os.path.exists(golden):
        z = np.load(golden, allow_pickle=False)
        out["rows_differing_from_oracle_selection"] = int(len(np.setxor1d(idx.cpu().numpy(), z["sampled_idx"])))
        out["oracle_seconds"] = json.loads(str(z["meta"]))["leverage_s"]
    log(f"[bench] cur: {ms:.2f} ms per selection ({out['tflops']:.1f} TFLOP/s)")
    return out


def bench_forces(args, gap, log):
    """The energies-forces-virials workload (synth.WORKLOADS["forces_fp64"]): whole
    fits (gap_build_knm_obs + gap_solve) in FP64 and mixed precision, timed like the
    main fit; c against the oracle's reference fit when it is available."""
    import numpy as np
    import torch

    from paper_2207_03803_amd import synth

    w = dict(synth.WORKLOADS["forces_fp64"])
    D = synth.make_deriv_inputs(seed=args.seed, **w)
    dev = "cuda"
    golden = os.path.join(ROOT, "tests", "golden", "forces_fp64_seed0.npz")
    z = np.load(golden, allow_pickle=False) if args.seed == 0 and os.path.exists(golden) else None
    y = torch.from_numpy(z["y"] if z is not None else D.sigma * np.concatenate([D.noise_E, D.noise_D])).to(dev)
    X, offs, XM = (torch.from_numpy(a).to(dev) for a in (D.X, D.offsets, D.XM))
    sig = torch.from_numpy(D.sigma).to(dev)
    obs = {k: torch.from_numpy(getattr(D, k)).to(dev)
           for k in ("x_grad", "grad_atom", "obs_offsets", "pos_grad", "pos_weight")}
    M, d, n_pos = D.XM.shape[0], w["d"], len(D.pos_grad)
    out = {"n_configs": D.n_configs, "n_atoms": D.n_atoms, "n_derivative_obs": D.n_obs, "n_positions": n_pos,
           "M": M, "d": d, "zeta": w["zeta"], "stacked_matrix": [D.n_configs + D.n_obs + M, M]}
    kdm_flops = 2.0 * n_pos * M * d + (2.0 * D.n_atoms * M * d if w["zeta"] > 1 else 0.0)
    for name, prec in (("fp64", gap.GAP_FP64), ("mixed", gap.GAP_MIXED_FP32)):
        with torch.cuda.stream(torch.cuda.Stream()):
            h = gap.Handle(gap.params(d, w["zeta"], w["sigma_w"], w["jitter"], precision=prec,
                                      flags=gap.GAP_FLAG_TIMING, max_refine_iters=30, refine_tol=1e-12))
            h.set_tuning(qr_free_cus=32)
            h.alloc_workspace_obs(D.n_configs, D.n_atoms, D.n_obs, n_pos, M)
            c = torch.empty(M, dtype=torch.float64, device=dev)
            stage_sum, per = {}, []
            for i in range(args.warmup + args.steps):
                ts = time.perf_counter()
                h.build_knm_obs(X, offs, obs, XM, sig)
                h.solve(y, c, info=False)
                st = h.stage_times()
                if i >= args.warmup:
                    per.append(time.perf_counter() - ts)
                    for k, v in st.items():
                        stage_sum[k] = stage_sum.get(k, 0.0) + v
            status, info = h.sync()
            h.close()
        stages = {k: v / args.steps for k, v in stage_sum.items() if v > 0}
        r = {"s_per_fit": float(np.mean(per)), "median_ms": 1e3 * float(np.median(per)), "stages_ms": stages,
             "status": gap.status_string(status), "refine_iters": info.refine_iters,
             "kdm_tflops": kdm_flops / (stages["kdm"] / 1e3) / 1e12}
        if z is not None:
            r["c_rel_err_vs_oracle"] = float(np.linalg.norm(c.cpu().numpy() - z["c"]) / np.linalg.norm(z["c"]))
        out[name] = r
        log(f"[bench] forces {name}: {1e3 * r['s_per_fit']:.1f} ms per fit (derivative rows "
            f"{stages['kdm']:.1f} ms, {r['kdm_tflops']:.1f} TFLOP/s)")
    return out


def fit_flops(n_atoms, N, M, d):
    m, n = N + M, M
    return {
        "knm": 2.0 * n_atoms * M * d,
        "kmm": 2.0 * M * M * d,
        "cholesky": M ** 3 / 3.0,
        "qr": 2.0 * m * n * n - 2.0 * n ** 3 / 3.0 + 4.0 * m * n,  # dense Householder QR (the oracle's)
        # the library skips the rows of the trailing L^T that are still zero (at column j the
        # reflector spans N + 1 rows): 4 (N + 1) (n - j) flops for column j and b
        "qr_tri": 2.0 * (N + 1) * n * (n + 1) + 4.0 * (N + 1) * n,
        "trsv": float(n * n),
    }


def cpu_baseline(workload, budget_note):
    """Time the CPU oracle on bounded samples of the workload and scale each
    stage by its flop count to one whole fit."""
    import numpy as np

    import oracle
    from paper_2207_03803_amd import synth

    orc = oracle.Oracle()
    w = dict(synth.WORKLOADS[workload])
    d, zeta = w["d"], w["zeta"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # K_NM sample: 6000 configurations x 3200 sparse points
    Ns, Ms = (6000, 3200) if workload != "tiny_fp64" else (w["n_configs"], w["M"])
    inp = synth.make_fit_inputs(n_configs=Ns, atoms=w["atoms"], d=d, M=Ms, seed=123)
    t0 = time.perf_counter()
    orc.knm(inp.X, inp.offsets, inp.XM, zeta)
    t_knm = time.perf_counter() - t0
    f_knm_s = 2.0 * inp.n_atoms * Ms * d
    # QR sample: m x n Householder QR with the b column, at the workload's full row count
    # (the oracle's column steps stream the trailing matrix: their rate depends on m)
    ms, ns = (w["n_configs"] + w["M"], 400) if workload != "tiny_fp64" else (w["n_configs"] + w["M"], w["M"])
    rng = np.random.default_rng(7)
    A = rng.standard_normal((ms, ns))
    b = rng.standard_normal(ms)
    t0 = time.perf_counter()
    orc.householder_qr(A, b)
    t_qr = time.perf_counter() - t0
    f_qr_s = 2.0 * ms * ns * ns - 2.0 * ns ** 3 / 3
    # Cholesky sample
    mc = min(2000, w["M"], inp.n_atoms)
    K = orc.kmm(inp.X[:mc], zeta, jitter=1e-8)
    t0 = time.perf_counter()
    orc.cholesky(K)
    t_ch = time.perf_counter() - t0
    f_ch_s = K.shape[0] ** 3 / 3.0
    # full workload flops (mean atoms per configuration from the recipe)
    lo, hi = w["atoms"]
    n_atoms = w["n_configs"] * (lo + hi) / 2.0
    f = fit_flops(n_atoms, w["n_configs"], w["M"], d)
    t_full = (f["knm"] + f["kmm"]) * t_knm / f_knm_s + f["qr"] * t_qr / f_qr_s + f["cholesky"] * t_ch / f_ch_s
    sample = (f"oracle K_NM on {Ns} configs x {Ms} sparse points (d={d}, zeta={zeta}) {t_knm:.2f}s; "
              f"unblocked Householder QR {ms}x{ns} {t_qr:.2f}s; Cholesky {K.shape[0]} {t_ch:.2f}s; "
              f"each scaled by flop count to the full fit")
    return {"value": t_full, "unit": "s", "cores": cores, "kind": "oracle", "sample": sample,
            "seconds_measured": t_knm + t_qr + t_ch, "note": budget_note}


def lapack_baseline(workload):
    """The paper's single-node CPU route on host LAPACK / BLAS (numpy and scipy,
    all cores): K_NM as a dgemm with the power and the per-configuration sums,
    dgeqrf on [A | b] (scipy.linalg.qr, R only), dpotrf; each timed on a sample
    and scaled by its flop count to one whole fit."""
    import numpy as np
    import scipy.linalg

    from paper_2207_03803_amd import synth

    w = dict(synth.WORKLOADS[workload])
    d, zeta = w["d"], w["zeta"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    Ns, Ms = (6000, 3200) if workload != "tiny_fp64" else (w["n_configs"], w["M"])
    inp = synth.make_fit_inputs(n_configs=Ns, atoms=w["atoms"], d=d, M=Ms, seed=123)
    from concurrent.futures import ThreadPoolExecutor

    def epilogue(G, offs):
        # power by repeated multiplication and the per-configuration sums (numpy
        # releases the GIL in these loops, so the slices run in parallel)
        P = G.copy()
        for _ in range(zeta - 1):
            P *= G
        return np.add.reduceat(P, offs, axis=0)

    t0 = time.perf_counter()
    step = 1000  # configurations per GEMM (bounds the atom-level block in host memory)
    with ThreadPoolExecutor(max_workers=cores) as pool:
        for c0 in range(0, Ns, step):
            c1 = min(Ns, c0 + step)
            a0, a1 = int(inp.offsets[c0]), int(inp.offsets[c1])
            G = inp.X[a0:a1] @ inp.XM.T  # multithreaded dgemm
            cuts = np.linspace(c0, c1, min(cores, c1 - c0) + 1).astype(np.int64)
            jobs = [pool.submit(epilogue, G[int(inp.offsets[u]) - a0:int(inp.offsets[v]) - a0],
                                inp.offsets[u:v] - inp.offsets[u]) for u, v in zip(cuts[:-1], cuts[1:]) if v > u]
            for j in jobs:
                j.result()
    t_knm = time.perf_counter() - t0
    f_knm_s = 2.0 * inp.n_atoms * Ms * d
    ms, ns = (20000, 2500) if workload != "tiny_fp64" else (w["n_configs"] + w["M"], w["M"])
    A = np.random.default_rng(7).standard_normal((ms, ns + 1))
    t0 = time.perf_counter()
    scipy.linalg.qr(A, mode="r", overwrite_a=True, check_finite=False)
    t_qr = time.perf_counter() - t0
    f_qr_s = 2.0 * ms * ns * ns - 2.0 * ns ** 3 / 3
    mc = min(6000, w["M"])
    B = np.random.default_rng(8).standard_normal((mc, mc))
    K = B @ B.T + mc * np.eye(mc)
    t0 = time.perf_counter()
    np.linalg.cholesky(K)
    t_ch = time.perf_counter() - t0
    f_ch_s = mc ** 3 / 3.0
    lo, hi = w["atoms"]
    f = fit_flops(w["n_configs"] * (lo + hi) / 2.0, w["n_configs"], w["M"], d)
    t_full = (f["knm"] + f["kmm"]) * t_knm / f_knm_s + f["qr"] * t_qr / f_qr_s + f["cholesky"] * t_ch / f_ch_s
    sample = (f"BLAS K_NM on {Ns} configs x {Ms} sparse points (d={d}, zeta={zeta}) {t_knm:.2f}s "
              f"({f_knm_s / t_knm / 1e9:.0f} GFLOP/s); dgeqrf {ms}x{ns + 1} {t_qr:.2f}s "
              f"({f_qr_s / t_qr / 1e9:.0f} GFLOP/s); dpotrf {mc} {t_ch:.2f}s; each scaled by flop count to the full fit")
    return {"value": t_full, "unit": "s", "cores": cores, "kind": "lapack", "sample": sample,
            "seconds_measured": t_knm + t_qr + t_ch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="realistic_fp64")
    ap.add_argument("--forms", default="mixed,bf16,fp16,int8,cur,forces,sweep,serve",
                    help="comma-separated forms to measure beside the FP64 fit, or none")
    ap.add_argument("--inputs", choices=("host", "device"), default="host",
                    help="host: numpy descriptors (the arrays the oracle's full-size reference fit used); "
                         "device: torch's generator on the GPU (faster to draw, no oracle reference)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only the serving loop: saturation throughput, then latency at 0.5/0.8/1.0/1.2 x it")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-summary", default=None,
                    help="with --serve-sweep: also write a markdown summary of the sweep to this path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the fit's hot path runs on a single MI355X here; "
              "multi-GPU sharding is a design note only (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2207_03803_amd import gap, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        # A plain copy of known size: 2^27 doubles (1 GiB) read and 1 GiB written per launch.
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 8 << 27, "launches": 3}), flush=True)
        return
    if args.serve_sweep:
        serve_sweep(args, dev)
        return
    w = dict(synth.WORKLOADS[args.workload])
    N, M, d, zeta = w["n_configs"], w["M"], w["d"], w["zeta"]
    log(f"[bench] generating {args.workload}: N={N} M={M} d={d} zeta={zeta} ({args.inputs})")
    t0 = time.perf_counter()
    ref = None
    if args.inputs == "host":
        # the oracle's reference fit was computed on exactly these arrays
        inp = synth.make_fit_inputs_blocked(seed=args.seed, workers=16, log=log, **w)
        X = torch.from_numpy(inp.X).to(dev)
        XM = torch.from_numpy(inp.XM).to(dev)
        inp.X = None
        ref = load_reference(args.workload, args.seed)
    else:
        inp = synth.make_fit_inputs_torch(seed=args.seed, device=dev, **w)
        X, XM = inp.X, inp.XM
    offsets = torch.from_numpy(inp.offsets).to(dev)
    sigma = torch.from_numpy(inp.sigma).to(dev)
    n_atoms = inp.n_atoms
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f}s (n_atoms={n_atoms}; oracle reference: "
        f"{'yes' if ref is not None else 'no'})")
    f = fit_flops(n_atoms, N, M, d)

    def run_fit(precision, steps, warmup, y=None, flags=0):
        """Time `steps` whole fits (build + solve) after `warmup` untimed ones, on a
        stream of the fit's own (beside it the QR look-ahead keeps CUs free for the
        panel chain)."""
        with torch.cuda.stream(torch.cuda.Stream()):
            return _run_fit(precision, steps, warmup, y, flags)

    def _run_fit(precision, steps, warmup, y=None, flags=0):
        iters = 30 if precision in (gap.GAP_FP64, gap.GAP_MIXED_FP32) else 200
        p = gap.params(d, zeta, w["sigma_w"], w["jitter"], precision=precision, flags=gap.GAP_FLAG_TIMING | flags,
                       max_refine_iters=iters, refine_tol=1e-12)
        h = gap.Handle(p)
        # one fit on a stream of its own and nothing on the legacy stream meanwhile:
        # keep CUs free of the QR look-ahead stream for the panel chain
        h.set_tuning(qr_free_cus=32)
        h.alloc_workspace(N, n_atoms, M)
        if y is None:
            # targets: model prediction with c_true (through the library) plus noise
            h.build_knm(X, offsets, XM, sigma)
            y = torch.empty(N, dtype=torch.float64, device=dev)
            h.predict(X, offsets, torch.from_numpy(inp.c_true).to(dev), y)
            y += sigma * torch.from_numpy(inp.noise).to(dev)
            torch.cuda.synchronize()
        c = torch.empty(M, dtype=torch.float64, device=dev)
        stage_sum = {}

        def step(record):
            h.build_knm(X, offsets, XM, sigma)
            h.solve(y, c, info=False)
            st = h.stage_times()  # waits for the stream
            if record:
                for k, v in st.items():
                    stage_sum[k] = stage_sum.get(k, 0.0) + v

        tag = {gap.GAP_FP64: "fp64", gap.GAP_MIXED_FP32: "mixed", gap.GAP_MIXED_BF16: "mixed_bf16",
               gap.GAP_MIXED_FP16: "mixed_fp16"}[precision] + ("_int8" if flags & gap.GAP_FLAG_KNM_INT8 else "")
        for i in range(warmup):
            step(False)
            log(f"[bench] {tag} warmup {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_step = []
        for i in range(steps):
            ts = time.perf_counter()
            step(True)  # ends with a wait for the stream (the stage timers)
            per_step.append(time.perf_counter() - ts)
            log(f"[bench] {tag} step {i + 1}/{steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        s_status, info = h.sync()
        if s_status != gap.GAP_OK and not (s_status == gap.GAP_ENOCONV and precision in (gap.GAP_MIXED_BF16,
                                                                                           gap.GAP_MIXED_FP16)):
            raise RuntimeError(f"{tag} fit: device status {gap.status_string(s_status)}")
        h.close()
        del h
        torch.cuda.empty_cache()
        stages_ms = {k: v / steps for k, v in stage_sum.items() if v > 0}
        return dict(ms=1e3 * elapsed / steps, ms_median=1e3 * float(np.median(per_step)),
                    ms_min=1e3 * min(per_step), stages_ms=stages_ms, info=info, c=c, y=y, status=s_status)

    def vs_oracle(res):
        """c and the minimum loss of a timed fit against the oracle's reference fit."""
        if ref is None:
            return {}
        c = res["c"].cpu().numpy()
        return {"c_rel_err_vs_oracle": float(np.linalg.norm(c - ref["c"]) / np.linalg.norm(ref["c"])),
                "loss_rel_err_vs_oracle": abs(res["info"].residual_norm2 - float(ref["loss_tail"]))
                / float(ref["loss_tail"])}

    y_ref = torch.from_numpy(ref["y"]).to(dev) if ref is not None else None
    fp = run_fit(gap.GAP_FP64, args.steps, args.warmup, y=y_ref)
    ms_per_step = fp["ms"]
    step_stats = {"median_ms": fp["ms_median"], "min_ms": fp["ms_min"]}
    stages_ms = fp["stages_ms"]
    knm_s = stages_ms["knm"] / 1e3
    achieved = f["knm"] / knm_s
    # With the QR look-ahead (M >= 2048) the K_MM and its Cholesky run on the look-ahead
    # stream beside the K_NM: their stage events then span the overlap (mostly waiting for
    # CUs), and the K_NM's own time includes sharing the GPU with them.
    kmm_overlapped = M >= 2048
    stage_rates = {
        "knm_tflops": f["knm"] / knm_s / 1e12,
        "qr_tflops": f["qr_tri"] / (stages_ms["qr"] / 1e3) / 1e12,
    }
    if kmm_overlapped:
        others = sum(v for k, v in stages_ms.items() if k not in ("kmm", "cholesky"))
        stage_rates["kmm_cholesky_overlapped"] = {
            "side_stream_span_ms": stages_ms["kmm"] + stages_ms["cholesky"],
            "exposed_ms": max(0.0, ms_per_step - others),
            "note": "K_MM + Cholesky on the look-ahead stream beside the K_NM; exposed_ms = fit time minus the "
                    "main stream's stages"}
    else:
        stage_rates["kmm_tflops"] = f["kmm"] / (stages_ms["kmm"] / 1e3) / 1e12
        stage_rates["cholesky_tflops"] = f["cholesky"] / (stages_ms["cholesky"] / 1e3) / 1e12
    fp_oracle = vs_oracle(fp)
    if fp_oracle:
        log(f"[bench] fp64: c rel err vs oracle {fp_oracle['c_rel_err_vs_oracle']:.2e}")
    rooflines = [
        {"stage": "knm", "kernel": "knm_kernel", "bound": "mfma", "dtype": "f64",
         "achieved": f["knm"] / knm_s / 1e12, "peak": PEAK_FP64_MFMA / 1e12},
        {"stage": "qr", "kernel": "qr_wpart_kernel + qr_update_kernel (+ panels)", "bound": "mfma", "dtype": "f64",
         "achieved": stage_rates["qr_tflops"], "peak": PEAK_FP64_MFMA / 1e12},
    ]
    if not kmm_overlapped:
        rooflines.append({"stage": "cholesky", "kernel": "chol_*", "bound": "mfma", "dtype": "f64",
                          "achieved": stage_rates["cholesky_tflops"], "peak": PEAK_FP64_MFMA / 1e12})
    # the forms are measured around the realistic workload only
    forms = [] if args.forms == "none" or args.workload != "realistic_fp64" else args.forms.split(",")
    extra = {}
    notes = {
        "mixed": "FP64 K_NM/Cholesky, FP32 Householder QR (FP64 reflector norms), FP64 refinement (corrected "
                 "semi-normal equations, then R-preconditioned CGLS) to ||dc||/||c|| <= 1e-12",
        "mixed_bf16": "as mixed, with the factored K_NM block from BF16 descriptor dot products on MFMA (FP32 "
                      "accumulation, power and sums); the FP64 K_NM is built too, for the refinement's residuals",
        "mixed_fp16": "as mixed_bf16 with FP16 descriptors",
    }
    for form, prec in (("mixed", gap.GAP_MIXED_FP32), ("bf16", gap.GAP_MIXED_BF16), ("fp16", gap.GAP_MIXED_FP16)):
        if form not in forms:
            continue
        key = "mixed" if form == "mixed" else f"mixed_{form}"
        mx = run_fit(prec, args.steps, args.warmup, y=fp["y"])
        err = float((mx["c"] - fp["c"]).norm() / fp["c"].norm())
        qr32 = f["qr_tri"] / (mx["stages_ms"]["qr"] / 1e3) / 1e12
        extra[key] = {
            "s_per_fit": mx["ms"] / 1e3, "median_ms": mx["ms_median"], "min_ms": mx["ms_min"],
            "speedup_vs_fp64": ms_per_step / mx["ms"], "stages_ms": mx["stages_ms"],
            "qr_tflops_fp32": qr32, "status": gap.status_string(mx["status"]),
            "refine_iters": mx["info"].refine_iters, "cgls_iters": mx["info"].cgls_iters,
            "last_dc_over_c": mx["info"].step_rel, "eta": mx["info"].grad_rel,
            "c_rel_err_vs_fp64_path": err, **vs_oracle(mx), "note": notes[key]}
        if form == "mixed":
            rooflines.append({"stage": "qr", "kernel": "qr_wpart32 + qr_update32 (+ panels)", "bound": "mfma",
                              "dtype": "f32", "achieved": qr32, "peak": PEAK_FP32_MFMA / 1e12})
        else:
            t_lp = mx["stages_ms"].get("knm_lp", 0.0) / 1e3
            if t_lp > 0:
                extra[key]["knm_lp_tflops"] = f["knm"] / t_lp / 1e12
                rooflines.append({"stage": "knm_lp", "kernel": "knm_lp_kernel (+ descriptor rounding)",
                                  "bound": "mfma", "dtype": form, "achieved": f["knm"] / t_lp / 1e12,
                                  "peak": PEAK_BF16_MFMA / 1e12})
        log(f"[bench] {key}: {mx['ms']:.1f} ms per fit ({gap.status_string(mx['status'])}, "
            f"{mx['info'].refine_iters} refinement steps), c rel err vs FP64 path {err:.2e}")
    if "int8" in forms:
        # the FP64 fit with its K_NM from INT8 slice products (Ozaki scheme)
        oz = run_fit(gap.GAP_FP64, args.steps, args.warmup, y=fp["y"], flags=gap.GAP_FLAG_KNM_INT8)
        t_oz = oz["stages_ms"]["knm"] / 1e3
        int8_ops = 28 * 2.0 * n_atoms * M * d  # 28 slice products of the d-term dot products
        extra["fp64_int8"] = {
            "s_per_fit": oz["ms"] / 1e3, "median_ms": oz["ms_median"], "min_ms": oz["ms_min"],
            "speedup_vs_fp64": ms_per_step / oz["ms"], "stages_ms": oz["stages_ms"],
            "knm_int8_tops": int8_ops / t_oz / 1e12, "knm_fp64_equivalent_tflops": f["knm"] / t_oz / 1e12,
            "c_rel_err_vs_fp64_path": float((oz["c"] - fp["c"]).norm() / fp["c"].norm()), **vs_oracle(oz),
            "note": "FP64 fit whose K_NM dot products come from 7 signed 8-bit slices per value, 28 slice "
                    "products on v_mfma_i32_32x32x32_i8 summed exactly in INT32 and combined in FP64"}
        rooflines.append({"stage": "knm_int8", "kernel": "knm_oz_kernel (+ slicing)", "bound": "mfma",
                          "dtype": "i8", "achieved": int8_ops / t_oz / 1e12, "peak": PEAK_INT8_MFMA / 1e12,
                          "unit": "TOP/s"})
        log(f"[bench] fp64_int8: {oz['ms']:.1f} ms per fit, K_NM {1e3 * t_oz:.1f} ms")
        del oz
        # the mixed fit (FP32 QR, FP64 refinement) on the same FP64-accurate K_NM
        mo = run_fit(gap.GAP_MIXED_FP32, args.steps, args.warmup, y=fp["y"], flags=gap.GAP_FLAG_KNM_INT8)
        extra["mixed_int8"] = {
            "s_per_fit": mo["ms"] / 1e3, "median_ms": mo["ms_median"], "min_ms": mo["ms_min"],
            "speedup_vs_fp64": ms_per_step / mo["ms"], "stages_ms": mo["stages_ms"],
            "status": gap.status_string(mo["status"]), "refine_iters": mo["info"].refine_iters,
            "cgls_iters": mo["info"].cgls_iters, "eta": mo["info"].grad_rel,
            "c_rel_err_vs_fp64_path": float((mo["c"] - fp["c"]).norm() / fp["c"].norm()), **vs_oracle(mo),
            "note": "mixed fit (FP32 Householder QR, FP64 refinement) whose FP64 K_NM comes from INT8 slice "
                    "products, as in fp64_int8"}
        log(f"[bench] mixed_int8: {mo['ms']:.1f} ms per fit ({gap.status_string(mo['status'])}, "
            f"{mo['info'].refine_iters} refinement steps)")
        del mo
    for r in rooflines:
        r.setdefault("unit", "TFLOP/s")
        r["frac"] = r["achieved"] / r["peak"]
    del fp
    torch.cuda.empty_cache()
    if "cur" in forms:
        extra["cur"] = bench_cur(args, X, n_atoms, d, M, ref is not None)
        r = extra["cur"]
        rooflines.append({"stage": "cur", "kernel": "cur_gram_kernel + cur_proj_kernel (+ selection)",
                          "bound": "mfma", "dtype": "f64", "achieved": r["tflops"], "peak": PEAK_FP64_MFMA / 1e12,
                          "unit": "TFLOP/s", "frac": r["tflops"] / (PEAK_FP64_MFMA / 1e12)})
    if "forces" in forms:
        extra["forces"] = bench_forces(args, gap, log)
        r = extra["forces"]["fp64"]
        rooflines.append({"stage": "kdm", "kernel": "kdm_kernel (+ the power block)", "bound": "mfma",
                          "dtype": "f64", "achieved": r["kdm_tflops"], "peak": PEAK_FP64_MFMA / 1e12,
                          "unit": "TFLOP/s", "frac": r["kdm_tflops"] / (PEAK_FP64_MFMA / 1e12)})
    if "sweep" in forms or "serve" in forms:
        from paper_2207_03803_amd import serve, sweep

        specs = sweep.make_sweep(seed=args.seed)
        pools = sweep.make_pools(specs, seed=args.seed, min_configs=sweep.SWEEP_RECIPE["pool_configs"])
    if "sweep" in forms:
        extra["sweep"] = bench_sweep(gap, sweep, specs, pools)
    if "serve" in forms:
        big = sweep.Pool(d, inp.offsets, X)
        extra["serve"] = bench_serve(gap, serve, sweep, pools, big, args.seed)
    traffic = knm_traffic() if args.workload == "realistic_fp64" else None
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.workload, "reported baseline, not a target")
        if ref is not None:
            m = ref["meta"]
            cpu["measured_full_fit"] = {
                "seconds": m["total_s"], "threads": m["threads"], "stages_s": {
                    k: m[k] for k in ("knm_s", "kmm_chol_s", "qr_s") if k in m},
                "host": "the build container's CPU (not this GPU host), by tests/golden/make_reference_fits.py"}
        log("[bench] timing host LAPACK / BLAS on a bounded sample")
        extra["cpu_lapack"] = lapack_baseline(args.workload)
    out = {
        "metric": "K_NM build+QR solve time at N=1e5,M=1e4 (FP64 vs mixed); fits/s + p99 latency",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "step_ms": step_stats,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_configs": N, "atoms_per_config": list(w["atoms"]),
                   "n_atoms": n_atoms, "d": d, "M": M, "zeta": zeta, "precision": "fp64",
                   "stacked_matrix": [N + M, M]},
        "fits_per_s": 1e3 / ms_per_step,
        "stages_ms": stages_ms,
        "stage_rates": stage_rates,
        "roofline": {"kernel": "knm_kernel", "bound": "mfma", "achieved": achieved / 1e12,
                     "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA,
                     "traffic": traffic},
        "roofline_stages": rooflines,
        "cpu_baseline": cpu,
    }
    if fp_oracle:
        out["parity_vs_oracle"] = dict(fp_oracle, kappa_A=float(ref["smax"] / ref["smin"]),
                                       kappa_u=float(ref["smax"] / ref["smin"]) * 2.0 ** -53)
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_sweep(gap, sweep, specs, pools, replays=2):
    """64 uneven fits: one HIP graph (mixed precision, launch shape from the tuning
    table) against the same fits one after another in plain FP64."""
    import torch

    table = sweep.load_table()
    tune = table.get(sweep.bucket(specs), dict(streams=16, grouped=False))
    total_flops = sum(s.flops() for s in specs)
    prec = gap.GAP_MIXED_FP32
    sw = sweep.Sweep(specs, pools, precision=prec, streams=tune["streams"], grouped=tune.get("grouped", False),
                     shapes=lambda s: sweep.shape_for(s, prec, table), max_refine_iters=30, refine_tol=1e-12)
    sw.capture(log=log)
    log("[bench] sweep: every fit's graph captured; first replay")
    sw.replay(1)
    log("[bench] sweep replayed once")
    t_graph = sw.replay(replays)
    st = sw.statuses()
    c_mixed = sw.weights()
    sw.close()
    del sw
    torch.cuda.empty_cache()
    log("[bench] sweep: the same fits one after another in plain FP64")
    seq = sweep.Sweep(specs, pools, precision=gap.GAP_FP64, streams=1)
    seq.run_eager()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq.run_eager()
    t_seq = time.perf_counter() - t0
    c_fp64 = seq.weights()
    st64 = seq.statuses()
    seq.close()
    del seq
    torch.cuda.empty_cache()
    import numpy as np

    errs = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(c_mixed, c_fp64)]
    log(f"[bench] sweep: graph {t_graph * 1e3:.0f} ms, sequential FP64 {t_seq * 1e3:.0f} ms")
    return {"n_fits": len(specs), "fits_per_s": len(specs) / t_graph, "s_per_sweep": t_graph,
            "fp64_sequential_fits_per_s": len(specs) / t_seq, "speedup_vs_fp64_sequential": t_seq / t_graph,
            "launch_shape": {"streams": tune["streams"], "grouped_knm": bool(tune.get("grouped", False)),
                             "per_fit_shapes": sum(1 for s in specs if sweep.shape_for(s, prec, table)),
                             "from_tuning_table": sweep.bucket(specs) in table},
            "tflops_effective": total_flops / t_graph / 1e12,
            "all_ok": all(s == gap.GAP_OK for s in st) and all(s == gap.GAP_OK for s in st64),
            "max_c_rel_err_vs_fp64": max(errs)}


def serve_sweep(args, dev):
    """Serving latency against load: a saturation run (every request at t = 0)
    gives the request throughput; then Poisson arrivals at fractions of it."""
    import torch

    from paper_2207_03803_amd import gap, serve, sweep, synth

    w = dict(synth.WORKLOADS["realistic_fp64"])
    inp = synth.make_fit_inputs_torch(seed=args.seed, device=dev, **w)
    big = sweep.Pool(w["d"], inp.offsets, inp.X)
    specs = sweep.make_sweep(seed=args.seed)
    pools = sweep.make_pools(specs, seed=args.seed, min_configs=sweep.SWEEP_RECIPE["pool_configs"])
    n = args.serve_requests
    out = {"mode": "serve-sweep", "n_requests_per_point": n, "precision": "mixed",
           "mix": "70% sweep-sized fits, 5% realistic-size fits, 25% predicts of 1..4096 configurations",
           "points": []}

    def one(rate, seed):
        reqs = serve.make_requests(n, rate=rate, seed=seed)
        srv = serve.Server(pools, slots=8, hbm_budget=96 << 30, precision=gap.GAP_MIXED_FP32,
                           predict_pool=(pools[400].offsets, pools[400].X), big_pool=big,
                           max_refine_iters=30, refine_tol=1e-12)
        for i, r in enumerate(reqs):
            srv.prepare(r)
            if (i + 1) % 250 == 0:
                log(f"[serve-sweep] {i + 1}/{n} requests prepared")
        torch.cuda.synchronize()
        log(f"[serve-sweep] {n} requests prepared (rate {rate:.3g}/s)")
        srv.run(reqs, log=log)
        torch.cuda.synchronize()
        rep = serve.latency_report(reqs)
        rep["all_fits_ok"] = all(r.meta.get("status") == gap.GAP_OK for r in reqs if r.kind == "fit")
        serve.close(srv)
        del srv, reqs
        torch.cuda.empty_cache()
        return rep

    sat = one(1e9, args.seed + 21)
    out["saturation"] = sat
    log(f"[serve-sweep] saturation: {sat['requests_per_s']:.2f} requests/s, {sat['fits_per_s']:.2f} fits/s")
    for k, f in enumerate((0.5, 0.8, 1.0, 1.2)):
        rate = f * sat["requests_per_s"]
        rep = one(rate, args.seed + 22 + k)
        rep["load"] = f
        rep["arrival_rate_per_s"] = rate
        out["points"].append(rep)
        log(f"[serve-sweep] load {f}: fit p50 {rep['fit']['p50_ms']:.0f} ms p99 {rep['fit']['p99_ms']:.0f} ms; "
            f"predict p50 {rep['predict']['p50_ms']:.0f} ms p99 {rep['predict']['p99_ms']:.0f} ms")
    print(json.dumps(out), flush=True)
    if args.serve_summary:
        with open(args.serve_summary, "w") as fh:
            fh.write(serve_sweep_md(out, args))


def serve_sweep_md(out, args):
    """Markdown summary of a serving load sweep."""
    n = out["n_requests_per_point"]
    sat = out["saturation"]
    runs = [("saturation", sat)] + [(f"load {p['load']}", p) for p in out["points"]]
    lines = [
        "# Serving latency against load (mixed-precision fits, realistic request mix)", "",
        "Command (repository root, one MI355X):", "", "```",
        f"python bench.py --serve-sweep --serve-requests {n} --serve-summary <path>", "```", "",
        f"{n} requests per point: {out['mix']}. Fit sizes as in the 64-fit sweep recipe; the realistic-size "
        "fits are N = 1e5, M = 1e4, d = 400. Latency is arrival to result on the host clock; p50/p99 by "
        "nearest rank. The saturation run releases every request at t = 0 and gives the throughput the load "
        "points are scaled from. Fits run in mixed precision (FP32 QR, FP64 refinement with the CGLS stage, at "
        "most 30 steps); a fit whose refinement still does not converge is solved again in FP64.", "",
        f"Saturation: {sat['requests_per_s']:.2f} requests/s, {sat['fits_per_s']:.2f} fits/s.", "",
        "| load | arrivals / s | fit p50 ms | fit p99 ms | predict p50 ms | predict p99 ms | fits / s "
        "| realistic fits (n, mean ms) |",
        "|---:|---:|---:|---:|---:|---:|---:|---|",
    ]
    for p in out["points"]:
        rf = p.get("realistic_fits")
        lines.append(f"| {p['load']} | {p['arrival_rate_per_s']:.2f} | {p['fit']['p50_ms']:.0f} | "
                     f"{p['fit']['p99_ms']:.0f} | {p['predict']['p50_ms']:.0f} | {p['predict']['p99_ms']:.0f} | "
                     f"{p['fits_per_s']:.2f} | {(str(rf['n']) + ', ' + format(rf['mean_ms'], '.0f')) if rf else '-'} |")
    lines += ["", "Fit outcomes per run (status counts; FP64 re-solves after a non-converged mixed refinement):", "",
              "| run | statuses | FP64 re-solves |", "|---|---|---:|"]
    for name, r in runs:
        st = ", ".join(f"{k}: {v}" for k, v in sorted(r.get("fit_status", {}).items()))
        lines.append(f"| {name} | {st} | {r.get('fp64_fallbacks', 0)} |")
    ok = all(r.get("all_fits_ok") for _, r in runs)
    lines += ["", "p99 of the fits is set by the realistic-size fits (5 % of the requests), each of which needs "
              f"the whole GPU for about 1.3 s on its own. Every fit ended GAP_OK in every run: {ok}.", ""]
    return "\n".join(lines)


def bench_serve(gap, serve, sweep, pools, big_pool, seed, n_requests=64, rate=6.0):
    """Poisson fit/predict requests through the serving loop, mixed and plain FP64."""
    import torch

    out = {"n_requests": n_requests, "arrival_rate_per_s": rate,
           "mix": "70% sweep-sized fits, 5% realistic-size fits, 25% predicts of 1..4096 configurations"}
    for name, prec in (("mixed", gap.GAP_MIXED_FP32), ("fp64", gap.GAP_FP64)):
        reqs = serve.make_requests(n_requests, rate=rate, seed=seed + 11)
        srv = serve.Server(pools, slots=8, hbm_budget=96 << 30, precision=prec,
                           predict_pool=(pools[400].offsets, pools[400].X), big_pool=big_pool,
                           max_refine_iters=30, refine_tol=1e-12)
        for r in reqs:
            srv.prepare(r)
        torch.cuda.synchronize()
        log(f"[bench] serve {name}: {n_requests} requests prepared")
        srv.run(reqs)
        torch.cuda.synchronize()
        rep = serve.latency_report(reqs)
        rep["all_fits_ok"] = all(r.meta.get("status") == gap.GAP_OK for r in reqs if r.kind == "fit")
        out[name] = rep
        log(f"[bench] serve {name}: {rep}")
        serve.close(srv)
        del srv, reqs
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
