"""Batched hyperparameter sweep: many independent GAP fits replayed as HIP graphs.

A sweep is a list of fits of different sizes and hyperparameters over shared
descriptor pools (one pool per descriptor length d; a fit with N_c
configurations takes the pool's first N_c, and draws its own sparse set from
their atoms).  The fits are spread over S streams by longest-processing-time
order on their flop counts.  Each fit's `gap_build_knm` + `gap_solve` is
captured once into its own graph (about a thousand kernel nodes for the
largest fits of the recipe), and a sweep replays every fit's graph on its
stream, so the fits of different streams overlap on the device.  Each fit
keeps its own handle and workspace; the library's kernels are deterministic,
so a fit's weights are bitwise the same alone, in a replay, or on any stream.

The autotuner times whole-sweep replays over a small grid of launch shapes
(stream count, split-K workgroup target of the QR, QR look-ahead) and keeps a
table keyed by the sweep's shape bucket.  Run it as a program of its own
(`python -m paper_2207_03803_amd.sweep`); it sets 16 hardware queues, like
the benchmark.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import gap

TUNING_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

# The sweep recipe: N_c ~ U[2000, 30000] configurations of U[8, 64] atoms,
# d in {128, 256, 400}, M ~ U[500, 4000], zeta in {2, 3, 4}, sigma_E in
# {1e-4, 1e-3, 1e-2} per atom; pools of 30000 configurations per d.
SWEEP_RECIPE = dict(n_fits=64, n_configs=(2000, 30000), atoms=(8, 64), ds=(128, 256, 400),
                    M=(500, 4000), zetas=(2, 3, 4), sigmas=(1e-4, 1e-3, 1e-2), pool_configs=30000)


@dataclass
class FitSpec:
    idx: int
    d: int
    n_configs: int
    M: int
    zeta: int
    sigma_per_atom: float
    seed: int

    def flops(self, atoms_mean=36.0):
        n_atoms = self.n_configs * atoms_mean
        m, n = self.n_configs + self.M, self.M
        return 2 * n_atoms * self.M * self.d + 2 * m * n * n


def make_sweep(seed=0, n_fits=None, scale=1.0, recipe=SWEEP_RECIPE):
    """Draw the sweep's fit specifications (sizes scaled by `scale` for tests)."""
    rng = np.random.default_rng(seed)
    n_fits = n_fits or recipe["n_fits"]
    lo_n, hi_n = recipe["n_configs"]
    lo_m, hi_m = recipe["M"]
    specs = []
    for i in range(n_fits):
        N = int(rng.integers(lo_n, hi_n + 1) * scale)
        M = int(rng.integers(lo_m, hi_m + 1) * scale)
        specs.append(FitSpec(i, int(rng.choice(recipe["ds"])), max(N, 8), max(M, 8), int(rng.choice(recipe["zetas"])),
                             float(rng.choice(recipe["sigmas"])), int(seed * 1000 + i)))
    return specs


@dataclass
class Pool:
    d: int
    offsets: np.ndarray     # int64 [n_configs + 1]
    X: object               # torch [n_atoms, d] float64 (cuda)


def make_pools(specs, seed=0, atoms=(8, 64), device="cuda", min_configs=0, host=False, log=None):
    """One descriptor pool per d, as large as the largest fit that uses it (and at
    least `min_configs` configurations).  host=False draws the descriptors on
    the device (torch Philox); host=True draws them on the host
    (synth.make_fit_inputs_blocked, numpy arrays), so that a CPU program can
    draw the same pool."""
    from . import synth

    pools = {}
    for d in sorted({s.d for s in specs}):
        n = max(max(s.n_configs for s in specs if s.d == d), min_configs)
        if host:
            inp = synth.make_fit_inputs_blocked(n_configs=n, atoms=atoms, d=d, M=1, seed=seed + d, log=log)
        else:
            inp = synth.make_fit_inputs_torch(n_configs=n, atoms=atoms, d=d, M=1, seed=seed + d, device=device)
        pools[d] = Pool(d, inp.offsets, inp.X)
    return pools


def draw_fit(spec, pool_offsets):
    """A fit's own draws over its pool (numpy, seeded by the fit): sparse rows
    (uniform without replacement over the fit's atoms), c_true, noise, and
    sigma_A = sigma_per_atom * N_A.  Returns a dict of numpy arrays."""
    n_atoms = int(pool_offsets[spec.n_configs])
    rng = np.random.default_rng(spec.seed)
    sparse_idx = np.sort(rng.choice(n_atoms, size=spec.M, replace=False))
    counts = np.diff(pool_offsets[:spec.n_configs + 1])
    sigma = spec.sigma_per_atom * counts.astype(np.float64)
    return dict(c_true=rng.standard_normal(spec.M), noise=rng.standard_normal(spec.n_configs),
                sparse_idx=sparse_idx, sigma=sigma, n_atoms=n_atoms)


@dataclass
class Fit:
    spec: FitSpec
    handle: object = None
    ws: object = None
    offsets: object = None
    XM: object = None
    sigma: object = None
    y: object = None
    c: object = None
    X: object = None
    host: dict = field(default_factory=dict)


class Sweep:
    """The fits of one sweep with their inputs resident on the device."""

    def __init__(self, specs, pools, precision=gap.GAP_MIXED_FP32, streams=8, split_wgs=0, lookahead=0,
                 max_refine_iters=20, refine_tol=1e-12, targets=None):
        import torch

        self.specs = specs
        self.pools = pools
        self.precision = precision
        self.n_streams = streams
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.root = torch.cuda.Stream()
        self.fits = []
        # positions in `specs` (and in self.fits), stream by stream
        order = sorted(range(len(specs)), key=lambda i: -specs[i].flops())
        loads = [0.0] * streams
        self.assign = [[] for _ in range(streams)]
        for i in order:  # longest processing time first, onto the least-loaded stream
            k = int(np.argmin(loads))
            loads[k] += specs[i].flops()
            self.assign[k].append(i)
        stream_of = {i: k for k, lst in enumerate(self.assign) for i in lst}
        for pos, s in enumerate(specs):
            pool = pools[s.d]
            dr = draw_fit(s, pool.offsets)
            n_atoms = dr["n_atoms"]
            f = Fit(s)
            f.X = pool.X[:n_atoms]
            f.offsets = torch.from_numpy(np.ascontiguousarray(pool.offsets[:s.n_configs + 1])).cuda()
            f.XM = pool.X[torch.from_numpy(dr["sparse_idx"]).cuda()].contiguous()
            f.sigma = torch.from_numpy(dr["sigma"]).cuda()
            f.host = dict(c_true=dr["c_true"], noise=dr["noise"], sparse_idx=dr["sparse_idx"], sigma=dr["sigma"])
            p = gap.params(s.d, s.zeta, 1.0, 1e-8, precision=precision, max_refine_iters=max_refine_iters,
                           refine_tol=refine_tol)
            f.handle = gap.Handle(p, stream=self.streams[stream_of[pos]])
            if split_wgs or lookahead:
                f.handle.set_tuning(qr_split_wgs=split_wgs, qr_lookahead=lookahead)
            f.ws = f.handle.alloc_workspace(s.n_configs, n_atoms, s.M)
            f.c = torch.empty(s.M, dtype=torch.float64, device="cuda")
            self.fits.append(f)
        self._targets(targets or {})
        self.graphs = None

    def _targets(self, given):
        """y = prediction with c_true plus sigma * noise, through the library;
        given[idx] (host array) is used instead where present."""
        import torch

        for f in self.fits:
            if f.spec.idx in given:
                f.y = torch.from_numpy(np.ascontiguousarray(given[f.spec.idx], dtype=np.float64)).cuda()
                continue
            with torch.cuda.stream(f.handle.stream):
                f.handle.build_knm(f.X, f.offsets, f.XM, f.sigma)
                y = torch.empty(f.spec.n_configs, dtype=torch.float64, device="cuda")
                f.handle.predict(f.X, f.offsets, torch.from_numpy(f.host["c_true"]).cuda(), y)
                y += f.sigma * torch.from_numpy(f.host["noise"]).cuda()
                f.y = y
        torch.cuda.synchronize()

    def enqueue(self):
        """Every fit's build + solve on its stream (no host synchronisation)."""
        for k, lst in enumerate(self.assign):
            for i in lst:
                f = self.fits[i]
                f.handle.build_knm(f.X, f.offsets, f.XM, f.sigma)
                f.handle.solve(f.y, f.c, info=False)

    def run_eager(self):
        import torch

        torch.cuda.synchronize()
        for st in self.streams:
            st.wait_stream(torch.cuda.current_stream())
        self.enqueue()
        for st in self.streams:
            torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()

    def capture(self, log=None):
        """Capture each fit's build + solve into a graph of its own, on its stream."""
        import torch

        torch.cuda.synchronize()
        self.graphs = [None] * len(self.fits)
        for k, lst in enumerate(self.assign):
            st = self.streams[k]
            for i in lst:
                f = self.fits[i]
                if log:
                    log(f"[sweep] capturing fit {i} (N={f.spec.n_configs} M={f.spec.M} d={f.spec.d}) on stream {k}")
                g = torch.cuda.CUDAGraph()
                with torch.cuda.stream(st):
                    g.capture_begin()
                    f.handle.build_knm(f.X, f.offsets, f.XM, f.sigma)
                    f.handle.solve(f.y, f.c, info=False)
                    g.capture_end()
                self.graphs[i] = g
        torch.cuda.synchronize()
        return self.graphs

    def replay(self, n=1):
        """Replay the whole sweep n times; returns seconds per sweep."""
        import torch

        torch.cuda.synchronize()
        cur = torch.cuda.current_stream()
        t0 = time.perf_counter()
        for _ in range(n):
            for st in self.streams:
                st.wait_stream(cur)
            for k, lst in enumerate(self.assign):
                with torch.cuda.stream(self.streams[k]):
                    for i in lst:
                        self.graphs[i].replay()
            for st in self.streams:
                cur.wait_stream(st)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    def statuses(self):
        return [f.handle.sync()[0] for f in self.fits]

    def weights(self):
        return [f.c.cpu().numpy() for f in self.fits]

    def close(self):
        for f in self.fits:
            f.handle.close()


def bucket(specs):
    """Shape bucket of a sweep for the tuning table."""
    n = len(specs)
    mm = int(np.median([s.M for s in specs]))
    nn = int(np.median([s.n_configs for s in specs]))
    return f"fits{n}_M{1 << max(0, mm.bit_length() - 1)}_N{1 << max(0, nn.bit_length() - 1)}"


def load_table(path=TUNING_TABLE):
    if os.path.exists(path):
        return json.load(open(path))
    return {}


def autotune(specs, pools, precision=gap.GAP_MIXED_FP32, candidates=None, replays=1, path=TUNING_TABLE,
             log=print):
    """Time whole-sweep graph replays for each candidate launch shape and keep the best.

    Returns (best, results); stores {bucket: best} in the table at `path`.
    """
    candidates = candidates or [dict(streams=s, split_wgs=w, lookahead=la) for s in (8, 16) for w in (1024, 2048)
                                for la in (0, 1)]
    results = []
    for cand in candidates:
        log(f"[autotune] building {cand}")
        sw = Sweep(specs, pools, precision=precision, streams=cand["streams"], split_wgs=cand["split_wgs"],
                   lookahead=cand.get("lookahead", 0))
        sw.capture()
        log(f"[autotune] captured {len(specs)} fit graphs; first replay")
        sw.replay(1)
        t = sw.replay(replays)
        results.append(dict(cand, seconds=t))
        log(f"[autotune] {cand} -> {t * 1e3:.1f} ms per sweep")
        sw.close()
        del sw
    best = min(results, key=lambda r: r["seconds"])
    table = load_table(path)
    table[bucket(specs)] = dict(streams=best["streams"], split_wgs=best["split_wgs"],
                                lookahead=best.get("lookahead", 0), seconds=best["seconds"],
                                precision=int(precision))
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    return best, results


def main():
    import argparse

    os.environ["GPU_MAX_HW_QUEUES"] = "16"  # before HIP starts: as many queues as streams

    ap = argparse.ArgumentParser(description="Autotune the sweep's launch shape and store it in the tuning table.")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n-fits", type=int, default=SWEEP_RECIPE["n_fits"])
    ap.add_argument("--replays", type=int, default=1)
    args = ap.parse_args()
    specs = make_sweep(seed=args.seed, n_fits=args.n_fits)
    pools = make_pools(specs, seed=args.seed, min_configs=SWEEP_RECIPE["pool_configs"])
    best, results = autotune(specs, pools, replays=args.replays, log=lambda m: print(m, flush=True))
    print(json.dumps(dict(bucket=bucket(specs), best=best, results=results)), flush=True)


if __name__ == "__main__":
    main()
