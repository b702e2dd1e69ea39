"""Serving loop: fit and predict requests arriving over time, batched continuously.

Requests arrive by a Poisson process.  A fit request carries a training set
(descriptors already resident on the device, its sparse set, targets); a
predict request carries a batch of configurations and names a resident model
(the sparse set and weights of an earlier fit, kept on the device with an LRU
bound).  The loop admits a waiting request as soon as a slot (a HIP stream) is
free and its device footprint (`gap_workspace_bytes` for a fit, its inputs and
outputs for a predict) fits in the remaining HBM budget; in-flight requests
overlap on the device.  Completion is observed by polling each slot's event,
so the host never blocks on one request while others are in flight.  Latency
is arrival -> result on the host clock.

The library's kernels are deterministic: a request's result is bitwise the
same whether it runs alone or in the mix.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import gap


@dataclass
class Request:
    rid: int
    kind: str                 # "fit" or "predict"
    arrival: float            # seconds after the start
    spec: object = None       # fit: a FitSpec-like with d, n_configs, M, zeta, sigma_per_atom, seed
    model: int = -1           # predict: index of the fit whose model it uses (resolved at admission)
    n_configs: int = 0        # predict: batch size
    seed: int = 0
    # filled by the loop
    admitted: float = -1.0
    done: float = -1.0
    result: object = None
    footprint: int = 0
    meta: dict = field(default_factory=dict)


def make_requests(n, rate, seed=0, mix=(0.70, 0.05, 0.25), small_scale=1.0, realistic=None):
    """Poisson arrivals at `rate` per second: fractions of sweep-sized fits,
    realistic-sized fits and predict batches (1..4096 configurations)."""
    from . import sweep

    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    small = sweep.make_sweep(seed=seed + 7, n_fits=n, scale=small_scale)
    realistic = realistic or dict(d=400, n_configs=100_000, M=10_000, zeta=4, sigma_per_atom=1e-3)
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        u = rng.random()
        if u < mix[0]:
            reqs.append(Request(i, "fit", t, spec=small[i]))
        elif u < mix[0] + mix[1]:
            s = sweep.FitSpec(i, realistic["d"], realistic["n_configs"], realistic["M"], realistic["zeta"],
                              realistic["sigma_per_atom"], seed * 1000 + 500 + i)
            reqs.append(Request(i, "fit", t, spec=s))
        else:
            reqs.append(Request(i, "predict", t, n_configs=int(rng.integers(1, 4097)), seed=seed * 1000 + i))
    return reqs


class Server:
    """Continuous-batching executor over `slots` streams and an HBM budget."""

    def __init__(self, pools, slots=8, hbm_budget=96 << 30, precision=gap.GAP_FP64, resident_max=64,
                 predict_pool=None, big_pool=None, max_refine_iters=20, refine_tol=1e-12):
        import torch

        self.pools = pools
        self.big_pool = big_pool                   # descriptors of the realistic-size fits
        self.refine = dict(max_refine_iters=max_refine_iters, refine_tol=refine_tol)
        self.slots = [torch.cuda.Stream() for _ in range(slots)]
        self.free = list(range(slots))
        self.budget = hbm_budget
        self.in_use = 0
        self.precision = precision
        self.models = collections.OrderedDict()   # rid -> (XM, c, zeta, d, handle)
        self.resident_max = resident_max
        self.predict_pool = predict_pool           # (offsets, X) for d=400 predict batches
        self.inflight = []                         # (req, slot, event, keep)

    # ---------------------------------------------------------------- helpers
    def _fit_inputs(self, spec):
        import torch

        pool = self.pools.get(spec.d)
        if pool is None or len(pool.offsets) <= spec.n_configs:
            pool = self.big_pool
        if pool is None or pool.d != spec.d or len(pool.offsets) <= spec.n_configs:
            raise ValueError(f"no descriptor pool of d={spec.d} with {spec.n_configs} configurations")
        n_atoms = int(pool.offsets[spec.n_configs])
        rng = np.random.default_rng(spec.seed)
        sparse_idx = np.sort(rng.choice(n_atoms, size=spec.M, replace=False))
        counts = np.diff(pool.offsets[:spec.n_configs + 1])
        sigma = spec.sigma_per_atom * counts.astype(np.float64)
        X = pool.X[:n_atoms]
        offsets = torch.from_numpy(np.ascontiguousarray(pool.offsets[:spec.n_configs + 1])).cuda()
        XM = pool.X[torch.from_numpy(sparse_idx).cuda()].contiguous()
        return X, offsets, XM, torch.from_numpy(sigma).cuda(), rng.standard_normal(spec.M), \
            rng.standard_normal(spec.n_configs)

    def prepare(self, req):
        """Device-resident inputs of a request (before the clock starts)."""
        import torch

        if req.kind == "fit":
            X, offsets, XM, sigma, c_true, noise = self._fit_inputs(req.spec)
            p = gap.params(req.spec.d, req.spec.zeta, 1.0, 1e-8, precision=self.precision, **self.refine)
            h = gap.Handle(p)
            h.alloc_workspace(req.spec.n_configs, X.shape[0], req.spec.M)
            h.build_knm(X, offsets, XM, sigma)
            y = torch.empty(req.spec.n_configs, dtype=torch.float64, device="cuda")
            h.predict(X, offsets, torch.from_numpy(c_true).cuda(), y)
            y += sigma * torch.from_numpy(noise).cuda()
            torch.cuda.synchronize()
            h.close()
            req.meta = dict(X=X, offsets=offsets, XM=XM, sigma=sigma, y=y)
            req.footprint = gap.workspace_bytes(p, req.spec.n_configs, X.shape[0], req.spec.M)
        else:
            offs_all, Xp = self.predict_pool
            rng = np.random.default_rng(req.seed)
            n_pool = len(offs_all) - 1
            start = int(rng.integers(0, max(1, n_pool - req.n_configs)))
            n = min(req.n_configs, n_pool - start)
            a0, a1 = int(offs_all[start]), int(offs_all[start + n])
            offsets = torch.from_numpy(offs_all[start:start + n + 1] - a0).cuda()
            req.meta = dict(X=Xp[a0:a1], offsets=offsets, n=n)
            req.footprint = (a1 - a0) * Xp.shape[1] * 8 + (n + 1) * 16

    def _launch(self, req, slot):
        import torch

        st = self.slots[slot]
        m = req.meta
        with torch.cuda.stream(st):
            if req.kind == "fit":
                p = gap.params(req.spec.d, req.spec.zeta, 1.0, 1e-8, precision=self.precision, **self.refine)
                h = gap.Handle(p, stream=st)
                h.alloc_workspace(req.spec.n_configs, m["X"].shape[0], req.spec.M)
                h.build_knm(m["X"], m["offsets"], m["XM"], m["sigma"])
                c = torch.empty(req.spec.M, dtype=torch.float64, device="cuda")
                h.solve(m["y"], c, info=False)
                keep = (h, c)
            else:
                XM, c, zeta, d, mh = self.models[req.model]
                mh.set_stream(st)
                out = torch.empty(m["n"], dtype=torch.float64, device="cuda")
                mh.predict(m["X"], m["offsets"], c, out)
                keep = (None, out)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev, keep

    def _finish(self, req, keep, now):
        h, out = keep
        req.done = now
        if req.kind == "fit":
            s, info = h.sync()
            req.result = out.cpu().numpy()
            req.meta["status"] = s
            # keep the model resident (sparse set + weights) and release the fit's workspace
            mh = gap.Handle(gap.params(req.spec.d, req.spec.zeta, 1.0, 1e-8))
            mh.set_model(req.meta["XM"])
            h.close()
            h.ws = None
            self.models[req.rid] = (req.meta["XM"], out, req.spec.zeta, req.spec.d, mh)
            while len(self.models) > self.resident_max:
                _, (_, _, _, _, h_old) = self.models.popitem(last=False)
                h_old.close()
        else:
            req.result = out.cpu().numpy()

    # ---------------------------------------------------------------- the loop
    def run(self, requests, log=None):
        """Serve `requests` (sorted by arrival).  Returns the requests, filled."""
        pending = collections.deque()
        todo = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        while todo or pending or self.inflight:
            now = time.perf_counter() - t0
            while todo and todo[0].arrival <= now:
                pending.append(todo.popleft())
            # completions
            still = []
            for req, slot, ev, keep in self.inflight:
                if ev.query():
                    self._finish(req, keep, time.perf_counter() - t0)
                    self.free.append(slot)
                    self.in_use -= req.footprint
                else:
                    still.append((req, slot, ev, keep))
            self.inflight = still
            # admission: first waiting request that fits, while slots are free
            admitted = True
            while self.free and pending and admitted:
                admitted = False
                for i, req in enumerate(pending):
                    if req.kind == "predict":
                        fits400 = [k for k, v in self.models.items() if v[3] == self.predict_pool[1].shape[1]]
                        if not fits400:
                            continue
                        req.model = fits400[req.seed % len(fits400)]
                    if self.in_use + req.footprint > self.budget and self.inflight:
                        continue
                    del pending[i]
                    slot = self.free.pop()
                    self.in_use += req.footprint
                    req.admitted = time.perf_counter() - t0
                    ev, keep = self._launch(req, slot)
                    self.inflight.append((req, slot, ev, keep))
                    admitted = True
                    break
            if not todo and not self.inflight and pending:
                # only predicts are left and no model exists yet: nothing can serve them
                if all(r.kind == "predict" for r in pending) and not self.models:
                    break
            if not admitted or not self.free:
                time.sleep(0.0002)
        return requests


def latency_report(requests):
    out = {}
    for kind in ("fit", "predict"):
        lat = np.array([r.done - r.arrival for r in requests if r.kind == kind and r.done >= 0])
        if len(lat):
            out[kind] = dict(n=int(len(lat)), p50_ms=float(np.percentile(lat, 50, method="inverted_cdf") * 1e3),
                             p99_ms=float(np.percentile(lat, 99, method="inverted_cdf") * 1e3),
                             mean_ms=float(lat.mean() * 1e3))
    done = [r for r in requests if r.done >= 0]
    if done:
        span = max(r.done for r in done) - min(r.arrival for r in done)
        out["fits_per_s"] = sum(r.kind == "fit" for r in done) / span
        out["requests_per_s"] = len(done) / span
    return out
