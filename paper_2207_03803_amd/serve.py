"""Serving loop: fit and predict requests arriving over time, batched continuously.

Requests arrive by a Poisson process.  A fit request carries a training set
(descriptors already resident on the device, its sparse set, targets); a
predict request carries a batch of configurations and names a resident model
(the sparse set and weights of an earlier fit, kept on the device with an LRU
bound).  The server owns one device arena of the HBM budget, allocated once;
a request's device memory (`gap_workspace_bytes` for a fit, weights, outputs)
is carved from it by a first-fit allocator, so serving never calls the device
allocator (whose calls can wait for work in flight).  The loop admits a
waiting request as soon as a slot (a HIP stream) is free and its footprint
fits in the arena, and hands it to that slot's host thread, which enqueues its
kernels (a large fit enqueues thousands, and an enqueue waits when the
hardware queue is full: the admission loop itself never does); in-flight
requests overlap on the device.  Completion is observed by polling each slot's event,
so the host never blocks on one request while others are in flight.  Latency
is arrival -> result on the host clock.

The library's kernels are deterministic: a request's result is bitwise the
same whether it runs alone or in the mix.
"""
from __future__ import annotations

import collections
import queue
import threading
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


class Arena:
    """First-fit allocator over one device buffer (offsets aligned to 256 bytes)."""

    ALIGN = 256

    def __init__(self, nbytes):
        import torch

        self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.size = int(nbytes)
        self.free = [(0, self.size)]   # sorted (offset, length), coalesced
        self.used = 0

    def alloc(self, nbytes):
        n = (int(nbytes) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for k, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[k]
                else:
                    self.free[k] = (off + n, ln - n)
                self.used += n
                return off, n
        return None

    def release(self, block):
        off, n = block
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def view(self, block, dtype=None, count=None):
        import torch

        off, n = block
        t = self.buf[off:off + n]
        if dtype is not None:
            t = t.view(dtype)
            if count is not None:
                t = t[:count]
        return t


class Server:
    """Continuous-batching executor over `slots` streams and an HBM budget."""

    def __init__(self, pools, slots=8, hbm_budget=96 << 30, precision=gap.GAP_FP64, resident_max=64,
                 predict_pool=None, big_pool=None, max_refine_iters=20, refine_tol=1e-12, fp64_fallback=True):
        import torch

        self.pools = pools
        self.big_pool = big_pool                   # descriptors of the realistic-size fits
        self.refine = dict(max_refine_iters=max_refine_iters, refine_tol=refine_tol)
        self.slots = [torch.cuda.Stream() for _ in range(slots)]
        self.free = list(range(slots))
        self.arena = Arena(hbm_budget)
        self.precision = precision
        # a mixed-precision fit whose refinement did not converge (kappa(A) beyond what
        # the FP32 factor can precondition) is solved again in FP64 in the same slot
        # and workspace (an FP64 workspace is smaller than a mixed one)
        self.fp64_fallback = fp64_fallback and precision != gap.GAP_FP64
        self.models = collections.OrderedDict()   # rid -> (XM, c, zeta, d, handle, c_block)
        self.resident_max = resident_max
        self.predict_pool = predict_pool           # (offsets, X) for d=400 predict batches
        self.inflight = []                         # (req, slot, event, keep, arena blocks)
        self.n_active = 0                          # admitted and not finished
        self.model_users = {}                      # model -> predicts admitted and not finished
        self.handles = {}                          # (d, zeta) -> predict-only handle
        self.handles_lock = threading.Lock()
        self.launched = queue.Queue()              # filled by the slot threads
        self.work = [queue.Queue() for _ in range(slots)]
        self.threads = [threading.Thread(target=self._slot_thread, args=(k,), daemon=True) for k in range(slots)]
        for t in self.threads:
            t.start()

    def _slot_thread(self, slot):
        while True:
            item = self.work[slot].get()
            if item is None:
                return
            req, blocks = item
            try:
                ev, keep = self._launch(req, slot, blocks)
                self.launched.put((req, slot, ev, keep, blocks, None))
            except Exception as exc:  # reported by the loop
                self.launched.put((req, slot, None, None, blocks, exc))

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
            # targets: the model's prediction with c_true (a predict-only handle) plus noise
            h = gap.Handle(gap.params(req.spec.d, req.spec.zeta, 1.0, 1e-8))
            h.set_model(XM)
            y = torch.empty(req.spec.n_configs, dtype=torch.float64, device="cuda")
            h.predict(X, offsets, torch.from_numpy(c_true).cuda(), y)
            torch.cuda.synchronize()
            h.close()
            y += sigma * torch.from_numpy(noise).cuda()
            torch.cuda.synchronize()
            req.meta = dict(X=X, offsets=offsets, XM=XM, sigma=sigma, y=y)
            req.footprint = gap.workspace_bytes(p, req.spec.n_configs, X.shape[0], req.spec.M) + 8 * req.spec.M + 512
        else:
            offs_all, Xp = self.predict_pool
            rng = np.random.default_rng(req.seed)
            n_pool = len(offs_all) - 1
            start = int(rng.integers(0, max(1, n_pool - req.n_configs)))
            n = min(req.n_configs, n_pool - start)
            a0, a1 = int(offs_all[start]), int(offs_all[start + n])
            offsets = torch.from_numpy(offs_all[start:start + n + 1] - a0).cuda()
            req.meta = dict(X=Xp[a0:a1], offsets=offsets, n=n)
            req.footprint = 8 * n

    def _launch(self, req, slot, blocks):
        import torch

        st = self.slots[slot]
        m = req.meta
        if req.kind == "fit":
            h = self._fit_handle(slot, req.spec.d, req.spec.zeta, fp64=req.meta.get("fallback", False))
            ws_block, c_block = blocks
            h.bind(self.arena.view(ws_block))
            h.build_knm(m["X"], m["offsets"], m["XM"], m["sigma"])
            c = self.arena.view(c_block, torch.float64, req.spec.M)
            h.solve(m["y"], c, info=False)
            keep = (h, c)
        else:
            XM, c, zeta, d, _, _ = self.models[req.model]
            mh = self._predict_handle(slot, d, zeta)
            mh.set_model(XM)
            mh.set_stream(st)
            out = self.arena.view(blocks[0], torch.float64, m["n"])
            mh.predict(m["X"], m["offsets"], c, out)
            keep = (None, out)
        ev = torch.cuda.Event()
        ev.record(st)
        return ev, keep

    def _fit_handle(self, slot, d, zeta, fp64=False):
        """A slot's handle for fits of (d, zeta), created once and reused (a handle
        owns HIP events and a stream: creating and destroying them per request
        would put those calls on the serving path)."""
        prec = gap.GAP_FP64 if fp64 else self.precision
        key = ("fit", slot, d, zeta, prec)
        with self.handles_lock:
            if key not in self.handles:
                p = gap.params(d, zeta, 1.0, 1e-8, precision=prec, **self.refine)
                self.handles[key] = gap.Handle(p, stream=self.slots[slot])
            return self.handles[key]

    def _predict_handle(self, slot, d, zeta):
        key = (slot, d, zeta)  # one per slot thread: set_model / set_stream are per call
        with self.handles_lock:
            if key not in self.handles:
                self.handles[key] = gap.Handle(gap.params(d, zeta, 1.0, 1e-8))
            return self.handles[key]

    def _blocks(self, req):
        """Arena blocks of a request (None when it does not fit now)."""
        if req.kind == "fit":
            p = gap.params(req.spec.d, req.spec.zeta, 1.0, 1e-8, precision=self.precision, **self.refine)
            ws = self.arena.alloc(gap.workspace_bytes(p, req.spec.n_configs, req.meta["X"].shape[0], req.spec.M))
            if ws is None:
                return None
            cb = self.arena.alloc(8 * req.spec.M)
            if cb is None:
                self.arena.release(ws)
                return None
            return (ws, cb)
        ob = self.arena.alloc(8 * req.meta["n"])
        return None if ob is None else (ob,)

    def _finish(self, req, slot, keep, blocks, now):
        """Complete a request; True when it was sent back to its slot instead."""
        h, out = keep
        if req.kind == "fit":
            s, info = h.sync()
            if s == gap.GAP_ENOCONV and self.fp64_fallback and not req.meta.get("fallback"):
                req.meta["fallback"] = True
                self.work[slot].put((req, blocks))
                return True
            req.done = now
            req.result = out.cpu().numpy()
            req.meta["status"] = s
            # release the workspace (the handle stays with its slot); the weights of a fit that
            # ended GAP_OK stay resident as a model, those of a failed fit are released
            self.arena.release(blocks[0])
            if s != gap.GAP_OK:
                self.arena.release(blocks[1])
                return False
            self.models[req.rid] = (req.meta["XM"], out, req.spec.zeta, req.spec.d, None, blocks[1])
            busy = {k for k, v in self.model_users.items() if v > 0}
            while len(self.models) > self.resident_max:
                victim = next((k for k in self.models if k not in busy), None)
                if victim is None:
                    break
                self.arena.release(self.models.pop(victim)[5])
        else:
            req.done = now
            req.result = out.cpu().numpy()
            self.arena.release(blocks[0])
            self.model_users[req.model] -= 1
        return False

    # ---------------------------------------------------------------- the loop
    def run(self, requests, log=None, log_every=100):
        """Serve `requests` (sorted by arrival).  Returns the requests, filled.
        `log(msg)`, when given, hears of every `log_every` completed requests."""
        pending = collections.deque()
        todo = collections.deque(sorted(requests, key=lambda r: r.arrival))
        n_done = 0
        t0 = time.perf_counter()
        while todo or pending or self.n_active:
            now = time.perf_counter() - t0
            while todo and todo[0].arrival <= now:
                pending.append(todo.popleft())
            # launches done by the slot threads, then completions
            while True:
                try:
                    req, slot, ev, keep, blocks, exc = self.launched.get_nowait()
                except queue.Empty:
                    break
                if exc is not None:
                    raise exc
                self.inflight.append((req, slot, ev, keep, blocks))
            still = []
            for req, slot, ev, keep, blocks in self.inflight:
                if ev.query():
                    if not self._finish(req, slot, keep, blocks, time.perf_counter() - t0):
                        self.free.append(slot)
                        self.n_active -= 1
                        n_done += 1
                        if log and n_done % log_every == 0:
                            log(f"[serve] {n_done}/{len(requests)} requests done at {time.perf_counter() - t0:.1f} s")
                else:
                    still.append((req, slot, ev, keep, blocks))
            self.inflight = still
            # admission: first waiting request whose memory fits, while slots are free
            admitted = True
            while self.free and pending and admitted:
                admitted = False
                for i, req in enumerate(pending):
                    if req.kind == "predict":
                        fits400 = [k for k, v in self.models.items() if v[3] == self.predict_pool[1].shape[1]]
                        if not fits400:
                            continue
                        req.model = fits400[req.seed % len(fits400)]
                    blocks = self._blocks(req)
                    if blocks is None:
                        if not self.n_active:
                            raise RuntimeError(f"request {req.rid} needs more than the whole arena")
                        continue
                    del pending[i]
                    slot = self.free.pop()
                    req.admitted = time.perf_counter() - t0
                    self.n_active += 1
                    if req.kind == "predict":
                        self.model_users[req.model] = self.model_users.get(req.model, 0) + 1
                    self.work[slot].put((req, blocks))
                    admitted = True
                    break
            if not todo and not self.n_active and pending:
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
            wait = np.array([r.admitted - r.arrival for r in requests if r.kind == kind and r.done >= 0])
            out[kind] = dict(n=int(len(lat)), p50_ms=float(np.percentile(lat, 50, method="inverted_cdf") * 1e3),
                             p99_ms=float(np.percentile(lat, 99, method="inverted_cdf") * 1e3),
                             mean_ms=float(lat.mean() * 1e3),
                             admission_wait_p50_ms=float(np.percentile(wait, 50, method="inverted_cdf") * 1e3))
    big = [r.done - r.arrival for r in requests if r.kind == "fit" and r.done >= 0 and r.spec.n_configs >= 50_000]
    if big:
        out["realistic_fits"] = dict(n=len(big), mean_ms=float(np.mean(big) * 1e3))
    st = collections.Counter(gap.status_string(r.meta["status"]) for r in requests
                             if r.kind == "fit" and "status" in r.meta)
    out["fit_status"] = dict(st)
    out["fp64_fallbacks"] = sum(1 for r in requests if r.kind == "fit" and r.meta.get("fallback"))
    bad = [r for r in requests if r.kind == "fit" and r.meta.get("status", 0) != gap.GAP_OK]
    if bad:
        out["failed_fits"] = [dict(rid=r.rid, n_configs=r.spec.n_configs, M=r.spec.M, d=r.spec.d, zeta=r.spec.zeta,
                                   sigma_per_atom=r.spec.sigma_per_atom, status=gap.status_string(r.meta["status"]))
                              for r in bad[:8]]
    done = [r for r in requests if r.done >= 0]
    if done:
        span = max(r.done for r in done) - min(r.arrival for r in done)
        out["fits_per_s"] = sum(r.kind == "fit" for r in done) / span
        out["requests_per_s"] = len(done) / span
    return out


def close(server):
    for q in server.work:
        q.put(None)
    for t in server.threads:
        t.join()
    for h in server.handles.values():
        h.close()
    server.handles.clear()
