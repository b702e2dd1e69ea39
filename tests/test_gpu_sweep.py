"""Batched sweep: many uneven fits captured in one HIP graph.  Each fit's
weights match the oracle, are bitwise the same as the fit run alone, and stay
the same over repeated replays with eager work in between."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def small_sweep():
    from paper_2207_03803_amd import gap, sweep

    specs = sweep.make_sweep(seed=3, n_fits=8, scale=0.05)
    pools = sweep.make_pools(specs, seed=3)
    sw = sweep.Sweep(specs, pools, precision=gap.GAP_MIXED_FP32, streams=4, max_refine_iters=30,
                     refine_tol=1e-14)
    sw.capture()
    sw.replay(1)
    yield sw
    sw.close()


def test_sweep_fits_match_oracle(small_sweep):
    from paper_2207_03803_amd import gap

    sw = small_sweep
    assert all(s == gap.GAP_OK for s in sw.statuses())
    orc = oracle.Oracle()
    for f, c in zip(sw.fits, sw.weights()):
        s = f.spec
        X = f.X.cpu().numpy()
        offs = f.offsets.cpu().numpy()
        XM = f.XM.cpu().numpy()
        y = f.y.cpu().numpy()
        ref = orc.fit(X, offs, XM, f.host["sigma"], y, s.zeta, jitter=1e-8)
        assert ref.status == 0
        err = rel(c, ref.c)
        log(f"  fit {s.idx}: N={s.n_configs} M={s.M} d={s.d} zeta={s.zeta} sigma_E={s.sigma_per_atom:g}: "
            f"c rel err {err:.2e}")
        assert err <= 1e-8


def test_sweep_is_batch_invariant_and_replays_identically(small_sweep):
    import torch

    sw = small_sweep
    in_graph = sw.weights()
    # eager work between replays, then replay again
    junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    junk.mul_(2.0).sum().item()
    sw.replay(2)
    again = sw.weights()
    for a, b in zip(in_graph, again):
        assert np.array_equal(a, b)
    # each fit alone, eagerly, on the default stream
    for f, c_graph in zip(sw.fits, in_graph):
        f.handle.build_knm(f.X, f.offsets, f.XM, f.sigma)
        c = torch.empty_like(f.c)
        f.handle.solve(f.y, c)
        assert np.array_equal(c.cpu().numpy(), c_graph), f.spec


def test_full_recipe_sweep_fits_match_oracle():
    """Three fits of the benchmark's 64-fit sweep at full recipe size (the largest M,
    the one with M > N_c, the smallest N_c at sigma_E = 1e-4 per atom) over host-drawn
    pools, captured as graphs with the tuning table's launch shape and replayed on
    their streams, against the oracle's reference fits
    (tests/golden/sweep_fits_seed0.npz): c within 1e-8, or within the FP64
    perturbation bound u (kappa + kappa^2 ||r|| / (||A|| ||c||)) of an
    ill-conditioned fit; the same fits in plain FP64, eagerly, within 1e-10 or that
    bound."""
    import json
    import os

    import torch

    from paper_2207_03803_amd import gap, sweep

    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sweep_fits_seed0.npz"),
                allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    specs = sweep.make_sweep(seed=0)
    pinned = [specs[m["idx"]] for m in meta["fits"]]
    log("full-recipe sweep fits: " + ", ".join(f"{s.idx} (N={s.n_configs} M={s.M} d={s.d})" for s in pinned))
    pools = sweep.make_pools(pinned, seed=0, min_configs=meta["pool_configs"], host=True)
    pools = {d: sweep.Pool(d, p.offsets, torch.from_numpy(p.X).cuda()) for d, p in pools.items()}
    targets = {s.idx: z[f"fit{s.idx}_y"] for s in pinned}
    table = sweep.load_table()
    tune = table.get(sweep.bucket(specs), dict(streams=16, grouped=False))
    u = 2.0 ** -53

    def bound(idx, floor):
        smax, smin = float(z[f"fit{idx}_smax"]), float(z[f"fit{idx}_smin"])
        kappa = smax / smin
        c = z[f"fit{idx}_c"]
        rn = np.sqrt(float(z[f"fit{idx}_loss_tail"]))
        return max(floor, 32 * u * (kappa + kappa ** 2 * rn / (smax * np.linalg.norm(c)))), kappa

    prec = gap.GAP_MIXED_FP32
    sw = sweep.Sweep(pinned, pools, precision=prec, streams=tune["streams"], grouped=tune.get("grouped", False),
                     shapes=lambda s: sweep.shape_for(s, prec, table), max_refine_iters=60, refine_tol=1e-12,
                     targets=targets)
    sw.capture()
    sw.replay(1)
    st = sw.statuses()
    for f, c, s in zip(sw.fits, sw.weights(), st):
        idx = f.spec.idx
        b, kappa = bound(idx, 1e-8)
        err = rel(c, z[f"fit{idx}_c"])
        log(f"  graph, mixed: fit {idx} shape {f.shape}: kappa(A) {kappa:.2e}; {gap.status_string(s)}; "
            f"c rel err {err:.2e} (allowed {b:.1e})")
        assert s == gap.GAP_OK
        assert err <= b
    sw.close()
    seq = sweep.Sweep(pinned, pools, precision=gap.GAP_FP64, streams=1, targets=targets)
    seq.run_eager()
    for f, c, s in zip(seq.fits, seq.weights(), seq.statuses()):
        idx = f.spec.idx
        b, kappa = bound(idx, 1e-10)
        err = rel(c, z[f"fit{idx}_c"])
        log(f"  eager, FP64: fit {idx}: c rel err {err:.2e} (allowed {b:.1e})")
        assert s == gap.GAP_OK
        assert err <= b
    seq.close()


def test_grouped_knm_and_tile_shapes_leave_results_bitwise_unchanged():
    """The K_NM of every fit in grouped launches (gap_build_knm_batch + gap_build_kmm)
    against one gap_build_knm per fit, and the K_NM column tile of 32 against 64:
    every fit's stacked matrix and weights are the same bit for bit; the batch
    also matches the oracle."""
    import torch

    from paper_2207_03803_amd import gap, sweep

    specs = sweep.make_sweep(seed=4, n_fits=10, scale=0.05)
    pools = sweep.make_pools(specs, seed=4)
    runs = {}
    for name, grouped, bn in (("per-fit", False, 64), ("grouped", True, 64), ("grouped bn32", True, 32)):
        sw = sweep.Sweep(specs, pools, precision=gap.GAP_FP64, streams=4, grouped=grouped,
                         shapes=lambda s, bn=bn: dict(knm_bn=bn))
        sw.capture()
        sw.replay(2)
        assert all(st == gap.GAP_OK for st in sw.statuses())
        runs[name] = sw.weights()
        # the stacked matrix of the first fit, from an eager rebuild in this mode
        f = sw.fits[0]
        if grouped:
            gap.build_knm_batch([f.handle], [(f.X, f.offsets, f.XM, f.sigma)])
            torch.cuda.synchronize()
            f.handle.build_kmm()
        else:
            f.handle.build_knm(f.X, f.offsets, f.XM, f.sigma)
        torch.cuda.synchronize()  # the rebuild ran on the fit's stream
        Av, lay = f.handle.A_view()  # [column, row]; rows past N + M are padding
        runs[name + " A"] = Av[:lay.M, :lay.N + lay.M].cpu().numpy()
        sw.close()
    for name in ("grouped", "grouped bn32"):
        a, b = runs[name + " A"], runs["per-fit A"]
        diff = np.argwhere(a != b)
        assert len(diff) == 0, (name, diff[:5], a.shape)
        for a, b in zip(runs[name], runs["per-fit"]):
            assert np.array_equal(a, b), name
    orc = oracle.Oracle()
    sw = sweep.Sweep(specs[:3], pools, precision=gap.GAP_FP64, streams=2, grouped=True)
    sw.run_eager()
    for f, c in zip(sw.fits, sw.weights()):
        ref = orc.fit(f.X.cpu().numpy(), f.offsets.cpu().numpy(), f.XM.cpu().numpy(), f.host["sigma"],
                      f.y.cpu().numpy(), f.spec.zeta, jitter=1e-8)
        err = rel(c, ref.c)
        log(f"  grouped build, fit {f.spec.idx}: c rel err vs oracle {err:.2e}")
        assert err <= 1e-10
    sw.close()
