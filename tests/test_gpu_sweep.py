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
