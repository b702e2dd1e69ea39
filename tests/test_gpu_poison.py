"""Workspace poisoning (GAP_FLAG_POISON_WORKSPACE): every numeric array of the
workspace is filled with all-ones bytes (a NaN in the floating-point formats)
at the start of each build.  A build or solve that reads workspace memory it
did not write first would then give a non-finite or different result.  Every
form, both QR panel methods and the derivative rows give the unpoisoned
weights bitwise, at the oracle's weights; so do the captured sweep graphs, with
per-fit and with grouped K_NM launches."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import GpuFit, log, to_dev

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


@pytest.fixture(scope="module")
def case(orc):
    # several K_NM tiles, a ragged last tile, three QR blocks and a ragged last panel
    inp = synth.make_fit_inputs(n_configs=1500, atoms=(16, 64), d=160, M=390, seed=21, sigma_per_atom=1e-3)
    y = oracle.targets(orc, inp, 3)
    ref = orc.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 3, jitter=1e-8)
    assert ref.status == 0
    return inp, y, ref


@pytest.mark.parametrize("precision,int8,panel,tol", [
    (0, False, 0, 1e-10),   # FP64, CholeskyQR3 panels
    (0, False, 1, 1e-10),   # FP64, TSQR panels
    (1, False, 0, 1e-8),    # FP32-storage QR + FP64 refinement
    (2, False, 0, 1e-8),    # BF16 K_NM block
    (3, False, 0, 1e-8),    # FP16 K_NM block
    (0, True, 0, 1e-10),    # INT8-emulated K_NM
    (1, True, 0, 1e-8),
])
def test_poisoned_workspace_gives_the_same_fit(case, precision, int8, panel, tol):
    from paper_2207_03803_amd import gap

    inp, y, ref = case
    flags = gap.GAP_FLAG_KNM_INT8 if int8 else 0
    out = {}
    for poison in (False, True):
        g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 3, precision=precision, max_refine_iters=60,
                   flags=flags | (gap.GAP_FLAG_POISON_WORKSPACE if poison else 0))
        g.h.set_tuning(qr_panel=panel)
        runs = []
        for _ in range(2):  # the second build poisons the workspace the first one left
            g.build()
            if poison:
                # the Householder scalars are written by the solve's QR only: NaN until then
                import torch

                torch.cuda.synchronize()
                assert bool(torch.isnan(g.h.tau_view()).all())
            c, info = g.solve()
            assert info.device_status == gap.GAP_OK
            runs.append(c)
        out[poison] = runs
        g.h.close()
    err = rel(out[True][0], ref.c)
    log(f"  precision {precision}{' INT8 K_NM' if int8 else ''} panel {panel}: poisoned c rel err vs oracle "
        f"{err:.2e}")
    assert np.all(np.isfinite(out[True][0]))
    assert err <= tol
    for c in out[True] + out[False][1:]:
        assert np.array_equal(c, out[False][0])


@pytest.mark.parametrize("precision", [0, 1])
def test_poisoned_workspace_with_derivative_rows(orc, precision):
    import torch

    from paper_2207_03803_amd import gap
    from tests.test_gpu_deriv import _build, _handle

    D = synth.make_deriv_inputs(12, atoms=(16, 30), d=64, M=80, n_neigh=8, seed=6)
    y = oracle.deriv_targets(orc, D, 2)
    c_ref, _, _ = orc.fit_deriv(D, y, 2)
    cs = []
    for poison in (False, True):
        h = _handle(D, 2, precision=precision, max_refine_iters=60, refine_tol=1e-12,
                    flags=gap.GAP_FLAG_POISON_WORKSPACE if poison else 0)
        _build(h, D)
        c = torch.empty(D.XM.shape[0], dtype=torch.float64, device="cuda")
        info = h.solve(to_dev(y), c)
        assert info.device_status == gap.GAP_OK
        cs.append(c.cpu().numpy())
        h.close()
    log(f"  precision {precision}: poisoned c rel err vs oracle {rel(cs[1], c_ref):.2e}")
    assert np.all(np.isfinite(cs[1]))
    assert np.array_equal(cs[0], cs[1])


@pytest.mark.parametrize("grouped", [False, True])
def test_poisoned_workspaces_in_captured_sweep_graphs(grouped):
    from paper_2207_03803_amd import gap, sweep

    specs = sweep.make_sweep(seed=4, n_fits=6, scale=0.05)
    pools = sweep.make_pools(specs, seed=4)
    out = {}
    for poison in (False, True):
        sw = sweep.Sweep(specs, pools, precision=gap.GAP_FP64, streams=3, grouped=grouped,
                         flags=gap.GAP_FLAG_POISON_WORKSPACE if poison else 0)
        sw.capture()
        sw.replay(2)
        assert all(st == gap.GAP_OK for st in sw.statuses())
        out[poison] = sw.weights()
        sw.close()
    log(f"  {'grouped' if grouped else 'per-fit'} K_NM: {len(out[True])} fits, poisoned weights bitwise equal")
    for a, b in zip(out[True], out[False]):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
