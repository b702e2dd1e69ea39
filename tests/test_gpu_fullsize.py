"""Parity at the realistic workload's full size (N = 1e5 configurations of
16..64 atoms, d = 400, M = 1e4, zeta = 4), in the launch configuration the
benchmark times.  The oracle cannot run the whole fit at this size, so it
checks sampled outputs one by one (K_NM entries, K_MM entries through the
Cholesky factor) and the solution is checked through properties that hold at
any size: the normal equations (zero loss gradient), the loss identity and
predict = K_NM c."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_fit():
    import torch

    from paper_2207_03803_amd import gap

    w = dict(synth.WORKLOADS["realistic_fp64"])
    log(f"full size: N={w['n_configs']} M={w['M']} d={w['d']} zeta={w['zeta']}")
    inp = synth.make_fit_inputs_torch(seed=0, device="cuda", **w)
    offsets = torch.from_numpy(inp.offsets).cuda()
    sigma = torch.from_numpy(inp.sigma).cuda()
    h = gap.Handle(gap.params(w["d"], w["zeta"], w["sigma_w"], w["jitter"]))
    h.alloc_workspace(inp.n_configs, inp.n_atoms, w["M"])
    h.build_knm(inp.X, offsets, inp.XM, sigma)
    y = torch.empty(inp.n_configs, dtype=torch.float64, device="cuda")
    h.predict(inp.X, offsets, torch.from_numpy(inp.c_true).cuda(), y)
    y += sigma * torch.from_numpy(inp.noise).cuda()
    h.build_knm(inp.X, offsets, inp.XM, sigma)
    Av, lay = h.A_view()
    A_host = Av.cpu().numpy()  # [ncols, lda] = column-major A before the QR
    log("  built; A copied to the host")
    c = torch.empty(w["M"], dtype=torch.float64, device="cuda")
    info = h.solve(y, c)
    assert info.device_status == 0
    log("  solved")
    yield dict(w=w, inp=inp, h=h, A=A_host, lay=lay, y=y.cpu().numpy(), c=c.cpu().numpy(), info=info,
               offsets=offsets, c_dev=c)
    h.close()


def test_sampled_knm_entries_match_oracle(full_fit):
    f = full_fit
    inp, w, A = f["inp"], f["w"], f["A"]
    rng = np.random.default_rng(1)
    cfgs = np.sort(rng.choice(inp.n_configs, 48, replace=False))
    cols = np.sort(rng.choice(w["M"], 48, replace=False))
    X = inp.X
    rows = np.concatenate([np.arange(inp.offsets[a], inp.offsets[a + 1]) for a in cfgs])
    import torch

    Xs = X[torch.from_numpy(rows).cuda()].cpu().numpy()
    counts = np.diff(inp.offsets)[cfgs]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    XMs = inp.XM[torch.from_numpy(cols).cuda()].cpu().numpy()
    K = oracle.Oracle().knm(Xs, offs, XMs, w["zeta"], w["sigma_w"])
    expect = K / inp.sigma[cfgs][:, None]
    got = A[cols][:, cfgs].T
    err = np.max(np.abs(got - expect) / np.abs(expect))
    log(f"  sampled K_NM/sigma max rel err {err:.2e}")
    assert err <= 1e-13


def test_sampled_kmm_through_cholesky_factor(full_fit):
    f = full_fit
    inp, w, A = f["inp"], f["w"], f["A"]
    N, M = inp.n_configs, w["M"]
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(M, 40, replace=False))
    U = A[:M, N:N + M]          # U[col, row] layout: U_T[j, i] = L^T[i, j]
    Ucols = U[idx].T            # L^T[:, idx], M x 40
    got = Ucols.T @ Ucols       # (L L^T)[idx, idx]
    import torch

    XMs = inp.XM[torch.from_numpy(idx).cuda()].cpu().numpy()
    expect = oracle.Oracle().kmm(XMs, w["zeta"], w["sigma_w"], w["jitter"])
    err = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    log(f"  sampled K_MM via L L^T rel err {err:.2e}")
    assert err <= 1e-12


def test_solution_satisfies_normal_equations(full_fit):
    f = full_fit
    inp, w, A, c = f["inp"], f["w"], f["A"], f["c"]
    N, M = inp.n_configs, w["M"]
    Amat = A[:M, :N + M].T       # (N+M) x M view, F-ordered
    b = np.zeros(N + M)
    b[:N] = f["y"] / inp.sigma
    r = b - Amat @ c
    g = Amat.T @ r
    nA = np.linalg.norm(Amat)
    eta = np.linalg.norm(g) / (nA * (nA * np.linalg.norm(c) + np.linalg.norm(b)))
    loss = float(r @ r)
    lerr = abs(loss - f["info"].residual_norm2) / loss
    log(f"  eta {eta:.2e}; loss identity rel err {lerr:.2e}")
    assert eta <= 1e-12
    assert lerr <= 1e-8


def test_predict_equals_knm_c_at_full_size(full_fit):
    import torch

    f = full_fit
    inp, w, A = f["inp"], f["w"], f["A"]
    N, M = inp.n_configs, w["M"]
    out = torch.empty(N, dtype=torch.float64, device="cuda")
    f["h"].predict(inp.X, f["offsets"], f["c_dev"], out)
    expect = inp.sigma * (A[:M, :N].T @ f["c"])
    got = out.cpu().numpy()
    err = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    log(f"  predict vs K_NM c rel err {err:.2e}")
    assert err <= 1e-12


def test_mixed_precision_at_full_size(full_fit):
    """FP32 QR + FP64 refinement at full size: the refined c satisfies the FP64
    normal equations as tightly as the FP64 path, and matches its loss."""
    import torch

    from paper_2207_03803_amd import gap

    f = full_fit
    inp, w, A = f["inp"], f["w"], f["A"]
    N, M = inp.n_configs, w["M"]
    h = gap.Handle(gap.params(w["d"], w["zeta"], w["sigma_w"], w["jitter"], precision=gap.GAP_MIXED_FP32,
                              max_refine_iters=30, refine_tol=1e-12))
    h.alloc_workspace(N, inp.n_atoms, M)
    sigma = torch.from_numpy(inp.sigma).cuda()  # read again by gap_solve: keep it alive
    h.build_knm(inp.X, f["offsets"], inp.XM, sigma)
    c = torch.empty(M, dtype=torch.float64, device="cuda")
    y = torch.from_numpy(f["y"]).cuda()
    info = h.solve(y, c)
    assert info.device_status == gap.GAP_OK
    cm = c.cpu().numpy()
    Amat = A[:M, :N + M].T
    b = np.zeros(N + M)
    b[:N] = f["y"] / inp.sigma
    r = b - Amat @ cm
    nA = np.linalg.norm(Amat)
    eta = np.linalg.norm(Amat.T @ r) / (nA * (nA * np.linalg.norm(cm) + np.linalg.norm(b)))
    loss = float(r @ r)
    log(f"  mixed: {info.refine_iters} refinement steps (last |dc|/|c| {info.step_rel:.1e}, eta {info.grad_rel:.1e}), eta {eta:.2e}, "
        f"loss rel diff vs FP64 path {abs(loss - f['info'].residual_norm2) / loss:.2e}")
    assert eta <= 1e-12
    assert abs(loss - f["info"].residual_norm2) <= 1e-8 * loss
    h.close()
