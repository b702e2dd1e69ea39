"""Parity at the realistic workload's full size (N = 1e5 configurations of
16..64 atoms, d = 400, M = 1e4, zeta = 4), in the launch configuration the
benchmark times (the fit on a stream of its own, 32 CUs kept free of the QR
look-ahead stream).

The oracle's reference fit at this size, tests/golden/realistic_fp64_seed0.npz
(written by tests/golden/make_reference_fits.py from the oracle alone, on the
same host-drawn arrays), gives y, c, |diag R|, the minimum loss and
kappa_2(A).  The FP64 path's weights must match it within 1e-10, the mixed
forms within 1e-8 (BF16/FP16: or end in GAP_ENOCONV).  Sampled K_NM and K_MM
entries are computed by the oracle one by one, and the normal equations, the
loss identity and predict = K_NM c are checked at this size."""
import os

import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "realistic_fp64_seed0.npz")
U = 2.0 ** -53


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ref():
    z = np.load(GOLDEN, allow_pickle=False)
    return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def full(ref):
    import torch

    from paper_2207_03803_amd import gap

    w = dict(synth.WORKLOADS["realistic_fp64"])
    log(f"full size: N={w['n_configs']} M={w['M']} d={w['d']} zeta={w['zeta']}; drawing the host arrays")
    inp = synth.make_fit_inputs_blocked(seed=0, workers=16, log=log, **w)
    X = torch.from_numpy(inp.X).cuda()
    XM = torch.from_numpy(inp.XM).cuda()
    offsets = torch.from_numpy(inp.offsets).cuda()
    sigma = torch.from_numpy(inp.sigma).cuda()
    y = torch.from_numpy(ref["y"]).cuda()
    N, M = inp.n_configs, w["M"]
    log("  inputs on the device")
    out = dict(w=w, inp=inp, X=X, XM=XM, offsets=offsets, sigma=sigma, y=y, N=N, M=M)
    with torch.cuda.stream(torch.cuda.Stream()):
        h = gap.Handle(gap.params(w["d"], w["zeta"], w["sigma_w"], w["jitter"]))
        h.set_tuning(qr_free_cus=32)
        h.alloc_workspace(N, inp.n_atoms, M)
        h.build_knm(X, offsets, XM, sigma)
        Av, lay = h.A_view()
        out["A"] = Av.cpu().numpy()  # [ncols, lda] = column-major A before the QR
        log("  built; A copied to the host")
        c = torch.empty(M, dtype=torch.float64, device="cuda")
        info = h.solve(y, c)
        assert info.device_status == gap.GAP_OK
        Av, _ = h.A_view()
        out["diagR"] = np.abs(torch.diagonal(Av[:M, :M]).cpu().numpy())
    out.update(h=h, c=c.cpu().numpy(), c_dev=c, info=info)
    log("  solved in FP64")
    yield out
    h.close()


def test_fp64_weights_match_the_oracle(full, ref):
    f = full
    c, info = f["c"], f["info"]
    kappa = float(ref["smax"] / ref["smin"])
    err = rel(c, ref["c"])
    loss_err = abs(info.residual_norm2 - float(ref["loss_tail"])) / float(ref["loss_tail"])
    N, M = f["N"], f["M"]
    Knm = f["A"][:M, :N].T * f["inp"].sigma[:, None]  # K_NM from the GPU's (checked) build
    pred_err = rel(Knm @ c, Knm @ ref["c"])
    dR = np.max(np.abs(f["diagR"] - ref["diagR_abs"]) / ref["diagR_abs"])
    log(f"  FP64: c rel err {err:.2e} (kappa(A) {kappa:.3e}, kappa u {kappa * U:.1e}); prediction-space "
        f"{pred_err:.2e}; loss {loss_err:.2e}; |diag R| {dR:.2e}; eta {info.grad_rel:.1e}")
    assert err <= 1e-10
    assert pred_err <= 1e-12
    assert loss_err <= 1e-10
    assert dR <= 1e-9
    assert info.grad_rel <= 1e-13


def test_sampled_knm_entries_match_oracle(full):
    f = full
    inp, w, A = f["inp"], f["w"], f["A"]
    rng = np.random.default_rng(1)
    cfgs = np.sort(rng.choice(inp.n_configs, 48, replace=False))
    cols = np.sort(rng.choice(w["M"], 48, replace=False))
    rows = np.concatenate([np.arange(inp.offsets[a], inp.offsets[a + 1]) for a in cfgs])
    counts = np.diff(inp.offsets)[cfgs]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    K = oracle.Oracle().knm(inp.X[rows], offs, inp.XM[cols], w["zeta"], w["sigma_w"])
    expect = K / inp.sigma[cfgs][:, None]
    got = A[cols][:, cfgs].T
    err = np.max(np.abs(got - expect) / np.abs(expect))
    log(f"  sampled K_NM/sigma max rel err {err:.2e}")
    assert err <= 1e-13


def test_sampled_kmm_through_cholesky_factor(full):
    f = full
    inp, w, A = f["inp"], f["w"], f["A"]
    N, M = f["N"], f["M"]
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(M, 40, replace=False))
    U_ = A[:M, N:N + M]         # U_[col, row] layout: U_[j, i] = L^T[i, j]
    Ucols = U_[idx].T           # L^T[:, idx], M x 40
    got = Ucols.T @ Ucols       # (L L^T)[idx, idx]
    expect = oracle.Oracle().kmm(inp.XM[idx], w["zeta"], w["sigma_w"], w["jitter"])
    err = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    log(f"  sampled K_MM via L L^T rel err {err:.2e}")
    assert err <= 1e-12


def test_solution_satisfies_normal_equations(full):
    f = full
    inp, A, c = f["inp"], f["A"], f["c"]
    N, M = f["N"], f["M"]
    Amat = A[:M, :N + M].T       # (N+M) x M view, F-ordered
    b = np.zeros(N + M)
    b[:N] = f["y"].cpu().numpy() / inp.sigma
    r = b - Amat @ c
    g = Amat.T @ r
    nA = np.linalg.norm(Amat)
    eta = np.linalg.norm(g) / (nA * (nA * np.linalg.norm(c) + np.linalg.norm(b)))
    loss = float(r @ r)
    lerr = abs(loss - f["info"].residual_norm2) / loss
    log(f"  eta {eta:.2e}; loss identity rel err {lerr:.2e}")
    assert eta <= 1e-12
    assert lerr <= 1e-10


def test_predict_equals_knm_c_at_full_size(full):
    import torch

    f = full
    inp, A = f["inp"], f["A"]
    N, M = f["N"], f["M"]
    out = torch.empty(N, dtype=torch.float64, device="cuda")
    f["h"].predict(f["X"], f["offsets"], f["c_dev"], out)
    assert f["h"].sync()[0] == 0  # waits for the handle's stream
    expect = inp.sigma * (A[:M, :N].T @ f["c"])
    got = out.cpu().numpy()
    err = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    log(f"  predict vs K_NM c rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("form", ["fp32", "bf16", "fp16"])
def test_mixed_forms_match_the_oracle_at_full_size(full, ref, form):
    """FP32 QR + FP64 refinement (the factored K_NM from the FP64 build, or from
    BF16/FP16 dot products): c within 1e-8 of the oracle's, or GAP_ENOCONV for the
    low-precision factors."""
    import torch

    from paper_2207_03803_amd import gap

    f = full
    w, N, M = f["w"], f["N"], f["M"]
    prec = {"fp32": gap.GAP_MIXED_FP32, "bf16": gap.GAP_MIXED_BF16, "fp16": gap.GAP_MIXED_FP16}[form]
    iters = 30 if form == "fp32" else 200
    with torch.cuda.stream(torch.cuda.Stream()):
        h = gap.Handle(gap.params(w["d"], w["zeta"], w["sigma_w"], w["jitter"], precision=prec,
                                  max_refine_iters=iters, refine_tol=1e-12))
        h.set_tuning(qr_free_cus=32)
        h.alloc_workspace(N, f["inp"].n_atoms, M)
        h.build_knm(f["X"], f["offsets"], f["XM"], f["sigma"])
        c = torch.empty(M, dtype=torch.float64, device="cuda")
        h.solve(f["y"], c, info=False)
        s, info = h.sync()
    err = rel(c.cpu().numpy(), ref["c"])
    loss_err = abs(info.residual_norm2 - float(ref["loss_tail"])) / float(ref["loss_tail"])
    log(f"  mixed {form}: {gap.status_string(s)} after {info.refine_iters} refinement steps ({info.cgls_iters} CGLS); "
        f"c rel err vs oracle {err:.2e}; loss {loss_err:.2e}; eta {info.grad_rel:.1e}")
    h.close()
    if form == "fp32" or s == gap.GAP_OK:
        assert s == gap.GAP_OK
        assert err <= 1e-8
        assert loss_err <= 1e-8
        assert info.grad_rel <= 1e-12
    else:
        assert s == gap.GAP_ENOCONV


def test_int8_knm_fit_at_full_size(full, ref):
    """The FP64 fit with its K_NM from INT8 slice products (GAP_FLAG_KNM_INT8) at the
    realistic size: every K_NM entry of 500 sampled columns within 1e-13 of the FP64
    build's, sampled entries against the oracle, c within 1e-10 of the oracle's."""
    import torch

    from paper_2207_03803_amd import gap

    f = full
    w, N, M = f["w"], f["N"], f["M"]
    with torch.cuda.stream(torch.cuda.Stream()):
        h = gap.Handle(gap.params(w["d"], w["zeta"], w["sigma_w"], w["jitter"], flags=gap.GAP_FLAG_KNM_INT8))
        h.set_tuning(qr_free_cus=32)
        h.alloc_workspace(N, f["inp"].n_atoms, M)
        h.build_knm(f["X"], f["offsets"], f["XM"], f["sigma"])
        cols = np.sort(np.random.default_rng(3).choice(M, 500, replace=False))
        Av, _ = h.A_view()
        got = Av[torch.from_numpy(cols).cuda(), :N].cpu().numpy()
        c = torch.empty(M, dtype=torch.float64, device="cuda")
        info = h.solve(f["y"], c)
    h.close()
    fp64 = f["A"][cols, :N]
    dk = np.max(np.abs(got - fp64) / np.abs(fp64))
    inp = f["inp"]
    rng = np.random.default_rng(4)
    cfgs = np.sort(rng.choice(N, 32, replace=False))
    rows = np.concatenate([np.arange(inp.offsets[a], inp.offsets[a + 1]) for a in cfgs])
    offs = np.concatenate([[0], np.cumsum(np.diff(inp.offsets)[cfgs])]).astype(np.int64)
    K = oracle.Oracle().knm(inp.X[rows], offs, inp.XM[cols[:32]], w["zeta"], w["sigma_w"])
    ko = np.max(np.abs(got[:32][:, cfgs].T - K / inp.sigma[cfgs][:, None]) / np.abs(K / inp.sigma[cfgs][:, None]))
    err = rel(c.cpu().numpy(), ref["c"])
    log(f"  INT8 K_NM: vs FP64 build max rel diff {dk:.2e}, vs oracle {ko:.2e}; c rel err vs oracle {err:.2e}")
    assert info.device_status == gap.GAP_OK
    assert dk <= 1e-13 and ko <= 1e-13
    assert err <= 1e-10


def test_cur_selection_at_full_size(full):
    """CUR sparse-point selection over the realistic workload's 4e6 descriptor rows
    (d = 400, M = 1e4) against the oracle's (tests/golden/cur_realistic_seed0.npz):
    8192 sampled leverages within 1e-10, their sum d, and both selections (sampled
    with the stored draws, and by largest leverage) equal to the oracle's except
    where a key lies within 1e-9 of the threshold."""
    import torch

    from paper_2207_03803_amd import gap

    z = np.load(os.path.join(HERE, "golden", "cur_realistic_seed0.npz"), allow_pickle=False)
    n = f_n = full["inp"].n_atoms
    M = 10_000
    draws = torch.from_numpy(synth.cur_draws(n, 0)).cuda()
    rows = z["rows"]
    for mode, dr in (("sampled", draws), ("top", None)):
        idx, lev = gap.cur_select(full["X"], M, draws=dr, leverage=True)
        idx, lev = idx.cpu().numpy(), lev.cpu().numpy()
        err = np.max(np.abs(lev[rows] - z["lev_rows"]) / z["lev_rows"])
        diff = np.setxor1d(idx, z[f"{mode}_idx"])
        kth = z[f"{mode}_kth"][0]
        keys = (synth.cur_draws(n, 0)[diff] if dr is not None else 1.0) / lev[diff]
        log(f"  CUR {mode}: {f_n} rows: sampled leverage max rel err {err:.2e}; sum {lev.sum():.12f}; "
            f"selection differs from the oracle's in {len(diff)} rows")
        assert err <= 1e-10
        assert abs(lev.sum() - 400.0) <= 1e-9 * 400
        assert np.all(np.abs(keys - kth) <= 1e-9 * kth)
