"""Derivative observations (forces, virials) on the GPU (gap_build_knm_obs)
against the oracle: the derivative rows of the stacked matrix elementwise, the
energy and L^T rows bitwise equal to an energy-only build, the weights of FP64
and mixed fits on [energies; forces; virials; L^T], out-of-range gradient
indices reported without a read outside the arrays, and the low-precision
forms rejected."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import log, to_dev

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _obs(D, pos_grad=None):
    return dict(x_grad=to_dev(D.x_grad), grad_atom=to_dev(D.grad_atom), obs_offsets=to_dev(D.obs_offsets),
                pos_grad=to_dev(D.pos_grad if pos_grad is None else pos_grad), pos_weight=to_dev(D.pos_weight))


def _handle(D, zeta, precision=0, sigma_w=1.0, flags=0, **kw):
    from paper_2207_03803_amd import gap

    h = gap.Handle(gap.params(D.X.shape[1], zeta, sigma_w, 1e-8, precision=precision, flags=flags, **kw))
    h.alloc_workspace_obs(D.n_configs, D.n_atoms, D.n_obs, len(D.pos_grad), D.XM.shape[0])
    return h


def _build(h, D, pos_grad=None):
    inputs = dict(X=to_dev(D.X), offsets=to_dev(D.offsets), XM=to_dev(D.XM), sigma=to_dev(D.sigma))
    h.build_knm_obs(inputs["X"], inputs["offsets"], _obs(D, pos_grad), inputs["XM"], inputs["sigma"])
    return inputs


def _rows(h, D):
    import torch

    torch.cuda.synchronize()
    Av, lay = h.A_view()
    return Av[:lay.M, :lay.N + lay.M].T.cpu().numpy()  # [N + M, M]


@pytest.mark.parametrize("n_configs,atoms,d,M,n_neigh,zeta,sigma_w,seed", [
    (12, (16, 30), 64, 80, 8, 1, 1.0, 5),
    (12, (16, 30), 64, 80, 8, 2, 0.8, 6),
    (40, (20, 60), 400, 300, 12, 4, 1.0, 7),   # realistic d and zeta; virial rows over 256 positions
])
def test_derivative_rows_match_oracle(orc, n_configs, atoms, d, M, n_neigh, zeta, sigma_w, seed):
    from paper_2207_03803_amd import gap

    D = synth.make_deriv_inputs(n_configs, atoms=atoms, d=d, M=M, n_neigh=n_neigh, seed=seed)
    log(f"derivative rows: {D.n_configs} configs, {D.n_atoms} atoms, {D.n_obs} observations over "
        f"{len(D.pos_grad)} positions, d={d} M={M} zeta={zeta}")
    h = _handle(D, zeta, sigma_w=sigma_w)
    _build(h, D)
    rows = _rows(h, D)
    assert h.sync()[0] == gap.GAP_OK
    NE, NO = D.n_configs, D.n_obs
    Kd = orc.kdm(D.X, D.x_grad, D.grad_atom, D.obs_offsets, D.pos_grad, D.pos_weight, D.XM, zeta, sigma_w)
    # the sum of absolute terms: |x_i . x_j| <= |x_i| . |x_j| and |x' . x_j| <= |x'| . |x_j|
    scale = orc.kdm(np.abs(D.X), np.abs(D.x_grad), D.grad_atom, D.obs_offsets, D.pos_grad, np.abs(D.pos_weight),
                    np.abs(D.XM), zeta, sigma_w)
    got = rows[NE:NE + NO] * D.sigma_D[:, None]
    err = np.max(np.abs(got - Kd) / scale)
    log(f"  derivative rows: max |error| / sum of |terms| {err:.2e}")
    assert err <= 1e-13
    # the energy rows and L^T are those of the energy-only build, bit for bit
    h2 = gap.Handle(gap.params(d, zeta, sigma_w, 1e-8))
    h2.alloc_workspace(D.n_configs, D.n_atoms, M)
    X, offs, XM, sig = to_dev(D.X), to_dev(D.offsets), to_dev(D.XM), to_dev(D.sigma_E)
    h2.build_knm(X, offs, XM, sig)
    e_rows = _rows(h2, D)
    assert np.array_equal(rows[:NE], e_rows[:NE])
    assert np.array_equal(rows[NE + NO:], e_rows[NE:])
    h.close()
    h2.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_fit_with_forces_and_virials_matches_oracle(orc, precision):
    """c of the fit on [energies; forces; virials; L^T] against the oracle's staged
    fit: within 1e-10 (FP64) / 1e-8 (mixed) or the FP64 perturbation bound
    u (kappa + kappa^2 ||r|| / (||A|| ||c||)) of this stacked matrix."""
    import torch

    from paper_2207_03803_amd import gap

    D = synth.make_deriv_inputs(40, atoms=(20, 60), d=400, M=300, n_neigh=12, seed=8)
    zeta = 4
    y = oracle.deriv_targets(orc, D, zeta)
    c_ref, tail, K = orc.fit_deriv(D, y, zeta)
    rc, L, _ = orc.cholesky(orc.kmm(D.XM, zeta, 1.0, 1e-8))
    A, b = orc.stack(K, D.sigma, y, L)
    sv = np.linalg.svd(A, compute_uv=False)
    r = b - A @ c_ref
    kappa = sv[0] / sv[-1]
    bound = 32 * U * (kappa + kappa ** 2 * np.linalg.norm(r) / (sv[0] * np.linalg.norm(c_ref)))
    h = _handle(D, zeta, precision=precision, max_refine_iters=60, refine_tol=1e-12)
    _build(h, D)
    c = torch.empty(D.XM.shape[0], dtype=torch.float64, device="cuda")
    info = h.solve(to_dev(y), c)
    err = float(np.linalg.norm(c.cpu().numpy() - c_ref) / np.linalg.norm(c_ref))
    lerr = abs(info.residual_norm2 - tail) / tail
    allowed = max(1e-10 if precision == 0 else 1e-8, bound)
    log(f"  precision {precision}: {gap.status_string(info.device_status)}, {info.refine_iters} refinement steps "
        f"({info.cgls_iters} CGLS); kappa(A) {kappa:.2e}; c rel err vs oracle {err:.2e} (allowed {allowed:.1e}); "
        f"loss {lerr:.2e}; eta {info.grad_rel:.1e}")
    assert info.device_status == gap.GAP_OK
    assert err <= allowed
    assert lerr <= 1e-8
    assert info.grad_rel <= 1e-12
    h.close()


def test_out_of_range_gradient_index_is_reported():
    """A position naming a gradient row past n_grad: GAP_EINVAL in the device status;
    the kernel reads only in-range rows (the position contributes nothing)."""
    from paper_2207_03803_amd import gap

    D = synth.make_deriv_inputs(6, atoms=(16, 20), d=32, M=30, n_neigh=6, seed=9)
    bad = D.pos_grad.copy()
    bad[5] = D.x_grad.shape[0] + 1000
    h = _handle(D, 2)
    _build(h, D, pos_grad=bad)
    status, _ = h.sync()
    assert status == gap.GAP_EINVAL
    h.close()


def test_low_precision_forms_reject_derivative_observations():
    from paper_2207_03803_amd import gap

    D = synth.make_deriv_inputs(4, atoms=(16, 20), d=32, M=30, n_neigh=6, seed=10)
    for prec in (gap.GAP_MIXED_BF16, gap.GAP_MIXED_FP16):
        h = _handle(D, 2, precision=prec)
        with pytest.raises(gap.GapError) as e:
            _build(h, D)
        assert e.value.status == gap.GAP_EINVAL
        h.close()


def test_forces_workload_at_full_size(orc):
    """The energies-forces-virials workload at full size (500 configurations,
    19,537 atoms, 61,611 derivative observations over 2.3e6 positions, d = 400,
    M = 4000, zeta = 4) against the oracle's reference fit
    (tests/golden/forces_fp64_seed0.npz): c within 1e-10 (FP64) and 1e-8 (mixed) or
    the FP64 perturbation bound (kappa(A) = 1.0e6 here), the minimum loss, and 24
    sampled derivative rows against the oracle one by one."""
    import os

    import torch

    from paper_2207_03803_amd import gap

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "forces_fp64_seed0.npz")
    z = np.load(path, allow_pickle=False)
    w = dict(synth.WORKLOADS["forces_fp64"])
    D = synth.make_deriv_inputs(seed=0, **w)
    log(f"forces workload: {D.n_atoms} atoms, {D.n_obs} derivative observations, {len(D.pos_grad)} positions")
    y = to_dev(z["y"])
    kappa = float(z["smax"] / z["smin"])
    bound = 32 * U * (kappa + kappa ** 2 * np.sqrt(float(z["loss_tail"])) / (float(z["smax"]) * np.linalg.norm(z["c"])))
    rng = np.random.default_rng(12)
    pick = np.sort(np.concatenate([rng.choice(3 * D.n_atoms, 16, replace=False),
                                   3 * D.n_atoms + rng.choice(6 * D.n_configs, 8, replace=False)]))
    sizes = np.diff(D.obs_offsets)[pick]
    sub_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    sub_pos = np.concatenate([np.arange(D.obs_offsets[o], D.obs_offsets[o + 1]) for o in pick])
    ref_rows = orc.kdm(D.X, D.x_grad, D.grad_atom, sub_off, D.pos_grad[sub_pos], D.pos_weight[sub_pos], D.XM,
                       w["zeta"], w["sigma_w"])
    for prec in (gap.GAP_FP64, gap.GAP_MIXED_FP32):
        h = _handle(D, w["zeta"], precision=prec, max_refine_iters=30, refine_tol=1e-12)
        h.set_tuning(qr_free_cus=32)
        _build(h, D)
        if prec == gap.GAP_FP64:
            rows = _rows(h, D)[D.n_configs + pick] * D.sigma_D[pick][:, None]
            err_rows = np.max(np.abs(rows - ref_rows)) / np.max(np.abs(ref_rows))
        c = torch.empty(D.XM.shape[0], dtype=torch.float64, device="cuda")
        info = h.solve(y, c)
        err = float(np.linalg.norm(c.cpu().numpy() - z["c"]) / np.linalg.norm(z["c"]))
        lerr = abs(info.residual_norm2 - float(z["loss_tail"])) / float(z["loss_tail"])
        log(f"  precision {prec}: {gap.status_string(info.device_status)}, {info.refine_iters} refinement steps; "
            f"c rel err vs oracle {err:.2e}; loss {lerr:.2e}; eta {info.grad_rel:.1e}"
            + (f"; sampled rows {err_rows:.2e}" if prec == gap.GAP_FP64 else ""))
        assert info.device_status == gap.GAP_OK
        assert err <= max(1e-10 if prec == gap.GAP_FP64 else 1e-8, bound)
        assert lerr <= 1e-9
        h.close()
    assert err_rows <= 1e-13
