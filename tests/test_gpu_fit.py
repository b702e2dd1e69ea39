"""GPU parity tests of the FP64 path (K_NM build, Cholesky, Householder QR,
back-substitution, predict) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import GpuFit, U, log, to_dev

pytestmark = pytest.mark.gpu

TOL_C = 1e-10          # FP64 path: relative error of c versus the oracle
TOL_K = 1e-13          # elementwise relative error of Sigma^-1/2 K_NM


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _case(orc, n_configs, atoms, d, M, zeta, seed, sigma_per_atom=1e-3, jitter=1e-8):
    inp = synth.make_fit_inputs(n_configs=n_configs, atoms=atoms, d=d, M=M, seed=seed,
                                sigma_per_atom=sigma_per_atom)
    y = oracle.targets(orc, inp, zeta)
    ref = orc.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, jitter=jitter, keep=True)
    assert ref.status == 0
    return inp, y, ref


def _compare_fit(orc, inp, y, ref, zeta, jitter=1e-8, check_blocks=True):
    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, jitter=jitter)
    g.build()
    if check_blocks:
        top, low = g.A_top_and_lower()
        expect_top = ref.Knm / inp.sigma[:, None]
        relK = np.max(np.abs(top - expect_top) / np.abs(expect_top))
        log(f"  K_NM/sigma max elementwise rel err {relK:.2e}")
        assert relK <= TOL_K
        Lt = ref.L.T
        errL = np.linalg.norm(low - Lt) / np.linalg.norm(Lt)
        log(f"  L^T rel err {errL:.2e}")
        assert np.all(np.tril(low, -1) == 0.0)
        assert errL <= 1e-12
    c, info = g.solve()
    assert info.device_status == 0
    err = rel(c, ref.c)
    pred_err = rel(ref.Knm @ c, ref.Knm @ ref.c)
    loss_err = abs(info.residual_norm2 - ref.loss_tail) / ref.loss_tail
    log(f"  c rel err {err:.2e}; prediction-space {pred_err:.2e}; loss {loss_err:.2e}; eta {info.grad_rel:.1e}")
    assert info.grad_rel <= 1e-13  # back-substitution residual in the factored basis
    assert err <= TOL_C
    assert pred_err <= 1e-12
    assert loss_err <= 1e-10
    # |diag R| against the oracle (R is unique up to row signs)
    Av, lay = g.h.A_view()
    dR = np.abs(np.diag(Av[:g.M, :g.M].T.cpu().numpy()))
    assert np.max(np.abs(dR - np.abs(ref.diagR)) / np.abs(ref.diagR)) <= 1e-9
    return g, c


@pytest.fixture(scope="module")
def orc_m():
    return oracle.Oracle()


def test_tiny_workload_parity(orc_m):
    w = synth.WORKLOADS["tiny_fp64"]
    log("tiny_fp64: 200 configs, d=64, M=256, zeta=2")
    inp, y, ref = _case(orc_m, 200, (8, 64), 64, 256, 2, seed=0)
    _compare_fit(orc_m, inp, y, ref, 2, jitter=w["jitter"])


@pytest.mark.parametrize("n_configs,atoms,d,M,zeta,seed", [
    (37, (1, 5), 13, 45, 3, 1),      # tiny odd shapes: M < one QR panel, d not a tile multiple
    (150, (8, 64), 64, 200, 2, 2),    # ragged M (3 panels + 8 columns)
    (400, (16, 64), 96, 333, 4, 3),   # several K_NM tiles, ragged everything
    (90, (1, 1), 32, 90, 2, 4),       # one atom per configuration, M = N
])
def test_ragged_shapes_parity(orc_m, n_configs, atoms, d, M, zeta, seed):
    log(f"ragged: N={n_configs} atoms={atoms} d={d} M={M} zeta={zeta}")
    inp, y, ref = _case(orc_m, n_configs, atoms, d, M, zeta, seed)
    _compare_fit(orc_m, inp, y, ref, zeta)


@pytest.mark.parametrize("M", [64, 128, 129, 192, 193])
def test_cholesky_step_pairing_boundaries(orc_m, M):
    """K_MM sizes where the Cholesky's 64-column steps pair up exactly, or leave
    one step or one column over: L^T and c against the oracle."""
    log(f"cholesky pairing: N=300 atoms=(1, 4) d=64 M={M} zeta=2")
    inp, y, ref = _case(orc_m, 300, (1, 4), 64, M, 2, 40 + M)
    _compare_fit(orc_m, inp, y, ref, 2)


def test_large_and_empty_configurations(orc_m):
    """Configurations larger than one 256-atom chunk, and empty ones."""
    rng = np.random.default_rng(9)
    counts = np.array([3, 0, 300, 17, 0, 0, 600, 64, 1, 257, 256, 5] * 3, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    d, M, zeta = 24, 70, 2
    X = np.abs(rng.standard_normal((offsets[-1], d)))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    XM = X[rng.choice(offsets[-1], M, replace=False)]
    sigma = 1e-3 * np.maximum(counts, 1).astype(float)
    y = orc_m.predict(X, offsets, XM, rng.standard_normal(M), zeta) + sigma * rng.standard_normal(len(counts))
    log("large/empty configurations: counts up to 600 atoms, empty rows")
    ref = orc_m.fit(X, offsets, XM, sigma, y, zeta, jitter=1e-8, keep=True)
    assert ref.status == 0
    g = GpuFit(X, offsets, XM, sigma, y, zeta)
    g.build()
    top, low = g.A_top_and_lower()
    expect = ref.Knm / sigma[:, None]
    nz = expect != 0
    assert np.all(top[~nz] == 0.0)
    assert np.max(np.abs(top[nz] - expect[nz]) / np.abs(expect[nz])) <= TOL_K
    c, info = g.solve()
    # empty configurations make zero rows: still a valid least-squares problem
    assert rel(c, ref.c) <= TOL_C


def test_mid_size_realistic_shape(orc_m):
    """d=400, zeta=4 at a size the oracle finishes in seconds (several tiles, ragged M)."""
    log("mid-size: N=2000 configs of 16..64 atoms, d=400, M=520, zeta=4")
    inp, y, ref = _case(orc_m, 2000, (16, 64), 400, 520, 4, seed=5)
    _compare_fit(orc_m, inp, y, ref, 4)


def test_predict_parity(orc_m):
    inp, y, ref = _case(orc_m, 150, (8, 64), 64, 200, 2, seed=6)
    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 2)
    c, info = g.run()
    import torch

    # new configurations, different sizes, including a 1-configuration batch
    for n_cfg, seed in ((1, 20), (7, 21), (333, 22)):
        q = synth.make_fit_inputs(n_configs=n_cfg, atoms=(8, 64), d=64, M=1, seed=seed)
        expect = orc_m.predict(q.X, q.offsets, inp.XM, ref.c, 2)
        out = torch.empty(n_cfg, dtype=torch.float64, device="cuda")
        g.h.predict(to_dev(q.X), to_dev(q.offsets), to_dev(ref.c), out)
        got = out.cpu().numpy()
        e = np.max(np.abs(got - expect) / np.abs(expect))
        log(f"  predict {n_cfg} configs: max rel err {e:.2e}")
        assert e <= 1e-12
    # on the training configurations, predict = K_NM c
    out = torch.empty(inp.n_configs, dtype=torch.float64, device="cuda")
    g.h.predict(g.X, g.offsets, g.c, out)
    assert rel(out.cpu().numpy(), ref.Knm @ c) <= 1e-13


def test_predict_at_the_serving_shape(orc_m):
    """A served model's shape (d=400, zeta=4, M=4,000) on a predict-only handle
    (gap_set_model), 4,096 configurations of 8..64 atoms: 256 sampled
    configurations against the oracle one by one.  Weights of both signs, so the
    error is measured against the sum of absolute terms (the oracle's predict
    with |c|; descriptors are non-negative, so every kernel value is)."""
    import torch

    from paper_2207_03803_amd import gap

    d, zeta, M, n = 400, 4, 4000, 4096
    q = synth.make_fit_inputs(n_configs=n, atoms=(8, 64), d=d, M=M, seed=31)
    c = np.random.default_rng(32).standard_normal(M)
    log(f"predict at serving shape: {n} configs ({q.n_atoms} atoms), d={d}, M={M}, zeta={zeta}")
    h = gap.Handle(gap.params(d, zeta))
    XM = to_dev(q.XM)
    h.set_model(XM)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    h.predict(to_dev(q.X), to_dev(q.offsets), to_dev(c), out)
    status, _ = h.sync()
    assert status == gap.GAP_OK
    got = out.cpu().numpy()
    h.close()
    pick = np.sort(np.random.default_rng(33).choice(n, 256, replace=False))
    rows = np.concatenate([np.arange(q.offsets[a], q.offsets[a + 1]) for a in pick])
    offs = np.concatenate([[0], np.cumsum(np.diff(q.offsets)[pick])]).astype(np.int64)
    expect = orc_m.predict(q.X[rows], offs, q.XM, c, zeta)
    scale = orc_m.predict(q.X[rows], offs, q.XM, np.abs(c), zeta)
    e = np.max(np.abs(got[pick] - expect) / scale)
    log(f"  max |error| / sum of |terms| {e:.2e}")
    assert e <= 1e-14 * np.sqrt(M)
    assert np.all(np.isfinite(got))


def test_not_positive_definite_is_reported(orc_m):
    inp, y, ref = _case(orc_m, 60, (8, 16), 16, 40, 2, seed=7)
    XM = np.vstack([inp.XM[:39], inp.XM[:1]])  # duplicated sparse point, no jitter
    g = GpuFit(inp.X, inp.offsets, XM, inp.sigma, y, 2, jitter=0.0)
    g.build()
    from paper_2207_03803_amd import gap

    with pytest.raises(gap.GapError) as e:
        g.solve()
    assert e.value.status == gap.GAP_ENOTPD


def test_bad_offsets_are_reported(orc_m):
    inp, y, ref = _case(orc_m, 20, (8, 16), 16, 10, 2, seed=8)
    offs = inp.offsets.copy()
    offs[5], offs[6] = offs[6], offs[5]  # decreasing
    g = GpuFit(inp.X, offs, inp.XM, inp.sigma, y, 2)
    g.build()
    s, info = g.h.sync()
    from paper_2207_03803_amd import gap

    assert s == gap.GAP_EINVAL


def test_predict_rejects_bad_offsets(orc_m):
    """Malformed offsets in a predict request (swapped, past n_atoms, offsets[0] != 0)
    give NaN energies where they occur and GAP_EINVAL, on a fit handle and on a
    predict-only handle with a status workspace; good requests are unaffected."""
    import torch

    from paper_2207_03803_amd import gap

    inp, y, ref = _case(orc_m, 600, (8, 64), 64, 40, 2, seed=9)
    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 2)
    g.build()
    c, info = g.solve()
    assert info.device_status == gap.GAP_OK
    n = inp.n_configs
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    swapped = inp.offsets.copy()
    swapped[400], swapped[401] = swapped[401], swapped[400]
    past = inp.offsets.copy()
    past[300:] += 10_000_000  # every range from configuration 299 on ends past the descriptors
    shifted = inp.offsets.copy()
    shifted[0] = 3
    ph = gap.Handle(gap.params(64, 2, 1.0, 1e-8))
    ph.set_model(g.XM)
    status_ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    ph.bind(status_ws)
    for name, offs in (("swapped", swapped), ("past n_atoms", past), ("offsets[0] != 0", shifted)):
        g.build()  # clears the fit handle's status word (the weights stay in g.c)
        for h in (g.h, ph):
            assert h.sync()[0] == gap.GAP_OK
            out.fill_(0.0)
            h.predict(g.X, to_dev(offs), g.c, out)
            s, _ = h.sync()
            got = out.cpu().numpy()
            log(f"  predict with {name} offsets: status {gap.status_string(s)}, {np.isnan(got).sum()} NaN of {n}")
            assert s == gap.GAP_EINVAL
            assert np.isnan(got).any()
        ph.bind(status_ws)  # clears the predict-only handle's status word
    # a good request on a fresh predict-only handle: finite, status OK
    ph2 = gap.Handle(gap.params(64, 2, 1.0, 1e-8))
    ph2.set_model(g.XM)
    ph2.bind(torch.zeros(256, dtype=torch.uint8, device="cuda"))
    ph2.predict(g.X, g.offsets, g.c, out)
    assert ph2.sync()[0] == gap.GAP_OK
    assert np.isfinite(out.cpu().numpy()).all()
    for h in (ph, ph2):
        h.close()


def test_repeat_runs_are_bitwise_identical(orc_m):
    inp, y, ref = _case(orc_m, 150, (8, 64), 64, 200, 2, seed=10)
    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 2)
    c1, _ = g.run()
    c2, _ = g.run()
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("panel,lookahead", [(0, 2), (0, 1), (1, 2), (1, 1)])
def test_qr_schedules_and_panels_agree(orc_m, panel, lookahead):
    """Both panel factorisations (shifted CholeskyQR3, TSQR) with and without the
    look-ahead schedule reach the oracle's weights; each is bitwise repeatable."""
    inp, y, ref = _case(orc_m, 1500, (16, 64), 160, 390, 3, 21)
    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 3)
    g.h.set_tuning(qr_panel=panel, qr_lookahead=lookahead)
    g.build()
    c1, info = g.solve()
    g.build()
    c2, _ = g.solve()
    err = rel(c1, ref.c)
    log(f"  panel={'TSQR' if panel else 'CholeskyQR3'} look-ahead={'off' if lookahead == 1 else 'on'}: "
        f"c rel err {err:.2e}")
    assert info.device_status == 0
    assert err <= TOL_C
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("precision", [0, 1])
def test_lookahead_free_cus_leave_results_bitwise_unchanged(orc_m, precision):
    """Keeping CUs free of the look-ahead stream (a CU mask, for a handle on a
    stream of its own) changes only where kernels run: c is bitwise the unmasked
    look-ahead's, at the oracle's weights."""
    import torch

    inp, y, ref = _case(orc_m, 1500, (16, 64), 160, 390, 3, 21)
    outs = {}
    with torch.cuda.stream(torch.cuda.Stream()):
        g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 3, precision=precision)
        for free in (0, 16, 32, 64, 0):
            g.h.set_tuning(qr_lookahead=2, qr_free_cus=free)
            g.build()
            g.h.solve(g.y, g.c, info=False)
            s, info = g.h.sync()
            assert s == 0
            outs.setdefault(free, []).append(g.c.cpu().numpy())
    base = outs[0][0]
    log(f"  precision {precision}: c rel err {rel(base, ref.c):.2e}")
    assert rel(base, ref.c) <= (TOL_C if precision == 0 else 1e-8)
    for free, cs in outs.items():
        for c in cs:
            assert np.array_equal(c, base), free


def test_atom_order_within_configurations(orc_m):
    """Permuting the atoms inside every configuration changes only the order of
    the segment sums (K_NM within a few ulps) and leaves c at the oracle's."""
    inp, y, ref = _case(orc_m, 300, (8, 64), 48, 180, 3, 31)
    rng = np.random.default_rng(5)
    X2 = inp.X.copy()
    for a in range(inp.n_configs):
        s, e = inp.offsets[a], inp.offsets[a + 1]
        X2[s:e] = X2[s:e][rng.permutation(e - s)]
    g1 = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 3)
    g1.build()
    k1, _ = g1.A_top_and_lower()
    g2 = GpuFit(X2, inp.offsets, inp.XM, inp.sigma, y, 3)
    g2.build()
    k2, _ = g2.A_top_and_lower()
    assert np.max(np.abs(k1 - k2) / np.abs(k1)) <= 64 * U
    c2, _ = g2.solve()
    assert rel(c2, ref.c) <= TOL_C


def test_configuration_order_gives_the_same_rows_bitwise(orc_m):
    """The tile plan packs configurations out of order; a row of K_NM depends only
    on its configuration's atoms, so permuting the configurations permutes the
    rows bit for bit, and c stays at the oracle's."""
    inp, y, ref = _case(orc_m, 700, (8, 64), 40, 150, 2, 33)
    rng = np.random.default_rng(6)
    order = rng.permutation(inp.n_configs)
    counts = np.diff(inp.offsets)
    offs2 = np.concatenate([[0], np.cumsum(counts[order])]).astype(np.int64)
    X2 = np.concatenate([inp.X[inp.offsets[a]:inp.offsets[a + 1]] for a in order])
    g1 = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 2)
    g1.build()
    k1, _ = g1.A_top_and_lower()
    g2 = GpuFit(X2, offs2, inp.XM, inp.sigma[order], y[order], 2)
    g2.build()
    k2, _ = g2.A_top_and_lower()
    assert np.array_equal(k2, k1[order])
    c2, _ = g2.solve()
    assert rel(c2, ref.c) <= TOL_C


def test_one_hot_descriptors_give_exact_counts(orc_m):
    """x = e_p makes every covariance 0 or sigma_w^2, so K_NM holds integer counts:
    the GPU's Sigma^-1/2 K_NM equals the oracle's bit for bit."""
    rng = np.random.default_rng(8)
    d, N, M = 16, 120, 12
    counts = rng.integers(1, 40, N)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    X = np.zeros((offsets[-1], d))
    X[np.arange(offsets[-1]), rng.integers(0, d, offsets[-1])] = 1.0
    XM = np.eye(d)[:M]
    sigma = 1e-3 * counts.astype(float)
    Knm = orc_m.knm(X, offsets, XM, 3)
    assert np.array_equal(Knm, np.round(Knm))
    g = GpuFit(X, offsets, XM, sigma, np.ones(N), 3)
    g.build()
    top, _ = g.A_top_and_lower()
    assert np.array_equal(top, Knm / sigma[:, None])


@pytest.mark.parametrize("name,args", [
    ("tiny", (200, (8, 64), 64, 256, 2, 0)),
    ("mid-size d=400 zeta=4", (2000, (16, 64), 400, 520, 4, 5)),
])
def test_error_estimate_against_the_oracle_condition_number(orc_m, name, args):
    """GAP_FLAG_ERROR_ESTIMATE: kappa_2(A) from 16 power / inverse iteration steps on
    the GPU's R against the oracle's converged estimate (which is pinned to LAPACK's
    SVD); the estimated error bounds the observed difference from the oracle's c."""
    from paper_2207_03803_amd import gap

    inp, y, ref = _case(orc_m, *args)
    zeta = args[4]
    n = args[3]
    smax, smin, _ = orc_m.singular_extremes(np.triu(ref.A[:n]))
    kappa = smax / smin
    for prec in (gap.GAP_FP64, gap.GAP_MIXED_FP32):
        g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, precision=prec, max_refine_iters=30,
                   refine_tol=1e-14)
        g.h.close()
        g.h = gap.Handle(gap.params(inp.X.shape[1], zeta, 1.0, 1e-8, precision=prec, max_refine_iters=30,
                                    refine_tol=1e-14, flags=gap.GAP_FLAG_ERROR_ESTIMATE))
        g.h.alloc_workspace(g.N, g.X.shape[0], g.M)
        c, info = g.run()
        assert info.device_status == gap.GAP_OK
        err = rel(c, ref.c)
        log(f"  {name} precision {prec}: kappa est {info.kappa_est:.3e} (oracle {kappa:.3e}); est_err "
            f"{info.est_err:.2e}, observed c rel err {err:.2e}; eta {info.grad_rel:.1e}")
        assert 0.05 * kappa <= info.kappa_est <= 1.01 * kappa
        assert info.est_err > 0 and err <= 10 * info.est_err
        assert info.grad_rel <= 1e-13
        g.h.close()
