"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: the expected side is an exact
rational solve, a closed form, a textbook special case, a numpy/LAPACK routine
the oracle never calls, or an invariance the paper states.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests import exact_ref

U = np.finfo(np.float64).eps / 2  # unit roundoff
HERE = os.path.dirname(os.path.abspath(__file__))


def tiny(seed=0, **kw):
    w = dict(synth.WORKLOADS["tiny_fp64"])
    w.update(kw)
    return w, synth.make_fit_inputs(seed=seed, **w)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def eta(A, b, c):
    """Normwise backward-error style residual of the normal equations."""
    r = b - A @ c
    nA = np.linalg.norm(A)
    return float(np.linalg.norm(A.T @ r) / (nA * (nA * np.linalg.norm(c) + np.linalg.norm(b))))


@pytest.fixture(scope="module")
def tiny_fit(orc):
    w, inp = tiny()
    y = oracle.targets(orc, inp, w["zeta"])
    res = orc.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, w["zeta"], jitter=w["jitter"], keep=True)
    assert res.status == oracle.ORACLE_OK
    A, b = orc.stack(res.Knm, inp.sigma, y, res.L)
    return w, inp, y, res, A, b


# ---------------------------------------------------------------- P1 exact


def _micro(seed, jitter=1e-8, zeta=2):
    rng = np.random.default_rng(1000 + seed)
    d, M = 3, 4
    counts = rng.integers(1, 4, size=6)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    X = np.abs(rng.standard_normal((offsets[-1], d)))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    XM = np.abs(rng.standard_normal((M, d)))
    XM /= np.linalg.norm(XM, axis=1, keepdims=True)
    sigma = 0.05 * counts.astype(float)
    y = rng.standard_normal(len(counts)) * counts
    return X, offsets, XM, sigma, y, zeta, jitter


@pytest.mark.parametrize("seed", range(4))
def test_p1_exact_rational_normal_equations(orc, seed):
    X, offsets, XM, sigma, y, zeta, jitter = _micro(seed)
    res = orc.fit(X, offsets, XM, sigma, y, zeta, jitter=jitter, keep=True)
    assert res.status == 0
    c_ex = np.array([float(v) for v in exact_ref.fit_exact(X.tolist(), offsets.tolist(), XM.tolist(),
                                                           sigma.tolist(), y.tolist(), zeta,
                                                           jitter=jitter)])
    A, b = orc.stack(res.Knm, sigma, y, res.L)
    kappa = np.linalg.cond(A)
    assert rel(res.c, c_ex) <= 10 * kappa * U
    Knm_ex = np.array([[float(v) for v in row] for row in
                       exact_ref.knm_exact(X.tolist(), offsets.tolist(), XM.tolist(), zeta)])
    assert np.max(np.abs(res.Knm - Knm_ex) / np.abs(Knm_ex)) <= 8 * U * (X.shape[1] + 3)


def test_p1_exact_with_large_jitter(orc):
    """A jitter large enough to move c well above rounding: pins where it enters."""
    X, offsets, XM, sigma, y, zeta, _ = _micro(7)
    res = orc.fit(X, offsets, XM, sigma, y, zeta, jitter=0.5)
    c_ex = np.array([float(v) for v in exact_ref.fit_exact(X.tolist(), offsets.tolist(), XM.tolist(),
                                                           sigma.tolist(), y.tolist(), zeta,
                                                           jitter=0.5)])
    c_nojit = np.array([float(v) for v in exact_ref.fit_exact(X.tolist(), offsets.tolist(),
                                                              XM.tolist(), sigma.tolist(),
                                                              y.tolist(), zeta, jitter=0.0)])
    assert rel(res.c, c_ex) <= 1e-12
    assert rel(c_nojit, c_ex) > 1e-3


# ---------------------------------------------------------------- P2 LAPACK


def test_p2_lapack_lstsq(tiny_fit):
    w, inp, y, res, A, b = tiny_fit
    c_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    assert rel(res.c, c_ls) <= 1e-10


def test_p2_normal_equations_within_kappa_squared(tiny_fit, orc):
    """FP64 normal equations agree only to ~kappa^2 u (why the paper uses QR)."""
    w, inp, y, res, A, b = tiny_fit
    Kmm = orc.kmm(inp.XM, w["zeta"], jitter=w["jitter"])
    Si = 1.0 / inp.sigma ** 2
    H = Kmm + res.Knm.T @ (Si[:, None] * res.Knm)
    c_ne = np.linalg.solve(H, res.Knm.T @ (Si * y))
    kappa = np.linalg.cond(A)
    assert rel(res.c, c_ne) <= kappa ** 2 * U


# ---------------------------------------------------------------- P3/P4


def test_p3_zero_gradient(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    assert eta(A, b, res.c) <= 1e-13
    # gradient of the paper's loss (Eq. loss), written without A or b
    Kmm = orc.kmm(inp.XM, w["zeta"], jitter=w["jitter"])
    g = orc.gradient(res.Knm, inp.sigma, y, Kmm, res.c)
    # the same gradient via the least-squares form: 2 A^T (A c - b)
    g_ls = 2.0 * A.T @ (A @ res.c - b)
    scale = 2 * np.linalg.norm(A) * (np.linalg.norm(A) * np.linalg.norm(res.c) + np.linalg.norm(b))
    assert np.linalg.norm(g) <= 1e-13 * scale
    assert np.linalg.norm(g - g_ls) <= 1e-13 * scale


def test_p4_loss_identity(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    Kmm = orc.kmm(inp.XM, w["zeta"], jitter=w["jitter"])
    L_paper = orc.loss(res.Knm, inp.sigma, y, Kmm, res.c)
    r = b - A @ res.c
    assert abs(r @ r - res.loss_tail) <= 1e-10 * res.loss_tail
    assert abs(L_paper - res.loss_tail) <= 1e-10 * res.loss_tail
    # and it is a minimum: any perturbation raises the loss
    rng = np.random.default_rng(5)
    for _ in range(3):
        dc = rng.standard_normal(len(res.c)) * 1e-3 * np.linalg.norm(res.c) / np.sqrt(len(res.c))
        assert orc.loss(res.Knm, inp.sigma, y, Kmm, res.c + dc) > L_paper


# ---------------------------------------------------------------- P5/P6 invariances


def test_p5_atom_order_invariance(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    rng = np.random.default_rng(11)
    X2 = inp.X.copy()
    for a in range(inp.n_configs):
        s, e = inp.offsets[a], inp.offsets[a + 1]
        X2[s:e] = X2[s:e][rng.permutation(e - s)]
    res2 = orc.fit(X2, inp.offsets, inp.XM, inp.sigma, y, w["zeta"], jitter=w["jitter"], keep=True)
    assert np.max(np.abs(res2.Knm - res.Knm) / np.abs(res.Knm)) <= 64 * U
    assert rel(res2.c, res.c) <= np.linalg.cond(A) * U * 100


def test_p6_row_permutation_and_zero_padding(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    rng = np.random.default_rng(12)
    perm = np.concatenate([rng.permutation(inp.n_configs), inp.n_configs + np.arange(len(res.c))])
    A2, b2 = A[perm], b[perm]
    pad = 37
    A2 = np.vstack([A2[:100], np.zeros((pad, A.shape[1])), A2[100:]])
    b2 = np.concatenate([b2[:100], np.zeros(pad), b2[100:]])
    R, qtb, _ = orc.householder_qr(A2, b2)
    n = A.shape[1]
    c2 = orc.back_substitution(R[:n], qtb[:n])
    assert rel(c2, res.c) <= np.linalg.cond(A) * U * 100
    # the same through the whole fit with the configurations reordered
    order = rng.permutation(inp.n_configs)
    counts = np.diff(inp.offsets)[order]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    X3 = np.concatenate([inp.X[inp.offsets[a]:inp.offsets[a + 1]] for a in order])
    res3 = orc.fit(X3, offs, inp.XM, inp.sigma[order], y[order], w["zeta"], jitter=w["jitter"])
    assert rel(res3.c, res.c) <= np.linalg.cond(A) * U * 100


# ---------------------------------------------------------------- P7/P8 special cases


def _single_atom_configs(n, d, seed):
    rng = np.random.default_rng(seed)
    X = np.abs(rng.standard_normal((n, d)))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return X, np.arange(n + 1, dtype=np.int64)


def test_p7_full_gp_special_case(orc):
    """One atom per configuration, sparse set = all atoms, no jitter, Sigma = s^2 I:
    the sparse-GP weights are the textbook GP weights (K + s^2 I)^-1 y."""
    n, d, zeta, s = 40, 16, 2, 0.3
    X, offsets = _single_atom_configs(n, d, 3)
    y = np.random.default_rng(4).standard_normal(n)
    res = orc.fit(X, offsets, X, np.full(n, s), y, zeta, jitter=0.0)
    assert res.status == 0
    K = (X @ X.T) ** zeta
    c_gp = np.linalg.solve(K + s * s * np.eye(n), y)
    assert rel(res.c, c_gp) <= 100 * np.linalg.cond(K + s * s * np.eye(n)) * U


def test_p8_interpolation_limit(orc):
    """M = N, sigma -> 0: the fit interpolates, residual shrinking as sigma^2."""
    n, d, zeta = 30, 16, 2
    X, offsets = _single_atom_configs(n, d, 5)
    y = np.random.default_rng(6).standard_normal(n)
    K = (X @ X.T) ** zeta
    resid = []
    for s in (1e-2, 1e-3):
        res = orc.fit(X, offsets, X, np.full(n, s), y, zeta, jitter=1e-8)
        resid.append(np.linalg.norm(K @ res.c - y) / np.linalg.norm(y))
    ratio = resid[0] / resid[1]
    assert 50 < ratio < 200, ratio
    assert resid[1] < 1e-2


# ---------------------------------------------------------------- P9-P11 kernel structure


def test_p9_one_hot_descriptors_give_exact_counts(orc):
    rng = np.random.default_rng(7)
    d, M, zeta, sw = 8, 8, 3, 1.5
    counts = rng.integers(1, 20, size=25)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    hot = rng.integers(0, d, size=offsets[-1])
    X = np.eye(d)[hot]
    XM = np.eye(d)
    K = orc.knm(X, offsets, XM, zeta, sw)
    expect = np.zeros((len(counts), M))
    for a in range(len(counts)):
        for i in range(offsets[a], offsets[a + 1]):
            expect[a, hot[i]] += 1
    assert np.array_equal(K, expect * sw * sw)


def test_p10_identical_atoms_and_self_similarity(orc):
    _, inp = tiny(seed=3)
    d = inp.X.shape[1]
    x = inp.X[0]
    counts = np.array([1, 5, 17, 64])
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    X = np.tile(x, (offsets[-1], 1))
    K = orc.knm(X, offsets, inp.XM[:10], 4, 1.0)
    single = orc.knm(x[None, :], np.array([0, 1]), inp.XM[:10], 4, 1.0)[0]
    for a, n in enumerate(counts):
        assert np.max(np.abs(K[a] - n * single) / (n * single)) <= 64 * U
    Kself = orc.kmm(inp.XM[:10], 4, 1.0, 0.0)
    assert np.max(np.abs(np.diag(Kself) - 1.0)) <= 4 * d * U


def test_p11_linear_kernel_is_a_sum_then_product(orc):
    _, inp = tiny(seed=4)
    K = orc.knm(inp.X, inp.offsets, inp.XM, 1, 1.0)
    S = np.add.reduceat(inp.X, inp.offsets[:-1], axis=0)
    expect = S @ inp.XM.T
    assert np.max(np.abs(K - expect) / np.abs(expect)) <= 2 * (inp.X.shape[1] + 64) * U


def test_knm_matches_numpy_segment_sum(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    G = (inp.X @ inp.XM.T) ** w["zeta"]
    expect = np.add.reduceat(G, inp.offsets[:-1], axis=0)
    assert np.max(np.abs(res.Knm - expect) / np.abs(expect)) <= 1e-13


# ---------------------------------------------------------------- P12/P13 factorisations


def test_p12_cholesky(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    Kmm = orc.kmm(inp.XM, w["zeta"], jitter=w["jitter"])
    L_np = np.linalg.cholesky(Kmm)
    M = Kmm.shape[0]
    assert np.linalg.norm(res.L @ res.L.T - Kmm) <= M * U * np.linalg.norm(Kmm)
    assert rel(res.L, L_np) <= np.linalg.cond(Kmm) * M * U
    assert np.all(np.triu(res.L, 1) == 0)


def test_p12_cholesky_reports_not_pd(orc):
    _, inp = tiny()
    XM = np.vstack([inp.XM[:20], inp.XM[:1]])      # a duplicated sparse point
    K = orc.kmm(XM, 2, 1.0, 0.0)
    rc, L, fail = orc.cholesky(K)
    assert rc == oracle.ORACLE_ENOTPD and fail == 20


def _form_q(Afact, tau):
    m, n = Afact.shape
    Q = np.eye(m)
    for k in range(n - 1, -1, -1):
        v = np.zeros(m)
        v[k] = 1.0
        v[k + 1:] = Afact[k + 1:, k]
        Q -= tau[k] * np.outer(v, v @ Q)
    return Q


def test_p13_householder_qr(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    m, n = A.shape
    Q = _form_q(res.A, res.tau)
    R = np.triu(res.A[:n])
    assert np.linalg.norm(A - Q[:, :n] @ R) <= m * U * np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= m * U * np.sqrt(m)
    assert np.linalg.norm(Q.T @ b - res.qtb) <= m * U * np.linalg.norm(b)
    R_np = np.linalg.qr(A, mode="r")
    assert np.max(np.abs(np.abs(np.diag(R)) - np.abs(np.diag(R_np))) / np.abs(np.diag(R_np))) \
        <= np.linalg.cond(A) * m * U
    # sign convention: beta = -sign(alpha) ||.||, so R's diagonal is never 0 here
    assert np.all(res.tau >= 0) and np.all(res.tau <= 2)


def test_p13_zero_column_gives_identity_reflector(orc):
    A = np.zeros((6, 3))
    A[:, 0] = [3.0, 0, 0, 0, 0, 0]
    A[:, 1] = np.arange(6.0)
    A[:, 2] = 1.0
    b = np.ones(6)
    R, qtb, tau = orc.householder_qr(A, b)
    assert tau[0] == 0.0 and R[0, 0] == 3.0


def test_kappa_estimate_matches_svd_of_the_stacked_matrix(tiny_fit, orc):
    """The singular-value estimator (power and inverse iteration on R) against
    LAPACK's SVD of A itself: A and its R share their singular values."""
    w, inp, y, res, A, b = tiny_fit
    n = A.shape[1]
    smax, smin, its = orc.singular_extremes(np.triu(res.A[:n]))
    sv = np.linalg.svd(A, compute_uv=False)
    kappa = sv[0] / sv[-1]
    assert abs(smax / sv[0] - 1) <= 1e-12
    assert abs(smin / sv[-1] - 1) <= 1e-9
    assert abs(smax / smin / kappa - 1) <= 1e-9
    assert its[0] < 2000 and its[1] < 2000  # converged, not capped


def test_kappa_estimate_closed_forms(orc):
    """Diagonal R: the extremes are its largest and smallest |entries|.
    A 2 x 2 triangle [[1, t], [0, e]]: sigma_max sigma_min = |det| = e and
    sigma_max^2 + sigma_min^2 = 1 + t^2 + e^2 (the Frobenius norm)."""
    s = np.array([3.0, -0.5, 2.0, 0.01, 1.0])
    smax, smin, _ = orc.singular_extremes(np.diag(s))
    assert abs(smax - 3.0) <= 1e-14 * 3.0 and abs(smin - 0.01) <= 1e-13 * 0.01
    t, e = 4.0, 1e-3
    smax, smin, _ = orc.singular_extremes(np.array([[1.0, t], [0.0, e]]))
    assert abs(smax * smin - e) <= 1e-12 * e
    assert abs(smax ** 2 + smin ** 2 - (1 + t * t + e * e)) <= 1e-14 * (1 + t * t)


# ---------------------------------------------------------------- P15 predict


def test_p15_predict_equals_knm_times_c(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    yp = orc.predict(inp.X, inp.offsets, inp.XM, res.c, w["zeta"])
    assert rel(yp, res.Knm @ res.c) <= 1e-13


def test_p15_predict_closed_form_numpy(tiny_fit, orc):
    w, inp, y, res, A, b = tiny_fit
    eps = ((inp.X @ inp.XM.T) ** w["zeta"]) @ inp.c_true
    expect = np.add.reduceat(eps, inp.offsets[:-1])
    got = orc.predict(inp.X, inp.offsets, inp.XM, inp.c_true, w["zeta"])
    assert rel(got, expect) <= 1e-13


# ---------------------------------------------------------------- P17 printed shapes


def test_p17_paper_printed_shapes():
    cases = json.load(open(os.path.join(HERE, "golden", "paper_shapes.json")))["cases"]
    for c in cases:
        assert c["N_energies"] + c["N_forces"] + c["N_virials"] == c["N"]
        assert sum(k * n for k, n in c["M_parts"]) == c["M"]
        assert (c["N"] + c["M"]) * c["M"] == c["n_A"]
        assert round(c["n_A"] * 8 / 1e9, 1) == c["GB"]


# ---------------------------------------------------------------- planted mistakes


PLANTS = ["ORACLE_PLANT_POWER", "ORACLE_PLANT_NO_JITTER", "ORACLE_PLANT_NO_ROW_SCALE",
          "ORACLE_PLANT_TRANSPOSE_L", "ORACLE_PLANT_TAU", "ORACLE_PLANT_BACKSUB", "ORACLE_PLANT_SEGMENT_END",
          "ORACLE_PLANT_B_UNSCALED", "ORACLE_PLANT_PREDICT_SEGMENT"]


@pytest.mark.parametrize("plant", PLANTS)
def test_planted_mistake_is_caught(plant, tmp_path):
    """Each planted mistake in the oracle makes at least one pin fail."""
    path = oracle.build(str(tmp_path / f"lib_{plant}.so"), defines=[plant])
    bad = oracle.Oracle(path)
    failures = 0
    # exact rational pin with a jitter large enough to matter
    X, offsets, XM, sigma, y, zeta, _ = _micro(7)
    res = bad.fit(X, offsets, XM, sigma, y, zeta, jitter=0.5)
    c_ex = np.array([float(v) for v in exact_ref.fit_exact(X.tolist(), offsets.tolist(), XM.tolist(),
                                                           sigma.tolist(), y.tolist(), zeta,
                                                           jitter=0.5)])
    if res.status != 0 or not np.all(np.isfinite(res.c)) or rel(res.c, c_ex) > 1e-12:
        failures += 1
    # prediction (Eqs. 1-2) against its closed form in numpy, with sigma_w != 1
    c = np.random.default_rng(3).standard_normal(XM.shape[0])
    eps = 1.3 ** 2 * (X @ XM.T) ** zeta @ c
    y_ref = np.array([eps[offsets[a]:offsets[a + 1]].sum() for a in range(len(offsets) - 1)])
    if rel(bad.predict(X, offsets, XM, c, zeta, sigma_w=1.3), y_ref) > 1e-13:
        failures += 1
    assert failures > 0


def test_the_planted_mistake_checks_pass_on_the_oracle(orc):
    """The checks the planted-mistake test relies on hold for the oracle as built."""
    X, offsets, XM, sigma, y, zeta, _ = _micro(7)
    res = orc.fit(X, offsets, XM, sigma, y, zeta, jitter=0.5)
    c_ex = np.array([float(v) for v in exact_ref.fit_exact(X.tolist(), offsets.tolist(), XM.tolist(),
                                                           sigma.tolist(), y.tolist(), zeta,
                                                           jitter=0.5)])
    assert res.status == 0 and rel(res.c, c_ex) <= 1e-12
    c = np.random.default_rng(3).standard_normal(XM.shape[0])
    eps = 1.3 ** 2 * (X @ XM.T) ** zeta @ c
    y_ref = np.array([eps[offsets[a]:offsets[a + 1]].sum() for a in range(len(offsets) - 1)])
    assert rel(orc.predict(X, offsets, XM, c, zeta, sigma_w=1.3), y_ref) <= 1e-13
