"""Mixed precision with a low-precision K_NM (GAP_MIXED_BF16, GAP_MIXED_FP16):
the factored matrix's Sigma^-1/2 K_NM block comes from BF16/FP16 descriptor
dot products (FP32 accumulation, FP32 power, sums and row scale).  It is
checked elementwise against the oracle's FP64 K_NM within the bound the
rounding fixes, exactly for one-hot descriptors, and the weights are reported
per refinement step against the FP64 oracle, ending within 1e-8 or in
GAP_ENOCONV."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import GpuFit, log

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-8
U32 = 2.0 ** -24


def _u(prec):
    from paper_2207_03803_amd import gap

    return {gap.GAP_MIXED_BF16: 2.0 ** -8, gap.GAP_MIXED_FP16: 2.0 ** -11}[prec]


def knm_bound(K, counts, d, zeta, prec, sigma_w=1.0):
    """Elementwise bound on |K_lp - K| for non-negative descriptors of unit norm.

    Each descriptor entry is rounded with relative error <= u (plus 2^-25 absolute
    for FP16 subnormals), products are exact in FP32, so a dot product g moves by
    <= (2u + u^2) g (+ 2^-24 sqrt(d) for FP16); g^zeta then moves by
    <= zeta (2u + u^2)(1 + 2u)^(zeta - 1) g^zeta (+ zeta 2^-24 sqrt(d), g <= 1).
    All terms are non-negative, so the relative part carries over to the
    per-configuration sums.  FP32 accumulation over d terms, the power, the sum
    over n_A atoms and the row scale add (d + zeta + n_A + 3) u_32 relative."""
    from paper_2207_03803_amd import gap

    u = _u(prec)
    n_a = np.asarray(counts, dtype=float)[:, None]
    rel = 1.01 * zeta * (2 * u + u * u) * (1 + 2 * u) ** (zeta - 1) + (d + zeta + n_a + 3) * U32
    absterm = 0.0
    if prec == gap.GAP_MIXED_FP16:
        absterm = 1.01 * n_a * zeta * sigma_w ** 2 * 2.0 ** -24 * np.sqrt(d)
    return np.abs(K) * rel + absterm


def _lp_top(g):
    """Sigma^-1/2 K_NM as the low-precision build left it in the FP32 copy."""
    A32 = g.h.A32_view()
    return A32[:g.M, :g.N].T.cpu().numpy().astype(np.float64)


def _check_knm(orc, X, offsets, XM, sigma, zeta, prec, label):
    g = GpuFit(X, offsets, XM, sigma, np.ones(len(offsets) - 1), zeta, precision=prec)
    g.build()
    got = _lp_top(g)
    K = orc.knm(X, offsets, XM, zeta)
    expect = K / sigma[:, None]
    counts = np.diff(offsets)
    bound = knm_bound(K, counts, X.shape[1], zeta, prec) / sigma[:, None]
    err = np.abs(got - expect)
    nz = expect != 0
    ratio = float(np.max(err / np.where(bound > 0, bound, 1.0)))
    relmax = float(np.max(err[nz] / np.abs(expect[nz]))) if nz.any() else 0.0
    log(f"  {label}: K_NM max rel err {relmax:.2e}, max err / bound {ratio:.2f}")
    assert np.all(got[~nz] == 0.0)
    assert ratio <= 1.0
    # the FP64 K_NM of the same build is untouched by the low-precision one
    top64, _ = g.A_top_and_lower()
    assert np.max(np.abs(top64[nz] - expect[nz]) / np.abs(expect[nz])) <= 1e-13
    g.h.close()
    return relmax


@pytest.fixture(scope="module")
def orc_m():
    return oracle.Oracle()


def _precs():
    from paper_2207_03803_amd import gap

    return [("bf16", gap.GAP_MIXED_BF16), ("fp16", gap.GAP_MIXED_FP16)]


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
@pytest.mark.parametrize("shape", [
    (200, (8, 64), 64, 256, 2, 0),       # tiny workload
    (300, (16, 64), 70, 333, 3, 1),      # d not a multiple of 32, M not a multiple of 128
    (1500, (16, 64), 400, 520, 4, 5),    # d = 400, zeta = 4
])
def test_lowprec_knm_within_rounding_bound(orc_m, pname, shape):
    prec = dict(_precs())[pname]
    n, atoms, d, M, zeta, seed = shape
    inp = synth.make_fit_inputs(n_configs=n, atoms=atoms, d=d, M=M, seed=seed)
    log(f"low-precision K_NM {pname}: N={n} d={d} M={M} zeta={zeta}")
    _check_knm(orc_m, inp.X, inp.offsets, inp.XM, inp.sigma, zeta, prec, pname)


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
def test_lowprec_knm_large_and_empty_configurations(orc_m, pname):
    """Configurations of more than one 256-atom chunk and empty ones."""
    prec = dict(_precs())[pname]
    rng = np.random.default_rng(19)
    counts = np.array([3, 0, 300, 17, 0, 600, 64, 1, 257, 256, 5] * 3, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    d, M, zeta = 40, 150, 2
    X = np.abs(rng.standard_normal((offsets[-1], d)))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    XM = X[rng.choice(offsets[-1], M, replace=False)]
    sigma = 1e-3 * np.maximum(counts, 1).astype(float)
    _check_knm(orc_m, X, offsets, XM, sigma, zeta, prec, f"{pname} large/empty")


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
def test_lowprec_one_hot_descriptors_are_exact(orc_m, pname):
    """x = e_p: every dot product is 0 or 1 in any precision, so K_NM holds integer
    counts; with sigma a power of two the FP32 rows equal the oracle's bit for bit."""
    prec = dict(_precs())[pname]
    rng = np.random.default_rng(8)
    d, N, M = 16, 120, 12
    counts = rng.integers(1, 40, N)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    X = np.zeros((offsets[-1], d))
    X[np.arange(offsets[-1]), rng.integers(0, d, offsets[-1])] = 1.0
    XM = np.eye(d)[:M]
    sigma = np.full(N, 0.25)
    Knm = orc_m.knm(X, offsets, XM, 3)
    g = GpuFit(X, offsets, XM, sigma, np.ones(N), 3, precision=prec)
    g.build()
    assert np.array_equal(_lp_top(g), Knm / sigma[:, None])
    g.h.close()


def _fit(inp, y, zeta, prec, iters, tol):
    from paper_2207_03803_amd import gap

    g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, precision=prec, max_refine_iters=iters,
               refine_tol=tol)
    g.build()
    g.h.solve(g.y, g.c, info=False)
    s, info = g.h.sync()
    c = g.c.cpu().numpy()
    g.h.close()
    assert s in (gap.GAP_OK, gap.GAP_ENOCONV)
    return c, s, info


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
@pytest.mark.parametrize("name,args", [
    ("tiny", (200, (8, 64), 64, 256, 2, 0)),
    ("mid-size d=400 zeta=4", (1500, (16, 64), 400, 520, 4, 5)),
])
def test_lowprec_fit_error_per_step(orc_m, pname, name, args):
    """c against the FP64 oracle after 0, 1, 2, 5, 10 and 20 refinement steps, then
    to convergence: within 1e-8 when the status is GAP_OK; GAP_ENOCONV otherwise
    (the low-precision factor may precondition too weakly; the status says so)."""
    from paper_2207_03803_amd import gap

    prec = dict(_precs())[pname]
    n, atoms, d, M, zeta, seed = args
    inp = synth.make_fit_inputs(n_configs=n, atoms=atoms, d=d, M=M, seed=seed)
    y = oracle.targets(orc_m, inp, zeta)
    ref = orc_m.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, zeta, jitter=1e-8)
    assert ref.status == 0
    rel = lambda c: float(np.linalg.norm(c - ref.c) / np.linalg.norm(ref.c))
    steps = {}
    for k in (0, 1, 2, 5, 10, 20):
        c, s, info = _fit(inp, y, zeta, prec, k, 0.0)  # tol 0: exactly k steps
        steps[k] = rel(c)
    c, s, info = _fit(inp, y, zeta, prec, 200, 1e-14)
    err = rel(c)
    log(f"  {pname} {name}: c rel err after " + ", ".join(f"{k}: {e:.1e}" for k, e in steps.items())
        + f"; final {gap.status_string(s)} after {info.refine_iters} steps ({info.cgls_iters} CGLS): {err:.2e}")
    assert steps[20] < steps[0]  # the refinement improves on the low-precision factor's solve
    if s == gap.GAP_OK:
        assert err <= TOL_MIXED
        assert abs(info.residual_norm2 - ref.loss_tail) <= 1e-8 * ref.loss_tail
    else:
        assert s == gap.GAP_ENOCONV and info.refine_iters == 200
