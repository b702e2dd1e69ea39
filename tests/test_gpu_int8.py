"""The FP64 K_NM from descriptor dot products emulated on INT8 MFMA
(GAP_FLAG_KNM_INT8, Ozaki scheme) against the oracle's FP64 K_NM (K_MN
definition, Sec. Theory): elementwise within 1e-13 for non-negative
descriptors, within 1e-13 of the sum of absolute terms for signed ones and
rows of very different scale, exact for one-hot descriptors; rows permute with
the configurations bit for bit; the weights of FP64 and mixed fits built on it
match the oracle's like those of the FP64 build."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth
from tests.gpu_helpers import GpuFit, log, to_dev

pytestmark = pytest.mark.gpu

TOL_K = 1e-13


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _int8_fit(inp_X, offsets, XM, sigma, y, zeta, **kw):
    from paper_2207_03803_amd import gap

    return GpuFit(inp_X, offsets, XM, sigma, y, zeta, flags=gap.GAP_FLAG_KNM_INT8, **kw)


def _knm_top(g):
    top, _ = g.A_top_and_lower()
    return top


@pytest.mark.parametrize("n_configs,atoms,d,M,zeta,seed", [
    (200, (8, 64), 64, 256, 2, 0),      # the tiny workload
    (150, (1, 9), 37, 70, 3, 1),        # d not a multiple of 64, one-atom configurations, M < one tile
    (120, (200, 300), 100, 140, 2, 2),  # configurations over one 256-atom tile
    (1500, (16, 64), 400, 520, 4, 3),   # realistic d and zeta, several column tiles and groups
])
def test_int8_knm_matches_oracle_elementwise(orc, n_configs, atoms, d, M, zeta, seed):
    inp = synth.make_fit_inputs(n_configs=n_configs, atoms=atoms, d=d, M=M, seed=seed)
    log(f"INT8 K_NM: N={n_configs} atoms {atoms} d={d} M={M} zeta={zeta}")
    g = _int8_fit(inp.X, inp.offsets, inp.XM, inp.sigma, np.ones(n_configs), zeta)
    g.build()
    got = _knm_top(g)
    expect = orc.knm(inp.X, inp.offsets, inp.XM, zeta) / inp.sigma[:, None]
    err = np.max(np.abs(got - expect) / np.abs(expect))
    log(f"  max elementwise rel err {err:.2e}")
    assert err <= TOL_K
    _, low = g.A_top_and_lower()
    Lt = np.linalg.cholesky(orc.kmm(inp.XM, zeta, 1.0, 1e-8)).T
    assert np.linalg.norm(low - Lt) / np.linalg.norm(Lt) <= 1e-12


def test_int8_knm_large_and_empty_configurations(orc):
    """Configurations over one and two 128-atom chunks of the kernel's tile, ending at
    or just past a chunk boundary, and empty ones between, before and after them: each
    row once, empty ones zero."""
    rng = np.random.default_rng(19)
    counts = np.array([0, 3, 0, 300, 17, 0, 0, 600, 128, 0, 129, 1, 257, 256, 0, 5, 0] * 2, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    d, M, zeta = 40, 150, 3
    X = rng.standard_normal((offsets[-1], d))
    XM = X[rng.choice(offsets[-1], M, replace=False)]
    sigma = 1e-3 * np.maximum(counts, 1).astype(float)
    log("INT8 K_NM: large and empty configurations, d=40, M=150")
    g = _int8_fit(X, offsets, XM, sigma, np.ones(len(counts)), zeta, jitter=1e-6)
    g.build()
    got = _knm_top(g) * sigma[:, None]
    expect = orc.knm(X, offsets, XM, zeta)
    scale = orc.knm(np.abs(X), offsets, np.abs(XM), zeta)
    empty = counts == 0
    assert np.all(got[empty] == 0.0)
    err = np.max(np.abs(got[~empty] - expect[~empty]) / scale[~empty])
    log(f"  max rel err (to the sum of absolute terms) {err:.2e}")
    assert err <= TOL_K


def test_int8_knm_signed_and_rescaled_rows(orc):
    """Entries of both signs and rows scaled by powers of two from 2^-40 to 2^40
    (each row's slices carry their own exponent): the error is bounded by 1e-13 of
    sigma_w^2 sum_i (|x_i| . |x_j|)^zeta, the oracle's K_NM of the absolute values."""
    rng = np.random.default_rng(7)
    inp = synth.make_fit_inputs(n_configs=300, atoms=(4, 40), d=96, M=150, seed=7)
    X = inp.X * rng.choice([-1.0, 1.0], size=inp.X.shape) * np.exp2(rng.integers(-40, 41, size=(inp.X.shape[0], 1)))
    XM = inp.XM * rng.choice([-1.0, 1.0], size=inp.XM.shape)
    for zeta in (1, 3):
        g = _int8_fit(X, inp.offsets, XM, inp.sigma, np.ones(300), zeta, jitter=1e-6)
        g.build()
        got = _knm_top(g) * inp.sigma[:, None]
        expect = orc.knm(X, inp.offsets, XM, zeta)
        scale = orc.knm(np.abs(X), inp.offsets, np.abs(XM), zeta)
        err = np.max(np.abs(got - expect) / scale)
        log(f"  signed, rescaled rows, zeta={zeta}: max |err| / sum of |terms| {err:.2e}")
        assert err <= TOL_K


def test_int8_knm_one_hot_counts_are_exact(orc):
    """One-hot descriptors: every dot product is 0 or 1, so K_NM holds integer
    counts of the sparse points' species in each configuration, exactly."""
    rng = np.random.default_rng(8)
    counts = rng.integers(1, 50, size=80)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    d = 16
    species = rng.integers(0, d, size=offsets[-1])
    X = np.eye(d)[species]
    XM = np.eye(d)[rng.integers(0, d, size=40)]
    sigma = np.ones(80)
    g = _int8_fit(X, offsets, XM, sigma, np.ones(80), 2, jitter=1.0)
    g.build()
    got = _knm_top(g)
    expect = orc.knm(X, offsets, XM, 2)
    assert np.array_equal(got, expect)


def test_int8_configuration_order_gives_the_same_rows_bitwise():
    inp = synth.make_fit_inputs(n_configs=400, atoms=(8, 64), d=64, M=130, seed=9)
    perm = np.random.default_rng(10).permutation(400)
    counts = np.diff(inp.offsets)
    rows = np.concatenate([np.arange(inp.offsets[a], inp.offsets[a + 1]) for a in perm])
    offs_p = np.concatenate([[0], np.cumsum(counts[perm])]).astype(np.int64)
    a = _int8_fit(inp.X, inp.offsets, inp.XM, inp.sigma, np.ones(400), 2)
    a.build()
    b = _int8_fit(inp.X[rows], offs_p, inp.XM, inp.sigma[perm], np.ones(400), 2)
    b.build()
    assert np.array_equal(_knm_top(a)[perm], _knm_top(b))


@pytest.mark.parametrize("precision", [0, 1])
def test_int8_fit_weights_match_oracle(orc, precision):
    """FP64 (c within 1e-10) and mixed FP32 (within 1e-8) fits whose FP64 K_NM
    comes from INT8 slice products, at d=400, zeta=4."""
    inp = synth.make_fit_inputs(n_configs=2000, atoms=(16, 64), d=400, M=520, seed=5)
    y = oracle.targets(orc, inp, 4)
    ref = orc.fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 4, jitter=1e-8)
    g = _int8_fit(inp.X, inp.offsets, inp.XM, inp.sigma, y, 4, precision=precision, max_refine_iters=30)
    c, info = g.run()
    assert info.device_status == 0
    err = rel(c, ref.c)
    log(f"  INT8 K_NM, precision {precision}: c rel err vs oracle {err:.2e}; eta {info.grad_rel:.1e}")
    assert err <= (1e-10 if precision == 0 else 1e-8)


def test_int8_fits_in_a_batch_match_their_own_builds():
    """gap_build_knm_batch over handles with and without GAP_FLAG_KNM_INT8: every
    stacked matrix equals the one its own gap_build_knm leaves, bit for bit."""
    import torch

    from paper_2207_03803_amd import gap

    fits = []
    for i, flags in enumerate((gap.GAP_FLAG_KNM_INT8, 0, gap.GAP_FLAG_KNM_INT8)):
        inp = synth.make_fit_inputs(n_configs=150 + 40 * i, atoms=(8, 64), d=64, M=100 + 30 * i, seed=20 + i)
        g = GpuFit(inp.X, inp.offsets, inp.XM, inp.sigma, np.ones(inp.n_configs), 2, flags=flags)
        fits.append(g)
    own = []
    for g in fits:
        g.build()
        torch.cuda.synchronize()
        Av, lay = g.h.A_view()
        own.append(Av[:lay.M, :lay.N + lay.M].cpu().numpy())
    gap.build_knm_batch([g.h for g in fits], [(g.X, g.offsets, g.XM, g.sigma) for g in fits])
    torch.cuda.synchronize()
    for g in fits:
        g.h.build_kmm()
    torch.cuda.synchronize()
    for g, a in zip(fits, own):
        Av, lay = g.h.A_view()
        assert np.array_equal(Av[:lay.M, :lay.N + lay.M].cpu().numpy(), a)
