"""Pins of the oracle's derivative observation rows (forces and virials; Sec.
Theory: derivative targets follow by differentiating the energy expression)
against central finite differences of the oracle's energies under the synthetic
descriptor model, the zeta = 1 closed form, translation invariance, and the fit
with derivative rows against LAPACK's least squares."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


@pytest.fixture(scope="module")
def data():
    return synth.make_deriv_inputs(8, atoms=(16, 24), d=24, M=40, n_neigh=6, seed=4)


def _kd(orc, D, zeta, sigma_w=1.0):
    return orc.kdm(D.X, D.x_grad, D.grad_atom, D.obs_offsets, D.pos_grad, D.pos_weight, D.XM, zeta, sigma_w)


def _energy(orc, D, R, c, zeta, sigma_w):
    X = synth.deriv_descriptors(R, D.offsets, D.species, D.nb, D.U0, D.U)
    return orc.predict(X, D.offsets, D.XM, c, zeta, sigma_w)  # per configuration


@pytest.mark.parametrize("zeta,sigma_w", [(1, 1.0), (2, 0.7), (4, 1.3)])
def test_force_rows_match_finite_differences(orc, data, zeta, sigma_w):
    """(K_F c)[k, alpha] = -dE/dr_{k, alpha} for every atom and direction, E the
    oracle's energy of the configuration at positions moved by +-h."""
    D = data
    c = np.random.default_rng(1).standard_normal(D.XM.shape[0])
    F = (_kd(orc, D, zeta, sigma_w) @ c)[:3 * D.n_atoms].reshape(D.n_atoms, 3)
    h = 1e-5
    cfg = np.repeat(np.arange(D.n_configs), np.diff(D.offsets))
    fd = np.empty_like(F)
    for k in range(D.n_atoms):
        for al in range(3):
            Rp, Rm = D.R.copy(), D.R.copy()
            Rp[k, al] += h
            Rm[k, al] -= h
            a = cfg[k]
            fd[k, al] = -(_energy(orc, D, Rp, c, zeta, sigma_w)[a] - _energy(orc, D, Rm, c, zeta, sigma_w)[a]) / (2 * h)
    assert np.max(np.abs(F - fd)) <= 1e-6 * np.max(np.abs(F))


def test_virial_rows_match_finite_differences_of_strain(orc, data):
    """(K_V c)[a, alpha, beta] = -dE_a/d eps for the homogeneous strain
    r_{k, beta} += eps r_{k, alpha} of configuration a (alpha <= beta)."""
    D, zeta = data, 3
    c = np.random.default_rng(2).standard_normal(D.XM.shape[0])
    V = (_kd(orc, D, zeta) @ c)[3 * D.n_atoms:].reshape(D.n_configs, 6)
    comps = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    h = 1e-6
    for a in range(D.n_configs):
        lo, hi = D.offsets[a], D.offsets[a + 1]
        for ci, (al, be) in enumerate(comps):
            Rp, Rm = D.R.copy(), D.R.copy()
            Rp[lo:hi, be] += h * D.R[lo:hi, al]
            Rm[lo:hi, be] -= h * D.R[lo:hi, al]
            fd = -(_energy(orc, D, Rp, c, zeta, 1.0)[a] - _energy(orc, D, Rm, c, zeta, 1.0)[a]) / (2 * h)
            assert abs(V[a, ci] - fd) <= 1e-6 * max(1.0, abs(fd)), (a, al, be)


def test_zeta_one_is_a_weighted_gradient_sum(orc, data):
    """zeta = 1: K_D[o] = sigma_w^2 sum_p w_p x'_{g(p)} . X_M^T (linear in the gradients)."""
    D = data
    W = np.zeros((D.n_obs, D.x_grad.shape[0]))
    o_of_p = np.repeat(np.arange(D.n_obs), np.diff(D.obs_offsets))
    np.add.at(W, (o_of_p, D.pos_grad), D.pos_weight)
    expect = 0.49 * (W @ D.x_grad) @ D.XM.T
    got = _kd(orc, D, 1, 0.7)
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.max(np.abs(expect))


def test_forces_sum_to_zero_per_configuration(orc, data):
    """E is unchanged by a translation of a configuration, so its force rows sum to
    zero in each direction (for every sparse point)."""
    D = data
    K = _kd(orc, D, 4)[:3 * D.n_atoms].reshape(D.n_atoms, 3, -1)
    scale = np.max(np.abs(K))
    for a in range(D.n_configs):
        s = K[D.offsets[a]:D.offsets[a + 1]].sum(axis=0)
        assert np.max(np.abs(s)) <= 1e-12 * scale


def test_fit_with_derivative_rows_against_lstsq(orc, data):
    """The staged fit on [energies ; forces ; virials ; L^T] against LAPACK's least
    squares on the same stacked matrix (within the FP64 perturbation bound; kappa(A)
    is about 6e7 here), and its normal-equation residual."""
    D, zeta = data, 2
    y = oracle.deriv_targets(orc, D, zeta)
    c, tail, K = orc.fit_deriv(D, y, zeta)
    rc, L, _ = orc.cholesky(orc.kmm(D.XM, zeta, 1.0, 1e-8))
    A, b = orc.stack(K, D.sigma, y, L)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    r = b - A @ c
    sv = np.linalg.svd(A, compute_uv=False)
    kappa, u = sv[0] / sv[-1], 2.0 ** -53
    bound = 32 * u * (kappa + kappa ** 2 * np.linalg.norm(r) / (sv[0] * np.linalg.norm(c)))
    assert np.linalg.norm(c - ref) / np.linalg.norm(ref) <= bound
    assert abs(r @ r - tail) <= 1e-9 * tail
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A.T @ r) / (nA * (nA * np.linalg.norm(c) + np.linalg.norm(b))) <= 1e-14
