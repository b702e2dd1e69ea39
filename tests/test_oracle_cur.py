"""Pins of the oracle's CUR sparse-point selection (Sec. Implementation: CUR-based
selection of the sparse points, after Mahoney & Drineas 2009): the leverage of a
descriptor row over the row space of X against an independent route (the row
norms of Q from LAPACK's QR), its closed forms and invariances, and the selection
against brute force and against the sampling law it implements."""
import numpy as np
import pytest

import oracle
from paper_2207_03803_amd import synth


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _x(n, d, seed):
    X = synth.make_fit_inputs(n_configs=(n + 29) // 30, atoms=(30, 30), d=d, M=1, seed=seed).X[:n]
    assert X.shape == (n, d)
    return X


def test_leverage_equals_row_norms_of_q(orc):
    """lev[i] = ||Q[i]||^2 for X = QR (LAPACK's Householder QR, another route to the
    hat matrix's diagonal), and the leverages sum to d (its trace)."""
    for n, d, seed in ((600, 20, 0), (3000, 64, 1), (900, 37, 2)):
        X = _x(n, d, seed)
        lev = orc.cur_leverage(X)
        Q, _ = np.linalg.qr(X)
        assert np.max(np.abs(lev - np.sum(Q * Q, axis=1))) <= 1e-12
        assert abs(lev.sum() - d) <= 1e-10 * d
        assert np.all(lev >= 0) and np.all(lev <= 1 + 1e-12)


def test_leverage_closed_forms(orc):
    """Orthonormal columns: lev[i] = ||x_i||^2.  X = [I_d ; 0]: one for the first d
    rows, zero for the rest.  A single column: x_i^2 / ||x||^2."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((400, 12)))
    assert np.max(np.abs(orc.cur_leverage(Q) - np.sum(Q * Q, axis=1))) <= 1e-14
    E = np.vstack([np.eye(9), np.zeros((31, 9))])
    assert np.array_equal(orc.cur_leverage(E), np.concatenate([np.ones(9), np.zeros(31)]))
    x = rng.standard_normal((50, 1))
    assert np.max(np.abs(orc.cur_leverage(x) - x[:, 0] ** 2 / np.sum(x * x))) <= 1e-15


def test_leverage_invariances(orc):
    """The row space does not change under X -> X S (S invertible), and permuting
    the rows permutes the leverages."""
    X = _x(800, 24, 4)
    lev = orc.cur_leverage(X)
    rng = np.random.default_rng(5)
    S = np.triu(rng.standard_normal((24, 24))) + 4 * np.eye(24)
    assert np.max(np.abs(orc.cur_leverage(X @ S) - lev)) <= 1e-12
    assert np.max(np.abs(orc.cur_leverage(X * np.exp2(rng.integers(-30, 30, 24))) - lev)) <= 1e-12
    perm = rng.permutation(800)
    assert np.max(np.abs(orc.cur_leverage(X[perm]) - lev[perm])) <= 1e-14


def test_rank_deficient_rows_are_reported(orc):
    X = _x(300, 10, 6)
    X[:, 7] = X[:, 2]
    with pytest.raises(np.linalg.LinAlgError):
        orc.cur_leverage(X)


def test_selection_against_brute_force(orc):
    """The selected rows are the M smallest keys (draws / lev, or 1 / lev without
    draws), equal keys in row order, returned ascending; zero rows (lev = 0, key
    +inf) come last; M = n takes every row."""
    X = _x(200, 8, 7)
    X[[5, 50, 150]] = 0.0
    X[60] = X[61]  # equal leverages
    rng = np.random.default_rng(8)
    draws = rng.standard_exponential(200)
    lev = orc.cur_leverage(X)
    for M in (1, 17, 196, 197, 200):
        for dr in (None, draws):
            idx, keys, _ = orc.cur_select(X, M, draws=dr, lev=lev)
            brute = sorted(range(200), key=lambda i: (keys[i], i))[:M]
            assert list(idx) == sorted(brute)
            if M <= 197:
                assert not set(idx) & {5, 50, 150}
    top, _, _ = orc.cur_select(X, 2, lev=lev)  # without draws: the largest leverages
    assert set(top) == set(sorted(range(200), key=lambda i: (-lev[i], i))[:2])


def test_selection_samples_rows_in_proportion_to_leverage(orc):
    """With M = 1 the exponential keys pick row i with probability lev[i] / sum(lev):
    over 40,000 independent draws the frequencies match within 5 standard errors
    (a key such as draws * lev, or draws / lev^2, fails this)."""
    X = _x(12, 4, 9)
    lev = orc.cur_leverage(X)
    p = lev / lev.sum()
    rng = np.random.default_rng(10)
    trials = 40_000
    draws = rng.standard_exponential((trials, 12))
    picks = np.argmin(draws / lev, axis=1)
    freq = np.bincount(picks, minlength=12) / trials
    se = np.sqrt(p * (1 - p) / trials)
    assert np.all(np.abs(freq - p) <= 5 * se + 1e-12)
    for t in range(50):  # the oracle's own selection agrees with argmin
        assert orc.cur_select(X, 1, draws=draws[t], lev=lev)[0][0] == picks[t]
