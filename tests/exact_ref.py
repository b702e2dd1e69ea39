"""Exact-rational solution of the sparse-GP normal equations on tiny inputs.

Independent of the oracle: it never forms A, never takes a square root and
never runs a QR.  The FP64 inputs are taken as exact binary fractions, the
kernel values, K_NM, the jittered K_MM and the normal equations
(K_MM + K_MN Sigma^-1 K_NM) c = K_MN Sigma^-1 y (Sec. Theory, Eq. GP_sparse)
are formed in exact arithmetic and solved by Gaussian elimination.
"""
from fractions import Fraction


def _kernel(a, b, zeta, sw2):
    g = sum((Fraction(p) * Fraction(q) for p, q in zip(a, b)), Fraction(0))
    return sw2 * g ** zeta


def knm_exact(X, offsets, XM, zeta, sigma_w=1.0):
    sw2 = Fraction(sigma_w) ** 2
    N = len(offsets) - 1
    return [[sum((_kernel(X[i], XM[j], zeta, sw2) for i in range(offsets[A], offsets[A + 1])),
                 Fraction(0)) for j in range(len(XM))] for A in range(N)]


def kmm_exact(XM, zeta, sigma_w=1.0, jitter=0.0):
    sw2 = Fraction(sigma_w) ** 2
    M = len(XM)
    K = [[_kernel(XM[i], XM[j], zeta, sw2) for j in range(M)] for i in range(M)]
    for i in range(M):
        K[i][i] += Fraction(jitter)
    return K


def solve_exact(Amat, rhs):
    n = len(rhs)
    A = [row[:] + [rhs[i]] for i, row in enumerate(Amat)]
    for k in range(n):
        p = next(i for i in range(k, n) if A[i][k] != 0)
        A[k], A[p] = A[p], A[k]
        for i in range(k + 1, n):
            f = A[i][k] / A[k][k]
            if f:
                for j in range(k, n + 1):
                    A[i][j] -= f * A[k][j]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = A[i][n] - sum((A[i][j] * x[j] for j in range(i + 1, n)), Fraction(0))
        x[i] = s / A[i][i]
    return x


def fit_exact(X, offsets, XM, sigma, y, zeta, sigma_w=1.0, jitter=0.0):
    """Exact c of the normal equations; returns a list of Fractions."""
    Knm = knm_exact(X, offsets, XM, zeta, sigma_w)
    Kmm = kmm_exact(XM, zeta, sigma_w, jitter)
    N, M = len(Knm), len(XM)
    w = [1 / Fraction(s) ** 2 for s in sigma]
    H = [[Kmm[i][j] + sum((Knm[A][i] * w[A] * Knm[A][j] for A in range(N)), Fraction(0))
          for j in range(M)] for i in range(M)]
    r = [sum((Knm[A][i] * w[A] * Fraction(y[A]) for A in range(N)), Fraction(0)) for i in range(M)]
    return solve_exact(H, r)
