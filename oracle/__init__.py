"""Plain FP64 CPU oracle for the sparse-GP (GAP) fit — test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never calls it; the two share no code.

The arithmetic lives in ``oracle.c`` (plain loops, fixed summation order); this
module only compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORACLE_OK, ORACLE_EINVAL, ORACLE_ENOTPD, ORACLE_ENOMEM = 0, 1, 2, 3

_lib = None
_lib_path = None


def build(out: str = _LIB, defines=()) -> str:
    """Compile oracle.c with gcc (no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c11", *[f"-D{d}" for d in defines], _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _bind(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_knm.argtypes = [P, P, I64, P, I64, I64, ctypes.c_int, ctypes.c_double, P]
    lib.oracle_kmm.argtypes = [P, I64, I64, ctypes.c_int, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_cholesky.argtypes = [P, I64, P, P]
    lib.oracle_stack.argtypes = [P, P, P, P, I64, I64, P, P]
    lib.oracle_householder_qr.argtypes = [P, P, I64, I64, P]
    lib.oracle_back_substitution.argtypes = [P, I64, P, I64, P]
    lib.oracle_predict.argtypes = [P, P, I64, P, I64, I64, ctypes.c_int, ctypes.c_double, P, P]
    lib.oracle_loss.argtypes = [P, P, P, P, P, I64, I64]
    lib.oracle_loss.restype = ctypes.c_double
    lib.oracle_gradient.argtypes = [P, P, P, P, P, I64, I64, P]
    lib.oracle_fit.argtypes = [P, P, I64, P, I64, I64, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, P, P, P, P, P, P, P, P, P, P]
    lib.oracle_singular_extremes.argtypes = [P, I64, I64, ctypes.c_int, ctypes.c_double, P, P, P]
    lib.oracle_cur_leverage.argtypes = [P, I64, I64, P]
    lib.oracle_kdm.argtypes = [P, P, P, P, I64, P, P, P, I64, I64, ctypes.c_int, ctypes.c_double, P]
    for name in ("oracle_knm", "oracle_kmm", "oracle_cholesky", "oracle_stack",
                 "oracle_householder_qr", "oracle_back_substitution", "oracle_predict",
                 "oracle_gradient", "oracle_fit", "oracle_singular_extremes", "oracle_cur_leverage",
                 "oracle_kdm"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """Load (building first if needed) the oracle shared library."""
    global _lib, _lib_path
    path = path or _LIB
    if _lib is not None and _lib_path == path:
        return _lib
    if path == _LIB and (not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)):
        build(path)
    _lib = _bind(ctypes.CDLL(path))
    _lib_path = path
    return _lib


class Oracle:
    """numpy front end over one loaded copy of the oracle library."""

    def __init__(self, path: str | None = None):
        if path is None:
            self.lib = load()
        else:
            self.lib = _bind(ctypes.CDLL(path))

    @staticmethod
    def _p(a):
        return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None

    @staticmethod
    def _f64(a):
        return np.ascontiguousarray(a, dtype=np.float64)

    @staticmethod
    def _i64(a):
        return np.ascontiguousarray(a, dtype=np.int64)

    def knm(self, X, offsets, XM, zeta, sigma_w=1.0):
        X, XM, offsets = self._f64(X), self._f64(XM), self._i64(offsets)
        N, M, d = len(offsets) - 1, XM.shape[0], X.shape[1]
        K = np.empty((N, M))
        rc = self.lib.oracle_knm(self._p(X), self._p(offsets), N, self._p(XM), M, d, zeta, sigma_w,
                                 self._p(K))
        assert rc == ORACLE_OK, rc
        return K

    def kmm(self, XM, zeta, sigma_w=1.0, jitter=0.0):
        XM = self._f64(XM)
        M, d = XM.shape
        K = np.empty((M, M))
        rc = self.lib.oracle_kmm(self._p(XM), M, d, zeta, sigma_w, jitter, self._p(K))
        assert rc == ORACLE_OK, rc
        return K

    def cholesky(self, K):
        K = self._f64(K)
        M = K.shape[0]
        L = np.empty((M, M))
        fail = np.array([-1], dtype=np.int64)
        rc = self.lib.oracle_cholesky(self._p(K), M, self._p(L), self._p(fail))
        return rc, L, int(fail[0])

    def stack(self, Knm, sigma, y, L):
        Knm, sigma, y, L = map(self._f64, (Knm, sigma, y, L))
        N, M = Knm.shape
        A = np.empty((N + M, M))
        b = np.empty(N + M)
        self.lib.oracle_stack(self._p(Knm), self._p(sigma), self._p(y), self._p(L), N, M,
                              self._p(A), self._p(b))
        return A, b

    def householder_qr(self, A, b, overwrite=False):
        """(A holding R and the reflectors, Q^T b, tau).  overwrite=True factors a
        C-contiguous float64 A (and b) in place instead of copies."""
        if not (overwrite and A.flags.c_contiguous and A.dtype == np.float64):
            A = np.array(A, dtype=np.float64, order="C")
        if not (overwrite and b.flags.c_contiguous and b.dtype == np.float64):
            b = np.array(b, dtype=np.float64)
        m, n = A.shape
        tau = np.empty(n)
        rc = self.lib.oracle_householder_qr(self._p(A), self._p(b), m, n, self._p(tau))
        assert rc == ORACLE_OK, rc
        return A, b, tau

    def back_substitution(self, R, rhs):
        R = self._f64(R)
        n = len(rhs)
        c = np.empty(n)
        self.lib.oracle_back_substitution(self._p(R), R.shape[1], self._p(self._f64(rhs)), n,
                                          self._p(c))
        return c

    def singular_extremes(self, R, max_iter=2000, tol=1e-14):
        """(smax, smin, (power steps, inverse steps)) of the upper triangle of R."""
        R = self._f64(R)
        n = R.shape[0]
        smax, smin = np.zeros(1), np.zeros(1)
        its = np.zeros(2, dtype=np.int32)
        rc = self.lib.oracle_singular_extremes(self._p(R), R.shape[1], n, max_iter, tol, self._p(smax),
                                               self._p(smin), self._p(its))
        assert rc == ORACLE_OK, rc
        return float(smax[0]), float(smin[0]), (int(its[0]), int(its[1]))

    def cur_leverage(self, X):
        """Leverage of every row of X over its row space (CUR sparse-point selection,
        Sec. Implementation): lev[i] = x_i^T (X^T X)^-1 x_i.  Raises on a rank-deficient X."""
        X = self._f64(X)
        lev = np.empty(X.shape[0])
        rc = self.lib.oracle_cur_leverage(self._p(X), X.shape[0], X.shape[1], self._p(lev))
        if rc != ORACLE_OK:
            raise np.linalg.LinAlgError(f"oracle_cur_leverage: status {rc}")
        return lev

    def cur_select(self, X, M, draws=None, lev=None):
        """The M sparse points CUR selection takes from the rows of X, ascending.

        Without draws: the M rows of largest leverage.  With draws (one Exp(1)
        variate per row, drawn by the caller): M rows sampled without replacement
        with probability proportional to the leverage, by the exponential-key
        method of Efraimidis & Spirakis (the M smallest draws[i] / lev[i]).  The
        key is draws[i] / lev[i] (1 / lev[i] without draws); equal keys are taken
        in row order.  Returns (indices, keys, lev)."""
        if lev is None:
            lev = self.cur_leverage(X)
        with np.errstate(divide="ignore"):
            keys = (np.asarray(draws, dtype=np.float64) if draws is not None else np.ones(len(lev))) / lev
        order = np.argsort(keys, kind="stable")  # library sort; ties keep row order
        return np.sort(order[:M]), keys, lev

    def kdm(self, X, x_grad, grad_atom, obs_offsets, pos_grad, pos_weight, XM, zeta, sigma_w=1.0):
        """Derivative observation rows of K [n_obs x M] (forces, virials)."""
        X, x_grad, XM, pos_weight = map(self._f64, (X, x_grad, XM, pos_weight))
        grad_atom, obs_offsets, pos_grad = map(self._i64, (grad_atom, obs_offsets, pos_grad))
        n_obs, M, d = len(obs_offsets) - 1, XM.shape[0], X.shape[1]
        K = np.empty((n_obs, M))
        rc = self.lib.oracle_kdm(self._p(X), self._p(x_grad), self._p(grad_atom), self._p(obs_offsets), n_obs,
                                 self._p(pos_grad), self._p(pos_weight), self._p(XM), M, d, zeta, sigma_w,
                                 self._p(K))
        assert rc == ORACLE_OK, rc
        return K

    def fit_deriv(self, D, y, zeta, sigma_w=1.0, jitter=1e-8):
        """The fit with energy and derivative rows (synth.DerivInputs D, targets y of
        all N_E + n_obs rows), in the paper's order: K_NM, the derivative rows, K_MM +
        jitter, Cholesky, the stacked problem A = [Sigma^-1/2 [K_NM ; K_D] ; L^T],
        Householder QR with Q^T b, back-substitution.  Returns (c, loss_tail, K_all)."""
        Knm = self.knm(D.X, D.offsets, D.XM, zeta, sigma_w)
        Kd = self.kdm(D.X, D.x_grad, D.grad_atom, D.obs_offsets, D.pos_grad, D.pos_weight, D.XM, zeta, sigma_w)
        K = np.vstack([Knm, Kd])
        rc, L, fail = self.cholesky(self.kmm(D.XM, zeta, sigma_w, jitter))
        assert rc == ORACLE_OK, (rc, fail)
        A, b = self.stack(K, D.sigma, y, L)
        A, qtb, _ = self.householder_qr(A, b, overwrite=True)
        M = K.shape[1]
        c = self.back_substitution(A, qtb[:M])
        return c, float(np.sum(qtb[M:] ** 2)), K

    def predict(self, X, offsets, XM, c, zeta, sigma_w=1.0):
        X, XM, c, offsets = self._f64(X), self._f64(XM), self._f64(c), self._i64(offsets)
        N, M, d = len(offsets) - 1, XM.shape[0], X.shape[1]
        y = np.empty(N)
        self.lib.oracle_predict(self._p(X), self._p(offsets), N, self._p(XM), M, d, zeta, sigma_w,
                                self._p(c), self._p(y))
        return y

    def loss(self, Knm, sigma, y, Kmm, c):
        Knm, sigma, y, Kmm, c = map(self._f64, (Knm, sigma, y, Kmm, c))
        return self.lib.oracle_loss(self._p(Knm), self._p(sigma), self._p(y), self._p(Kmm),
                                    self._p(c), Knm.shape[0], Knm.shape[1])

    def gradient(self, Knm, sigma, y, Kmm, c):
        Knm, sigma, y, Kmm, c = map(self._f64, (Knm, sigma, y, Kmm, c))
        g = np.empty(Knm.shape[1])
        self.lib.oracle_gradient(self._p(Knm), self._p(sigma), self._p(y), self._p(Kmm),
                                 self._p(c), Knm.shape[0], Knm.shape[1], self._p(g))
        return g

    def fit(self, X, offsets, XM, sigma, y, zeta, sigma_w=1.0, jitter=1e-8, keep=False):
        X, XM, sigma, y = map(self._f64, (X, XM, sigma, y))
        offsets = self._i64(offsets)
        N, M, d = len(offsets) - 1, XM.shape[0], X.shape[1]
        c = np.empty(M)
        tail = np.zeros(1)
        diagR = np.empty(M)
        extra = dict(Knm=None, L=None, A=None, qtb=None, tau=None)
        if keep:
            extra = dict(Knm=np.empty((N, M)), L=np.empty((M, M)), A=np.empty((N + M, M)),
                         qtb=np.empty(N + M), tau=np.empty(M))
        rc = self.lib.oracle_fit(self._p(X), self._p(offsets), N, self._p(XM), M, d, zeta, sigma_w,
                                 jitter, self._p(sigma), self._p(y), self._p(c), self._p(tail),
                                 self._p(diagR), self._p(extra["Knm"]), self._p(extra["L"]),
                                 self._p(extra["A"]), self._p(extra["qtb"]), self._p(extra["tau"]))
        return FitResult(rc, c, float(tail[0]), diagR, **extra)


@dataclass
class FitResult:
    status: int
    c: np.ndarray
    loss_tail: float
    diagR: np.ndarray
    Knm: np.ndarray | None = None
    L: np.ndarray | None = None
    A: np.ndarray | None = None
    qtb: np.ndarray | None = None
    tau: np.ndarray | None = None


def deriv_targets(orc: Oracle, D, zeta, sigma_w=1.0):
    """y for every row of a synth.DerivInputs: K c_true + sigma * noise (energies,
    then derivative observations), computed by the oracle."""
    yE = orc.predict(D.X, D.offsets, D.XM, D.c_true, zeta, sigma_w)
    Kd = orc.kdm(D.X, D.x_grad, D.grad_atom, D.obs_offsets, D.pos_grad, D.pos_weight, D.XM, zeta, sigma_w)
    return np.concatenate([yE, Kd @ D.c_true]) + D.sigma * np.concatenate([D.noise_E, D.noise_D])


def targets(orc: Oracle, inputs, zeta, sigma_w=1.0):
    """y = prediction with c_true plus sigma * noise, computed by the oracle."""
    y0 = orc.predict(inputs.X, inputs.offsets, inputs.XM, inputs.c_true, zeta, sigma_w)
    return y0 + inputs.sigma * inputs.noise
