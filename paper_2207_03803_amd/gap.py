"""Thin ctypes binding of libgap.so (declared in include/gap.h).

Argument marshalling only: every step of the fit runs in the library's HIP
kernels.  PyTorch supplies device memory (tensor data pointers) and streams.
The library must have been built (``python -m paper_2207_03803_amd.build``);
loading fails loudly otherwise, and nothing here falls back to a CPU path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgap.so")

GAP_OK, GAP_EINVAL, GAP_ENOMEM, GAP_ENOTPD, GAP_ENONFINITE, GAP_ENOCONV, GAP_EDEVICE, GAP_ESTATE, GAP_ERANK = range(9)
GAP_FP64, GAP_MIXED_FP32, GAP_MIXED_BF16, GAP_MIXED_FP16 = 0, 1, 2, 3
GAP_FLAG_TIMING = 1
GAP_FLAG_ERROR_ESTIMATE = 2
GAP_FLAG_KNM_INT8 = 4
GAP_FLAG_POISON_WORKSPACE = 8

# Every entry point include/gap.h declares.
EXPORTS = ["gap_create", "gap_workspace_bytes", "gap_bind_workspace", "gap_build_knm", "gap_solve",
           "gap_predict", "gap_sync", "gap_layout", "gap_stage_times", "gap_status_string",
           "gap_set_tuning", "gap_set_model", "gap_set_stream", "gap_destroy", "gap_fit_static",
           "gap_static_scratch_bytes", "gap_build_knm_batch", "gap_build_kmm", "gap_cur_workspace_bytes",
           "gap_cur_select", "gap_workspace_bytes_obs", "gap_build_knm_obs"]

STAGES = ["knm", "kmm", "cholesky", "assemble_b", "qr", "trsv", "refine", "knm_lp", "diag", "kdm"]


class GapParams(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("zeta", ctypes.c_int32), ("sigma_w", ctypes.c_double),
                ("jitter", ctypes.c_double), ("precision", ctypes.c_int32),
                ("max_refine_iters", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


class GapSolveInfo(ctypes.Structure):
    _fields_ = [("device_status", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
                ("residual_norm2", ctypes.c_double), ("grad_rel", ctypes.c_double),
                ("cgls_iters", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("step_rel", ctypes.c_double), ("est_err", ctypes.c_double), ("kappa_est", ctypes.c_double)]


class GapBatchFit(ctypes.Structure):
    _fields_ = [("x_atoms", ctypes.c_void_p), ("n_atoms", ctypes.c_int64), ("config_offsets", ctypes.c_void_p),
                ("n_configs", ctypes.c_int64), ("x_sparse", ctypes.c_void_p), ("M", ctypes.c_int64),
                ("sigma", ctypes.c_void_p)]


class GapDerivObs(ctypes.Structure):
    _fields_ = [("x_grad", ctypes.c_void_p), ("n_grad", ctypes.c_int64), ("grad_atom", ctypes.c_void_p),
                ("obs_offsets", ctypes.c_void_p), ("n_obs", ctypes.c_int64), ("pos_grad", ctypes.c_void_p),
                ("pos_weight", ctypes.c_void_p), ("n_pos", ctypes.c_int64)]


class GapTuning(ctypes.Structure):
    _fields_ = [("qr_split_wgs", ctypes.c_int32), ("qr_panel", ctypes.c_int32), ("qr_lookahead", ctypes.c_int32),
                ("qr_free_cus", ctypes.c_int32), ("knm_bn", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class GapLayoutInfo(ctypes.Structure):
    _fields_ = [("A_aug", ctypes.c_void_p), ("lda", ctypes.c_int64), ("ncols", ctypes.c_int64),
                ("N", ctypes.c_int64), ("M", ctypes.c_int64), ("n_atoms", ctypes.c_int64),
                ("tau", ctypes.c_void_p), ("device_status", ctypes.c_void_p), ("A32", ctypes.c_void_p)]


class GapError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def lib():
    """Load libgap.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2207_03803_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.gap_create.argtypes = [ctypes.POINTER(GapParams), P, ctypes.POINTER(P)]
    L.gap_workspace_bytes.argtypes = [ctypes.POINTER(GapParams), I64, I64, I64]
    L.gap_workspace_bytes.restype = ctypes.c_size_t
    L.gap_bind_workspace.argtypes = [P, P, ctypes.c_size_t]
    L.gap_build_knm.argtypes = [P, P, I64, P, I64, P, I64, P]
    L.gap_solve.argtypes = [P, P, P, ctypes.POINTER(GapSolveInfo)]
    L.gap_predict.argtypes = [P, P, I64, P, I64, P, P]
    L.gap_sync.argtypes = [P, ctypes.POINTER(GapSolveInfo)]
    L.gap_layout.argtypes = [P, ctypes.POINTER(GapLayoutInfo)]
    L.gap_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_float), I32]
    L.gap_status_string.argtypes = [I32]
    L.gap_status_string.restype = ctypes.c_char_p
    L.gap_destroy.argtypes = [P]
    L.gap_set_tuning.argtypes = [P, ctypes.POINTER(GapTuning)]
    L.gap_set_model.argtypes = [P, P, I64]
    L.gap_set_stream.argtypes = [P, P]
    L.gap_fit_static.argtypes = [ctypes.POINTER(GapParams), P, P, I64, P, I64, P, I64, P, P, P,
                                 ctypes.POINTER(GapSolveInfo)]
    L.gap_fit_static.restype = I32
    L.gap_static_scratch_bytes.argtypes = []
    L.gap_static_scratch_bytes.restype = ctypes.c_size_t
    L.gap_build_knm_batch.argtypes = [ctypes.POINTER(P), I32, ctypes.POINTER(GapBatchFit), P]
    L.gap_build_knm_batch.restype = I32
    L.gap_build_kmm.argtypes = [P]
    L.gap_build_kmm.restype = I32
    L.gap_workspace_bytes_obs.argtypes = [ctypes.POINTER(GapParams), I64, I64, I64, I64, I64]
    L.gap_workspace_bytes_obs.restype = ctypes.c_size_t
    L.gap_build_knm_obs.argtypes = [P, P, I64, P, I64, ctypes.POINTER(GapDerivObs), P, I64, P]
    L.gap_build_knm_obs.restype = I32
    L.gap_cur_workspace_bytes.argtypes = [I64, I32]
    L.gap_cur_workspace_bytes.restype = ctypes.c_size_t
    L.gap_cur_select.argtypes = [P, I64, I32, P, I64, P, P, P, ctypes.c_size_t, P, I32]
    L.gap_cur_select.restype = I32
    for n in ("gap_create", "gap_bind_workspace", "gap_build_knm", "gap_solve", "gap_predict", "gap_sync",
              "gap_layout", "gap_stage_times", "gap_set_tuning", "gap_set_model", "gap_set_stream",
              "gap_destroy"):
        getattr(L, n).restype = I32
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().gap_status_string(int(s)).decode()


def params(d, zeta, sigma_w=1.0, jitter=1e-8, precision=GAP_FP64, max_refine_iters=20,
           refine_tol=1e-12, flags=0) -> GapParams:
    return GapParams(d, zeta, sigma_w, jitter, precision, max_refine_iters, refine_tol, flags)


def workspace_bytes(p: GapParams, n_configs: int, n_atoms: int, M: int) -> int:
    return int(lib().gap_workspace_bytes(ctypes.byref(p), n_configs, n_atoms, M))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check(s, where):
    if s != GAP_OK:
        raise GapError(s, where)


def fit_static(p: GapParams, X, offsets, XM, sigma, y, c_out, info=True, stream=None):
    """gap_fit_static: one fit with the library's static scratch (no workspace,
    no handle).  Returns the GapSolveInfo (info=True: waits for the stream)."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream()
    inf = GapSolveInfo() if info else None
    s = lib().gap_fit_static(ctypes.byref(p), ctypes.c_void_p(st.cuda_stream), _ptr(X), X.shape[0], _ptr(offsets),
                             offsets.numel() - 1, _ptr(XM), XM.shape[0], _ptr(sigma), _ptr(y), _ptr(c_out),
                             ctypes.byref(inf) if info else None)
    _check(s, "gap_fit_static")
    return inf


def build_knm_batch(handles, inputs, stream=None):
    """gap_build_knm_batch: the K_NM of every fit as grouped launches on `stream`
    (torch stream, default: the current one).  inputs[i] = (X, offsets, XM, sigma)
    for handles[i]; each handle keeps its tensors alive until its next build.
    Each handle then needs build_kmm() on its own stream, ordered after `stream`."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream()
    n = len(handles)
    fits = (GapBatchFit * n)()
    hs = (ctypes.c_void_p * n)()
    for i, (h, (X, offsets, XM, sigma)) in enumerate(zip(handles, inputs)):
        h._inputs = (X, offsets, XM, sigma)
        hs[i] = h.h
        fits[i] = GapBatchFit(X.data_ptr(), X.shape[0], offsets.data_ptr(), offsets.numel() - 1, XM.data_ptr(),
                              XM.shape[0], sigma.data_ptr())
    _check(lib().gap_build_knm_batch(hs, n, fits, ctypes.c_void_p(st.cuda_stream)), "gap_build_knm_batch")


def cur_workspace_bytes(n_rows: int, d: int) -> int:
    return int(lib().gap_cur_workspace_bytes(int(n_rows), int(d)))


def cur_select(X, M, draws=None, leverage=False, stream=None, workspace=None, wait=True):
    """gap_cur_select: CUR sparse-point selection over the rows of X (n x d device
    FP64).  draws: Exp(1) variates per row (device FP64) or None for the M rows of
    largest leverage.  Returns (selected row indices [M] int64, leverage [n] or
    None).  wait=True synchronises and raises on a device error (GAP_ENOTPD for a
    rank-deficient X)."""
    import torch

    n, d = X.shape
    st = stream if stream is not None else torch.cuda.current_stream()
    nb = cur_workspace_bytes(n, d)
    if nb == 0:
        raise GapError(GAP_EINVAL, "gap_cur_workspace_bytes")
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=X.device)
    out = torch.empty(int(M), dtype=torch.int64, device=X.device)
    lev = torch.empty(n, dtype=torch.float64, device=X.device) if leverage else None
    _check(lib().gap_cur_select(_ptr(X), n, d, _ptr(draws) if draws is not None else None, int(M), _ptr(out),
                                _ptr(lev) if lev is not None else None, _ptr(workspace), workspace.numel(),
                                ctypes.c_void_p(st.cuda_stream), 1 if wait else 0), "gap_cur_select")
    return out, lev


def static_scratch_bytes() -> int:
    return int(lib().gap_static_scratch_bytes())


class Handle:
    """One fit context: gap_create / gap_bind_workspace / gap_destroy.

    Tensor arguments are torch CUDA tensors (float64 / int64, contiguous); the
    stream defaults to torch's current stream at creation.
    """

    def __init__(self, p: GapParams, stream=None):
        import torch

        self.p = p
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().gap_create(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "gap_create")
        self.h = h
        self.ws = None

    def bind(self, ws):
        self.ws = ws
        _check(lib().gap_bind_workspace(self.h, _ptr(ws), ws.numel() * ws.element_size()),
               "gap_bind_workspace")

    def alloc_workspace(self, n_configs, n_atoms, M):
        import torch

        nbytes = workspace_bytes(self.p, n_configs, n_atoms, M)
        if nbytes == 0:
            raise GapError(GAP_EINVAL, "gap_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.bind(ws)
        return ws

    def alloc_workspace_obs(self, n_configs, n_atoms, n_obs, n_pos, M):
        """Workspace for a fit with derivative observations (gap_workspace_bytes_obs)."""
        import torch

        nbytes = int(lib().gap_workspace_bytes_obs(ctypes.byref(self.p), n_configs, n_atoms, n_obs, n_pos, M))
        if nbytes == 0:
            raise GapError(GAP_EINVAL, "gap_workspace_bytes_obs")
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.bind(ws)
        return ws

    def build_knm_obs(self, X, offsets, obs, XM, sigma):
        """gap_build_knm_obs: energies and derivative observations.  obs: dict of device
        tensors x_grad [n_grad, d], grad_atom [n_grad], obs_offsets [n_obs + 1],
        pos_grad [n_pos], pos_weight [n_pos]; sigma covers every row (energies, then
        the derivative observations)."""
        o = GapDerivObs(obs["x_grad"].data_ptr(), obs["x_grad"].shape[0], obs["grad_atom"].data_ptr(),
                        obs["obs_offsets"].data_ptr(), obs["obs_offsets"].numel() - 1, obs["pos_grad"].data_ptr(),
                        obs["pos_weight"].data_ptr(), obs["pos_grad"].numel())
        self._inputs = (X, offsets, XM, sigma, obs)
        _check(lib().gap_build_knm_obs(self.h, _ptr(X), X.shape[0], _ptr(offsets), offsets.numel() - 1,
                                       ctypes.byref(o), _ptr(XM), XM.shape[0], _ptr(sigma)), "gap_build_knm_obs")

    def build_knm(self, X, offsets, XM, sigma):
        # the library keeps these pointers (sigma for gap_solve, XM for gap_predict):
        # hold the tensors until the next build
        self._inputs = (X, offsets, XM, sigma)
        _check(lib().gap_build_knm(self.h, _ptr(X), X.shape[0], _ptr(offsets), offsets.numel() - 1,
                                   _ptr(XM), XM.shape[0], _ptr(sigma)), "gap_build_knm")

    def build_kmm(self):
        _check(lib().gap_build_kmm(self.h), "gap_build_kmm")

    def solve(self, y, c_out, info=True):
        inf = GapSolveInfo() if info else None
        s = lib().gap_solve(self.h, _ptr(y), _ptr(c_out), ctypes.byref(inf) if info else None)
        _check(s, "gap_solve")
        return inf

    def predict(self, X, offsets, c, y_out):
        _check(lib().gap_predict(self.h, _ptr(X), X.shape[0], _ptr(offsets), offsets.numel() - 1, _ptr(c),
                                 _ptr(y_out)), "gap_predict")

    def sync(self):
        inf = GapSolveInfo()
        s = lib().gap_sync(self.h, ctypes.byref(inf))
        return s, inf

    def layout(self) -> GapLayoutInfo:
        out = GapLayoutInfo()
        _check(lib().gap_layout(self.h, ctypes.byref(out)), "gap_layout")
        return out

    def stage_times(self):
        arr = (ctypes.c_float * len(STAGES))()
        _check(lib().gap_stage_times(self.h, arr, len(STAGES)), "gap_stage_times")
        return dict(zip(STAGES, [float(v) for v in arr]))

    def A_view(self):
        """The workspace's augmented matrix as a torch view [ncols, lda] (column-major)."""
        import torch

        lay = self.layout()
        off = lay.A_aug - self.ws.data_ptr()
        n = lay.lda * lay.ncols
        flat = self.ws[off:off + 8 * n].view(torch.float64)
        return flat.view(lay.ncols, lay.lda), lay

    def A32_view(self):
        """Mixed precision: the FP32 copy of [A | b] as a torch view [ncols, lda]."""
        import torch

        lay = self.layout()
        if not lay.A32:
            return None
        off = lay.A32 - self.ws.data_ptr()
        n = lay.lda * lay.ncols
        return self.ws[off:off + 4 * n].view(torch.float32).view(lay.ncols, lay.lda)

    def tau_view(self):
        import torch

        lay = self.layout()
        off = lay.tau - self.ws.data_ptr()
        return self.ws[off:off + 8 * lay.M].view(torch.float64)

    def set_tuning(self, qr_split_wgs=0, qr_panel=0, qr_lookahead=0, qr_free_cus=0, knm_bn=0):
        """qr_lookahead: 0 automatic, 1 off, 2 on; qr_free_cus: CUs kept from the look-ahead stream (0 none);
        knm_bn: K_NM column tile (0 = 64, or 32)."""
        t = GapTuning()
        t.qr_split_wgs = int(qr_split_wgs)
        t.qr_panel = int(qr_panel)
        t.qr_lookahead = int(qr_lookahead)
        t.qr_free_cus = int(qr_free_cus)
        t.knm_bn = int(knm_bn)
        _check(lib().gap_set_tuning(self.h, ctypes.byref(t)), "gap_set_tuning")

    def set_model(self, XM):
        """Predict-only use: bind a resident sparse set (keep XM alive)."""
        self.model_XM = XM
        _check(lib().gap_set_model(self.h, _ptr(XM), XM.shape[0]), "gap_set_model")

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().gap_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "gap_set_stream")

    def close(self):
        if self.h:
            lib().gap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
