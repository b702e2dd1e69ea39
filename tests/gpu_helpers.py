"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI."""
import sys

import numpy as np

U = np.finfo(np.float64).eps / 2


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch

    dtype = dtype or (torch.int64 if np.asarray(a).dtype.kind in "iu" else torch.float64)
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


class GpuFit:
    """Build + solve one fit on the GPU; keeps the handle and the A copy."""

    def __init__(self, X, offsets, XM, sigma, y, zeta, sigma_w=1.0, jitter=1e-8, keep_A=False,
                 timing=False, precision=0, max_refine_iters=20, refine_tol=1e-12, flags=0):
        import torch

        from paper_2207_03803_amd import gap

        self.gap = gap
        flags = flags | (gap.GAP_FLAG_TIMING if timing else 0)
        self.X = X if isinstance(X, torch.Tensor) else to_dev(X)
        self.XM = XM if isinstance(XM, torch.Tensor) else to_dev(XM)
        self.offsets = to_dev(np.asarray(offsets, dtype=np.int64))
        self.sigma = to_dev(sigma)
        self.y = y if isinstance(y, torch.Tensor) else to_dev(y)
        self.N = self.offsets.numel() - 1
        self.M = self.XM.shape[0]
        d = self.X.shape[1]
        self.h = gap.Handle(gap.params(d, zeta, sigma_w, jitter, precision=precision, flags=flags,
                                       max_refine_iters=max_refine_iters, refine_tol=refine_tol))
        self.h.alloc_workspace(self.N, self.X.shape[0], self.M)
        self.c = torch.empty(self.M, dtype=torch.float64, device="cuda")

    def build(self):
        self.h.build_knm(self.X, self.offsets, self.XM, self.sigma)

    def A_top_and_lower(self):
        """(Sigma^-1/2 K_NM [N x M], L^T [M x M]) read from the workspace (host numpy)."""
        Av, lay = self.h.A_view()
        N, M = self.N, self.M
        top = Av[:M, :N].T.cpu().numpy()
        low = Av[:M, N:N + M].T.cpu().numpy()
        return top, low

    def solve(self):
        info = self.h.solve(self.y, self.c)
        return self.c.cpu().numpy(), info

    def run(self):
        self.build()
        return self.solve()
