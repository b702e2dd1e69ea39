"""Seeded synthetic inputs shaped like GAP training sets (energies only).

This module draws random numbers and nothing else: per-configuration atom
counts, per-atom descriptors (i.i.d. |N(0,1)| entries, then scaled to unit L2
norm, which is the form the dot-product kernel expects its inputs in), the
indices of the sparse points (uniform, without replacement), a "true" weight
vector and standard-normal noise draws.  It holds none of the fit's arithmetic:
targets y = (model prediction with c_true) + sigma * noise are formed by the
caller, with whichever implementation it is testing or timing.

Both the CPU oracle (through the tests) and the GPU path read the same arrays.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["FitInputs", "make_fit_inputs", "make_fit_inputs_blocked", "make_fit_inputs_torch", "WORKLOADS"]


# Workload recipes (atom-count range, descriptor length, sparse-set size,
# kernel exponent, noise scale per atom).  Names say what they are.
WORKLOADS = {
    # 200 configurations, 8..64 atoms, d=64, M=256, zeta=2: runs on a CPU in seconds.
    "tiny_fp64": dict(n_configs=200, atoms=(8, 64), d=64, M=256, zeta=2,
                      sigma_w=1.0, sigma_per_atom=1e-3, jitter=1e-8),
    # 1e5 configurations, 16..64 atoms (~4e6 descriptors), d=400, M=1e4, zeta=4:
    # stacked least-squares matrix 110,000 x 10,000 in FP64.
    "realistic_fp64": dict(n_configs=100_000, atoms=(16, 64), d=400, M=10_000, zeta=4,
                           sigma_w=1.0, sigma_per_atom=1e-3, jitter=1e-8),
}


@dataclass
class FitInputs:
    offsets: np.ndarray      # int64 [N+1], CSR offsets of each configuration's atoms
    X: object                # [n_atoms, d] float64, unit rows (numpy or torch)
    sparse_idx: np.ndarray   # int64 [M], rows of X chosen as sparse points
    XM: object               # [M, d] float64 copy of X[sparse_idx]
    c_true: np.ndarray       # float64 [M], N(0,1)
    noise: np.ndarray        # float64 [N], N(0,1) draws (scaled by sigma by the caller)
    sigma: np.ndarray        # float64 [N], sigma_A = sigma_per_atom * N_A

    @property
    def n_configs(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])


def _counts(rng, n_configs, atoms):
    lo, hi = atoms
    return rng.integers(lo, hi + 1, size=n_configs).astype(np.int64)


def make_fit_inputs(n_configs: int, atoms=(8, 64), d: int = 64, M: int = 256,
                    seed: int = 0, sigma_per_atom: float = 1e-3,
                    chunk: int = 1 << 20, **_unused) -> FitInputs:
    """Host (numpy PCG64) generator; every array is drawn from one seeded stream.

    Draw order: atom counts, descriptors (in chunks of ``chunk`` atoms), sparse
    indices, c_true, noise.
    """
    rng = np.random.default_rng(seed)
    counts = _counts(rng, n_configs, atoms)
    offsets = np.zeros(n_configs + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n_atoms = int(offsets[-1])
    if M > n_atoms:
        raise ValueError(f"M={M} exceeds the number of descriptors {n_atoms}")
    X = np.empty((n_atoms, d), dtype=np.float64)
    for s in range(0, n_atoms, chunk):
        e = min(n_atoms, s + chunk)
        blk = rng.standard_normal((e - s, d))
        np.abs(blk, out=blk)
        blk /= np.sqrt(np.einsum("ij,ij->i", blk, blk))[:, None]
        X[s:e] = blk
    sparse_idx = np.sort(rng.choice(n_atoms, size=M, replace=False)).astype(np.int64)
    XM = np.ascontiguousarray(X[sparse_idx])
    c_true = rng.standard_normal(M)
    noise = rng.standard_normal(n_configs)
    sigma = sigma_per_atom * counts.astype(np.float64)
    return FitInputs(offsets, X, sparse_idx, XM, c_true, noise, sigma)


BLOCK_ATOMS = 1 << 16  # descriptors per independent stream of make_fit_inputs_blocked


def _draw_block(seed: int, b: int, rows: int, d: int) -> np.ndarray:
    blk = np.random.default_rng(np.random.SeedSequence([seed, 1, b])).standard_normal((rows, d))
    np.abs(blk, out=blk)
    blk /= np.sqrt(np.einsum("ij,ij->i", blk, blk))[:, None]
    return blk


def cur_draws(n: int, seed: int = 0) -> np.ndarray:
    """One Exp(1) variate per descriptor row for the sampled CUR selection, from
    PCG64 seeded with SeedSequence([seed, 2]) (a stream of its own)."""
    return np.random.default_rng(np.random.SeedSequence([seed, 2])).standard_exponential(n)


def make_fit_inputs_blocked(n_configs: int, atoms=(16, 64), d: int = 400, M: int = 10_000,
                            seed: int = 0, sigma_per_atom: float = 1e-3, workers: int = 8,
                            log=None, **_unused) -> FitInputs:
    """Same recipe on the host, drawn by several threads: for sizes whose
    descriptors take minutes to draw from one stream.

    Counts, sparse indices, c_true and noise come from numpy PCG64 (seed), in
    that order (the descriptors are not on this stream); descriptor block b
    (BLOCK_ATOMS rows) comes
    from its own PCG64 stream seeded with SeedSequence([seed, 1, b]), so the
    arrays do not depend on ``workers``.  ``log`` (optional) is called with a
    progress string every 16 blocks.
    """
    from concurrent.futures import ThreadPoolExecutor

    rng = np.random.default_rng(seed)
    counts = _counts(rng, n_configs, atoms)
    offsets = np.zeros(n_configs + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n_atoms = int(offsets[-1])
    if M > n_atoms:
        raise ValueError(f"M={M} exceeds the number of descriptors {n_atoms}")
    X = np.empty((n_atoms, d), dtype=np.float64)
    n_blocks = (n_atoms + BLOCK_ATOMS - 1) // BLOCK_ATOMS

    def fill(b):
        s = b * BLOCK_ATOMS
        e = min(n_atoms, s + BLOCK_ATOMS)
        X[s:e] = _draw_block(seed, b, e - s, d)
        return b

    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        for done, _ in enumerate(ex.map(fill, range(n_blocks)), 1):
            if log and (done % 16 == 0 or done == n_blocks):
                log(f"descriptors: {done}/{n_blocks} blocks")
    sparse_idx = np.sort(rng.choice(n_atoms, size=M, replace=False)).astype(np.int64)
    XM = np.ascontiguousarray(X[sparse_idx])
    c_true = rng.standard_normal(M)
    noise = rng.standard_normal(n_configs)
    sigma = sigma_per_atom * counts.astype(np.float64)
    return FitInputs(offsets, X, sparse_idx, XM, c_true, noise, sigma)


def make_fit_inputs_torch(n_configs: int, atoms=(16, 64), d: int = 400, M: int = 10_000,
                          seed: int = 0, sigma_per_atom: float = 1e-3, device="cuda",
                          chunk: int = 1 << 20, **_unused) -> FitInputs:
    """Same recipe for sizes too large to draw on the host quickly.

    Counts, sparse indices, c_true and noise come from numpy PCG64 (seed);
    descriptors come from torch's Philox generator on ``device`` (seed + 1),
    drawn in chunks, folded to |.| and scaled to unit L2 norm in FP64.
    X and XM are torch tensors on ``device``.
    """
    import torch

    rng = np.random.default_rng(seed)
    counts = _counts(rng, n_configs, atoms)
    offsets = np.zeros(n_configs + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n_atoms = int(offsets[-1])
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 1)
    X = torch.empty((n_atoms, d), dtype=torch.float64, device=device)
    for s in range(0, n_atoms, chunk):
        e = min(n_atoms, s + chunk)
        blk = torch.randn((e - s, d), dtype=torch.float64, device=device, generator=gen)
        blk.abs_()
        blk /= torch.sqrt((blk * blk).sum(dim=1, keepdim=True))
        X[s:e] = blk
    sparse_idx = np.sort(rng.choice(n_atoms, size=M, replace=False)).astype(np.int64)
    XM = X[torch.from_numpy(sparse_idx).to(device)].contiguous()
    c_true = rng.standard_normal(M)
    noise = rng.standard_normal(n_configs)
    sigma = sigma_per_atom * counts.astype(np.float64)
    return FitInputs(offsets, X, sparse_idx, XM, c_true, noise, sigma)
