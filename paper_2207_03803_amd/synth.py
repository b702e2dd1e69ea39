"""Seeded synthetic inputs shaped like GAP training sets.

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

__all__ = ["FitInputs", "make_fit_inputs", "make_fit_inputs_blocked", "make_fit_inputs_torch", "WORKLOADS",
           "DerivInputs", "make_deriv_inputs", "deriv_descriptors", "cur_draws"]


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
    # energies, forces and virials: 500 configurations of 20..60 atoms (~2e4 atoms, 12
    # neighbours each), d=400, M=4000, zeta=4: about 6.3e4 observation rows, most of them
    # force components, as in the paper's training sets.
    "forces_fp64": dict(n_configs=500, atoms=(20, 60), d=400, M=4000, zeta=4, n_neigh=12,
                        sigma_w=1.0, sigma_per_atom=1e-3, sigma_force=0.05, sigma_virial_per_atom=0.05,
                        jitter=1e-8),
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


# ---------------------------------------------------------------------------
# Derivative observations (forces, virials).  A smooth synthetic descriptor
# model supplies descriptors together with their exact position gradients:
# atoms sit in a cube per configuration, each has a species (one of
# N_SPECIES) and its n_neigh nearest atoms of the configuration as neighbours
# (fixed lists), and
#   x_i = (U0[t_i] + sum_{k in nb(i)} sum_b phi_b(|r_i - r_k|^2) U[t_k, b]) / C,
#   phi_b(s) = exp(-s / (2 w_b^2)),  C = 1 + 0.3 n_neigh N_RADIAL,
# with U0, U fixed random unit vectors (per species and radial function b;
# entries of both signs, so that descriptors of different environments are far
# from parallel and K stays well conditioned).  The gradients dx_i / dr_{k, alpha} follow by the chain rule.  The fit's
# arithmetic on them (the derivative rows of K) is left to the caller.
# ---------------------------------------------------------------------------
N_SPECIES = 8
RADIAL_WIDTHS = np.array([0.6, 0.9, 1.3, 2.0])
N_RADIAL = len(RADIAL_WIDTHS)


@dataclass
class DerivInputs:
    offsets: np.ndarray      # int64 [N_E + 1]: atoms of each configuration
    R: np.ndarray            # float64 [n_atoms, 3] positions
    species: np.ndarray      # int64 [n_atoms]
    nb: np.ndarray           # int64 [n_atoms, n_neigh] neighbour lists (global atom indices)
    U0: np.ndarray           # float64 [N_SPECIES, d]
    U: np.ndarray            # float64 [N_SPECIES, N_RADIAL, d]
    X: np.ndarray            # float64 [n_atoms, d] descriptors at R
    sparse_idx: np.ndarray   # int64 [M]
    XM: np.ndarray           # float64 [M, d] = X[sparse_idx] (held fixed)
    x_grad: np.ndarray       # float64 [n_grad, d]: rows dx_i / dr_{k, alpha}
    grad_atom: np.ndarray    # int64 [n_grad]: i
    grad_k: np.ndarray       # int64 [n_grad]: k
    grad_alpha: np.ndarray   # int64 [n_grad]: alpha
    obs_offsets: np.ndarray  # int64 [n_obs + 1]: positions of each derivative observation
    pos_grad: np.ndarray     # int64 [n_pos]: gradient row of each position
    pos_weight: np.ndarray   # float64 [n_pos]: -1 (force) or -r_{k, alpha} (virial)
    obs_kind: np.ndarray     # int64 [n_obs]: 0 force component, 1 virial component
    obs_config: np.ndarray   # int64 [n_obs]
    sigma_E: np.ndarray      # float64 [N_E]
    sigma_D: np.ndarray      # float64 [n_obs]
    c_true: np.ndarray       # float64 [M]
    noise_E: np.ndarray      # float64 [N_E]
    noise_D: np.ndarray      # float64 [n_obs]

    @property
    def n_configs(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_obs(self) -> int:
        return len(self.obs_offsets) - 1

    @property
    def sigma(self) -> np.ndarray:
        """Standard deviations of all observation rows: energies, then derivatives."""
        return np.concatenate([self.sigma_E, self.sigma_D])


def _radial(R, nb):
    diff = R[:, None, :] - R[nb]                                        # r_i - r_k, [n, n_neigh, 3]
    s2 = np.sum(diff * diff, axis=2)                                    # [n, n_neigh]
    phi = np.exp(-s2[:, :, None] / (2.0 * RADIAL_WIDTHS ** 2))          # [n, n_neigh, N_RADIAL]
    return diff, phi


def deriv_descriptors(R, offsets, species, nb, U0, U):
    """Descriptors of the synthetic model at positions R (neighbour lists fixed)."""
    C = 1.0 + 0.3 * nb.shape[1] * N_RADIAL
    _, phi = _radial(R, nb)
    return (U0[species] + np.einsum("nkb,nkbd->nd", phi, U[species[nb]])) / C


def make_deriv_inputs(n_configs: int, atoms=(20, 60), d: int = 64, M: int = 128, n_neigh: int = 12,
                      seed: int = 0, sigma_per_atom: float = 1e-3, sigma_force: float = 0.05,
                      sigma_virial_per_atom: float = 0.05, virials: bool = True, **_unused) -> DerivInputs:
    """Energies, force components and (optionally) the six virial components per
    configuration, for the synthetic descriptor model above (numpy PCG64, seed)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    counts = _counts(rng, n_configs, atoms)
    if counts.min() <= n_neigh:
        raise ValueError("every configuration needs more atoms than neighbours")
    offsets = np.zeros(n_configs + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n = int(offsets[-1])
    R = np.empty((n, 3))
    nb = np.empty((n, n_neigh), dtype=np.int64)
    for a in range(n_configs):
        lo, na = offsets[a], counts[a]
        side = (na / 0.8) ** (1.0 / 3.0)  # about 0.8 atoms per unit volume
        r = rng.uniform(0.0, side, size=(na, 3))
        R[lo:lo + na] = r
        dist = np.sum((r[:, None, :] - r[None, :, :]) ** 2, axis=2)
        np.fill_diagonal(dist, np.inf)
        nb[lo:lo + na] = lo + np.argsort(dist, axis=1, kind="stable")[:, :n_neigh]
    species = rng.integers(0, N_SPECIES, size=n)
    U0 = rng.standard_normal((N_SPECIES, d))
    U0 /= np.linalg.norm(U0, axis=1, keepdims=True)
    U = rng.standard_normal((N_SPECIES, N_RADIAL, d))
    U /= np.linalg.norm(U, axis=2, keepdims=True)
    X = deriv_descriptors(R, offsets, species, nb, U0, U)
    sparse_idx = np.sort(rng.choice(n, size=M, replace=False)).astype(np.int64)
    XM = np.ascontiguousarray(X[sparse_idx])
    # gradient rows (i, k, alpha): k = i first, then i's neighbours
    C = 1.0 + 0.3 * n_neigh * N_RADIAL
    diff, phi = _radial(R, nb)
    dphi = -phi / (2.0 * RADIAL_WIDTHS ** 2)                       # phi_b'(s), [n, nn, N_RADIAL]
    # d x_i / d r_{k, alpha} = sum_b phi_b'(s_ik) 2 (r_k - r_i)_alpha U[t_k, b] / C for a neighbour k
    v = np.einsum("nkb,nkbd->nkd", dphi, U[species[nb]])           # [n, nn, d]
    g_nb = (-2.0 * diff)[:, :, :, None] * v[:, :, None, :] / C     # [n, nn, 3, d]
    g_self = -np.sum(g_nb, axis=1)                                 # [n, 3, d]
    n_grad = n * (n_neigh + 1) * 3
    x_grad = np.empty((n, n_neigh + 1, 3, d))
    x_grad[:, 0] = g_self
    x_grad[:, 1:] = g_nb
    x_grad = x_grad.reshape(n_grad, d)
    grad_atom = np.repeat(np.arange(n, dtype=np.int64), (n_neigh + 1) * 3)
    ks = np.concatenate([np.arange(n, dtype=np.int64)[:, None], nb], axis=1)  # [n, nn + 1]
    grad_k = np.repeat(ks.reshape(-1), 3)
    grad_alpha = np.tile(np.arange(3, dtype=np.int64), n * (n_neigh + 1))
    # store the gradient rows by (configuration, alpha, k, i): the rows of one force
    # component, and those of one virial component, are then contiguous
    g_cfg = np.repeat(np.arange(n_configs, dtype=np.int64), counts)[grad_atom]
    order = np.lexsort((grad_atom, grad_k, grad_alpha, g_cfg))
    x_grad = x_grad[order]
    grad_atom, grad_k, grad_alpha = grad_atom[order], grad_k[order], grad_alpha[order]
    # force rows (k, alpha), in atom order: positions = gradient rows with that (k, alpha), ascending
    fkey = grad_k * 3 + grad_alpha
    order = np.argsort(fkey, kind="stable")
    f_counts = np.bincount(fkey, minlength=3 * n)
    pos_grad = [order]
    pos_weight = [-np.ones(len(order))]
    obs_sizes = [f_counts]
    obs_kind = [np.zeros(3 * n, dtype=np.int64)]
    obs_config = [np.repeat(np.repeat(np.arange(n_configs, dtype=np.int64), counts), 3)]
    if virials:
        # virial (alpha, beta), alpha <= beta: -sum_k r_{k, alpha} dE / dr_{k, beta}
        comps = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
        g_cfg = np.repeat(np.arange(n_configs, dtype=np.int64), counts)[grad_atom]  # sorted
        vp, vw, vs = [], [], []
        for a in range(n_configs):
            rows = np.nonzero(g_cfg == a)[0]
            for al, be in comps:
                sel = rows[grad_alpha[rows] == be]
                vp.append(sel)
                vw.append(-R[grad_k[sel], al])
                vs.append(len(sel))
        pos_grad.append(np.concatenate(vp))
        pos_weight.append(np.concatenate(vw))
        obs_sizes.append(np.array(vs, dtype=np.int64))
        obs_kind.append(np.ones(6 * n_configs, dtype=np.int64))
        obs_config.append(np.repeat(np.arange(n_configs, dtype=np.int64), 6))
    sizes = np.concatenate(obs_sizes)
    obs_offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=obs_offsets[1:])
    obs_kind = np.concatenate(obs_kind)
    obs_config = np.concatenate(obs_config)
    sigma_E = sigma_per_atom * counts.astype(np.float64)
    sigma_D = np.where(obs_kind == 0, sigma_force, sigma_virial_per_atom * counts[obs_config].astype(np.float64))
    c_true = rng.standard_normal(M)
    noise_E = rng.standard_normal(n_configs)
    noise_D = rng.standard_normal(len(sizes))
    return DerivInputs(offsets, R, species, nb, U0, U, np.ascontiguousarray(X), sparse_idx, XM,
                       np.ascontiguousarray(x_grad), grad_atom, grad_k, grad_alpha, obs_offsets,
                       np.concatenate(pos_grad).astype(np.int64), np.concatenate(pos_weight), obs_kind,
                       obs_config, sigma_E, sigma_D, c_true, noise_E, noise_D)
