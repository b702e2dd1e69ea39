"""The seeded input recipe: shapes, value distributions and structure of the
synthetic GAP training sets, on the host (numpy) and through torch on the CPU."""
import numpy as np
import pytest
import torch

from paper_2207_03803_amd import synth


def _check(inp, n_configs, atoms, d, M, sigma_per_atom, X, XM):
    counts = np.diff(inp.offsets)
    assert inp.offsets.dtype == np.int64 and inp.offsets[0] == 0 and len(inp.offsets) == n_configs + 1
    assert counts.min() >= atoms[0] and counts.max() <= atoms[1]
    assert X.shape == (inp.n_atoms, d) and XM.shape == (M, d)
    assert X.min() >= 0.0  # |N(0,1)| entries
    assert np.abs(np.linalg.norm(X, axis=1) - 1.0).max() <= 4e-16 * np.sqrt(d)
    idx = inp.sparse_idx
    assert idx.dtype == np.int64 and len(idx) == M and np.all(np.diff(idx) > 0)
    assert idx[0] >= 0 and idx[-1] < inp.n_atoms
    assert np.array_equal(XM, X[idx])  # sparse points are copies of atom rows
    assert np.array_equal(inp.sigma, sigma_per_atom * counts.astype(np.float64))
    assert inp.c_true.shape == (M,) and inp.noise.shape == (n_configs,)


def test_host_recipe_structure_and_determinism():
    w = dict(synth.WORKLOADS["tiny_fp64"])
    a = synth.make_fit_inputs(seed=3, **w)
    _check(a, w["n_configs"], w["atoms"], w["d"], w["M"], w["sigma_per_atom"], a.X, a.XM)
    b = synth.make_fit_inputs(seed=3, **w)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.noise, b.noise) and np.array_equal(a.sparse_idx, b.sparse_idx)
    c = synth.make_fit_inputs(seed=4, **w)
    assert not np.array_equal(a.X[:8], c.X[:8])


def test_host_recipe_is_independent_of_the_drawing_chunk():
    w = dict(synth.WORKLOADS["tiny_fp64"])
    a = synth.make_fit_inputs(seed=1, **w)
    b = synth.make_fit_inputs(seed=1, chunk=1000, **w)  # several chunks, a ragged last one
    assert a.n_atoms > 3000
    # the stream is drawn in the same order, so only the normalisation's blocking differs
    assert np.array_equal(a.X, b.X)


def test_host_recipe_rejects_more_sparse_points_than_atoms():
    with pytest.raises(ValueError):
        synth.make_fit_inputs(n_configs=2, atoms=(1, 1), d=4, M=3)


def test_torch_recipe_on_the_cpu():
    inp = synth.make_fit_inputs_torch(n_configs=300, atoms=(16, 64), d=40, M=100, seed=2, device="cpu",
                                      chunk=2048)
    X, XM = inp.X.numpy(), inp.XM.numpy()
    _check(inp, 300, (16, 64), 40, 100, 1e-3, X, XM)
    again = synth.make_fit_inputs_torch(n_configs=300, atoms=(16, 64), d=40, M=100, seed=2, device="cpu",
                                        chunk=2048)
    assert torch.equal(inp.X, again.X)
    # counts, sparse indices, c_true and noise share the host stream with make_fit_inputs
    host = synth.make_fit_inputs(n_configs=300, atoms=(16, 64), d=40, M=100, seed=2)
    assert np.array_equal(inp.offsets, host.offsets)


def test_workload_recipes_have_the_stated_sizes():
    t, r = synth.WORKLOADS["tiny_fp64"], synth.WORKLOADS["realistic_fp64"]
    assert (t["n_configs"], t["d"], t["M"], t["zeta"]) == (200, 64, 256, 2)
    assert (r["n_configs"], r["atoms"], r["d"], r["M"], r["zeta"]) == (100_000, (16, 64), 400, 10_000, 4)
    assert r["jitter"] == t["jitter"] == 1e-8


def test_blocked_recipe_is_independent_of_the_worker_count():
    w = dict(n_configs=4000, atoms=(8, 64), d=24, M=50)
    a = synth.make_fit_inputs_blocked(seed=5, workers=1, **w)
    b = synth.make_fit_inputs_blocked(seed=5, workers=5, **w)
    assert a.n_atoms > 2 * synth.BLOCK_ATOMS  # several blocks and a ragged last one
    for f in ("offsets", "X", "sparse_idx", "XM", "c_true", "noise", "sigma"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.allclose(np.linalg.norm(a.X, axis=1), 1.0, rtol=0, atol=1e-12) and (a.X >= 0).all()
    assert np.array_equal(a.XM, a.X[a.sparse_idx])
    # counts come from the same host stream as the single-stream recipe
    h = synth.make_fit_inputs(seed=5, **w)
    assert np.array_equal(h.offsets, a.offsets)
