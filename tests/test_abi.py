"""Host-side checks of the C ABI: the library loads and exports every symbol
include/gap.h declares; pure host functions behave (no GPU needed)."""
import ctypes
import json
import os
import re

import pytest

from paper_2207_03803_amd import gap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gap.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(gap_[a-z_]+)\s*\(", src, re.M)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(gap.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = gap.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings():
    for s in range(9):
        assert gap.status_string(s) != "unknown status"
    assert gap.status_string(gap.GAP_ENOTPD).startswith("K_MM")
    assert "rank" in gap.status_string(gap.GAP_ERANK)


def test_create_rejects_bad_params_without_a_gpu():
    lib = gap.lib()
    h = ctypes.c_void_p()
    for p in (gap.params(0, 2), gap.params(8, 0), gap.params(8, 9), gap.params(8, 2, sigma_w=0.0),
              gap.params(8, 2, jitter=-1.0), gap.params(8, 2, precision=7),
              gap.params(4097, 2, flags=gap.GAP_FLAG_KNM_INT8)):
        assert lib.gap_create(ctypes.byref(p), None, ctypes.byref(h)) == gap.GAP_EINVAL


def test_int8_knm_descriptor_length_limit():
    """The INT8-emulated K_NM takes rows up to 4096 components (exact INT32 sums)."""
    assert gap.workspace_bytes(gap.params(4096, 2, flags=gap.GAP_FLAG_KNM_INT8), 10, 100, 10) > 0
    assert gap.workspace_bytes(gap.params(4097, 2, flags=gap.GAP_FLAG_KNM_INT8), 10, 100, 10) == 0
    assert gap.workspace_bytes(gap.params(4097, 2), 10, 100, 10) > 0


def test_poison_flag_leaves_the_workspace_size_unchanged():
    """GAP_FLAG_POISON_WORKSPACE only fills arrays the workspace already has."""
    for prec in (gap.GAP_FP64, gap.GAP_MIXED_FP32, gap.GAP_MIXED_BF16):
        for extra in (0, gap.GAP_FLAG_KNM_INT8):
            plain = gap.workspace_bytes(gap.params(64, 2, precision=prec, flags=extra), 30, 900, 200)
            poisoned = gap.workspace_bytes(
                gap.params(64, 2, precision=prec, flags=extra | gap.GAP_FLAG_POISON_WORKSPACE), 30, 900, 200)
            assert plain > 0 and poisoned == plain


def test_workspace_bytes_bad_inputs():
    p = gap.params(64, 2)
    assert gap.workspace_bytes(p, 0, 10, 10) == 0
    assert gap.workspace_bytes(p, 10, 10, 0) == 0
    assert gap.workspace_bytes(gap.params(64, 0), 10, 10, 10) == 0


def test_workspace_holds_the_paper_sized_stacked_matrix():
    """A of (N+M) x M in FP64 (the printed element counts) plus b, within the bound workspace."""
    cases = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_shapes.json")))["cases"]
    p = gap.params(400, 2)
    for c in cases:
        N, M = c["N"], c["M"]
        nb = gap.workspace_bytes(p, N, 40 * N, M)
        assert nb >= 8 * c["n_A"] + 8 * (N + M)
        # overhead beyond [A | b] (padding, QR scratch, tile plan) stays small
        assert nb <= 1.05 * 8 * (N + M + 64) * (M + 1)


@pytest.mark.parametrize("N,M", [(200, 256), (100_000, 10_000)])
def test_workspace_fits_one_mi355x(N, M):
    nb = gap.workspace_bytes(gap.params(400, 4), N, 40 * N, M)
    assert nb < 288e9 * 0.5


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with the library absent, the first call raises."""
    monkeypatch.setattr(gap, "_lib", None)
    monkeypatch.setattr(gap, "LIB_PATH", str(tmp_path / "libgap.so"))
    with pytest.raises(RuntimeError, match="not built"):
        gap.lib()
    with pytest.raises(RuntimeError, match="not built"):
        gap.workspace_bytes(gap.params(64, 2, 1.0, 1e-8), 10, 100, 8)


def test_fit_static_checks_arguments_and_size_without_a_gpu():
    """The allocation-free fit rejects bad parameters, timing events and shapes whose
    scratch would exceed the static array before it touches the GPU."""
    lib = gap.lib()
    dummy = ctypes.c_void_p(256)  # never dereferenced: every check here fails first
    cap = gap.static_scratch_bytes()
    assert cap == 256 << 20

    def call(p, n_atoms, N, M):
        return lib.gap_fit_static(ctypes.byref(p), None, dummy, n_atoms, dummy, N, dummy, M, dummy, dummy,
                                  dummy, None)

    assert call(gap.params(0, 2), 100, 10, 8) == gap.GAP_EINVAL
    assert call(gap.params(64, 2, flags=gap.GAP_FLAG_TIMING), 100, 10, 8) == gap.GAP_EINVAL
    assert call(gap.params(64, 2), 0, 10, 8) == gap.GAP_EINVAL
    big = (100_000, 10_000)
    assert gap.workspace_bytes(gap.params(64, 2), big[0], 40 * big[0], big[1]) > cap
    assert call(gap.params(64, 2), 40 * big[0], *big) == gap.GAP_ENOMEM
    assert gap.workspace_bytes(gap.params(64, 2), 200, 7200, 256) <= cap


def test_cur_select_argument_checks_without_a_gpu():
    """gap_cur_workspace_bytes is a pure host function; gap_cur_select rejects bad
    shapes and a short workspace before touching the device."""
    lib = gap.lib()
    assert gap.cur_workspace_bytes(0, 8) == 0
    assert gap.cur_workspace_bytes(100, 0) == 0
    assert gap.cur_workspace_bytes(7, 8) == 0        # fewer rows than columns
    assert gap.cur_workspace_bytes(100, 5000) == 0   # d above the supported 4096
    nb = gap.cur_workspace_bytes(4_000_000, 400)
    assert 8 * 4_000_000 * 5 <= nb <= 8 * 4_000_000 * 8  # keys + row parts, a few MB besides
    fake = ctypes.c_void_p(0x1000)
    call = lambda x, n, d, M, ws, wsb: lib.gap_cur_select(x, n, d, None, M, fake, None, ws, wsb, None, 1)
    assert call(None, 100, 8, 10, fake, 1 << 30) == gap.GAP_EINVAL
    assert call(fake, 100, 8, 0, fake, 1 << 30) == gap.GAP_EINVAL
    assert call(fake, 100, 8, 101, fake, 1 << 30) == gap.GAP_EINVAL
    assert call(fake, 100, 8, 10, None, 1 << 30) == gap.GAP_EINVAL
    assert call(fake, 100, 8, 10, fake, gap.cur_workspace_bytes(100, 8) - 1) == gap.GAP_ENOMEM
