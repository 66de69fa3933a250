"""The C ABI on the CPU: the library loads, exports every entry point that
include/epm.h declares, and rejects bad arguments on the host before any
device work (no GPU needed for any of this)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(epm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2603_18401_amd as E
    if not os.path.exists(E.library_path()):
        pytest.skip("libepm.so not built")
    return E.load_library()


def test_header_declares_the_three_calls():
    f = declared_functions()
    for name in ("epm_build_intervals", "epm_query_candidates", "epm_match"):
        assert name in f


def test_library_exports_every_declared_symbol(lib):
    import paper_2603_18401_amd as E
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(E.EXPORTS) == declared_functions()


def test_status_strings(lib):
    for s in range(7):
        assert lib.epm_status_string(s).startswith(b"EPM_")
    assert b"gfx950" in lib.epm_version()


def _pairs(specs):
    import paper_2603_18401_amd as E
    return E._pair_array(specs)


def _build(lib, arr, num, kp2=16, eps2=None, eps=2.0, ws=256, ws_bytes=1 << 40):
    h = ctypes.c_void_p()
    st = lib.epm_build_intervals(arr, num, ctypes.c_void_p(kp2) if kp2 else None,
                                 ctypes.c_void_p(eps2) if eps2 else None, eps,
                                 ctypes.c_void_p(ws) if ws else None, ws_bytes, ctypes.byref(h),
                                 None)
    return st, h


def test_workspace_size_rejects_bad_slices(lib):
    import paper_2603_18401_amd as E
    F = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0]], float)
    arr, _, _ = _pairs([E.PairSpec(F, 640, 480, 10, 20), E.PairSpec(F, 640, 480, 5, 5)])
    assert lib.epm_workspace_bytes(arr, 2) > 0
    arr[1].q_begin = 3  # not contiguous
    assert lib.epm_workspace_bytes(arr, 2) == 0
    arr, _, _ = _pairs([E.PairSpec(F, 0, 480, 10, 20)])
    assert lib.epm_workspace_bytes(arr, 1) == 0
    assert lib.epm_workspace_bytes(None, 1) == 0
    assert lib.epm_workspace_bytes(arr, 0) == 0


def test_build_argument_errors(lib):
    import paper_2603_18401_amd as E
    F = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0]], float)
    arr, _, _ = _pairs([E.PairSpec(F, 640, 480, 10, 20)])
    assert _build(lib, arr, 1, eps=0.0)[0] == 1          # eps_scalar must be > 0
    assert _build(lib, arr, 1, eps=float("nan"))[0] == 1
    assert _build(lib, arr, 1, kp2=0)[0] == 1            # kp2 missing
    assert _build(lib, arr, 1, ws=0)[0] == 4             # no workspace
    assert _build(lib, arr, 1, ws=300)[0] == 4           # misaligned
    assert _build(lib, arr, 1, ws_bytes=1024)[0] == 4    # too small


@pytest.mark.parametrize("F", [np.zeros((3, 3)), np.full((3, 3), np.nan),
                               np.outer([1.0, 2.0, 3.0], [0.5, -1.0, 2.0])])
def test_degenerate_F(lib, F):
    """Zero, non-finite or rank-1 F has no epipole: refused before any launch."""
    import paper_2603_18401_amd as E
    arr, _, _ = _pairs([E.PairSpec(F, 640, 480, 10, 20)])
    assert _build(lib, arr, 1)[0] == 2


def test_query_and_match_argument_errors(lib):
    V = ctypes.c_void_p
    nnz = ctypes.c_int64(0)
    assert lib.epm_query_candidates(None, V(16), V(16), V(16), 10, ctypes.byref(nnz), None) == 1
    assert lib.epm_match(None, V(16), V(16), 0, 128, V(16), V(16), None, None, None, None, 0.0,
                         V(16), V(16), V(16), None, None) == 1
    assert lib.epm_get_query_stats(None, None) == 1
    assert lib.epm_point_line_terms(None, None, None, None, 0.0, None, None, 5, None, None,
                                    None) == 1
