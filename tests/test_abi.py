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


LAYOUT_PROGRAM = r"""
#include <stdio.h>
#include <stddef.h>
#include "epm.h"
#define S(t) printf(#t " size %zu\n", sizeof(t))
#define O(t, f) printf(#t " " #f " %zu\n", offsetof(t, f))
int main(void) {
  S(epm_pair); O(epm_pair, w2); O(epm_pair, q_begin); O(epm_pair, n);
  S(epm_match_opts); O(epm_match_opts, check_capacity); O(epm_match_opts, col_capacity);
  S(epm_sched); O(epm_sched, lpt);
  S(epm_query_stats); S(epm_match_stats);
  S(epm_batch_desc);
  O(epm_batch_desc, eps_scalar); O(epm_batch_desc, row_offsets); O(epm_batch_desc, capacity);
  O(epm_batch_desc, dtype); O(epm_batch_desc, dim); O(epm_batch_desc, desc1);
  O(epm_batch_desc, ratio); O(epm_batch_desc, best_idx); O(epm_batch_desc, algo);
  O(epm_batch_desc, sched); O(epm_batch_desc, F_dev); O(epm_batch_desc, err2);
  S(epm_pose_prior); O(epm_pose_prior, t); O(epm_pose_prior, cov); O(epm_pose_prior, w1);
  O(epm_pose_prior, zmin); O(epm_pose_prior, zmax);
  O(epm_match_opts, qerr1); O(epm_match_opts, qerr2);
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout."""
    import shutil
    import subprocess

    import paper_2603_18401_amd as E
    if shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("gcc or the ROCm headers are missing")
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text(LAYOUT_PROGRAM)
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__=1", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    c = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True,
                               check=True).stdout.splitlines():
        *name, v = line.split()
        c[" ".join(name)] = int(v)
    mirrors = {"epm_pair": E._Pair, "epm_match_opts": E._MatchOpts, "epm_sched": E._Sched,
               "epm_query_stats": E._QueryStats, "epm_match_stats": E._MatchStats,
               "epm_batch_desc": E._BatchDesc, "epm_pose_prior": E._PosePrior}
    for key, v in c.items():
        parts = key.split()
        cls = mirrors[parts[0]]
        if parts[1] == "size":
            assert ctypes.sizeof(cls) == v, key
        else:
            assert getattr(cls, parts[1]).offset == v, key


def test_batch_and_sched_argument_errors(lib):
    import paper_2603_18401_amd as E
    V = ctypes.c_void_p
    pairs = (E._Pair * 1)()
    pairs[0].F[:] = [0, 0, 0, 0, 0, -1, 0, 1, 0]
    pairs[0].w2, pairs[0].h2, pairs[0].m, pairs[0].n = 640, 480, 10, 10
    h = V()
    d = E._BatchDesc()
    lib.epm_batch_create.argtypes = [V, ctypes.c_int32, V, V, ctypes.c_size_t,
                                     ctypes.POINTER(V), V]
    # no descriptor, no output pointer
    assert lib.epm_batch_create(pairs, 1, None, V(256), 1 << 20, ctypes.byref(h), None) == 1
    assert lib.epm_batch_create(pairs, 1, ctypes.byref(d), V(256), 1 << 20, None, None) == 1
    # missing inputs and outputs are caught before anything is enqueued
    d.kp1_xy, d.kp2_xy, d.eps_scalar = 256, 256, 2.0
    assert lib.epm_batch_create(pairs, 1, ctypes.byref(d), V(256), 1 << 20, ctypes.byref(h),
                                None) == 1
    d.row_offsets, d.col_indices, d.capacity = 256, 256, 100
    d.dtype, d.dim = 0, 64  # float descriptors need dim 128
    assert lib.epm_batch_create(pairs, 1, ctypes.byref(d), V(256), 1 << 20, ctypes.byref(h),
                                None) == 1
    d.dim = 128
    d.sched.lpt = 2
    assert lib.epm_batch_create(pairs, 1, ctypes.byref(d), V(256), 1 << 20, ctypes.byref(h),
                                None) == 1
    assert h.value is None
    assert lib.epm_batch_launch(None, None) == 1
    nnz = ctypes.c_int64(0)
    assert lib.epm_batch_nnz(None, ctypes.byref(nnz), None) == 1
    assert lib.epm_batch_index(None) is None
    lib.epm_batch_destroy(None)
    s = E._Sched()
    assert lib.epm_index_set_sched(None, ctypes.byref(s)) == 1


def test_learned_eps_argument_errors(lib):
    import paper_2603_18401_amd as E
    V = ctypes.c_void_p
    assert lib.epm_eps_workspace_bytes(-1) == 0
    assert lib.epm_eps_workspace_bytes(0) >= 256 * 4674 * 4
    assert lib.epm_eps_infer(V(256), -1, V(256), V(256), None) == 1
    assert lib.epm_eps_infer(None, 10, V(256), V(256), None) == 1
    assert lib.epm_eps_infer(None, 0, None, None, None) == 0  # nothing to do
    ws = lib.epm_eps_workspace_bytes(0)
    args = [V(256), 100, None, V(256), 100, V(256), 64, 0.99, V(256), V(256), V(256), V(256),
            ws, None]
    bad = list(args)
    bad[6] = 0  # empty batch
    assert lib.epm_eps_grad(*bad) == 1
    bad = list(args)
    bad[1] = 0  # no feature rows
    assert lib.epm_eps_grad(*bad) == 1
    for q in (0.0, 1.0, float("nan")):
        bad = list(args)
        bad[7] = q
        assert lib.epm_eps_grad(*bad) == 1
    bad = list(args)
    bad[12] = ws - 1
    assert lib.epm_eps_grad(*bad) == 4
    bad = list(args)
    bad[11] = V(258)  # misaligned workspace
    assert lib.epm_eps_grad(*bad) == 4
    assert lib.epm_eps_adam(V(256), V(256), V(256), V(256), 0, 1e-3, 0.9, 0.999, 1e-8,
                            None) == 1
    assert lib.epm_eps_adam(V(256), V(256), V(256), V(256), 1, 1e-3, 1.0, 0.999, 1e-8,
                            None) == 1
    pairs = (E._Pair * 1)()
    pairs[0].F[:] = [0, 0, 0, 0, 0, -1, 0, 1, 0]
    pairs[0].w2, pairs[0].h2, pairs[0].m, pairs[0].n = 640, 480, 10, 10
    wsp = lib.epm_eps_workspace_bytes(1)
    assert lib.epm_eps_features(pairs, 1, None, V(256), V(256), V(256), wsp, None) == 1
    assert lib.epm_eps_features(pairs, 1, V(256), V(256), V(256), V(256), wsp - 1, None) == 4
    pairs[0].F[:] = [0] * 9
    assert lib.epm_eps_features(pairs, 1, V(256), V(256), V(256), V(256), wsp, None) == 2
    assert lib.epm_match_residuals(None, V(256), V(256), V(256), V(256), None, None) == 1


def test_timing_kernel_argument_errors(lib):
    assert lib.epm_index_set_timing_kernel(None, 0) == 1
    assert lib.epm_index_set_timing_kernel(None, 1) == 1


def test_mutual_check_argument_errors(lib):
    assert lib.epm_mutual_check(None, None, None, None, None) == 1


def test_gms_argument_errors(lib):
    import ctypes
    size1 = (ctypes.c_int32 * 2)(640, 480)
    assert lib.epm_gms_workspace_bytes(None, 20) == 0
    assert lib.epm_gms(None, size1, 20, 6.0, None, None, None, None, None, 0, None) == 1


def test_noalloc_refuses_batches_beyond_its_scratch(lib):
    """epm_query_match_noalloc checks the index size against its fixed array
    on the host: a batch that needs more is refused before anything runs."""
    import paper_2603_18401_amd as E
    F = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0]], float)
    big = [E.PairSpec(F, 640, 480, 150000, 1000)]
    arr, n1, _ = _pairs(big)
    assert lib.epm_workspace_bytes(arr, 1) > E.NOALLOC_SCRATCH_BYTES
    V = ctypes.c_void_p
    nnz = ctypes.c_int64(0)
    st = lib.epm_query_match_noalloc(arr, 1, V(256), V(256), None, 2.0, V(256), V(256), 10,
                                     ctypes.byref(nnz), V(256), V(256), 0.0, V(256), V(256),
                                     V(256), None)
    assert st == 4  # EPM_ERR_WORKSPACE
    st = lib.epm_query_match_noalloc(arr, 1, None, V(256), None, 2.0, V(256), V(256), 10,
                                     ctypes.byref(nnz), V(256), V(256), 0.0, V(256), V(256),
                                     V(256), None)
    assert st == 1  # kp1 missing: EPM_ERR_ARG
