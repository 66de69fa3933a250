"""Python binding of libepm: exact epipolar-guided matching on MI355X.

Argument marshalling only.  Every step of the matching path runs in the HIP
kernels of libepm.so (built in-tree by paper_2603_18401_amd.build); torch is
used for device memory and streams.  Importing this package does not load the
library; the first call does, and fails loudly if it has not been built or if
no GPU is present -- there is no CPU fallback.

The three entry points mirror include/epm.h:

    idx = Index(pairs, kp2, eps2=None, eps=2.0)      # epm_build_intervals
    offs, cols = idx.query(kp1)                       # epm_query_candidates
    best, d1, d2 = idx.match(offs, cols, desc1, desc2)  # epm_match

and a whole batch can be recorded once and replayed as one HIP graph:

    b = Batch(pairs, kp1, kp2, desc1, desc2, capacity=..., eps=2.0)  # epm_batch_create
    b.launch()                                                       # epm_batch_launch
"""

import ctypes
import os

import numpy as np

__all__ = ["EpmError", "Index", "Batch", "Sched", "PairSpec", "load_library", "library_path",
           "point_line_terms", "descriptor_distances", "quantize", "query_match_noalloc",
           "DTYPES", "ALGOS"]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libepm.so")
_lib = None

STATUS = {0: "EPM_OK", 1: "EPM_ERR_ARG", 2: "EPM_ERR_DEGENERATE_F", 3: "EPM_ERR_CAPACITY",
          4: "EPM_ERR_WORKSPACE", 5: "EPM_ERR_HIP", 6: "EPM_ERR_UNSUPPORTED"}
DTYPES = {"f32": 0, "bf16": 1, "fp8": 2, "bin256": 3}
ALGOS = {"auto": 0, "plain": 1, "tiled": 2}
EXPORTS = ["epm_workspace_bytes", "epm_build_intervals", "epm_query_candidates", "epm_match",
           "epm_index_destroy", "epm_status_string", "epm_version", "epm_point_line_terms",
           "epm_get_query_stats", "epm_get_match_stats", "epm_index_set_sched",
           "epm_batch_create", "epm_batch_launch", "epm_batch_nnz", "epm_batch_index",
           "epm_batch_destroy", "epm_eps_workspace_bytes", "epm_eps_features", "epm_eps_infer",
           "epm_eps_grad", "epm_eps_adam", "epm_match_residuals", "epm_query_match",
           "epm_index_set_timing_events", "epm_index_set_timing_kernel", "epm_quantize",
           "epm_mutual_check", "epm_gms_workspace_bytes", "epm_gms", "epm_query_match_noalloc",
           "epm_query_match_bf16", "epm_query_match_fp8", "epm_descriptor_distances",
           "epm_rounding_error",
           "epm_pose_eps_workspace_bytes", "epm_pose_eps"]


class EpmError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{what}: {self.name}" if what else self.name)


class _Pair(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double * 9), ("w2", ctypes.c_int32), ("h2", ctypes.c_int32),
                ("q_begin", ctypes.c_int64), ("m", ctypes.c_int64),
                ("k_begin", ctypes.c_int64), ("n", ctypes.c_int64)]


class _QueryStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("queries", "empty_queries", "scanned_queries",
                                               "records_scanned", "angle_hits", "candidates")]


class _MatchStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("queries", "reranked_rows", "fallback_rows",
                                               "long_rows", "exact_distances")]


class _MatchOpts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("check_capacity", ctypes.c_int32),
                ("col_capacity", ctypes.c_int64), ("reserved", ctypes.c_int32 * 4),
                ("qerr1", ctypes.c_void_p), ("qerr2", ctypes.c_void_p)]


class _PosePrior(ctypes.Structure):
    _fields_ = [("K1", ctypes.c_double * 9), ("K2", ctypes.c_double * 9),
                ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("cov", ctypes.c_double * 36), ("w1", ctypes.c_int32), ("h1", ctypes.c_int32),
                ("zmin", ctypes.c_double), ("zmax", ctypes.c_double)]


class _Sched(ctypes.Structure):
    _fields_ = [("stab_workgroups", ctypes.c_int32), ("match_workgroups", ctypes.c_int32),
                ("lpt", ctypes.c_int32), ("stab_chunk", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


_V = ctypes.c_void_p


class _BatchDesc(ctypes.Structure):
    _fields_ = [("kp1_xy", _V), ("kp2_xy", _V), ("eps2", _V), ("eps_scalar", ctypes.c_float),
                ("row_offsets", _V), ("col_indices", _V), ("capacity", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("dim", ctypes.c_int32), ("desc1", _V), ("desc2", _V),
                ("scale1", _V), ("scale2", _V), ("desc1_f32", _V), ("desc2_f32", _V),
                ("ratio", ctypes.c_float), ("best_idx", _V), ("best_dist", _V),
                ("second_dist", _V), ("algo", ctypes.c_int32), ("sched", _Sched),
                ("F_dev", _V), ("err2", _V)]


class Sched:
    """Work distribution and tile shape of the tile kernels (epm_sched):
    0 workgroups = one workgroup per angle tile; n > 0 = persistent launch of
    n workgroups; lpt = take tiles longest first (persistent launches);
    stab_chunk = window records staged per round of the stabbing pass (256,
    512 or 1024; 0 = 256 for the fused BF16 pass, 512 for the others)."""

    def __init__(self, stab_workgroups=0, match_workgroups=0, lpt=0, stab_chunk=0):
        self.stab_workgroups = int(stab_workgroups)
        self.match_workgroups = int(match_workgroups)
        self.lpt = int(lpt)
        self.stab_chunk = int(stab_chunk)

    def as_dict(self):
        return {"stab_workgroups": self.stab_workgroups,
                "match_workgroups": self.match_workgroups, "lpt": self.lpt,
                "stab_chunk": self.stab_chunk}

    @classmethod
    def from_dict(cls, d):
        return cls(d.get("stab_workgroups", 0), d.get("match_workgroups", 0), d.get("lpt", 0),
                   d.get("stab_chunk", 0))

    def _c(self):
        c = _Sched()
        c.stab_workgroups, c.match_workgroups, c.lpt, c.stab_chunk = (
            self.stab_workgroups, self.match_workgroups, self.lpt, self.stab_chunk)
        return c

    def __repr__(self):
        return (f"Sched({self.stab_workgroups}, {self.match_workgroups}, lpt={self.lpt}, "
                f"stab_chunk={self.stab_chunk})")


def library_path():
    return _LIB_PATH


def load_library(path=None):
    """Loads libepm.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: run `python -m paper_2603_18401_amd.build`")
    # torch first: the library must bind to the HIP runtime torch uses (the
    # wheel ships its own), or torch's device pointers are foreign to it
    import torch  # noqa: F401
    lib = ctypes.CDLL(p)
    V, P, i64, i32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.epm_workspace_bytes.argtypes = [P, i32]
    lib.epm_workspace_bytes.restype = ctypes.c_size_t
    lib.epm_build_intervals.argtypes = [P, i32, V, V, ctypes.c_float, V, ctypes.c_size_t,
                                        ctypes.POINTER(V), V]
    lib.epm_build_intervals.restype = ctypes.c_int
    lib.epm_query_candidates.argtypes = [V, V, V, V, i64, ctypes.POINTER(i64), V]
    lib.epm_query_candidates.restype = ctypes.c_int
    lib.epm_match.argtypes = [V, V, V, ctypes.c_int, i32, V, V, V, V, V, V, ctypes.c_float,
                              V, V, V, P, V]
    lib.epm_match.restype = ctypes.c_int
    lib.epm_index_destroy.argtypes = [V]
    lib.epm_index_destroy.restype = None
    lib.epm_status_string.argtypes = [ctypes.c_int]
    lib.epm_status_string.restype = ctypes.c_char_p
    lib.epm_version.restype = ctypes.c_char_p
    lib.epm_point_line_terms.argtypes = [P, V, V, V, ctypes.c_float, V, V, i64, V, V, V]
    lib.epm_point_line_terms.restype = ctypes.c_int
    lib.epm_get_query_stats.argtypes = [V, ctypes.POINTER(_QueryStats)]
    lib.epm_get_query_stats.restype = ctypes.c_int
    lib.epm_get_match_stats.argtypes = [V, ctypes.POINTER(_MatchStats)]
    lib.epm_get_match_stats.restype = ctypes.c_int
    lib.epm_index_set_sched.argtypes = [V, ctypes.POINTER(_Sched)]
    lib.epm_index_set_sched.restype = ctypes.c_int
    lib.epm_batch_create.argtypes = [P, i32, ctypes.POINTER(_BatchDesc), V, ctypes.c_size_t,
                                     ctypes.POINTER(V), V]
    lib.epm_batch_create.restype = ctypes.c_int
    lib.epm_batch_launch.argtypes = [V, V]
    lib.epm_batch_launch.restype = ctypes.c_int
    lib.epm_batch_nnz.argtypes = [V, ctypes.POINTER(i64), V]
    lib.epm_batch_nnz.restype = ctypes.c_int
    lib.epm_batch_index.argtypes = [V]
    lib.epm_batch_index.restype = V
    lib.epm_batch_destroy.argtypes = [V]
    lib.epm_batch_destroy.restype = None
    f32 = ctypes.c_float
    lib.epm_eps_workspace_bytes.argtypes = [i32]
    lib.epm_eps_workspace_bytes.restype = ctypes.c_size_t
    lib.epm_eps_features.argtypes = [P, i32, V, V, V, V, ctypes.c_size_t, V]
    lib.epm_eps_features.restype = ctypes.c_int
    lib.epm_eps_infer.argtypes = [V, i64, V, V, V]
    lib.epm_eps_infer.restype = ctypes.c_int
    lib.epm_eps_grad.argtypes = [V, i64, V, V, i64, V, i32, f32, V, V, V, V, ctypes.c_size_t, V]
    lib.epm_eps_grad.restype = ctypes.c_int
    lib.epm_eps_adam.argtypes = [V, V, V, V, i32, f32, f32, f32, f32, V]
    lib.epm_eps_adam.restype = ctypes.c_int
    lib.epm_match_residuals.argtypes = [V, V, V, V, V, V, V]
    lib.epm_match_residuals.restype = ctypes.c_int
    lib.epm_mutual_check.argtypes = [V, V, V, V, V]
    lib.epm_mutual_check.restype = ctypes.c_int
    lib.epm_gms_workspace_bytes.argtypes = [V, i32]
    lib.epm_gms_workspace_bytes.restype = ctypes.c_size_t
    lib.epm_gms.argtypes = [V, P, i32, ctypes.c_float, V, V, V, V, V, ctypes.c_size_t, V]
    lib.epm_gms.restype = ctypes.c_int
    lib.epm_query_match.argtypes = [V, V, V, V, i64, ctypes.POINTER(i64), V, V, f32, V, V, V, V]
    lib.epm_query_match.restype = ctypes.c_int
    lib.epm_query_match_bf16.argtypes = [V, V, V, V, i64, ctypes.POINTER(i64), V, V, V, V, f32,
                                         V, V, V, V]
    lib.epm_query_match_bf16.restype = ctypes.c_int
    lib.epm_query_match_fp8.argtypes = [V, V, V, V, i64, ctypes.POINTER(i64), V, V, V, V, V,
                                        f32, V, V, V, V]
    lib.epm_query_match_fp8.restype = ctypes.c_int
    lib.epm_index_set_timing_events.argtypes = [V, V, V]
    lib.epm_index_set_timing_events.restype = ctypes.c_int
    lib.epm_index_set_timing_kernel.argtypes = [V, i32]
    lib.epm_index_set_timing_kernel.restype = ctypes.c_int
    lib.epm_quantize.argtypes = [V, i64, i32, ctypes.c_int, V, V, V]
    lib.epm_quantize.restype = ctypes.c_int
    lib.epm_query_match_noalloc.argtypes = [P, i32, V, V, V, f32, V, V, i64,
                                            ctypes.POINTER(i64), V, V, f32, V, V, V, V]
    lib.epm_query_match_noalloc.restype = ctypes.c_int
    lib.epm_descriptor_distances.argtypes = [ctypes.c_int, i32, V, V, V, V, V, V, i64, V, V]
    lib.epm_descriptor_distances.restype = ctypes.c_int
    lib.epm_rounding_error.argtypes = [V, i64, i32, ctypes.c_int, V, V, V, V]
    lib.epm_rounding_error.restype = ctypes.c_int
    lib.epm_pose_eps_workspace_bytes.argtypes = [i32]
    lib.epm_pose_eps_workspace_bytes.restype = ctypes.c_size_t
    lib.epm_pose_eps.argtypes = [P, P, i32, V, f32, f32, f32, V, V, ctypes.c_size_t, V]
    lib.epm_pose_eps.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libepm needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(torch, device, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _check(st, what):
    if st != 0:
        raise EpmError(st, what)


class PairSpec:
    """One image pair: F (3x3, row-major), image-2 size, keypoint counts."""

    def __init__(self, F, w2, h2, m, n):
        self.F = np.asarray(F, dtype=np.float64).reshape(9)
        self.w2, self.h2, self.m, self.n = int(w2), int(h2), int(m), int(n)


def _pair_array(specs):
    arr = (_Pair * len(specs))()
    q = k = 0
    for a, s in zip(arr, specs):
        a.F[:] = [float(v) for v in s.F]
        a.w2, a.h2 = s.w2, s.h2
        a.q_begin, a.m, a.k_begin, a.n = q, s.m, k, s.n
        q += s.m
        k += s.n
    return arr, q, k


class Index:
    """epm_build_intervals over a batch of pairs; owns its device workspace."""

    def __init__(self, pairs, kp2, eps2=None, eps=0.0, stream=None, workspace=None):
        torch = _torch()
        self._torch = torch
        self.lib = load_library()
        self.device = kp2.device
        self.specs = list(pairs)
        self._pairs, self.n1, self.n2 = _pair_array(self.specs)
        if tuple(kp2.shape) != (self.n2, 2) or kp2.dtype != torch.float32 or not kp2.is_contiguous():
            raise ValueError("kp2 must be a contiguous float32 [N2, 2] device tensor")
        if eps2 is not None and (tuple(eps2.shape) != (self.n2,) or eps2.dtype != torch.float32):
            raise ValueError("eps2 must be a float32 [N2] device tensor")
        nbytes = self.lib.epm_workspace_bytes(self._pairs, len(self.specs))
        if nbytes == 0:
            raise EpmError(1, "epm_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        self._keep = (kp2, eps2)
        h = ctypes.c_void_p()
        st = self.lib.epm_build_intervals(self._pairs, len(self.specs), _dptr(kp2), _dptr(eps2),
                                          float(eps), _dptr(workspace), workspace.numel(),
                                          ctypes.byref(h), _stream(torch, self.device, stream))
        _check(st, "epm_build_intervals")
        self.handle = h
        self.stream = stream

    def close(self):
        if getattr(self, "handle", None):
            self.lib.epm_index_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, kp1, capacity=None, row_offsets=None, col_indices=None, sync=True):
        """Candidate CSR (row_offsets int64 [N1+1], col_indices int32 [nnz]).

        capacity: initial guess for nnz (grown and retried on EPM_ERR_CAPACITY).
        sync=False with preallocated row_offsets/col_indices skips the host
        synchronisation (the caller guarantees the capacity)."""
        torch = self._torch
        if tuple(kp1.shape) != (self.n1, 2) or kp1.dtype != torch.float32 or not kp1.is_contiguous():
            raise ValueError("kp1 must be a contiguous float32 [N1, 2] device tensor")
        if row_offsets is None:
            row_offsets = torch.empty(self.n1 + 1, dtype=torch.int64, device=self.device)
        if col_indices is None:
            cap = int(capacity) if capacity is not None else max(1024, 64 * self.n1)
            col_indices = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        st_ptr = _stream(torch, self.device, self.stream)
        if not sync:
            st = self.lib.epm_query_candidates(self.handle, _dptr(kp1), _dptr(row_offsets),
                                               _dptr(col_indices), col_indices.numel(), None,
                                               st_ptr)
            _check(st, "epm_query_candidates")
            return row_offsets, col_indices
        nnz = ctypes.c_int64(0)
        st = self.lib.epm_query_candidates(self.handle, _dptr(kp1), _dptr(row_offsets),
                                           _dptr(col_indices), col_indices.numel(),
                                           ctypes.byref(nnz), st_ptr)
        if st == 3:
            col_indices = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=self.device)
            st = self.lib.epm_query_candidates(self.handle, _dptr(kp1), _dptr(row_offsets),
                                               _dptr(col_indices), col_indices.numel(),
                                               ctypes.byref(nnz), st_ptr)
        _check(st, "epm_query_candidates")
        return row_offsets, col_indices[: nnz.value]

    def _fused_query(self, name, kp1, args, ratio, capacity, row_offsets, col_indices, out,
                     sync):
        """The shared body of the fused query calls: output buffers, the call
        (entry point `name`, descriptor arguments `args` between nnz_host and
        the ratio), and one retry with a CSR buffer of the reported size."""
        torch = self._torch
        if tuple(kp1.shape) != (self.n1, 2) or kp1.dtype != torch.float32 or not kp1.is_contiguous():
            raise ValueError("kp1 must be a contiguous float32 [N1, 2] device tensor")
        dev = self.device
        if row_offsets is None:
            row_offsets = torch.empty(self.n1 + 1, dtype=torch.int64, device=dev)
        if col_indices is None:
            cap = int(capacity) if capacity is not None else max(1024, 64 * self.n1)
            col_indices = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        if out is None:
            out = (torch.empty(self.n1, dtype=torch.int32, device=dev),
                   torch.empty(self.n1, dtype=torch.float32, device=dev),
                   torch.empty(self.n1, dtype=torch.float32, device=dev))
        best, bd, sd = out
        st_ptr = _stream(torch, dev, self.stream)
        fn = getattr(self.lib, name)

        def call(cols, nnz_ref):
            return fn(self.handle, _dptr(kp1), _dptr(row_offsets), _dptr(cols), cols.numel(),
                      nnz_ref, *[_dptr(a) for a in args], float(ratio), _dptr(best), _dptr(bd),
                      _dptr(sd), st_ptr)

        if not sync:
            _check(call(col_indices, None), name)
            return row_offsets, col_indices, best, bd, sd
        nnz = ctypes.c_int64(0)
        st = call(col_indices, ctypes.byref(nnz))
        if st == 3:
            col_indices = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
            st = call(col_indices, ctypes.byref(nnz))
        _check(st, name)
        return row_offsets, col_indices[: nnz.value], best, bd, sd

    def query_match(self, kp1, desc1, desc2, ratio=0.0, capacity=None, row_offsets=None,
                    col_indices=None, out=None, sync=True):
        """epm_query_match: the candidate CSR and the FP32 matches in one pass.
        Returns (row_offsets, col_indices, best_idx, best_dist, second_dist);
        capacity / sync as in query()."""
        return self._fused_query("epm_query_match", kp1, (desc1, desc2), ratio, capacity,
                                 row_offsets, col_indices, out, sync)

    def query_match_bf16(self, kp1, desc1, desc2, desc1_f32, desc2_f32, ratio=0.0,
                         capacity=None, row_offsets=None, col_indices=None, out=None,
                         sync=True):
        """epm_query_match_bf16: the candidate CSR and the matches of the FP32
        masters, selected through BF16 MFMA bounds (desc1/desc2: int16 BF16
        codes [N, 128], the round-to-nearest-even values of the masters).
        Returns (row_offsets, col_indices, best_idx, best_dist, second_dist)."""
        return self._fused_query("epm_query_match_bf16", kp1,
                                 (desc1, desc2, desc1_f32, desc2_f32), ratio, capacity,
                                 row_offsets, col_indices, out, sync)

    def query_match_fp8(self, kp1, desc2, scale2, err2, desc1_f32, desc2_f32, ratio=0.0,
                        capacity=None, row_offsets=None, col_indices=None, out=None,
                        sync=True):
        """epm_query_match_fp8: the candidate CSR and the matches of the FP32
        masters, selected through MFMA bounds over FP8 image-2 rows (desc2:
        uint8 E4M3FN codes [N2, 128] with float32 scales scale2 [N2] and
        rounding-error bounds err2 [N2], see rounding_error).
        Returns (row_offsets, col_indices, best_idx, best_dist, second_dist)."""
        torch = self._torch
        for name, t, shape, dt in (("desc2", desc2, (self.n2, 128), torch.uint8),
                                   ("scale2", scale2, (self.n2,), torch.float32),
                                   ("err2", err2, (self.n2,), torch.float32),
                                   ("desc1_f32", desc1_f32, (self.n1, 128), torch.float32),
                                   ("desc2_f32", desc2_f32, (self.n2, 128), torch.float32)):
            if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} {list(shape)} device tensor")
        return self._fused_query("epm_query_match_fp8", kp1,
                                 (desc2, scale2, err2, desc1_f32, desc2_f32), ratio, capacity,
                                 row_offsets, col_indices, out, sync)

    def stats(self):
        """Counters of the last query (dict; waits for its stream)."""
        st = _QueryStats()
        _check(self.lib.epm_get_query_stats(self.handle, ctypes.byref(st)), "epm_get_query_stats")
        return {k: int(getattr(st, k)) for k, _ in st._fields_}

    def match_stats(self):
        """Counters of the last BF16/FP8 match (dict; waits for its stream)."""
        st = _MatchStats()
        _check(self.lib.epm_get_match_stats(self.handle, ctypes.byref(st)), "epm_get_match_stats")
        return {k: int(getattr(st, k)) for k, _ in st._fields_}

    def set_timing_events(self, start=None, stop=None, kernel=None):
        """Records two torch.cuda.Events (enable_timing=True) around the
        dominant kernel of later query / query_match / match calls; None, None
        turns it off.  kernel: "stab" (the stabbing-tile kernel of the query
        calls, the default) or "wide" (their wide-row kernel)."""
        if kernel is not None:
            k = {"stab": 0, "wide": 1}[kernel]
            _check(self.lib.epm_index_set_timing_kernel(self.handle, k),
                   "epm_index_set_timing_kernel")
        handles = []
        for ev in (start, stop):
            if ev is None:
                handles.append(None)
                continue
            if not ev.cuda_event:  # created lazily by the first record
                ev.record()
            handles.append(ctypes.c_void_p(ev.cuda_event))
        self._timing = (start, stop)
        _check(self.lib.epm_index_set_timing_events(self.handle, *handles),
               "epm_index_set_timing_events")

    def mutual(self, best12, best21, out=None):
        """epm_mutual_check: best12 [N1] from this index, best21 [N2] from the
        reversed index (image 2 against image 1 with the transposed F);
        returns the mutual matches [N1] (-1 where not mutual)."""
        torch = self._torch
        if out is None:
            out = torch.empty(self.n1, dtype=torch.int32, device=self.device)
        _check(self.lib.epm_mutual_check(self.handle, _dptr(best12), _dptr(best21), _dptr(out),
                                         _stream(torch, self.device, self.stream)),
               "epm_mutual_check")
        return out

    def gms(self, sizes1, kp1, kp2, best, grid=20, alpha=6.0, out=None):
        """epm_gms: GMS validation of the matches `best` of this index.
        sizes1: image-1 (width, height) of every pair.  Returns the kept
        matches (-1 elsewhere)."""
        torch = self._torch
        if len(sizes1) != len(self.specs):
            raise ValueError("one image-1 size per pair")
        size1 = (ctypes.c_int32 * (2 * len(sizes1)))(*[int(v) for wh in sizes1 for v in wh])
        nbytes = self.lib.epm_gms_workspace_bytes(self.handle, int(grid))
        if nbytes == 0:
            raise EpmError(1, "epm_gms_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if out is None:
            out = torch.empty(self.n1, dtype=torch.int32, device=self.device)
        _check(self.lib.epm_gms(self.handle, size1, int(grid), float(alpha), _dptr(kp1),
                                _dptr(kp2), _dptr(best), _dptr(out), _dptr(ws), ws.numel(),
                                _stream(torch, self.device, self.stream)), "epm_gms")
        return out

    def set_sched(self, sched):
        """Work distribution of later query/match calls (a Sched)."""
        c = sched._c()
        _check(self.lib.epm_index_set_sched(self.handle, ctypes.byref(c)), "epm_index_set_sched")

    def match(self, row_offsets, col_indices, desc1, desc2, dtype="f32", scale1=None,
              scale2=None, desc1_f32=None, desc2_f32=None, ratio=0.0, algo="auto", out=None,
              check_capacity=False, qerr1=None, qerr2=None):
        """Nearest neighbour per query: (best_idx int32, best_dist f32, second_dist f32).

        check_capacity: the launch writes nothing when row_offsets[N1] exceeds
        col_indices.numel() (a CSR from query(..., sync=False) that did not fit)."""
        torch = self._torch
        dim = 256 if dtype == "bin256" else 128
        if out is None:
            best = torch.empty(self.n1, dtype=torch.int32, device=self.device)
            bd = torch.empty(self.n1, dtype=torch.float32, device=self.device)
            sd = torch.empty(self.n1, dtype=torch.float32, device=self.device)
        else:
            best, bd, sd = out
        opts = _MatchOpts()
        opts.algo = ALGOS[algo]
        if check_capacity:
            opts.check_capacity = 1
            opts.col_capacity = col_indices.numel()
        if qerr1 is not None:
            opts.qerr1, opts.qerr2 = qerr1.data_ptr(), qerr2.data_ptr()
        st = self.lib.epm_match(self.handle, _dptr(row_offsets), _dptr(col_indices), DTYPES[dtype],
                                dim, _dptr(desc1), _dptr(desc2), _dptr(scale1), _dptr(scale2),
                                _dptr(desc1_f32), _dptr(desc2_f32), float(ratio), _dptr(best),
                                _dptr(bd), _dptr(sd), ctypes.byref(opts),
                                _stream(torch, self.device, self.stream))
        _check(st, "epm_match")
        return best, bd, sd


def reversed_specs(specs, sizes1):
    """PairSpecs of the other direction (image 2 against image 1): the
    transposed F, the image-1 sizes [(w1, h1), ...], m and n exchanged."""
    return [PairSpec(np.asarray(s.F, dtype=np.float64).reshape(3, 3).T, w, h, s.n, s.m)
            for s, (w, h) in zip(specs, sizes1)]


def mutual_match(specs, sizes1, kp1, kp2, desc1, desc2, eps=0.0, eps2=None, eps1=None,
                 ratio=0.0):
    """Mutual guided matching over a batch (FP32 descriptors): the
    candidates and matches of image 1 against image 2 (tolerances eps2 per
    image-2 keypoint, or eps), of image 2 against image 1 (eps1 per image-1
    keypoint, or eps), and the cross-check.  Returns (best12, best21, mutual);
    every step runs in the library."""
    fwd = Index(specs, kp2, eps2=eps2, eps=eps)
    rev = Index(reversed_specs(specs, sizes1), kp1, eps2=eps1, eps=eps)
    _, _, best12, _, _ = fwd.query_match(kp1, desc1, desc2, ratio=ratio)
    _, _, best21, _, _ = rev.query_match(kp2, desc2, desc1, ratio=ratio)
    mutual = fwd.mutual(best12, best21)
    return best12, best21, mutual


class Batch:
    """epm_batch_create: the whole build / query / match pipeline over a batch
    of pairs, recorded once as a HIP graph and replayed by launch().

    Inputs and outputs are fixed device tensors (new contents of the same
    sizes may be written between launches).  F_dev (float64 [P, 9], device):
    when given, every launch redoes the pair setup on the device from it, so
    new F may be written there between launches.  dtype "fp8" with err2
    (float32 [N2], the image-2 rows' rounding-error bounds): the fused FP8
    pass of query_match_fp8 (desc1 may then be None).  capacity: length of the CSR
    column buffer; nnz() reports the total of the last launch and raises
    EpmError(EPM_ERR_CAPACITY) when it did not fit."""

    def __init__(self, pairs, kp1, kp2, desc1, desc2, capacity, eps2=None, eps=0.0,
                 dtype="f32", scale1=None, scale2=None, desc1_f32=None, desc2_f32=None,
                 ratio=0.0, algo="auto", sched=None, stream=None, workspace=None,
                 F_dev=None, err2=None):
        torch = _torch()
        self._torch = torch
        self.lib = load_library()
        self.device = kp2.device
        self.specs = list(pairs)
        self._pairs, self.n1, self.n2 = _pair_array(self.specs)
        for name, t, n in (("kp1", kp1, self.n1), ("kp2", kp2, self.n2)):
            if tuple(t.shape) != (n, 2) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 [{n}, 2] device tensor")
        nbytes = self.lib.epm_workspace_bytes(self._pairs, len(self.specs))
        if nbytes == 0:
            raise EpmError(1, "epm_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        dev = self.device
        self.row_offsets = torch.empty(self.n1 + 1, dtype=torch.int64, device=dev)
        self.col_indices = torch.empty(max(int(capacity), 1), dtype=torch.int32, device=dev)
        self.best_idx = torch.empty(self.n1, dtype=torch.int32, device=dev)
        self.best_dist = torch.empty(self.n1, dtype=torch.float32, device=dev)
        self.second_dist = torch.empty(self.n1, dtype=torch.float32, device=dev)
        self.sched = sched or Sched()
        d = _BatchDesc()
        d.kp1_xy, d.kp2_xy, d.eps2 = kp1.data_ptr(), kp2.data_ptr(), (
            eps2.data_ptr() if eps2 is not None else None)
        d.eps_scalar = float(eps)
        d.row_offsets, d.col_indices = self.row_offsets.data_ptr(), self.col_indices.data_ptr()
        d.capacity = int(capacity)
        d.dtype, d.dim = DTYPES[dtype], 256 if dtype == "bin256" else 128
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        d.desc1, d.desc2, d.scale1, d.scale2 = ptr(desc1), ptr(desc2), ptr(scale1), ptr(scale2)
        d.desc1_f32, d.desc2_f32 = ptr(desc1_f32), ptr(desc2_f32)
        d.err2 = ptr(err2)
        d.ratio = float(ratio)
        d.best_idx, d.best_dist, d.second_dist = (self.best_idx.data_ptr(),
                                                  self.best_dist.data_ptr(),
                                                  self.second_dist.data_ptr())
        d.algo = ALGOS[algo]
        d.sched = self.sched._c()
        if F_dev is not None:
            if tuple(F_dev.shape) != (len(self.specs), 9) or F_dev.dtype != torch.float64 \
                    or not F_dev.is_contiguous():
                raise ValueError("F_dev must be a contiguous float64 [num_pairs, 9] device tensor")
            d.F_dev = F_dev.data_ptr()
        # the graph reads these buffers on every replay
        self._keep = (kp1, kp2, eps2, desc1, desc2, scale1, scale2, desc1_f32, desc2_f32, F_dev,
                      err2)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.epm_batch_create(self._pairs, len(self.specs), ctypes.byref(d),
                                       _dptr(workspace), workspace.numel(), ctypes.byref(h),
                                       _stream(torch, dev, stream))
        _check(st, "epm_batch_create")
        self.handle = h

    def launch(self):
        _check(self.lib.epm_batch_launch(self.handle, _stream(self._torch, self.device,
                                                              self.stream)), "epm_batch_launch")

    def nnz(self):
        v = ctypes.c_int64(0)
        st = self.lib.epm_batch_nnz(self.handle, ctypes.byref(v),
                                    _stream(self._torch, self.device, self.stream))
        _check(st, f"epm_batch_nnz ({v.value} candidates)")
        return v.value

    def outputs(self):
        """(row_offsets, col_indices[:nnz], best_idx, best_dist, second_dist)."""
        n = self.nnz()
        return (self.row_offsets, self.col_indices[:n], self.best_idx, self.best_dist,
                self.second_dist)

    def _index_handle(self):
        return ctypes.c_void_p(self.lib.epm_batch_index(self.handle))

    def stats(self):
        st = _QueryStats()
        _check(self.lib.epm_get_query_stats(self._index_handle(), ctypes.byref(st)),
               "epm_get_query_stats")
        return {k: int(getattr(st, k)) for k, _ in st._fields_}

    def match_stats(self):
        st = _MatchStats()
        _check(self.lib.epm_get_match_stats(self._index_handle(), ctypes.byref(st)),
               "epm_get_match_stats")
        return {k: int(getattr(st, k)) for k, _ in st._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.epm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 64 << 20


def query_match_noalloc(pairs, kp1, kp2, desc1, desc2, eps2=None, eps=0.0, ratio=0.0,
                        row_offsets=None, col_indices=None, out=None, stream=None):
    """epm_query_match_noalloc: build + fused query/match with the index in the
    library's static device array (no workspace, no device allocation by the
    library).  row_offsets [N1+1] and col_indices (its length is the capacity)
    may be preallocated by the caller; the call synchronises once to read nnz.
    Returns (row_offsets, col_indices[:nnz], best_idx, best_dist, second_dist)."""
    torch = _torch()
    lib = load_library()
    specs = list(pairs)
    arr, n1, n2 = _pair_array(specs)
    dev = kp2.device
    if row_offsets is None:
        row_offsets = torch.empty(n1 + 1, dtype=torch.int64, device=dev)
    if col_indices is None:
        col_indices = torch.empty(max(1024, 64 * n1), dtype=torch.int32, device=dev)
    if out is None:
        out = (torch.empty(n1, dtype=torch.int32, device=dev),
               torch.empty(n1, dtype=torch.float32, device=dev),
               torch.empty(n1, dtype=torch.float32, device=dev))
    best, bd, sd = out
    nnz = ctypes.c_int64(0)
    st = lib.epm_query_match_noalloc(arr, len(specs), _dptr(kp1), _dptr(kp2), _dptr(eps2),
                                     float(eps), _dptr(row_offsets), _dptr(col_indices),
                                     col_indices.numel(), ctypes.byref(nnz), _dptr(desc1),
                                     _dptr(desc2), float(ratio), _dptr(best), _dptr(bd),
                                     _dptr(sd), _stream(torch, dev, stream))
    _check(st, "epm_query_match_noalloc")
    return row_offsets, col_indices[: nnz.value], best, bd, sd


def quantize(desc, dtype, stream=None):
    """epm_quantize on the device: FP32 rows [N, D] -> BF16 bit patterns
    (int16 [N, D]), or FP8-E4M3 codes (uint8 [N, D]) and per-row scales."""
    torch = _torch()
    lib = load_library()
    if desc.dtype != torch.float32 or desc.dim() != 2 or not desc.is_contiguous():
        raise ValueError("desc must be a contiguous float32 [N, D] device tensor")
    n, d = desc.shape
    if dtype == "bf16":
        out, scale = torch.empty((n, d), dtype=torch.int16, device=desc.device), None
    elif dtype == "fp8":
        out = torch.empty((n, d), dtype=torch.uint8, device=desc.device)
        scale = torch.empty(n, dtype=torch.float32, device=desc.device)
    else:
        raise ValueError("dtype must be 'bf16' or 'fp8'")
    st = lib.epm_quantize(_dptr(desc), n, d, DTYPES[dtype], _dptr(out), _dptr(scale),
                          _stream(torch, desc.device, stream))
    _check(st, "epm_quantize")
    return (out, scale) if dtype == "fp8" else out


class PosePrior:
    """Estimated relative pose of one pair (X2 = R X1 + t), its intrinsics, the
    6 x 6 covariance of (rotation vector, translation), the image-1 size and
    optionally the scene's depth range in camera 2 (zmin = 0: none)."""

    def __init__(self, K1, K2, R, t, cov, w1, h1, zmin=0.0, zmax=float("inf")):
        self.K1 = np.asarray(K1, np.float64).reshape(9)
        self.K2 = np.asarray(K2, np.float64).reshape(9)
        self.R = np.asarray(R, np.float64).reshape(9)
        self.t = np.asarray(t, np.float64).reshape(3)
        self.cov = np.asarray(cov, np.float64).reshape(36)
        self.w1, self.h1 = int(w1), int(h1)
        self.zmin, self.zmax = float(zmin), float(zmax)


def pose_eps(pairs, priors, kp2, eps0, k_sigma, eps_max, stream=None):
    """epm_pose_eps: per image-2 keypoint tolerance (float32 [N2]) from the
    pose covariance of every pair (a list of PosePrior)."""
    torch = _torch()
    lib = load_library()
    specs = list(pairs)
    arr, _, n2 = _pair_array(specs)
    pri = (_PosePrior * len(specs))()
    for c, p in zip(pri, priors):
        c.K1[:], c.K2[:], c.R[:] = list(p.K1), list(p.K2), list(p.R)
        c.t[:], c.cov[:] = list(p.t), list(p.cov)
        c.w1, c.h1 = p.w1, p.h1
        c.zmin, c.zmax = p.zmin, p.zmax
    ws = torch.empty(lib.epm_pose_eps_workspace_bytes(len(specs)), dtype=torch.uint8,
                     device=kp2.device)
    eps2 = torch.empty(n2, dtype=torch.float32, device=kp2.device)
    st = lib.epm_pose_eps(arr, pri, len(specs), _dptr(kp2), float(eps0), float(k_sigma),
                          float(eps_max), _dptr(eps2), _dptr(ws), ws.numel(),
                          _stream(torch, kp2.device, stream))
    _check(st, "epm_pose_eps")
    return eps2


def rounding_error(src, codes, dtype, scale=None, stream=None):
    """epm_rounding_error: per-row bounds on |x - dequant(x^)| (float32 [N])."""
    torch = _torch()
    lib = load_library()
    n, d = src.shape
    err = torch.empty(n, dtype=torch.float32, device=src.device)
    st = lib.epm_rounding_error(_dptr(src), n, d, DTYPES[dtype], _dptr(codes), _dptr(scale),
                                _dptr(err), _stream(torch, src.device, stream))
    _check(st, "epm_rounding_error")
    return err


def descriptor_distances(desc1, desc2, qi, kj, dtype="f32", scale1=None, scale2=None,
                         stream=None):
    """epm_descriptor_distances: for listed pairs (qi[t], kj[t]) the canonical
    FP32 distance (dtype "f32") or the MFMA approximation of BF16 / FP8 codes
    (dtype "bf16" / "fp8") as the matching kernels compute them (float32 [count])."""
    torch = _torch()
    lib = load_library()
    out = torch.empty(qi.numel(), dtype=torch.float32, device=qi.device)
    st = lib.epm_descriptor_distances(DTYPES[dtype], 128, _dptr(desc1), _dptr(desc2),
                                      _dptr(scale1), _dptr(scale2), _dptr(qi), _dptr(kj),
                                      qi.numel(), _dptr(out), _stream(torch, qi.device, stream))
    _check(st, "epm_descriptor_distances")
    return out


def point_line_terms(F, kp1, kp2, qi, kj, eps2=None, eps=0.0, stream=None):
    """Device values of both sides of the Eq. 3 test for listed pairs."""
    torch = _torch()
    lib = load_library()
    Fh = (ctypes.c_double * 9)(*[float(v) for v in np.asarray(F, np.float64).reshape(9)])
    num = torch.empty(qi.numel(), dtype=torch.float64, device=kp1.device)
    rhs = torch.empty(qi.numel(), dtype=torch.float64, device=kp1.device)
    st = lib.epm_point_line_terms(Fh, _dptr(kp1), _dptr(kp2), _dptr(eps2), float(eps),
                                  _dptr(qi), _dptr(kj), qi.numel(), _dptr(num), _dptr(rhs),
                                  _stream(torch, kp1.device, stream))
    _check(st, "epm_point_line_terms")
    return num, rhs
