"""CPU oracle for exact epipolar-guided matching -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library: the brute-force
candidate search and the descriptor selection are in plain C (oracle.c,
FP64, no contraction), the paper's angular formulation (Sec. 4.2 Eq. 5-7,
Sec. 4.4) and the tolerance network are restated here in NumPy.

Parity status of each function (pins are the tests in tests/test_oracle*.py):
  candidates        pinned: rectified-stereo 1-D range query, pure forward
                    motion closed form, wrap-around worked case, circles
                    containing the epipole, eps >= diagonal, invariants
                    (true matches, monotonicity, scaling, permutation,
                    image swap), agreement with the paper's angular form.
  match (float)     pinned: canonical FP32 chain vs exact rational rounding,
                    selection vs sorted (distance, j), brute-force NN limit.
  match (binary)    pinned: Hamming vs numpy bit counts.
  point_line_dist,  pinned: hand values of the wrap-around case (Sec. 4.4),
  candidate_terms   integer lines with exact terms, the scanline case with
                    scalar and per-keypoint eps.
  desc_dist_f64     pinned: hand cases with exact dyadic sums, and exact
                    rational distances within its FP64 rounding bound.
  paper_angle_*     pinned against the brute-force candidates (agreement
                    outside a 1e-6 px boundary band).
  mutual.*          pinned: both directions keep noiseless true matches only
                    with the transposed matrix; the cross-check on a hand case.
  gms.*             pinned: hand-built motions, the threshold boundary, the
                    tie rule, invariance under the query order.
  pose_eps.*        pinned: zero covariance, the rectified-stereo closed form,
                    sqrt(Sigma) scaling, the spread under sampled poses, hand
                    cases of the reverse epipolar segment.
"""

import ctypes
import os
import subprocess

import numpy as np

from .paper_angle import paper_angle_candidates, paper_query_angle  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "oracle.c")
GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread"]


def build(force=True, src=None, out=None):
    """Compile oracle.c (or a given source) with gcc: plain C, no contraction."""
    src = src or _SRC_PATH
    out = out or _LIB_PATH
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc"] + GCC_FLAGS + [src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class OracleLib:
    """ctypes view of one build of oracle.c."""

    def __init__(self, path):
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_candidates.argtypes = [P, P, i64, P, i64, P, ctypes.c_float, P, P, i64, P,
                                          P, ctypes.c_int]
        lib.oracle_candidates.restype = ctypes.c_int
        lib.oracle_point_line_dist.argtypes = [P, P, P, P, P, i64, P]
        lib.oracle_point_line_dist.restype = None
        lib.oracle_match.argtypes = [ctypes.c_int, P, P, ctypes.c_int, P, P, P, P, i64,
                                     ctypes.c_float, P, P, P, ctypes.c_int]
        lib.oracle_match.restype = None
        lib.oracle_desc_dist_f32.argtypes = [P, P, ctypes.c_int]
        lib.oracle_desc_dist_f32.restype = ctypes.c_float
        lib.oracle_desc_dist_f64_pairs.argtypes = [P, P, ctypes.c_int, P, P, i64, P]
        lib.oracle_desc_dist_f64_pairs.restype = None
        lib.oracle_default_threads.restype = ctypes.c_int
        lib.oracle_candidate_terms.argtypes = [P, P, P, P, ctypes.c_float, P, P, i64, P, P]
        lib.oracle_candidate_terms.restype = None
        self.lib = lib
        self.path = path

    def default_threads(self):
        return int(self.lib.oracle_default_threads())

    def candidates(self, F, kp1, kp2, eps, nthreads=0):
        """Brute-force candidate sets (Eq. 3-4) for one pair.

        F: (3,3) float64; kp1 (m,2) / kp2 (n,2) float32; eps: scalar or (n,)
        float32 per image-2 keypoint.  Returns (row_offsets int64[m+1],
        col_indices int32[nnz] ascending per row, degenerate uint8[m])."""
        lib = self.lib
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
        kp1 = np.ascontiguousarray(kp1, dtype=np.float32).reshape(-1, 2)
        kp2 = np.ascontiguousarray(kp2, dtype=np.float32).reshape(-1, 2)
        m, n = kp1.shape[0], kp2.shape[0]
        if np.ndim(eps) == 0:
            eps_arr, eps_s = None, float(np.float32(eps))
        else:
            eps_arr = np.ascontiguousarray(eps, dtype=np.float32).reshape(n)
            eps_s = 0.0
        offs = np.zeros(m + 1, np.int64)
        deg = np.zeros(max(m, 1), np.uint8)
        nnz = ctypes.c_int64(0)
        cols = np.zeros(1, np.int32)
        rc = lib.oracle_candidates(_ptr(F), _ptr(kp1), m, _ptr(kp2), n, _ptr(eps_arr), eps_s,
                                   _ptr(offs), _ptr(cols), 0, ctypes.byref(nnz), _ptr(deg),
                                   int(nthreads))
        if rc == 1:
            cols = np.zeros(max(nnz.value, 1), np.int32)
            rc = lib.oracle_candidates(_ptr(F), _ptr(kp1), m, _ptr(kp2), n, _ptr(eps_arr),
                                       eps_s, _ptr(offs), _ptr(cols), nnz.value,
                                       ctypes.byref(nnz), _ptr(deg), int(nthreads))
            assert rc == 0
        return offs, cols[: nnz.value].copy(), deg[:m].copy()

    def point_line_dist(self, F, kp1, kp2, qi, kj):
        """FP64 Eq. 3 distance for each listed (query i, keypoint j) pair."""
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
        kp1 = np.ascontiguousarray(kp1, dtype=np.float32)
        kp2 = np.ascontiguousarray(kp2, dtype=np.float32)
        qi = np.ascontiguousarray(qi, dtype=np.int64)
        kj = np.ascontiguousarray(kj, dtype=np.int64)
        out = np.zeros(len(qi), np.float64)
        self.lib.oracle_point_line_dist(_ptr(F), _ptr(kp1), _ptr(kp2), _ptr(qi), _ptr(kj),
                                        len(qi), _ptr(out))
        return out

    def candidate_terms(self, F, kp1, kp2, eps, qi, kj):
        """Both sides of the Eq. 3 comparison, (|a x + b y + c|, eps sqrt(a^2+b^2)),
        for listed (i, j) pairs; j is a candidate of i iff num <= rhs."""
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
        kp1 = np.ascontiguousarray(kp1, dtype=np.float32)
        kp2 = np.ascontiguousarray(kp2, dtype=np.float32)
        if np.ndim(eps) == 0:
            e_arr, e_s = None, float(np.float32(eps))
        else:
            e_arr, e_s = np.ascontiguousarray(eps, dtype=np.float32), 0.0
        qi = np.ascontiguousarray(qi, dtype=np.int64)
        kj = np.ascontiguousarray(kj, dtype=np.int64)
        num = np.zeros(len(qi), np.float64)
        rhs = np.zeros(len(qi), np.float64)
        self.lib.oracle_candidate_terms(_ptr(F), _ptr(kp1), _ptr(kp2), _ptr(e_arr), e_s,
                                        _ptr(qi), _ptr(kj), len(qi), _ptr(num), _ptr(rhs))
        return num, rhs

    def match(self, desc1, desc2, row_offsets, col_indices, ratio=0.0, binary=False,
              col_base=None, row_base1=None, nthreads=0):
        """Nearest neighbour over candidate rows (Sec. 4.3).

        Float descriptors: canonical FP32 squared L2.  Binary (uint32 words):
        Hamming.  Returns (best_idx int32, best_dist float32, second_dist float32)."""
        row_offsets = np.ascontiguousarray(row_offsets, dtype=np.int64)
        col_indices = np.ascontiguousarray(col_indices, dtype=np.int32)
        if col_indices.size == 0:
            col_indices = np.zeros(1, np.int32)
        m = row_offsets.shape[0] - 1
        dt = np.uint32 if binary else np.float32
        desc1 = np.ascontiguousarray(desc1, dtype=dt)
        desc2 = np.ascontiguousarray(desc2, dtype=dt)
        dim = desc1.shape[1]
        cb = None if col_base is None else np.ascontiguousarray(col_base, dtype=np.int64)
        rb = None if row_base1 is None else np.ascontiguousarray(row_base1, dtype=np.int64)
        bi = np.zeros(max(m, 1), np.int32)
        bd = np.zeros(max(m, 1), np.float32)
        sd = np.zeros(max(m, 1), np.float32)
        self.lib.oracle_match(1 if binary else 0, _ptr(desc1), _ptr(desc2), dim,
                              _ptr(row_offsets), _ptr(col_indices), _ptr(cb), _ptr(rb), m,
                              float(ratio), _ptr(bi), _ptr(bd), _ptr(sd), int(nthreads))
        return bi[:m].copy(), bd[:m].copy(), sd[:m].copy()

    def desc_dist_f32(self, a, b):
        a = np.ascontiguousarray(a, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        return float(self.lib.oracle_desc_dist_f32(_ptr(a), _ptr(b), a.shape[0]))

    def desc_dist_f64(self, desc1, desc2, qi, kj):
        desc1 = np.ascontiguousarray(desc1, dtype=np.float32)
        desc2 = np.ascontiguousarray(desc2, dtype=np.float32)
        qi = np.ascontiguousarray(qi, dtype=np.int64)
        kj = np.ascontiguousarray(kj, dtype=np.int64)
        out = np.zeros(len(qi), np.float64)
        self.lib.oracle_desc_dist_f64_pairs(_ptr(desc1), _ptr(desc2), desc1.shape[1],
                                            _ptr(qi), _ptr(kj), len(qi), _ptr(out))
        return out

    def candidates_batch(self, pairs_F, kp1, kp2, eps, q_begin, m, k_begin, n, nthreads=0):
        """Per-pair brute force over a concatenated batch; one CSR whose column
        indices are local to each pair."""
        offs_all = [np.zeros(1, np.int64)]
        cols_all, deg_all = [], []
        base = 0
        for F, qb, mm, kb, nn in zip(pairs_F, q_begin, m, k_begin, n):
            e = eps if np.ndim(eps) == 0 else eps[kb:kb + nn]
            o, c, d = self.candidates(F, kp1[qb:qb + mm], kp2[kb:kb + nn], e, nthreads)
            offs_all.append(o[1:] + base)
            base += int(o[-1])
            cols_all.append(c)
            deg_all.append(d)
        offs = np.concatenate(offs_all)
        cols = np.concatenate(cols_all) if cols_all else np.zeros(0, np.int32)
        deg = np.concatenate(deg_all) if deg_all else np.zeros(0, np.uint8)
        return offs, cols, deg


_default = None


def _lib():
    global _default
    if _default is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _default = OracleLib(_LIB_PATH)
    return _default


def default_threads():
    return _lib().default_threads()


def candidates(*a, **k):
    return _lib().candidates(*a, **k)


def point_line_dist(*a, **k):
    return _lib().point_line_dist(*a, **k)


def match(*a, **k):
    return _lib().match(*a, **k)


def candidate_terms(*a, **k):
    return _lib().candidate_terms(*a, **k)


def desc_dist_f32(*a, **k):
    return _lib().desc_dist_f32(*a, **k)


def desc_dist_f64(*a, **k):
    return _lib().desc_dist_f64(*a, **k)


def candidates_batch(*a, **k):
    return _lib().candidates_batch(*a, **k)
