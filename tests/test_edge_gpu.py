"""Edge cases through every path (separate calls, fused call, recorded
graph): empty pairs and batches, the textbook special cases of the paper's
geometry, and a tolerance that covers the whole image."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, fp8_rows, specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_all(pairs, eps, ratio=0.0):
    """CSR and matches of the three paths, as NumPy arrays."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    b = synth.batch_pairs(pairs)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    kp1 = g(b.kp1.reshape(-1, 2).astype(np.float32))
    kp2 = g(b.kp2.reshape(-1, 2).astype(np.float32))
    d1 = g(b.desc1.reshape(-1, 128).astype(np.float32))
    d2 = g(b.desc2.reshape(-1, 128).astype(np.float32))
    specs = specs_of(pairs)
    out = {}
    idx = E.Index(specs, kp2, eps=eps)
    o, c = idx.query(kp1)
    res = idx.match(o, c, d1, d2, ratio=ratio)
    out["separate"] = [x.cpu().numpy() for x in (o, c) + tuple(res)]
    out["fused"] = [x.cpu().numpy() for x in idx.query_match(kp1, d1, d2, ratio=ratio)]
    # the BF16 and FP8 selections fused into the stabbing pass (exact on the masters)
    h1, h2 = b.desc1.reshape(-1, 128), b.desc2.reshape(-1, 128)
    q1 = g(synth.f32_to_bf16(h1).view(np.int16))
    q2 = g(synth.f32_to_bf16(h2).view(np.int16))
    out["fused_bf16"] = [x.cpu().numpy()
                         for x in idx.query_match_bf16(kp1, q1, q2, d1, d2, ratio=ratio)]
    if h2.shape[0] > 0:
        c2, s2, e2 = fp8_rows(h2)
        out["fused_fp8"] = [x.cpu().numpy()
                            for x in idx.query_match_fp8(kp1, g(c2), g(s2), g(e2), d1, d2,
                                                         ratio=ratio)]
    nnz = int(out["separate"][0][-1])
    bt = E.Batch(specs, kp1, kp2, d1, d2, nnz + 8, eps=eps, ratio=ratio)
    bt.launch()
    out["graph"] = [x.cpu().numpy() for x in bt.outputs()]
    bt.close()
    return out


def _oracle(pairs, eps, ratio=0.0):
    b = synth.batch_pairs(pairs)
    offs, cols = [np.zeros(1, np.int64)], []
    base = 0
    for p in pairs:
        if p.m == 0:
            continue
        if p.n == 0:
            offs.append(np.full(p.m, base, np.int64))
            continue
        o, c, _ = oracle.candidates(p.F, p.kp1, p.kp2, eps)
        offs.append(o[1:] + base)
        base += int(o[-1])
        cols.append(c)
    ro = np.concatenate(offs)
    rc = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    rows = np.repeat(np.arange(len(pairs)), [p.m for p in pairs])
    if len(rows) == 0:
        z = np.zeros(0)
        return ro, rc, z.astype(np.int32), z.astype(np.float32), z.astype(np.float32)
    rb, rbd, rsd = oracle.match(b.desc1.reshape(-1, 128), b.desc2.reshape(-1, 128), ro, rc,
                                ratio=ratio, col_base=b.k_begin[rows])
    return ro, rc, rb, rbd, rsd


def _check(out, ref, what):
    for path, got in out.items():
        assert_csr_equal((got[0], got[1]), (ref[0], ref[1]), f"{what} {path}")
        for a, r in zip(got[2:], ref[2:]):
            assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(r).view(np.uint8)), \
                f"{what} {path}"


def _cut(p, m, n):
    """A copy of pair p keeping the first m image-1 and n image-2 keypoints."""
    import copy
    q = copy.copy(p)
    q.kp1, q.desc1 = p.kp1[:m].copy(), p.desc1[:m].copy()
    q.kp2, q.desc2 = p.kp2[:n].copy(), p.desc2[:n].copy()
    q.gt12 = np.where(p.gt12[:m] < n, p.gt12[:m], -1)
    return q


def test_empty_pairs_inside_a_batch():
    base = [synth.cfg0_pair(r) for r in range(4)]
    pairs = [_cut(base[0], 0, 500), base[1], _cut(base[2], 700, 0), _cut(base[3], 0, 0),
             _cut(base[0], 300, 1000)]
    log("batch with empty pairs")
    _check(_run_all(pairs, 2.0, 0.8), _oracle(pairs, 2.0, 0.8), "empty pairs")


def test_batch_without_queries():
    pairs = [_cut(synth.cfg0_pair(0), 0, 800)]
    log("no queries at all")
    out = _run_all(pairs, 2.0)
    for path, got in out.items():
        assert list(got[0]) == [0] and got[1].size == 0 and got[2].size == 0, path


def _hand_pair(F, W, H, m, n, seed):
    rng = np.random.default_rng(seed)
    p = synth.cfg0_pair(0)
    import copy
    q = copy.copy(p)
    q.F = np.asarray(F, np.float64)
    q.W, q.H = W, H
    q.kp1 = np.stack([rng.uniform(0, W, m), rng.uniform(0, H, m)], 1).astype(np.float32)
    q.kp2 = np.stack([rng.uniform(0, W, n), rng.uniform(0, H, n)], 1).astype(np.float32)
    q.desc1 = p.desc1[:m].copy()
    q.desc2 = p.desc2[:n].copy()
    q.gt12 = np.full(m, -1, np.int32)
    return q


def test_rectified_stereo_is_a_range_query():
    """Epipole at infinity (t = (1, 0, 0), K = I): the candidates of query i are
    exactly {j : |y_j - y_i| <= eps}, a 1-D range query."""
    F = [[0, 0, 0], [0, 0, -1], [0, 1, 0]]
    p = _hand_pair(F, 640, 480, 900, 1000, 3)
    log("rectified stereo")
    out = _run_all([p], 1.5)
    y1, y2 = p.kp1[:, 1].astype(np.float64), p.kp2[:, 1].astype(np.float64)
    for path, got in out.items():
        o, c = got[0], got[1]
        for i in range(0, p.m, 37):
            want = np.nonzero(np.abs(y2 - y1[i]) <= 1.5)[0]
            assert np.array_equal(c[o[i]:o[i + 1]], want), (path, i)
    _check(out, _oracle([p], 1.5), "rectified")


def test_forward_motion_keeps_circles_around_the_epipole():
    """Pure forward motion (epipole at the origin, K = I): every keypoint
    within eps of the epipole is a candidate of every query."""
    F = [[0, -1, 0], [1, 0, 0], [0, 0, 0]]
    p = _hand_pair(F, 640, 480, 800, 900, 4)
    p.kp1 -= np.float32([320, 240])
    p.kp2 -= np.float32([320, 240])
    p.kp2[:5] = np.float32([[0.5, 0.5], [-1.0, 0.2], [0.0, 0.0], [1.4, -0.1], [0.0, -1.9]])
    log("forward motion")
    out = _run_all([p], 2.0)
    for path, got in out.items():
        o, c = got[0], got[1]
        for i in range(p.m):
            row = set(c[o[i]:o[i + 1]].tolist())
            assert {0, 1, 2, 3, 4} <= row, (path, i)
    _check(out, _oracle([p], 2.0), "forward")


def test_tolerance_covering_the_image_is_brute_force_matching():
    p = synth.cfg0_pair(1)
    log("eps beyond the image diagonal")
    out = _run_all([p], 2000.0)
    for path, got in out.items():
        assert np.all(np.diff(got[0]) == p.n), path
    _check(out, _oracle([p], 2000.0), "full rows")


def test_tiny_tolerance_keeps_noiseless_true_matches():
    """eps = 1e-3 px on noiseless keypoints: every true match is still a
    candidate (the FP32 storage error is far below 1e-3 px at 640 px)."""
    import copy
    p0 = synth.cfg0_pair(2)
    p = copy.copy(p0)
    p.kp1, p.kp2 = p0.clean1.copy(), p0.clean2.copy()
    log("eps 1e-3 on noiseless keypoints")
    out = _run_all([p], 1e-3)
    o, c = out["fused"][0], out["fused"][1]
    t = np.nonzero(p.gt12 >= 0)[0]
    for i in t:
        assert p.gt12[i] in c[o[i]:o[i + 1]]
    _check(out, _oracle([p], 1e-3), "tiny eps")


def test_single_keypoint_and_keypoints_outside_the_image():
    p = _cut(synth.cfg0_pair(3), 600, 1)
    log("one image-2 keypoint")
    _check(_run_all([p], 50.0), _oracle([p], 50.0), "n = 1")
    import copy
    q = copy.copy(synth.cfg0_pair(4))
    rng = np.random.default_rng(8)
    q.kp1 = q.kp1 + rng.uniform(-900, 900, q.kp1.shape).astype(np.float32)
    q.kp2 = q.kp2 + rng.uniform(-900, 900, q.kp2.shape).astype(np.float32)
    log("keypoints outside the image")
    _check(_run_all([q], 4.0), _oracle([q], 4.0), "outside")


def test_epipole_on_the_image_border():
    """Translation towards a point on the right border of image 2."""
    W, H, f = 640, 480, 500.0
    # camera 2 centre along the ray of the border pixel (W, H/2)
    ray = np.array([(W - W / 2) / f, 0.0, 1.0])
    C2 = ray / np.linalg.norm(ray)
    p = synth.make_pair(W, H, f, np.eye(3), C2, 800, 200, 200, 77)
    e = p.e2 / p.e2[2]
    assert abs(e[0] - W) < 1e-6 and abs(e[1] - H / 2) < 1e-6
    log("epipole on the border")
    _check(_run_all([p], 2.0), _oracle([p], 2.0), "border epipole")
