"""Pins for the CPU oracle: each test checks the oracle against something the
paper or plain mathematics fixes, never against a retyped copy of itself."""

import math
from fractions import Fraction

import numpy as np
import pytest

import synth


def rows_of(offs, cols):
    return [cols[offs[i]:offs[i + 1]].tolist() for i in range(len(offs) - 1)]


def rand_kp(rng, k, w, h):
    return np.stack([rng.uniform(0, w, k), rng.uniform(0, h, k)], 1).astype(np.float32)


# --------------------------------------------------------------- hand cases

def test_h1_rectified_stereo_is_1d_range_query(oracle_lib):
    """K = I, R = I, t = (1,0,0): F = [t]x, every line is y = y_i (the
    1-D scanline case of the introduction); candidates are a 1-D range query
    answered here by sorting and bisection."""
    F = synth.skew([1.0, 0.0, 0.0])
    rng = np.random.default_rng(1)
    kp1 = rand_kp(rng, 300, 640, 480)
    kp2 = rand_kp(rng, 400, 640, 480)
    eps = np.float32(2.5)
    offs, cols, deg = oracle_lib.candidates(F, kp1, kp2, eps)
    assert not deg.any()
    order = np.argsort(kp2[:, 1].astype(np.float64), kind="stable")
    ys = kp2[order, 1].astype(np.float64)
    for i in range(len(kp1)):
        y = float(kp1[i, 1])
        lo = np.searchsorted(ys, y - float(eps), side="left")
        hi = np.searchsorted(ys, y + float(eps), side="right")
        expect = sorted(order[lo:hi].tolist())
        assert cols[offs[i]:offs[i + 1]].tolist() == expect


def test_h1_per_keypoint_tolerance(oracle_lib):
    """Per-keypoint eps (Sec. 4.2): in the scanline case j is a candidate of
    i exactly when the closed interval [y_j - eps_j, y_j + eps_j] holds y_i."""
    F = synth.skew([1.0, 0.0, 0.0])
    rng = np.random.default_rng(2)
    kp1 = rand_kp(rng, 200, 640, 480)
    kp2 = rand_kp(rng, 300, 640, 480)
    eps = rng.uniform(0.25, 6.0, 300).astype(np.float32)
    offs, cols, _ = oracle_lib.candidates(F, kp1, kp2, eps)
    lo = kp2[:, 1].astype(np.float64) - eps
    hi = kp2[:, 1].astype(np.float64) + eps
    for i in range(len(kp1)):
        y = float(kp1[i, 1])
        expect = [j for j in range(300) if lo[j] <= y <= hi[j]]
        got = cols[offs[i]:offs[i + 1]].tolist()
        # lo/hi are rounded sums: only points inside a 1e-9 band may differ
        diff = set(expect) ^ set(got)
        for j in diff:
            assert abs(abs(y - float(kp2[j, 1])) - float(eps[j])) < 1e-9
        assert got == sorted(got)


def test_h2_forward_motion_closed_form(oracle_lib):
    """K = I, R = I, t = (0,0,1): F = [t]x, epipole at the origin, l_i =
    (-y_i, x_i, 0) and dist = |x_i y_j - y_i x_j| / |p_i|."""
    F = synth.skew([0.0, 0.0, 1.0])
    rng = np.random.default_rng(3)
    kp1 = rand_kp(rng, 200, 200, 200) - np.float32(100)
    kp2 = rand_kp(rng, 300, 200, 200) - np.float32(100)
    kp1[0] = (0.0, 0.0)  # query on the image-1 epipole: zero line
    eps = 1.5
    offs, cols, deg = oracle_lib.candidates(F, kp1, kp2, eps)
    assert deg[0] == 1 and offs[1] == offs[0]
    assert deg[1:].sum() == 0
    x1, y1 = kp1[:, 0].astype(np.float64), kp1[:, 1].astype(np.float64)
    x2, y2 = kp2[:, 0].astype(np.float64), kp2[:, 1].astype(np.float64)
    d = np.abs(np.outer(x1, y2) - np.outer(y1, x2)) / np.hypot(x1, y1)[:, None]
    near = np.hypot(x2, y2) <= eps
    for i in range(1, len(kp1)):
        got = set(cols[offs[i]:offs[i + 1]].tolist())
        # circles containing the epipole are hit by every line (Sec. 4.4)
        assert set(np.where(near)[0].tolist()) <= got
        for j in range(len(kp2)):
            if abs(d[i, j] - eps) > 1e-9:
                assert (j in got) == (d[i, j] <= eps)


def test_h3_wraparound_worked_case(oracle_lib):
    """Epipole at the origin, eps = 1, keypoint (10, 0.5).  Eq. 5-6 give
    theta = atan(0.05), delta = asin(1/|p|); the interval wraps below 0 and
    splits at 0/pi (Sec. 4.4).  Lines at angles 3.12, 0.15, 0.20 and 0 rad
    lie at distances |10 sin a - 0.5 cos a| = 0.7158, 0.99999579, 1.4967, 0.5:
    in, in (on the boundary side), out, in."""
    import oracle
    F = synth.skew([0.0, 0.0, 1.0])
    kp2 = np.array([[10.0, 0.5]], np.float32)
    alphas = [3.12, 0.15, 0.20, 0.0]
    expect = [True, True, False, True]
    kp1 = np.array([[math.cos(a), math.sin(a)] for a in alphas], np.float32)
    offs, cols, _ = oracle_lib.candidates(F, kp1, kp2, 1.0)
    got = [offs[i + 1] > offs[i] for i in range(4)]
    assert got == expect
    for a, dd in zip(alphas, [0.715793201, 0.999995786, 1.496660019, 0.5]):
        assert abs(abs(10 * math.sin(a) - 0.5 * math.cos(a)) - dd) < 1e-8
    # the paper's intervals for this keypoint: split into two pieces
    iv = oracle.paper_angle.paper_intervals(kp2.astype(np.float64), (0.0, 0.0), 1.0)[0]
    theta, delta = math.atan2(0.5, 10.0), math.asin(1.0 / math.hypot(10.0, 0.5))
    assert abs(theta - 0.049958396) < 1e-9 and abs(delta - 0.100042027) < 1e-9
    assert len(iv) == 2
    assert abs(iv[0][0] - 3.091509022) < 1e-8 and iv[0][1] == math.pi
    assert iv[1][0] == 0.0 and abs(iv[1][1] - 0.150000423) < 1e-8
    rows = oracle.paper_angle_candidates(F, kp1, kp2, 1.0)
    assert [len(r) > 0 for r in rows] == expect


def test_h4_circles_containing_the_epipole(oracle_lib):
    """Sec. 4.4: a keypoint within eps of e2 is returned by every query."""
    p = synth.cfg1_pair("forward_yaw", n_kp=2000)
    e = p.e2[:2] / p.e2[2]
    rng = np.random.default_rng(4)
    ang = rng.uniform(0, 2 * np.pi, 20)
    rad = rng.uniform(0, 1.9, 20)
    extra = np.stack([e[0] + rad * np.cos(ang), e[1] + rad * np.sin(ang)], 1).astype(np.float32)
    kp2 = np.concatenate([p.kp2[:500], extra])
    offs, cols, deg = oracle_lib.candidates(p.F, p.kp1[:400], kp2, 2.0)
    for i in range(400):
        if deg[i]:
            continue
        row = set(cols[offs[i]:offs[i + 1]].tolist())
        assert set(range(500, 520)) <= row


def test_h5_eps_beyond_diagonal_is_brute_force(oracle_lib):
    """eps >= image diagonal: every row holds every keypoint, and guided
    nearest neighbour equals unguided brute-force nearest neighbour."""
    p = synth.cfg0_pair(0)
    m = 120
    offs, cols, deg = oracle_lib.candidates(p.F, p.kp1[:m], p.kp2, 1.0e4)
    n = p.n
    assert (np.diff(offs) == n).all()
    assert (cols.reshape(m, n) == np.arange(n)).all()
    bi, bd, sd = oracle_lib.match(p.desc1[:m], p.desc2, offs, cols)
    d64 = ((p.desc1[:m, None, :].astype(np.float64) - p.desc2[None].astype(np.float64)) ** 2).sum(-1)
    srt = np.sort(d64, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-5 * srt[:, 1]
    assert clear.sum() > m // 2
    assert (bi[clear] == d64.argmin(1)[clear]).all()
    assert np.allclose(bd, srt[:, 0], rtol=1e-5) and np.allclose(sd, srt[:, 1], rtol=1e-5)


# --------------------------------------------------------------- invariants

def test_i1_noiseless_true_matches_are_candidates(oracle_lib):
    """x2^T F x1 = 0 for true correspondences (Sec. 3, Eq. 2): with the
    noiseless projections stored in FP32 every true partner lies within
    1e-3 px of its epipolar line (FP32 storage error at 6048 px is ~2.4e-4)."""
    for motion in ("sideways", "forward", "forward_yaw"):
        p = synth.cfg1_pair(motion, n_kp=3000)
        offs, cols, _ = oracle_lib.candidates(p.F, p.clean1, p.clean2, 1e-3)
        for i in np.where(p.gt12 >= 0)[0]:
            assert p.gt12[i] in cols[offs[i]:offs[i + 1]]


def test_i2_monotone_in_eps(oracle_lib):
    p = synth.cfg0_pair(1)
    rows = []
    for eps in (0.5, 1.0, 2.0, 4.0):
        o, c, _ = oracle_lib.candidates(p.F, p.kp1, p.kp2, eps)
        rows.append([set(r) for r in rows_of(o, c)])
    for a, b in zip(rows, rows[1:]):
        assert all(x <= y for x, y in zip(a, b))
    assert sum(map(len, rows[0])) < sum(map(len, rows[-1]))


def test_i3_scaling_and_sign_of_F(oracle_lib):
    p = synth.cfg1_pair("forward_yaw", n_kp=1500)
    ref = oracle_lib.candidates(p.F, p.kp1, p.kp2, 2.0)
    for s in (2.0 ** 20, 2.0 ** -30, -1.0, -(2.0 ** 7)):
        got = oracle_lib.candidates(p.F * s, p.kp1, p.kp2, 2.0)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])


def test_i4_permutation_equivariance(oracle_lib):
    p = synth.cfg0_pair(2)
    rng = np.random.default_rng(5)
    pq = rng.permutation(p.m)
    pk = rng.permutation(p.n)
    inv = np.empty_like(pk)
    inv[pk] = np.arange(p.n)
    o, c, _ = oracle_lib.candidates(p.F, p.kp1, p.kp2, 2.0)
    o2, c2, _ = oracle_lib.candidates(p.F, p.kp1[pq], p.kp2[pk], 2.0)
    r1, r2 = rows_of(o, c), rows_of(o2, c2)
    for new_i, old_i in enumerate(pq):
        assert sorted(pk[r2[new_i]].tolist()) == r1[old_i]


def test_i5_image_swap_symmetry(oracle_lib):
    """Swapping the images and using F^T: e1 = null(F) becomes the swapped
    problem's e2; x2^T F x1 = x1^T F^T x2; noiseless true matches are
    candidates both ways; and the two candidate relations coincide once the
    tolerance is rescaled by |(F^T x2)_12| / |(F x1)_12|."""
    from oracle.paper_angle import epipole_image2
    p = synth.cfg1_pair("sideways", n_kp=1500)
    e1 = epipole_image2(p.F.T)
    assert np.allclose(np.cross(e1, p.e1 / np.linalg.norm(p.e1)), 0, atol=1e-9)
    o, c, _ = oracle_lib.candidates(p.F.T, p.clean2, p.clean1, 1e-3)
    inv = {int(g): i for i, g in enumerate(p.gt12) if g >= 0}
    for j, i in inv.items():
        assert i in c[o[j]:o[j + 1]]
    # rescaled tolerance: brute force on a tiny sample
    rng = np.random.default_rng(6)
    eps = 3.0
    qi = rng.choice(p.m, 25, replace=False)
    kj = rng.choice(p.n, 40, replace=False)
    o, c, _ = oracle_lib.candidates(p.F, p.kp1[qi], p.kp2[kj], eps)
    rows = rows_of(o, c)
    F = p.F
    checked = 0
    for a, i in enumerate(qi):
        x1 = np.array([p.kp1[i, 0], p.kp1[i, 1], 1.0], np.float64)
        l1 = F @ x1
        for b, j in enumerate(kj):
            x2 = np.array([p.kp2[j, 0], p.kp2[j, 1], 1.0], np.float64)
            l2 = F.T @ x2
            eps_sw = eps * math.hypot(l1[0], l1[1]) / math.hypot(l2[0], l2[1])
            d = abs(x2 @ l1) / math.hypot(l1[0], l1[1])
            if abs(d - eps) < 1e-6:
                continue
            o2, c2, _ = oracle_lib.candidates(F.T, p.kp2[j:j + 1], p.kp1[i:i + 1], eps_sw)
            assert (b in rows[a]) == (o2[1] == 1)
            checked += 1
    assert checked > 900


# ------------------------------------------------- paper angular formulation

@pytest.mark.parametrize("where", ["inside", "outside", "far1e6", "far1e8", "centre"])
def test_paper_angle_form_agrees_with_brute_force(oracle_lib, where):
    """The paper's tangent-angle stabbing (Eq. 5-7, Algorithm 1, Sec. 4.4)
    returns the brute-force sets except within 1e-6 px of the boundary."""
    import oracle
    W, H, f = 640, 480, 500.0
    if where == "inside":
        R, C2 = synth.rot_axis_angle([0, 1, 0], 0.05), [0.2, 0.1, 1.0]
    elif where == "outside":
        R, C2 = synth.rot_axis_angle([0, 1, 0], 0.17), [1.0, 0.0, 0.0]
    elif where == "far1e6":
        R, C2 = synth.rot_axis_angle([0, 1, 0], 5e-4), [1.0, 0.0, 0.0]
    elif where == "far1e8":
        R, C2 = synth.rot_axis_angle([0, 1, 0], 5e-6), [1.0, 0.0, 0.0]
    else:
        R, C2 = np.eye(3), [0.0, 0.0, 1.0]
    p = synth.make_pair(W, H, f, R, C2, 150, 50, 50, seed=77, float_desc=False)
    rng = np.random.default_rng(8)
    eps = rng.uniform(0.5, 8.0, p.n).astype(np.float32)
    o, c, deg = oracle_lib.candidates(p.F, p.kp1, p.kp2, eps)
    brute = rows_of(o, c)
    for mode in ("direction", "paper"):
        if mode == "paper" and where == "centre":
            continue  # Eq. 7 degenerates: q_i is the epipole itself
        ang = oracle.paper_angle_candidates(p.F, p.kp1, p.kp2, eps, mode=mode,
                                            centre=(W / 2.0, H / 2.0))
        bad = 0
        for i in range(p.m):
            for j in set(ang[i]) ^ set(brute[i]):
                d = oracle_lib.point_line_dist(p.F, p.kp1, p.kp2, [i], [j])[0]
                assert abs(d - eps[j]) <= 1e-6, (mode, i, j, d, eps[j])
                bad += 1
        assert bad <= 2


# ----------------------------------------------------------------- matching

def _round_f32(fr):
    x = np.float32(float(fr))
    cands = [np.nextafter(x, np.float32(-np.inf)), x, np.nextafter(x, np.float32(np.inf))]
    return min(cands, key=lambda v: (abs(Fraction(float(v)) - fr),
                                     int(np.array(v, np.float32).view(np.uint32)) & 1))


def test_canonical_fp32_distance_is_exactly_rounded_chain(oracle_lib):
    """Each step of the canonical FP32 distance is one correctly rounded
    operation: checked with exact rational arithmetic."""
    rng = np.random.default_rng(9)
    for _ in range(6):
        a = synth.pairs._unit_rows(rng.standard_normal((1, 128)))[0]
        b = synth.pairs._unit_rows(rng.standard_normal((1, 128)))[0]
        acc = np.float32(0.0)
        for k in range(128):
            t = _round_f32(Fraction(float(a[k])) - Fraction(float(b[k])))
            acc = _round_f32(Fraction(float(t)) * Fraction(float(t)) + Fraction(float(acc)))
        got = np.float32(oracle_lib.desc_dist_f32(a, b))
        assert got.view(np.uint32) == np.float32(acc).view(np.uint32)
        ref = float(((a.astype(np.float64) - b.astype(np.float64)) ** 2).sum())
        assert abs(float(got) - ref) <= 1e-5 * ref


def test_selection_orders_by_distance_then_index(oracle_lib):
    rng = np.random.default_rng(10)
    base = synth.pairs._unit_rows(rng.standard_normal((6, 128)))
    d2 = base[rng.integers(0, 6, 40)]  # many exact ties
    d1 = base[rng.integers(0, 6, 25)] + np.float32(0.01)
    offs = [0]
    cols = []
    for i in range(25):
        k = int(rng.integers(0, 9))
        row = sorted(rng.choice(40, k, replace=False).tolist())
        cols += row
        offs.append(len(cols))
    offs = np.array(offs, np.int64)
    cols = np.array(cols, np.int32)
    bi, bd, sd = oracle_lib.match(d1, d2, offs, cols)
    for i in range(25):
        row = cols[offs[i]:offs[i + 1]].tolist()
        ds = sorted((oracle_lib.desc_dist_f32(d1[i], d2[j]), j) for j in row)
        if not ds:
            assert bi[i] == -1 and np.isinf(bd[i]) and np.isinf(sd[i])
            continue
        assert bi[i] == ds[0][1] and bd[i] == np.float32(ds[0][0])
        assert sd[i] == (np.float32(ds[1][0]) if len(ds) > 1 else np.inf)


def test_ratio_test(oracle_lib):
    d1 = np.zeros((3, 128), np.float32)
    d2 = np.zeros((4, 128), np.float32)
    d2[0, 0], d2[1, 0], d2[2, 0], d2[3, 0] = 0.5, 0.6, 0.1, 0.12
    # row 0: {0,1}: 0.25 vs 0.36: 0.25 < 0.64*0.36=0.2304? no -> rejected
    # row 1: {2,1}: 0.01 vs 0.36 -> accepted; row 2: {3}: singleton -> accepted
    offs = np.array([0, 2, 4, 5], np.int64)
    cols = np.array([0, 1, 1, 2, 3], np.int32)
    bi, bd, sd = oracle_lib.match(d1, d2, offs, cols, ratio=0.8)
    assert bi.tolist() == [-1, 2, 3]
    assert np.isinf(sd[2]) and bd[0] == np.float32(0.25)


def test_hamming_against_numpy_bitcount(oracle_lib):
    p = synth.cfg0_pair(3, binary=True)
    o, c, _ = oracle_lib.candidates(p.F, p.kp1, p.kp2, 3.0)
    bi, bd, sd = oracle_lib.match(p.bin1, p.bin2, o, c, binary=True)
    for i in range(p.m):
        row = c[o[i]:o[i + 1]]
        if len(row) == 0:
            assert bi[i] == -1
            continue
        h = np.bitwise_count(p.bin1[i][None, :] ^ p.bin2[row]).sum(1)
        order = np.lexsort((row, h))
        assert bi[i] == row[order[0]] and bd[i] == h[order[0]]
        if len(row) > 1:
            assert sd[i] == h[order[1]]
    # true partners with 8% flips are usually the best Hamming match
    ok = (p.gt12 >= 0) & (bi >= 0)
    assert (bi[ok] == p.gt12[ok]).mean() > 0.95


def test_closed_boundary_on_integer_grid(oracle_lib):
    """Eq. 3 uses <=: keypoints exactly eps away from the line are candidates
    (scanline case with integer coordinates, where every distance is exact)."""
    F = synth.skew([1.0, 0.0, 0.0])
    ys = np.arange(0, 40, dtype=np.float32)
    kp1 = np.stack([np.full(40, 3.0, np.float32), ys], 1)
    kp2 = np.stack([np.full(40, 7.0, np.float32), ys], 1)
    offs, cols, _ = oracle_lib.candidates(F, kp1, kp2, 2.0)
    for i in range(40):
        assert cols[offs[i]:offs[i + 1]].tolist() == [j for j in range(40) if abs(i - j) <= 2]
