"""Pins of the oracle's listed-pair helpers: the Eq. 3 distance and the two
sides of the Eq. 3-4 comparison for listed (query, keypoint) pairs, and the
FP64 descriptor distance used as the error reference of the reduced-precision
paths.  Each value comes from a hand computation or from exact rational
arithmetic, never from a retyped copy of the oracle's formula."""

import math
from fractions import Fraction

import numpy as np

import synth


def _unit(a):
    return (math.cos(a), math.sin(a))


def test_point_line_dist_wraparound_hand_values(oracle_lib):
    """Epipole at the origin (F = [t]x with t = (0, 0, 1)): the query at
    3 (cos a, sin a) has the line (-3 sin a, 3 cos a, 0), whose distance to
    (10, 0.5) is |10 sin a - 0.5 cos a|, computed by hand for the wrap-around
    case of Sec. 4.4: 0.715793201, 0.999995786, 1.496660019 and 0.5 at
    a = 3.12, 0.15, 0.20 and 0.  The factor 3 makes sqrt(a^2 + b^2) = 3, so a
    missing square root or a wrong norm cannot pass."""
    F = synth.skew([0.0, 0.0, 1.0])
    alphas = [3.12, 0.15, 0.20, 0.0]
    hand = [0.715793201, 0.999995786, 1.496660019, 0.5]
    kp1 = np.array([[3.0 * c, 3.0 * s] for c, s in map(_unit, alphas)], np.float32)
    kp2 = np.array([[10.0, 0.5]], np.float32)
    d = oracle_lib.point_line_dist(F, kp1, kp2, np.arange(4), np.zeros(4, np.int64))
    # kp1 is rounded to FP32 (relative 6e-8): the distance moves by at most
    # |p2| * 1e-7 ~ 1e-6
    for got, want in zip(d, hand):
        assert abs(got - want) < 2e-6, (got, want)
    num, rhs = oracle_lib.candidate_terms(F, kp1, kp2, 1.0, np.arange(4), np.zeros(4, np.int64))
    for t, want in enumerate(hand):
        assert abs(rhs[t] - 3.0) < 1e-6
        assert abs(num[t] / 3.0 - want) < 2e-6
    assert [bool(x <= y) for x, y in zip(num, rhs)] == [True, True, False, True]


def test_terms_on_integer_lines_are_exact(oracle_lib):
    """F = [[0,0,3],[0,0,4],[0,1,0]] gives every query the line
    (3, 4, y_i): with integer coordinates |3 x_j + 4 y_j + y_i| and
    eps * 5 are exact integers (times eps), and the distance is that integer
    over 5.  Columns of F, transposition, sign and norm mistakes all change
    these values."""
    F = np.array([[0.0, 0.0, 3.0], [0.0, 0.0, 4.0], [0.0, 1.0, 0.0]])
    rng = np.random.default_rng(21)
    kp1 = rng.integers(-50, 50, (30, 2)).astype(np.float32)
    kp2 = rng.integers(-50, 50, (40, 2)).astype(np.float32)
    eps = rng.integers(1, 9, 40).astype(np.float32) / np.float32(4)  # dyadic
    qi = np.repeat(np.arange(30), 40)
    kj = np.tile(np.arange(40), 30)
    num, rhs = oracle_lib.candidate_terms(F, kp1, kp2, eps, qi, kj)
    dist = oracle_lib.point_line_dist(F, kp1, kp2, qi, kj)
    for t in range(len(qi)):
        i, j = int(qi[t]), int(kj[t])
        v = abs(3 * int(kp2[j, 0]) + 4 * int(kp2[j, 1]) + int(kp1[i, 1]))
        assert num[t] == float(v)
        assert rhs[t] == float(Fraction(float(eps[j])) * 5)
        assert dist[t] == v / 5.0  # one correctly rounded division
    # the closed comparison of Eq. 3-4 agrees with the brute-force CSR
    offs, cols, _ = oracle_lib.candidates(F, kp1, kp2, eps)
    for i in range(30):
        want = [j for j in range(40) if num[i * 40 + j] <= rhs[i * 40 + j]]
        assert cols[offs[i]:offs[i + 1]].tolist() == want
    # some pairs sit exactly on the boundary (closed: they are candidates)
    assert (num == rhs).any()


def test_terms_scalar_and_per_keypoint_eps(oracle_lib):
    """A scalar tolerance is the per-keypoint tolerance with all eps_j equal
    (the reading of Sec. 4.2); rectified stereo (F = [t]x, t = (1, 0, 0))
    has the line (0, -1, y_i): num = |y_i - y_j|, rhs = eps."""
    F = synth.skew([1.0, 0.0, 0.0])
    kp1 = np.array([[1.0, 10.0], [2.0, -3.0]], np.float32)
    kp2 = np.array([[5.0, 12.5], [7.0, 10.0], [0.0, -6.0]], np.float32)
    qi = np.array([0, 0, 0, 1, 1, 1])
    kj = np.array([0, 1, 2, 0, 1, 2])
    num, rhs = oracle_lib.candidate_terms(F, kp1, kp2, 2.5, qi, kj)
    assert num.tolist() == [2.5, 0.0, 16.0, 15.5, 13.0, 3.0]
    assert rhs.tolist() == [2.5] * 6
    num2, rhs2 = oracle_lib.candidate_terms(F, kp1, kp2, np.full(3, 2.5, np.float32), qi, kj)
    assert num2.tolist() == num.tolist() and rhs2.tolist() == rhs.tolist()
    d = oracle_lib.point_line_dist(F, kp1, kp2, qi, kj)
    assert d.tolist() == num.tolist()


def test_desc_dist_f64_hand_cases(oracle_lib):
    """Squared L2 in FP64: orthogonal unit vectors are 2 apart, a vector is 0
    from itself, and dyadic entries give exact sums."""
    e = np.eye(128, dtype=np.float32)
    d1 = np.stack([e[0], e[5], 0.5 * e[0] + 0.25 * e[1]]).astype(np.float32)
    d2 = np.stack([e[1], e[5], -0.5 * e[0] + 0.75 * e[2]]).astype(np.float32)
    got = oracle_lib.desc_dist_f64(d1, d2, np.array([0, 1, 2, 0]), np.array([0, 1, 2, 2]))
    # (0.5 + 0.5)^2 + 0.25^2 + 0.75^2 = 1.625; e0 vs (-0.5, 0, 0.75): 2.25 + 0.5625
    assert got.tolist() == [2.0, 0.0, 1.625, 2.8125]


def test_desc_dist_f64_within_its_rounding_bound(oracle_lib):
    """Random unit rows: the FP64 result is within 128 * 2^-53 (relative) of
    the exact rational squared distance of the FP32 inputs; the canonical
    FP32 distance is within its own 130 * 2^-24 bound of it."""
    rng = np.random.default_rng(22)
    d1 = synth.pairs._unit_rows(rng.standard_normal((5, 128)))
    d2 = synth.pairs._unit_rows(rng.standard_normal((7, 128)))
    qi = np.array([0, 1, 2, 3, 4, 4])
    kj = np.array([0, 6, 2, 3, 1, 5])
    got = oracle_lib.desc_dist_f64(d1, d2, qi, kj)
    for t in range(len(qi)):
        a, b = d1[qi[t]], d2[kj[t]]
        exact = sum((Fraction(float(x)) - Fraction(float(y))) ** 2 for x, y in zip(a, b))
        assert abs(Fraction(got[t]) - exact) <= exact * Fraction(128, 2 ** 53)
        f32 = oracle_lib.desc_dist_f32(a, b)
        assert abs(Fraction(f32) - exact) <= exact * Fraction(130, 2 ** 24)
