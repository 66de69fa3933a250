"""Pins of the pose-uncertainty tolerance oracle (oracle/pose_eps.py): closed
forms, the spread of the distance under sampled poses, and hand cases of the
reverse epipolar segment -- never a retyped copy of its formulas."""

import numpy as np

from oracle import pose_eps as P


def _K(f, W, H):
    return np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])


def test_zero_covariance_gives_the_base_tolerance():
    K = _K(500.0, 640, 480)
    R0 = P.rodrigues(np.array([0.01, -0.02, 0.005]))
    t0 = np.array([0.9, 0.1, 0.2])
    kp2 = np.array([[10.0, 20.0], [320.0, 240.0], [630.0, 470.0]])
    eps = P.pose_eps(kp2, K, K, R0, t0, np.zeros((6, 6)), 640, 480, 1.5, 3.0, 50.0)
    assert eps.tolist() == [1.5, 1.5, 1.5]


def test_rectified_stereo_translation_y_closed_form():
    """K1 = K2, R = I, t = (1, 0, 0): every epipolar line is a pixel row.
    With only t_y uncertain (variance s2), the distance of x2 = (x', y') from
    the line of x1 = (x, y') moves by (x' - x) per unit t_y (the disparity),
    so sigma = sqrt(s2) * max(|x'|, |W1 - x'|) over the row."""
    W, H, f = 640, 480, 500.0
    K = _K(f, W, H)
    cov = np.zeros((6, 6))
    cov[4, 4] = 0.03 ** 2
    kp2 = np.array([[0.0, 17.0], [100.0, 240.0], [320.0, 300.0], [600.0, 479.0], [700.0, 5.0]])
    eps = P.pose_eps(kp2, K, K, np.eye(3), np.array([1.0, 0.0, 0.0]), cov, W, H, 2.0, 3.0, 1e9)
    want = 2.0 + 3.0 * 0.03 * np.maximum(np.abs(kp2[:, 0]), np.abs(W - kp2[:, 0]))
    assert np.allclose(eps, want, rtol=1e-7, atol=1e-9)


def test_sigma_scales_with_the_square_root_of_the_covariance():
    K = _K(800.0, 1024, 768)
    R0 = P.rodrigues(np.array([0.0, 0.1, 0.0]))
    t0 = np.array([1.0, 0.05, 0.1])
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6)) * 1e-3
    cov = A @ A.T
    kp2 = rng.uniform([0, 0], [1024, 768], (8, 2))
    e1 = P.pose_eps(kp2, K, K, R0, t0, cov, 1024, 768, 0.0, 1.0, 1e9)
    e4 = P.pose_eps(kp2, K, K, R0, t0, 4.0 * cov, 1024, 768, 0.0, 1.0, 1e9)
    assert np.allclose(e4, 2.0 * e1, rtol=1e-6)
    capped = P.pose_eps(kp2, K, K, R0, t0, cov, 1024, 768, 0.5, 2.0, 1.0)
    assert (capped <= 1.0).all() and (capped >= 0.5).all()


def test_spread_matches_sampled_poses():
    """The first-order spread g^T Sigma g against the standard deviation of
    the distance under poses drawn from N(0, Sigma) (small Sigma, so the
    distance is nearly linear): within 3 % on 20000 draws."""
    K = _K(700.0, 1000, 800)
    R0 = P.rodrigues(np.array([0.02, 0.15, -0.01]))
    t0 = np.array([0.8, -0.1, 0.3])
    rng = np.random.default_rng(5)
    L = np.diag([2e-4, 3e-4, 1e-4, 5e-3, 4e-3, 6e-3])
    cov = L @ L.T
    x1 = np.array([420.0, 310.0])
    F0 = P.F_of(np.zeros(6), K, K, R0, t0)
    l2 = F0 @ np.array([x1[0], x1[1], 1.0])
    # a point on the epipolar line of x1 (a true match at the mean pose)
    x2 = np.array([500.0, -(l2[0] * 500.0 + l2[2]) / l2[1]])
    g = P.gradient(x1, x2, K, K, R0, t0)
    pred = np.sqrt(g @ cov @ g)
    th = rng.standard_normal((20000, 6)) @ L.T
    d = np.array([P.distance(P.F_of(t, K, K, R0, t0), x1, x2) for t in th])
    assert abs(d.std() - pred) < 0.03 * pred


def test_segment_hand_cases():
    # x - y = 0 in a 10 x 5 image: from (0, 0) to (5, 5)
    seg = P.segment((1.0, -1.0, 0.0), 10, 5)
    assert sorted(seg) == [(0.0, 0.0), (5.0, 5.0)]
    # a horizontal row y = 2: the full width
    assert sorted(P.segment((0.0, 1.0, -2.0), 10, 5)) == [(0.0, 2.0), (10.0, 2.0)]
    # a line missing the image: its point nearest the centre, one sample
    line = (1.0, 1.0, 100.0)
    assert P.segment(line, 10, 5) is None
    (x, y), = P.samples(line, 10, 5)
    assert abs(x + y + 100.0) < 1e-9 and abs((x - 5.0) - (y - 2.5)) < 1e-9
    # 16 evenly spaced samples including both ends
    s = P.samples((0.0, 1.0, -2.0), 10, 5)
    assert len(s) == 16 and s[0] == (0.0, 2.0) and s[-1] == (10.0, 2.0)


def test_depth_range_rectified_stereo_closed_form():
    """Rectified stereo (f = 500, baseline 1 along x) with a depth range of
    [4, 16] m: the partner of x2 = (x', y') at depth Z is x1 = x' - f / Z, so
    sigma = sigma_ty * (largest disparity whose partner is inside image 1).
    The 16 inverse depths 1/16 + k (1/4 - 1/16) / 15 give disparities
    31.25 + 6.25 k: x' >= 125 reaches 125; x' = 60 reaches 56.25 (k = 4);
    x' = 10 has no partner in the image and takes the segment
    (max(10, 640 - 10) = 630)."""
    W, H, f = 640, 480, 500.0
    K = _K(f, W, H)
    cov = np.zeros((6, 6))
    cov[4, 4] = 0.03 ** 2
    kp2 = np.array([[125.0, 17.0], [400.0, 240.0], [639.0, 300.0], [60.0, 5.0], [10.0, 100.0]])
    eps = P.pose_eps(kp2, K, K, np.eye(3), np.array([1.0, 0.0, 0.0]), cov, W, H, 2.0, 3.0, 1e9,
                     4.0, 16.0)
    want = 2.0 + 3.0 * 0.03 * np.array([125.0, 125.0, 125.0, 56.25, 630.0])
    assert np.allclose(eps, want, rtol=1e-9, atol=1e-9)


def test_depth_samples_are_projections_of_points_at_those_depths():
    """A 3-D point placed in front of both cameras at camera-2 depth
    Z = 1 / (1/12 + 5 (1/3 - 1/12) / 15) (the sixth of the 16 inverse depths of
    [3, 12]) projects into image 1 onto one of the sample points of its image-2
    projection."""
    K1 = _K(600.0, 800, 600)
    K2 = _K(650.0, 800, 600)
    R0 = P.rodrigues(np.array([0.03, -0.2, 0.05]))
    t0 = np.array([-0.9, 0.1, 0.25])
    Z = 1.0 / (1.0 / 12.0 + 5.0 * (1.0 / 3.0 - 1.0 / 12.0) / 15.0)
    X2 = Z * np.array([0.05, -0.04, 1.0])
    X1 = R0.T @ (X2 - t0)
    x2 = (K2 @ X2)[:2] / X2[2]
    x1 = (K1 @ X1)[:2] / X1[2]
    assert 0 <= x1[0] <= 800 and 0 <= x1[1] <= 600
    pts = np.array(P.depth_samples(x2, K1, K2, R0, t0, 800, 600, 3.0, 12.0))
    assert np.min(np.hypot(*(pts - x1).T)) < 1e-9
    # every sample lies on the reverse epipolar line of x2
    F0 = P.fundamental(K1, K2, R0, t0)
    l = F0.T @ np.array([x2[0], x2[1], 1.0])
    assert np.all(np.abs(pts @ l[:2] + l[2]) / np.hypot(l[0], l[1]) < 1e-9)
    # an infinite far end: the first sample is the image of the direction
    inf_pts = P.depth_samples(x2, K1, K2, R0, t0, 800, 600, 3.0, np.inf)
    d = K1 @ R0.T @ np.linalg.inv(K2) @ np.array([x2[0], x2[1], 1.0])
    assert np.allclose(inf_pts[0], d[:2] / d[2], atol=1e-9)
