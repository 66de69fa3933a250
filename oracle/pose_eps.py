"""Oracle of the pose-uncertainty tolerance -- TEST INFRASTRUCTURE ONLY.

The paper's noise experiment (Sec. 5) perturbs the relative pose and widens
the tolerance to absorb it, and Sec. 6 names a tolerance adapted to each
keypoint as future work.  This module restates, in plain NumPy FP64, the
per-keypoint tolerance the GPU library derives from a pose covariance:

  pose      R(theta) = Exp([w]x) R0, t(theta) = t0 + tau, theta = (w, tau) in R^6,
            with covariance Sigma (6 x 6);
  F         F(theta) = K2^-T [t(theta)]x R(theta) K1^-1 (Eq. 1);
  distance  d(theta; x1, x2) = x2^T F(theta) x1 / |(F(theta) x1)_12| (Eq. 3,
            signed), so that a true match has d(0) = 0 up to keypoint noise;
  spread    s^2(x1, x2) = g^T Sigma g with g the gradient of d at theta = 0,
            here by central differences of the FP64 distance;
  segment   the true image-1 partner of an image-2 keypoint x2 lies on its
            reverse epipolar line F(0)^T x2 inside image 1 (0 <= x <= W1,
            0 <= y <= H1): sigma_j is the largest s over S = 16 evenly spaced
            points of that segment (one point, the line's point nearest the
            image centre, when the line misses the image; points where
            (F x1)_12 vanishes are skipped);
  depths    with a scene depth range 0 < zmin < zmax <= inf in camera 2
            given, the partner is instead the projection into image 1 of the
            3-D point seen at x2 with depth Z in that range:
            X1 ~ R0^T (K2^-1 x2 - rho t0), rho = 1 / Z, at S = 16 inverse
            depths evenly spaced from 1 / zmax to 1 / zmin, keeping those in
            front of camera 1 and inside image 1 (the segment's spread grows
            without bound towards the epipole, where the implied depth
            vanishes); a keypoint with no such point takes the segment;
  tolerance eps_j = min(eps0 + k sigma_j, eps_max).

Parity status (pins are tests/test_oracle_pose_eps.py):
  pose_eps        pinned: Sigma = 0 gives eps0 for every keypoint; rectified
                  stereo with only the translation's y uncertain has the
                  closed form sigma = sigma_ty * max(|x'|, |W1 - x'|) (the
                  disparity to the ends of the scanline); sigma scales as
                  sqrt(Sigma); the segment of a hand case; with a depth
                  range, rectified stereo has sigma = sigma_ty * f / zmin
                  (the largest disparity) and the sample points are the
                  projections of points at known depths.
"""

import numpy as np

SAMPLES = 16
STEP = 1e-6  # central-difference step: radians for w, the unit of t for tau


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def rodrigues(w):
    """Exp([w]x) for a rotation vector w (radians)."""
    th = float(np.linalg.norm(w))
    if th == 0.0:
        return np.eye(3)
    k = skew(np.asarray(w, dtype=np.float64) / th)
    return np.eye(3) + np.sin(th) * k + (1.0 - np.cos(th)) * (k @ k)


def fundamental(K1, K2, R, t):
    """Eq. 1: F = K2^-T [t]x R K1^-1."""
    return np.linalg.inv(K2).T @ skew(t) @ R @ np.linalg.inv(K1)


def F_of(theta, K1, K2, R0, t0):
    theta = np.asarray(theta, dtype=np.float64)
    return fundamental(K1, K2, rodrigues(theta[:3]) @ R0, t0 + theta[3:])


def distance(F, x1, x2):
    """Signed point-line distance of x2 (pixels) from the line F (x1, 1)."""
    l = F @ np.array([x1[0], x1[1], 1.0])
    return (l[0] * x2[0] + l[1] * x2[1] + l[2]) / np.hypot(l[0], l[1])


def gradient(x1, x2, K1, K2, R0, t0):
    """Gradient of the distance with respect to theta at 0 (central differences)."""
    g = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = STEP
        g[k] = (distance(F_of(e, K1, K2, R0, t0), x1, x2)
                - distance(F_of(-e, K1, K2, R0, t0), x1, x2)) / (2.0 * STEP)
    return g


def segment(line, W1, H1):
    """Endpoints of the part of the line a x + b y + c = 0 inside
    [0, W1] x [0, H1], or None when it has fewer than two points there."""
    a, b, c = line
    pts = []
    if b != 0.0:
        for x in (0.0, float(W1)):
            y = -(a * x + c) / b
            if 0.0 <= y <= H1:
                pts.append((x, y))
    if a != 0.0:
        for y in (0.0, float(H1)):
            x = -(b * y + c) / a
            if 0.0 <= x <= W1:
                pts.append((x, y))
    best, far = None, 0.0
    for i in range(len(pts)):
        for j in range(i + 1, len(pts)):
            dd = np.hypot(pts[i][0] - pts[j][0], pts[i][1] - pts[j][1])
            if dd > far:
                far, best = dd, (pts[i], pts[j])
    return best


def nearest_to_centre(line, W1, H1):
    a, b, c = line
    cx, cy = W1 / 2.0, H1 / 2.0
    s = (a * cx + b * cy + c) / (a * a + b * b)
    return (cx - a * s, cy - b * s)


def samples(line, W1, H1, S=SAMPLES):
    seg = segment(line, W1, H1)
    if seg is None:
        return [nearest_to_centre(line, W1, H1)]
    (px, py), (qx, qy) = seg
    return [(px + (qx - px) * s / (S - 1), py + (qy - py) * s / (S - 1)) for s in range(S)]


def depth_samples(x2, K1, K2, R0, t0, W1, H1, zmin, zmax, S=SAMPLES):
    """Image-1 projections of the 3-D points seen at image-2 pixel x2 at S
    inverse depths evenly spaced over [1 / zmax, 1 / zmin] (camera-2 depths,
    X2 = R0 X1 + t0), those in front of camera 1 and inside [0, W1] x [0, H1]."""
    ray = np.linalg.inv(K2) @ np.array([x2[0], x2[1], 1.0])
    lo, hi = 1.0 / zmax, 1.0 / zmin
    out = []
    for s in range(S):
        rho = lo + (hi - lo) * s / (S - 1)
        X1 = R0.T @ (ray - rho * np.asarray(t0, dtype=np.float64))  # X1 / Z
        if not X1[2] > 0.0:
            continue
        p = K1 @ X1
        x, y = p[0] / p[2], p[1] / p[2]
        if 0.0 <= x <= W1 and 0.0 <= y <= H1:
            out.append((x, y))
    return out


def sigma(x2, K1, K2, R0, t0, cov, W1, H1, zmin=0.0, zmax=np.inf):
    """Largest first-order spread of the distance of image-2 keypoint x2 over
    its possible partners in image 1 (the reverse epipolar segment, or the
    points of the depth range when zmin > 0)."""
    F0 = F_of(np.zeros(6), K1, K2, R0, t0)
    line = F0.T @ np.array([x2[0], x2[1], 1.0])
    best = 0.0
    pts = depth_samples(x2, K1, K2, R0, t0, W1, H1, zmin, zmax) if zmin > 0.0 else []
    if not pts:
        pts = samples(line, W1, H1)
    for x1 in pts:
        l = F0 @ np.array([x1[0], x1[1], 1.0])
        if not np.hypot(l[0], l[1]) > 1e-12 * np.abs(F0).max():
            continue
        g = gradient(x1, x2, K1, K2, R0, t0)
        best = max(best, float(g @ cov @ g))
    return np.sqrt(best)


def pose_eps(kp2, K1, K2, R0, t0, cov, W1, H1, eps0, k, eps_max, zmin=0.0, zmax=np.inf):
    """Tolerance of every image-2 keypoint (pixels), FP64."""
    kp2 = np.asarray(kp2, dtype=np.float64).reshape(-1, 2)
    cov = np.asarray(cov, dtype=np.float64).reshape(6, 6)
    out = np.empty(len(kp2))
    for j, x2 in enumerate(kp2):
        out[j] = min(eps0 + k * sigma(x2, K1, K2, R0, t0, cov, W1, H1, zmin, zmax), eps_max)
    return out
