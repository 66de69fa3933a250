"""The paper's own angular formulation, restated in NumPy for tiny inputs.

TEST INFRASTRUCTURE ONLY (cross-check of the brute-force oracle).

Section 4.2 (Eq. 5-7), Algorithm 1 and Section 4.4:
  * epipole e2 = null(F^T) (Algorithm 1, preprocessing);
  * a keypoint whose distance to e2 is at most eps is visible in every
    direction (full interval, Sec. 4.4 "Keypoints near the epipole");
  * otherwise theta_j = atan2(y_j - y_e, x_j - x_e) (Eq. 5) and
    delta_j = arcsin(eps_j / |p_j - e2|) (Eq. 6); theta_j is reduced to
    [0, pi) and the interval [theta - delta, theta + delta] is split at 0/pi
    when it wraps (Sec. 4.4 "Discontinuity at 0/pi");
  * a query's angle alpha_i is the direction of its epipolar line seen from
    e2, reduced mod pi (Sec. 4.2, Eq. 7 and the undirected-line remark).

Eq. 7 measures alpha from e2 to q_i, the point of the line closest to the
image centre.  That point coincides with e2 when the epipole is the image
centre, where Eq. 7 is undefined; the direction of the line itself gives the
same angle mod pi whenever q_i != e2.  Both are implemented
(mode='paper' / mode='direction').  The form is undefined for an epipole at
infinity (the paper assumes a finite epipole, Sec. 6).
"""

import math

import numpy as np


def epipole_image2(F):
    """Left null vector of F (F^T e2 = 0), via the SVD (smallest singular value)."""
    U, S, Vt = np.linalg.svd(np.asarray(F, dtype=np.float64))
    return U[:, 2]


def _line(F, x, y):
    return (F[0, 0] * x + F[0, 1] * y + F[0, 2],
            F[1, 0] * x + F[1, 1] * y + F[1, 2],
            F[2, 0] * x + F[2, 1] * y + F[2, 2])


def paper_query_angle(line, e_xy, centre=None, mode="direction"):
    """alpha mod pi for one line (a, b, c) seen from the finite epipole e_xy."""
    a, b, c = line
    if mode == "direction":
        alpha = math.atan2(-a, b)
    else:
        cx, cy = centre
        s = (a * cx + b * cy + c) / (a * a + b * b)
        qx, qy = cx - s * a, cy - s * b
        alpha = math.atan2(qy - e_xy[1], qx - e_xy[0])
    return alpha % math.pi


def paper_intervals(kp2, e_xy, eps):
    """One entry per keypoint: None for the full interval, else a list of
    closed [lo, hi] sub-intervals of [0, pi] (two when the interval wraps)."""
    out = []
    for j in range(kp2.shape[0]):
        x, y = float(kp2[j, 0]), float(kp2[j, 1])
        ej = float(eps if np.ndim(eps) == 0 else eps[j])
        r = math.hypot(x - e_xy[0], y - e_xy[1])
        if r <= ej:
            out.append(None)
            continue
        theta = math.atan2(y - e_xy[1], x - e_xy[0]) % math.pi
        delta = math.asin(ej / r)
        lo, hi = theta - delta, theta + delta
        if lo < 0.0:
            out.append([(lo + math.pi, math.pi), (0.0, hi)])
        elif hi > math.pi:
            out.append([(lo, math.pi), (0.0, hi - math.pi)])
        else:
            out.append([(lo, hi)])
    return out


def paper_angle_candidates(F, kp1, kp2, eps, mode="direction", centre=None):
    """Candidate rows (ascending j) by stabbing the angular intervals."""
    F = np.asarray(F, dtype=np.float64)
    e = epipole_image2(F)
    if e[2] == 0.0:
        raise ValueError("the angular form needs a finite epipole")
    e_xy = (e[0] / e[2], e[1] / e[2])
    ivs = paper_intervals(np.asarray(kp2, dtype=np.float64), e_xy, eps)
    rows = []
    for i in range(kp1.shape[0]):
        a, b, c = _line(F, float(kp1[i, 0]), float(kp1[i, 1]))
        if a == 0.0 and b == 0.0:
            rows.append([])
            continue
        alpha = paper_query_angle((a, b, c), e_xy, centre, mode)
        row = []
        for j, iv in enumerate(ivs):
            if iv is None or any(lo <= alpha <= hi for lo, hi in iv):
                row.append(j)
        rows.append(row)
    return rows
