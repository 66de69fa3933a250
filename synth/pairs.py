"""Synthetic image pairs shaped like the paper's multi-megapixel SfM workloads.

Scene recipe (shared by every workload):

* Camera 1: K = [[f,0,W/2],[0,f,H/2],[0,0,1]], R = I, centre at the origin.
* Camera 2: X2 = R X1 + t with t = -R C2 (the convention of Eq. 1), the
  baseline |C2| = 1 m unless stated otherwise.
* F12 = K2^-T [t]x R K1^-1 (Eq. 1), evaluated in FP64.
* 3-D points: a pixel drawn uniformly in image 1 and a depth Z ~ U(5, 15) m,
  back-projected; kept when in front of camera 2 and inside image 2.
* Keypoints: the projections plus N(0, sigma^2) noise per coordinate, stored
  as FP32 pixel coordinates (no half-pixel shift); outliers uniform in each
  image; each image's keypoint order is shuffled and the ground-truth map kept.
* Float descriptors: per true point g ~ N(0, I_128)/|.|, each view
  g + N(0, 0.05^2 I) renormalised; outliers independent random unit vectors.
* Binary descriptors: 256 random bits per true point; view 2 flips every bit
  independently with probability 0.08; outliers random.

Seeds are NumPy PCG64; workload k uses seed 1000*(k+1) + r.
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

DESC_DIM = 128
BIN_WORDS = 8


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def intrinsics(f, W, H):
    return np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])


def _intrinsics_inv(K):
    f, cx, cy = K[0, 0], K[0, 2], K[1, 2]
    return np.array([[1.0 / f, 0.0, -cx / f], [0.0, 1.0 / f, -cy / f], [0.0, 0.0, 1.0]])


def skew(t):
    return np.array([[0.0, -t[2], t[1]], [t[2], 0.0, -t[0]], [-t[1], t[0], 0.0]])


def rot_axis_angle(axis, angle):
    """Rodrigues rotation about a (not necessarily unit) axis, angle in radians."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    Kx = skew(a)
    return np.eye(3) + np.sin(angle) * Kx + (1.0 - np.cos(angle)) * (Kx @ Kx)


def fundamental_from_cameras(K1, K2, R, t):
    """Eq. 1: F12 = K2^-T [t]x R K1^-1 (FP64)."""
    return _intrinsics_inv(K2).T @ skew(t) @ R @ _intrinsics_inv(K1)


@dataclass
class Pair:
    W: int
    H: int
    f: float
    K1: np.ndarray
    K2: np.ndarray
    R: np.ndarray
    t: np.ndarray
    C2: np.ndarray
    F: np.ndarray          # (3,3) float64, row-major, l2 = F (x1, y1, 1)^T
    e1: np.ndarray         # homogeneous epipole in image 1 (projection of C2)
    e2: np.ndarray         # homogeneous epipole in image 2 (projection of C1)
    kp1: np.ndarray        # (m,2) float32
    kp2: np.ndarray        # (n,2) float32
    gt12: np.ndarray       # (m,) int32: true partner in image 2, or -1
    clean1: np.ndarray     # (m,2) float32 noiseless projections (outliers: as kp1)
    clean2: np.ndarray     # (n,2) float32
    desc1: Optional[np.ndarray] = None  # (m,128) float32 unit rows
    desc2: Optional[np.ndarray] = None
    bin1: Optional[np.ndarray] = None   # (m,8) uint32
    bin2: Optional[np.ndarray] = None
    scale1: Optional[np.ndarray] = None  # (m,) float32 keypoint scale (px)
    scale2: Optional[np.ndarray] = None
    resp2: Optional[np.ndarray] = None   # (n,) float32 detector response
    ori2: Optional[np.ndarray] = None    # (n,) float32 orientation (rad)
    tag: str = ""

    @property
    def m(self):
        return int(self.kp1.shape[0])

    @property
    def n(self):
        return int(self.kp2.shape[0])


def _project(K, X):
    p = (K @ X.T).T
    return p[:, :2] / p[:, 2:3]


def _sample_points(rng, W, H, K1, K2, R, t, n_true, zmin=5.0, zmax=15.0):
    Kinv = _intrinsics_inv(K1)
    out1, out2 = [], []
    have = 0
    for _ in range(2000):
        need = n_true - have
        if need <= 0:
            break
        k = max(64, 2 * need)
        u = rng.uniform(0.0, W, k)
        v = rng.uniform(0.0, H, k)
        z = rng.uniform(zmin, zmax, k)
        X1 = (Kinv @ np.stack([u, v, np.ones(k)])).T * z[:, None]
        X2 = (R @ X1.T).T + t
        ok = X2[:, 2] > 1e-3
        p2 = np.full((k, 2), -1.0)
        p2[ok] = _project(K2, X2[ok])
        ok &= (p2[:, 0] >= 0) & (p2[:, 0] < W) & (p2[:, 1] >= 0) & (p2[:, 1] < H)
        p1 = np.stack([u, v], axis=1)
        out1.append(p1[ok][:need])
        out2.append(p2[ok][:need])
        have += int(min(ok.sum(), need))
    if have < n_true:
        raise RuntimeError("scene sampler could not place enough visible points")
    return np.concatenate(out1)[:n_true], np.concatenate(out2)[:n_true]


def _unit_rows(x):
    x = np.asarray(x, dtype=np.float64)
    return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)


def make_pair(W, H, f, R, C2, n_true, n_out1, n_out2, seed, sigma=0.5,
              float_desc=True, binary=False, scale_noise=None, tag=""):
    """One synthetic pair.

    scale_noise: None for isotropic N(0, sigma^2) noise; otherwise a tuple
    (lo, hi, k): each true point gets a keypoint scale s ~ logU[lo, hi] px
    (shared by both views) and noise N(0, (k s)^2) per coordinate; outliers
    get their own scales from the same law.
    """
    rng = _rng(seed)
    K1 = intrinsics(f, W, H)
    K2 = intrinsics(f, W, H)
    R = np.asarray(R, dtype=np.float64)
    C2 = np.asarray(C2, dtype=np.float64)
    t = -R @ C2
    F = fundamental_from_cameras(K1, K2, R, t)
    e2 = K2 @ t
    e1 = K1 @ C2
    p1, p2 = _sample_points(rng, W, H, K1, K2, R, t, n_true)

    if scale_noise is None:
        s_true = None
        sig = np.full(n_true, sigma)
    else:
        lo, hi, kk = scale_noise
        s_true = np.exp(rng.uniform(np.log(lo), np.log(hi), n_true))
        sig = kk * s_true
    n1 = p1 + rng.standard_normal(p1.shape) * sig[:, None]
    n2 = p2 + rng.standard_normal(p2.shape) * sig[:, None]
    o1 = np.stack([rng.uniform(0, W, n_out1), rng.uniform(0, H, n_out1)], axis=1)
    o2 = np.stack([rng.uniform(0, W, n_out2), rng.uniform(0, H, n_out2)], axis=1)

    m, n = n_true + n_out1, n_true + n_out2
    perm1 = rng.permutation(m)   # new position of source row r is inv; rows[perm] order
    perm2 = rng.permutation(n)
    inv1 = np.empty(m, np.int64)
    inv1[perm1] = np.arange(m)
    inv2 = np.empty(n, np.int64)
    inv2[perm2] = np.arange(n)

    def arrange(src, perm):
        return np.ascontiguousarray(src[perm])

    kp1 = arrange(np.concatenate([n1, o1]).astype(np.float32), perm1)
    kp2 = arrange(np.concatenate([n2, o2]).astype(np.float32), perm2)
    clean1 = arrange(np.concatenate([p1, o1]).astype(np.float32), perm1)
    clean2 = arrange(np.concatenate([p2, o2]).astype(np.float32), perm2)
    gt_src = np.concatenate([inv2[:n_true], np.full(n_out1, -1)])
    gt12 = arrange(gt_src, perm1).astype(np.int32)

    pair = Pair(W=W, H=H, f=f, K1=K1, K2=K2, R=R, t=t, C2=C2, F=F, e1=e1, e2=e2,
                kp1=kp1, kp2=kp2, gt12=gt12, clean1=clean1, clean2=clean2, tag=tag)

    if float_desc:
        g = rng.standard_normal((n_true, DESC_DIM))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        d1 = _unit_rows(g + 0.05 * rng.standard_normal(g.shape))
        d2 = _unit_rows(g + 0.05 * rng.standard_normal(g.shape))
        r1 = _unit_rows(rng.standard_normal((n_out1, DESC_DIM)))
        r2 = _unit_rows(rng.standard_normal((n_out2, DESC_DIM)))
        pair.desc1 = arrange(np.concatenate([d1, r1]), perm1)
        pair.desc2 = arrange(np.concatenate([d2, r2]), perm2)
    if binary:
        base = rng.integers(0, 2 ** 32, (n_true, BIN_WORDS), dtype=np.uint32)
        flips = rng.random((n_true, 256)) < 0.08
        fw = np.packbits(flips, axis=1, bitorder="little").view("<u4").astype(np.uint32)
        b1 = base
        b2 = base ^ fw
        r1 = rng.integers(0, 2 ** 32, (n_out1, BIN_WORDS), dtype=np.uint32)
        r2 = rng.integers(0, 2 ** 32, (n_out2, BIN_WORDS), dtype=np.uint32)
        pair.bin1 = arrange(np.concatenate([b1, r1]), perm1)
        pair.bin2 = arrange(np.concatenate([b2, r2]), perm2)
    if scale_noise is not None:
        lo, hi, _ = scale_noise
        so1 = np.exp(rng.uniform(np.log(lo), np.log(hi), n_out1))
        so2 = np.exp(rng.uniform(np.log(lo), np.log(hi), n_out2))
        pair.scale1 = arrange(np.concatenate([s_true, so1]).astype(np.float32), perm1)
        pair.scale2 = arrange(np.concatenate([s_true, so2]).astype(np.float32), perm2)
        pair.resp2 = rng.uniform(0.0, 1.0, n).astype(np.float32)
        pair.ori2 = rng.uniform(-np.pi, np.pi, n).astype(np.float32)
    return pair


# ---------------------------------------------------------------- workloads

def _yaw(deg):
    return rot_axis_angle([0.0, 1.0, 0.0], np.deg2rad(deg))


def cfg0_pair(r=0, float_desc=True, binary=False):
    """640x480, f=500, 800 true + 200 outliers, sideways baseline with a
    relative yaw of magnitude U[1, 10] deg and random sign, sigma 0.5 px."""
    seed = 1000 * 1 + r
    rng = _rng(seed + 7_000_000)
    yaw = rng.uniform(1.0, 10.0) * (1 if rng.random() < 0.5 else -1)
    return make_pair(640, 480, 500.0, _yaw(yaw), [1.0, 0.0, 0.0], 800, 200, 200,
                     seed, float_desc=float_desc, binary=binary, tag=f"cfg0 yaw={yaw:.2f}")


def cfg1_pair(motion="sideways", r=0, n_kp=20000, float_desc=True, binary=False):
    """6048x4032, f=3400, 70% true / 30% outliers.

    motion: 'sideways' (yaw 10 deg, epipole far left of the image),
    'forward' (pure forward translation: epipole exactly at the image centre),
    'forward_yaw' (forward translation with a 3 deg yaw)."""
    seed = 1000 * 2 + r + {"sideways": 0, "forward": 100, "forward_yaw": 200}[motion]
    n_true = int(round(0.7 * n_kp))
    n_out = n_kp - n_true
    if motion == "sideways":
        R, C2 = _yaw(10.0), [1.0, 0.0, 0.0]
    elif motion == "forward":
        R, C2 = np.eye(3), [0.0, 0.0, 1.0]
    elif motion == "forward_yaw":
        R, C2 = _yaw(3.0), [0.0, 0.0, 1.0]
    else:
        raise ValueError(motion)
    return make_pair(6048, 4032, 3400.0, R, C2, n_true, n_out, n_out, seed,
                     float_desc=float_desc, binary=binary, tag=f"cfg1 {motion}")


def cfg2_pair(r=0, n_kp=60000):
    """cfg1 sideways geometry with 60k keypoints, float and binary descriptors."""
    seed = 1000 * 3 + r
    n_true = int(round(0.7 * n_kp))
    return make_pair(6048, 4032, 3400.0, _yaw(10.0), [1.0, 0.0, 0.0], n_true,
                     n_kp - n_true, n_kp - n_true, seed, binary=True, tag="cfg2")


_SIZES = [(1920, 1080), (4032, 3024), (6048, 4032)]


def _cfg3_pose(rng, kind):
    if kind == "sideways_far":
        yaw = 10.0 ** rng.uniform(-4.0, -2.0) * (1 if rng.random() < 0.5 else -1)
        return _yaw(yaw), np.array([1.0, 0.0, 0.0])
    if kind == "sideways_inf":
        return np.eye(3), np.array([1.0, 0.0, 0.0])
    if kind == "forward":
        c = np.array([rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), 1.0])
        axis = rng.standard_normal(3)
        return rot_axis_angle(axis, np.deg2rad(rng.uniform(0.0, 2.0))), c / np.linalg.norm(c)
    if kind == "general":
        c = rng.standard_normal(3)
        axis = rng.standard_normal(3)
        return rot_axis_angle(axis, np.deg2rad(rng.uniform(0.0, 15.0))), c / np.linalg.norm(c)
    raise ValueError(kind)


def cfg3_pair(r, float_desc=True, max_kp=30000, min_kp=500):
    """One pair of the batching workload (pair index r of the batch)."""
    seed = 1000 * 4 + r
    rng = _rng(seed + 9_000_000)
    W, H = _SIZES[int(rng.integers(0, 3))]
    f = 0.5622 * W
    m = int(round(np.exp(rng.uniform(np.log(min_kp), np.log(max_kp)))))
    n = int(round(np.exp(rng.uniform(np.log(min_kp), np.log(max_kp)))))
    kinds = ["sideways_far", "forward", "general"]
    kind = "sideways_inf" if r == 0 else kinds[r % 3]
    R, C2 = _cfg3_pose(rng, kind)
    n_true = int(round(0.7 * min(m, n)))
    return make_pair(W, H, f, R, C2, n_true, m - n_true, n - n_true, seed,
                     float_desc=float_desc, tag=f"cfg3 {kind} {W}x{H} m={m} n={n}")


def cfg3_batch(num_pairs=512, float_desc=True, max_kp=30000, min_kp=500, workers=8):
    """The pairs 0 .. num_pairs-1 of the batching workload, generated on a
    thread pool (every pair draws from its own seed, so the result does not
    depend on the number of workers)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(r):
        return cfg3_pair(r, float_desc=float_desc, max_kp=max_kp, min_kp=min_kp)

    if workers <= 1:
        return [one(r) for r in range(num_pairs)]
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, range(num_pairs)))


def cfg4_pair(r, n_kp=10000, float_desc=True):
    """Learned-tolerance workload: 6048x4032, f=3400, 70/30, poses as the
    batching mix, heteroscedastic noise sigma = 0.15 * scale with
    scale ~ logU[1, 12] px.  Training pairs use r in [0, 2000), held-out pairs
    r in [10000, 10200) (seeds 50000+r)."""
    seed = 50_000 + r
    rng = _rng(seed + 9_000_000)
    kinds = ["sideways_far", "forward", "general"]
    R, C2 = _cfg3_pose(rng, kinds[r % 3])
    n_true = int(round(0.7 * n_kp))
    return make_pair(6048, 4032, 3400.0, R, C2, n_true, n_kp - n_true, n_kp - n_true,
                     seed, float_desc=float_desc, scale_noise=(1.0, 12.0, 0.15),
                     tag=f"cfg4 {kinds[r % 3]}")


# ------------------------------------------------------------------ batches

@dataclass
class PairBatch:
    pairs: List[Pair]
    q_begin: np.ndarray = field(default=None)
    k_begin: np.ndarray = field(default=None)
    kp1: np.ndarray = field(default=None)
    kp2: np.ndarray = field(default=None)
    desc1: Optional[np.ndarray] = None
    desc2: Optional[np.ndarray] = None
    bin1: Optional[np.ndarray] = None
    bin2: Optional[np.ndarray] = None

    @property
    def m(self):
        return np.array([p.m for p in self.pairs], dtype=np.int64)

    @property
    def n(self):
        return np.array([p.n for p in self.pairs], dtype=np.int64)


def batch_pairs(pairs):
    """Concatenate pairs along the keypoint axis (image 1 and image 2 arrays
    separately) and record each pair's slice."""
    m = np.array([p.m for p in pairs], dtype=np.int64)
    n = np.array([p.n for p in pairs], dtype=np.int64)
    b = PairBatch(pairs=list(pairs))
    b.q_begin = np.concatenate([[0], np.cumsum(m)[:-1]]).astype(np.int64)
    b.k_begin = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    b.kp1 = np.ascontiguousarray(np.concatenate([p.kp1 for p in pairs]))
    b.kp2 = np.ascontiguousarray(np.concatenate([p.kp2 for p in pairs]))
    if all(p.desc1 is not None for p in pairs):
        b.desc1 = np.ascontiguousarray(np.concatenate([p.desc1 for p in pairs]))
        b.desc2 = np.ascontiguousarray(np.concatenate([p.desc2 for p in pairs]))
    if all(p.bin1 is not None for p in pairs):
        b.bin1 = np.ascontiguousarray(np.concatenate([p.bin1 for p in pairs]))
        b.bin2 = np.ascontiguousarray(np.concatenate([p.bin2 for p in pairs]))
    return b


def perturbed_pose(pair, level, seed):
    """A relative pose perturbed at a noise level (the paper's noise
    sensitivity experiment, Sec. 5): level 1 rotates by angles U(-1, 1) deg
    about each axis (applied before the true rotation) and moves the
    translation by U(-0.25, 0.25) m per component; level L scales both ranges
    by L.  Returns (R, t)."""
    rng = _rng(seed)
    ang = np.deg2rad(rng.uniform(-1.0, 1.0, 3) * level)
    Rn = (rot_axis_angle([1.0, 0.0, 0.0], ang[0]) @ rot_axis_angle([0.0, 1.0, 0.0], ang[1])
          @ rot_axis_angle([0.0, 0.0, 1.0], ang[2]))
    return Rn @ pair.R, pair.t + rng.uniform(-0.25, 0.25, 3) * level


def perturbed_F(pair, level, seed):
    """F of perturbed_pose(pair, level, seed); the keypoints keep the true
    geometry."""
    R, t = perturbed_pose(pair, level, seed)
    return fundamental_from_cameras(pair.K1, pair.K2, R, t)


def noise_covariance(level):
    """Covariance of the perturbation law of perturbed_pose as (rotation
    vector, translation), to first order: independent uniforms of half-widths
    level deg and 0.25 level m, whose variances are a^2 / 3."""
    r = np.deg2rad(level) ** 2 / 3.0
    t = (0.25 * level) ** 2 / 3.0
    return np.diag([r, r, r, t, t, t])
