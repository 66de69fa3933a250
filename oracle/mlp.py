"""Oracle of the learned per-keypoint tolerance -- TEST INFRASTRUCTURE ONLY.

The paper leaves a learned, per-keypoint tolerance as future work (Sec. 6):
the tolerance of image-2 keypoint j is predicted from its own attributes.
This module restates, in plain NumPy FP64, the network the GPU library
trains and evaluates:

  features  f_j = (scale, response, orientation, (x - W/2)/(W/2),
                   (y - H/2)/(W/2), log1p(min(|p_j - e2| / diag, 1000)))
            with e2 the image-2 epipole (left null vector of F, Eq. 1-2) and
            diag the image-2 diagonal; an epipole at infinity gives the
            clipped value.
  network   h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3
            (6 -> 64 -> 64 -> 1);
            eps = clamp(softplus(z), 0.5, 8) px at inference.
  loss      pinball (quantile) loss at level q of the unclamped softplus(z)
            against a target residual r (the point-line distance, Eq. 3, of
            a match the method itself accepted), averaged over the batch.
  update    Adam.

Parity status (pins are tests/test_oracle_mlp.py):
  features          pinned: pure forward motion (epipole at the origin,
                    distance = |p|), rectified stereo (epipole at infinity),
                    the image centre, and the epipole of the generating
                    cameras.
  forward/infer     pinned: zero network with output bias beta gives the
                    constant clamp(softplus(beta), 0.5, 8); BF16 rounding on
                    hand-worked ties.
  loss, gradients   pinned: hand-worked pinball values and subgradients,
                    the pinball minimiser over constants is the q-quantile,
                    central finite differences of the FP64 loss.
  adam              pinned: the first two steps under a constant gradient
                    move every parameter by lr * g / (|g| + eps).

Parameter vector (float, 4673 entries), in this order: W1 [64][6], b1 [64],
W2 [64][64], b2 [64], w3 [64], b3 [1]; matrices row-major (row = output unit).
"""

import numpy as np

H1 = 64
H2 = 64
NIN = 6
SIZES = (("W1", (H1, NIN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("w3", (H2,)),
         ("b3", ()))
NPARAM = sum(int(np.prod(s)) if s else 1 for _, s in SIZES)
EPS_MIN, EPS_MAX = 0.5, 8.0
DIST_CLIP = 1000.0


def unpack(theta):
    """Views of the named tensors of a flat parameter vector (FP64 copy)."""
    theta = np.asarray(theta, dtype=np.float64).reshape(-1)
    assert theta.size == NPARAM
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape)) if shape else 1
        out[name] = theta[o:o + k].reshape(shape) if shape else theta[o]
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1)
                           for name, _ in SIZES])


# ------------------------------------------------------------------ features

def epipole2(F):
    """Image-2 epipole: the unit left null vector of F (F^T e = 0), from the
    SVD (singular vector of the smallest singular value)."""
    U, _, _ = np.linalg.svd(np.asarray(F, np.float64).reshape(3, 3))
    return U[:, 2]


def features(F, kp2, scale, response, orientation, W, H):
    """[n][6] FP64 features of image-2 keypoints of one pair."""
    kp2 = np.asarray(kp2, np.float64).reshape(-1, 2)
    e = epipole2(F)
    x, y = kp2[:, 0], kp2[:, 1]
    diag = np.hypot(float(W), float(H))
    if e[2] == 0.0:
        d = np.full(len(x), np.inf)
    else:
        d = np.hypot(x - e[0] / e[2], y - e[1] / e[2])
    rel = np.minimum(d / diag, DIST_CLIP)
    half = 0.5 * float(W)
    return np.stack([np.asarray(scale, np.float64), np.asarray(response, np.float64),
                     np.asarray(orientation, np.float64), (x - half) / half,
                     (y - 0.5 * float(H)) / half, np.log1p(rel)], axis=1)


# ------------------------------------------------------------------- network

def softplus(z):
    z = np.asarray(z, np.float64)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    z = np.asarray(z, np.float64)
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(theta, X):
    """Layer values for inputs X [n][6]: dict with a1, h1, a2, h2, z, yhat
    (= softplus(z), the training output) and eps (the clamped tolerance)."""
    P = unpack(theta)
    X = np.asarray(X, np.float64)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["w3"] + P["b3"]
    yhat = softplus(z)
    return {"a1": a1, "h1": h1, "a2": a2, "h2": h2, "z": z, "yhat": yhat,
            "eps": np.clip(yhat, EPS_MIN, EPS_MAX)}


def pinball(y, yhat, q):
    """Mean pinball loss: rho_q(u) = q u for u >= 0, (q - 1) u for u < 0,
    u = y - yhat."""
    u = np.asarray(y, np.float64) - np.asarray(yhat, np.float64)
    return float(np.mean(np.where(u >= 0.0, q * u, (q - 1.0) * u)))


def pinball_grad(y, yhat, q):
    """d(mean pinball)/d yhat per sample: -q/B where y > yhat, else (1-q)/B
    (at the kink y == yhat the subgradient (1-q)/B is taken)."""
    y = np.asarray(y, np.float64)
    yhat = np.asarray(yhat, np.float64)
    return np.where(yhat >= y, 1.0 - q, -q) / float(len(y))


def loss_and_grad(theta, X, y, q):
    """Mean pinball loss of softplus(z) and its gradient with respect to the
    parameter vector, by the chain rule layer by layer."""
    P = unpack(theta)
    f = forward(theta, X)
    X = np.asarray(X, np.float64)
    dyhat = pinball_grad(y, f["yhat"], q)
    dz = dyhat * sigmoid(f["z"])
    g = {"b3": np.sum(dz), "w3": f["h2"].T @ dz}
    da2 = np.outer(dz, P["w3"]) * (f["a2"] > 0.0)
    g["W2"] = da2.T @ f["h1"]
    g["b2"] = np.sum(da2, axis=0)
    da1 = (da2 @ P["W2"]) * (f["a1"] > 0.0)
    g["W1"] = da1.T @ X
    g["b1"] = np.sum(da1, axis=0)
    return pinball(y, f["yhat"], q), pack(g)


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns (theta, m, v)."""
    grad = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ----------------------------------------------------------------- inference

def bf16_round(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float64.
    Finite inputs only."""
    b = np.asarray(x, np.float32).reshape(-1).view(np.uint32).astype(np.uint64)
    low = b & 0xFFFF
    keep = b >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((keep & 1) == 1))
    keep = keep + up.astype(np.uint64)
    out = (keep << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(x))


def infer_bf16(theta_f32, X):
    """Tolerances with the weights rounded to BF16 (from their float32
    values) and the features rounded to float32; arithmetic in FP64."""
    w = bf16_round(np.asarray(theta_f32, np.float32))
    Xf = np.asarray(X, np.float32).astype(np.float64)
    return forward(w, Xf)["eps"]
