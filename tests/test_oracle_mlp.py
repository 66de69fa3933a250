"""Pins of the tolerance-network oracle (oracle/mlp.py) against hand-worked
values, closed forms and finite differences -- none of them re-types the
oracle's own formulas."""

import math

import numpy as np
import pytest

import synth
from oracle import mlp

W, H = 640, 480


def test_parameter_layout():
    assert mlp.NPARAM == 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1 == 4673
    x = np.arange(mlp.NPARAM, dtype=np.float64)
    P = mlp.unpack(x)
    assert P["W1"][1, 0] == 6 and P["b1"][0] == 384 and P["W2"][0, 1] == 449
    assert P["b3"] == 4672
    assert np.array_equal(mlp.pack(P), x)


def test_features_forward_motion_closed_form():
    # K = I, R = I, t = (0, 0, 1): F = [t]x, epipole at the origin, distance |p|
    F = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    kp = np.array([[3.0, 4.0], [320.0, 240.0], [-6.0, 8.0]])
    f = mlp.features(F, kp, [1.5, 2.0, 3.0], [0.1, 0.2, 0.3], [-1.0, 0.0, 1.0], W, H)
    assert np.allclose(f[:, 0], [1.5, 2.0, 3.0]) and np.allclose(f[:, 1], [0.1, 0.2, 0.3])
    assert np.allclose(f[:, 2], [-1.0, 0.0, 1.0])
    assert np.allclose(f[:, 3], [(3 - 320) / 320, 0.0, (-6 - 320) / 320], rtol=0, atol=1e-15)
    assert np.allclose(f[:, 4], [(4 - 240) / 320, 0.0, (8 - 240) / 320], rtol=0, atol=1e-15)
    assert np.allclose(f[:, 5], [math.log1p(5 / 800), math.log1p(400 / 800),
                                 math.log1p(10 / 800)], rtol=1e-12)


def test_features_rectified_stereo_epipole_at_infinity():
    # t = (1, 0, 0): epipole (1, 0, 0), at infinity -> clipped distance
    F = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    f = mlp.features(F, [[10.0, 20.0], [600.0, 5.0]], [1, 1], [0, 0], [0, 0], W, H)
    assert np.allclose(f[:, 5], math.log1p(1000.0))


def test_epipole_matches_the_generating_cameras():
    for r in (0, 1, 2):
        p = synth.cfg4_pair(r, n_kp=200)
        e = mlp.epipole2(p.F)
        e2 = np.asarray(p.e2, np.float64)
        c = np.cross(e, e2 / np.linalg.norm(e2))
        assert np.linalg.norm(c) < 1e-9, (r, e, e2)


def test_constant_network_gives_clamped_softplus_of_the_bias():
    X = np.random.default_rng(0).normal(size=(50, 6)) * 5
    for beta, want in ((math.log(math.expm1(2.0)), 2.0), (-10.0, 0.5), (20.0, 8.0),
                       (math.log(math.expm1(3.3)), 3.3)):
        theta = np.zeros(mlp.NPARAM)
        theta[-1] = beta
        assert np.allclose(mlp.forward(theta, X)["eps"], want, rtol=1e-12)
    # BF16 inference rounds the bias first: 1.8545866 -> 1.8515625
    theta = np.zeros(mlp.NPARAM, np.float32)
    theta[-1] = math.log(math.expm1(2.0))
    want = math.log1p(math.exp(1.8515625))
    assert np.allclose(mlp.infer_bf16(theta, X), want, rtol=1e-12)


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 1 + 2 ** -8 + 2 ** -20, 3.0,
                  2 ** -130], np.float32)
    want = [1.0, 1.0, 1 + 2 ** -6, -1.0, 1 + 2 ** -7, 3.0, 2 ** -130]
    assert list(mlp.bf16_round(x)) == want
    # agrees with the independent encoder of the input generator
    r = np.random.default_rng(1).normal(size=10000).astype(np.float32) * 10
    assert np.array_equal(mlp.bf16_round(r), synth.bf16_to_f32(synth.f32_to_bf16(r)))


def test_pinball_hand_values():
    y = np.array([0.0, 1.0, 2.0, 3.0])
    # u = -1.5, -0.5, 0.5, 1.5: 0.01*1.5 + 0.01*0.5 + 0.99*0.5 + 0.99*1.5 = 2.0
    assert mlp.pinball(y, 1.5, 0.99) == pytest.approx(0.5, abs=1e-15)
    assert mlp.pinball(y, 1.5, 0.5) == pytest.approx(0.5, abs=1e-15)
    g = mlp.pinball_grad(y, np.full(4, 1.5), 0.99)
    assert np.allclose(g, [0.01 / 4, 0.01 / 4, -0.99 / 4, -0.99 / 4], rtol=1e-12)


def test_pinball_minimiser_over_constants_is_the_quantile():
    y = np.sort(np.random.default_rng(2).exponential(1.0, 1000))
    q = 0.99
    k = math.ceil(q * len(y)) - 1  # smallest c with empirical CDF(c) >= q
    best = mlp.pinball(y, y[k], q)
    for c in (y[k - 1], y[k + 1], y[k] - 1e-3, y[k] + 1e-3, np.mean(y), np.median(y)):
        assert best <= mlp.pinball(y, c, q) + 1e-15


def _safe_case(seed, n=120, margin=1e-3):
    """Inputs where no ReLU pre-activation and no residual lies near a kink."""
    rng = np.random.default_rng(seed)
    theta = synth.mlp_init(seed).astype(np.float64)
    theta[-65:-1] *= 20.0  # a larger output layer, so the gradients are not tiny
    p = synth.cfg4_pair(seed % 3, n_kp=400)
    X = mlp.features(p.F, p.kp2, p.scale2, p.resp2, p.ori2, p.W, p.H)
    f = mlp.forward(theta, X)
    ok = (np.abs(f["a1"]).min(axis=1) > margin) & (np.abs(f["a2"]).min(axis=1) > margin)
    X = X[ok][:n]
    yhat = mlp.forward(theta, X)["yhat"]
    sign = rng.choice([-1.0, 1.0], size=len(X))
    y = yhat + sign * rng.uniform(0.05, 1.0, size=len(X))
    return theta, X, y


@pytest.mark.parametrize("q", [0.99, 0.5])
def test_gradient_matches_central_differences(q):
    theta, X, y = _safe_case(5)
    assert len(X) >= 60
    _, g = mlp.loss_and_grad(theta, X, y, q)
    h = 1e-6
    fd = np.empty_like(g)
    for k in range(mlp.NPARAM):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (mlp.pinball(y, mlp.forward(tp, X)["yhat"], q)
                 - mlp.pinball(y, mlp.forward(tm, X)["yhat"], q)) / (2 * h)
    err = np.abs(fd - g)
    assert np.all(err <= 1e-6 * np.abs(g) + 1e-9), (err.max(), int(np.argmax(err)))
    assert np.count_nonzero(g) > 1000


def test_adam_first_steps_under_a_constant_gradient():
    rng = np.random.default_rng(3)
    theta = rng.normal(size=mlp.NPARAM)
    g = rng.normal(size=mlp.NPARAM)
    m = v = np.zeros(mlp.NPARAM)
    lr, eps = 1e-3, 1e-8
    step = lr * g / (np.abs(g) + eps)
    t1, m, v = mlp.adam(theta, g, m, v, 1, lr=lr, eps=eps)
    assert np.allclose(t1, theta - step, rtol=0, atol=1e-15)
    t2, m, v = mlp.adam(t1, g, m, v, 2, lr=lr, eps=eps)
    assert np.allclose(t2, theta - 2 * step, rtol=0, atol=1e-14)


MUTANTS = [
    ("loss_and_grad", 'da1 = (da2 @ P["W2"])', 'da1 = (da2 @ P["W2"].T)'),  # transposed operand
    ("loss_and_grad", '* (f["a1"] > 0.0)', ''),                            # dropped ReLU mask
    ("loss_and_grad", 'dz = dyhat * sigmoid(f["z"])', 'dz = dyhat'),        # dropped factor
    ("loss_and_grad", 'g["W2"] = da2.T @ f["h1"]', 'g["W2"] = da2.T @ f["h2"]'),  # wrong index
    ("pinball_grad", 'np.where(yhat >= y, 1.0 - q, -q)', 'np.where(yhat >= y, -q, 1.0 - q)'),
]


@pytest.mark.parametrize("fn,old,new", MUTANTS)
def test_finite_difference_pin_catches_planted_mistakes(fn, old, new, monkeypatch):
    """A mistake planted in the oracle's backward pass fails the central
    difference check (run on a subset of the parameters)."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(getattr(mlp, fn)))
    assert old in src
    ns = dict(vars(mlp))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    monkeypatch.setattr(mlp, fn, ns[fn])
    if fn == "pinball_grad":
        ns["loss_and_grad"].__globals__["pinball_grad"] = ns[fn]
    theta, X, y = _safe_case(5)
    q = 0.99
    _, g = (ns if fn == "loss_and_grad" else vars(mlp))["loss_and_grad"](theta, X, y, q)
    idx = np.concatenate([np.arange(0, 448, 7), np.arange(448, 4544, 41),
                          np.arange(4544, mlp.NPARAM)])
    h = 1e-6
    bad = 0
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.pinball(y, mlp.forward(tp, X)["yhat"], q)
              - mlp.pinball(y, mlp.forward(tm, X)["yhat"], q)) / (2 * h)
        bad += abs(fd - g[k]) > 1e-6 * abs(g[k]) + 1e-9
    assert bad > 0
