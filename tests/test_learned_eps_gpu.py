"""Learned per-keypoint tolerance on the GPU: features, BF16 inference,
gradients and Adam against the FP64 oracle, residual targets bit for bit, and
what the trained network gains over a fixed tolerance on held-out pairs."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from tests.gpu_util import specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _attrs(p):
    return np.stack([p.scale2, p.resp2, p.ori2], axis=1).astype(np.float32)


def _oracle_features(pairs):
    return np.concatenate([mlp.features(p.F, p.kp2, p.scale2, p.resp2, p.ori2, p.W, p.H)
                           for p in pairs])


def _rectified_pair():
    # sideways translation with no rotation: the epipole is at infinity
    return synth.make_pair(1920, 1080, 1000.0, np.eye(3), np.array([1.0, 0.0, 0.0]), 600, 200,
                           200, 123, scale_noise=(1.0, 12.0, 0.15), tag="rectified")


def test_features_match_oracle():
    from paper_2603_18401_amd import learned_eps as L
    torch = torch_gpu()
    pairs = [synth.cfg4_pair(r, n_kp=2000) for r in range(6)] + [_rectified_pair()]
    log("eps features: 6 cfg4 pairs + rectified")
    dev = torch.device("cuda:0")
    kp2 = torch.from_numpy(np.concatenate([p.kp2 for p in pairs])).to(dev)
    at = torch.from_numpy(np.concatenate([_attrs(p) for p in pairs])).to(dev)
    got = L.features(specs_of(pairs), kp2, at).cpu().numpy()
    ref = _oracle_features(pairs)
    assert np.all(np.abs(got - ref) <= 2e-6 * np.abs(ref) + 2e-7), np.abs(got - ref).max()
    assert np.allclose(got[-800:, 5], np.log1p(1000.0))


def _net(seed, out_scale=20.0):
    theta = synth.mlp_init(seed).astype(np.float32)
    theta[-65:-1] *= out_scale
    return theta


def test_bf16_inference_matches_oracle():
    from paper_2603_18401_amd import learned_eps as L
    torch = torch_gpu()
    pairs = [synth.cfg4_pair(r, n_kp=3000) for r in range(3)]
    X = _oracle_features(pairs).astype(np.float32)
    dev = torch.device("cuda:0")
    for seed in (1, 2):
        theta = _net(seed, out_scale=4.0 * seed)
        got = L.infer(torch.from_numpy(X).to(dev), torch.from_numpy(theta).to(dev))
        got = got.cpu().numpy()
        ref = mlp.infer_bf16(theta, X)
        # FP32 accumulation of 64-term dot products against FP64
        assert np.all(np.abs(got - ref) <= 1e-5 * ref + 5e-5), np.abs(got - ref).max()
        assert got.min() >= 0.5 and got.max() <= 8.0
        assert np.ptp(ref) > 0.5  # the network is not constant on these inputs


def _safe_samples(theta, X, rng, margin=1e-3):
    """Rows whose ReLU pre-activations and residual stay clear of the kinks
    (decided by the FP64 oracle), with targets 0.05-1 px from the output."""
    f = mlp.forward(theta.astype(np.float64), X.astype(np.float64))
    ok = (np.abs(f["a1"]).min(axis=1) > margin) & (np.abs(f["a2"]).min(axis=1) > margin)
    rows = np.nonzero(ok)[0]
    yhat = f["yhat"][rows]
    y = yhat + rng.choice([-1.0, 1.0], size=len(rows)) * rng.uniform(0.05, 1.0, size=len(rows))
    return rows, y.astype(np.float32)


@pytest.mark.parametrize("q", [0.99, 0.5])
def test_gradient_matches_oracle(q):
    from paper_2603_18401_amd import learned_eps as L
    torch = torch_gpu()
    rng = np.random.default_rng(4)
    pairs = [synth.cfg4_pair(r, n_kp=4000) for r in range(2)]
    X = _oracle_features(pairs).astype(np.float32)
    theta = _net(7)
    rows, y = _safe_samples(theta, X, rng)
    assert len(rows) > 2000
    # slots -> feature rows through feat_index; the batch lists slots in a random order
    batch = rng.permutation(len(rows))[:3000].astype(np.int32)
    log(f"eps gradient q={q}: {len(batch)} samples")
    dev = torch.device("cuda:0")
    tr = L.Trainer(theta, dev, q=q)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    feat, fidx, tgt, sidx = g(X), g(rows.astype(np.int64)), g(y), g(batch)
    grad, loss = tr.grad(feat, tgt, sidx, feat_index=fidx)
    got = grad.cpu().numpy().astype(np.float64)
    got_loss = float(loss.item())
    again = tr.grad(feat, tgt, sidx, feat_index=fidx)[0].cpu().numpy().astype(np.float64)
    assert np.array_equal(got, again)  # deterministic reductions
    rl, rg = mlp.loss_and_grad(theta.astype(np.float64),
                               X[rows[batch]].astype(np.float64), y[batch].astype(np.float64), q)
    assert abs(got_loss - rl) <= 1e-5 * abs(rl)
    gmax = np.abs(rg).max()
    assert np.abs(got - rg).max() <= 1e-4 * gmax
    big = np.abs(rg) >= 1e-2 * gmax
    assert np.all(np.abs(got - rg)[big] <= 1e-4 * np.abs(rg)[big])


def test_adam_matches_oracle():
    from paper_2603_18401_amd import learned_eps as L
    torch = torch_gpu()
    rng = np.random.default_rng(9)
    dev = torch.device("cuda:0")
    theta = rng.normal(size=mlp.NPARAM).astype(np.float32)
    tr = L.Trainer(theta, dev)
    m = rng.normal(size=mlp.NPARAM).astype(np.float32) * 1e-2
    v = rng.uniform(0, 1e-3, size=mlp.NPARAM).astype(np.float32)
    grad = rng.normal(size=mlp.NPARAM).astype(np.float32) * 1e-2
    tr.m.copy_(torch.from_numpy(m))
    tr.v.copy_(torch.from_numpy(v))
    tr.grad_buf.copy_(torch.from_numpy(grad))
    tr.t = 2
    tr.adam()  # step 3
    # the hyperparameters reach the device as float32 values: use those
    f = lambda x: float(np.float32(x))  # noqa: E731
    rt, rm, rv = mlp.adam(theta, grad, m, v, 3, lr=f(1e-3), beta1=f(0.9), beta2=f(0.999),
                          eps=f(1e-8))
    assert np.allclose(tr.params.cpu().numpy(), rt, rtol=0, atol=2e-7)
    # FP32 moments: a few roundings of 2^-24 relative to the two terms (and of
    # beta1 / beta2 themselves), which can cancel
    g64 = grad.astype(np.float64)
    bm = 3e-7 * (0.9 * np.abs(m) + 0.1 * np.abs(g64))
    bv = 3e-7 * (0.999 * np.abs(v) + 0.001 * g64 * g64)
    assert np.all(np.abs(tr.m.cpu().numpy() - rm) <= bm)
    assert np.all(np.abs(tr.v.cpu().numpy() - rv) <= bv)


def test_residuals_equal_oracle():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg4_pair(3, n_kp=3000)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 8.0)
    best, _, _ = oracle.match(p.desc1, p.desc2, ro, rc, ratio=0.8)
    log(f"residuals: {int((best >= 0).sum())} matches")
    dev = torch.device("cuda:0")
    k1, k2 = torch.from_numpy(p.kp1).to(dev), torch.from_numpy(p.kp2).to(dev)
    idx = E.Index(specs_of([p]), k2, eps=8.0)
    res = torch.empty(p.m, dtype=torch.float32, device=dev)
    fidx = torch.empty(p.m, dtype=torch.int64, device=dev)
    lib = E.load_library()
    st = lib.epm_match_residuals(idx.handle, E._dptr(k1), E._dptr(k2),
                                 E._dptr(torch.from_numpy(best).to(dev)), E._dptr(res),
                                 E._dptr(fidx), E._stream(torch, dev))
    assert st == 0
    res, fidx = res.cpu().numpy(), fidx.cpu().numpy()
    has = best >= 0
    qi = np.nonzero(has)[0]
    ref = oracle.point_line_dist(p.F, p.kp1, p.kp2, qi, best[has]).astype(np.float32)
    assert np.array_equal(res[has], ref)
    assert np.all(res[~has] == -1.0) and np.all(fidx[~has] == -1)
    assert np.array_equal(fidx[has], best[has])
    assert ref.max() <= 8.0


# ----------------------------------------------------------- the gain test

def _recall_kbar(pairs, eps2_list, torch, dev):
    """Candidate recall of the true matches and candidates per query over a
    set of pairs, each with its own per-keypoint tolerances."""
    import paper_2603_18401_amd as E
    hit = tot = nnz = nq = 0
    for p, e2 in zip(pairs, eps2_list):
        k1, k2 = torch.from_numpy(p.kp1).to(dev), torch.from_numpy(p.kp2).to(dev)
        idx = E.Index(specs_of([p]), k2, eps2=e2)
        offs, cols = idx.query(k1)
        o, c = offs.cpu().numpy(), cols.cpu().numpy()
        idx.close()
        rows = np.repeat(np.arange(p.m), np.diff(o))
        keys = rows.astype(np.int64) * (p.n + 1) + c
        t = np.nonzero(p.gt12 >= 0)[0]
        want = t.astype(np.int64) * (p.n + 1) + p.gt12[t]
        pos = np.searchsorted(keys, want)
        found = (pos < len(keys)) & (keys[np.minimum(pos, len(keys) - 1)] == want)
        hit += int(found.sum())
        tot += len(t)
        nnz += int(o[-1])
        nq += p.m
    return hit / tot, nnz / nq


def train_and_compare(n_train, n_test, epochs, torch, dev, log=log, batch=65536):
    """Trains the tolerance network on the method's own matches of n_train
    pairs and measures held-out recall / candidates per query for the learned
    tolerance and for a sweep of fixed tolerances."""
    from paper_2603_18401_amd import learned_eps as L
    Xs, ys = [], []
    for c0 in range(0, n_train, 16):
        pairs = [synth.cfg4_pair(r) for r in range(c0, min(n_train, c0 + 16))]
        b = synth.batch_pairs(pairs)
        g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        specs = specs_of(pairs)
        res, fidx = L.residual_targets(specs, g(b.kp1), g(b.kp2), g(b.desc1), g(b.desc2))
        at = np.concatenate([_attrs(p) for p in pairs])
        feat = L.features(specs, g(b.kp2), g(at)).cpu().numpy()
        res, fidx = res.cpu().numpy(), fidx.cpu().numpy()
        ok = fidx >= 0
        Xs.append(feat[fidx[ok]])
        ys.append(res[ok])
        log(f"training data: {c0 + len(pairs)} pairs")
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    tr = L.Trainer(synth.mlp_init(0), dev, q=0.99)
    hist = tr.fit(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), epochs, batch=batch,
                  seed=1)
    log(f"trained on {len(y)} residuals: loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    test = [synth.cfg4_pair(10000 + r) for r in range(n_test)]
    learned = []
    for p in test:
        f = L.features(specs_of([p]), torch.from_numpy(p.kp2).to(dev),
                       torch.from_numpy(_attrs(p)).to(dev))
        learned.append(L.infer(f, tr.params))
    rl, kl = _recall_kbar(test, learned, torch, dev)
    sweep = []
    for e in (0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 5.0, 6.0, 8.0):
        fixed = [torch.full((p.n,), e, dtype=torch.float32, device=dev) for p in test]
        r, k = _recall_kbar(test, fixed, torch, dev)
        sweep.append((e, r, k))
    mean_eps = float(np.mean(np.concatenate([x.cpu().numpy() for x in learned])))
    return {"train_samples": int(len(y)), "loss_first": hist[0], "loss_last": hist[-1],
            "learned": {"recall": rl, "kbar": kl, "mean_eps": mean_eps},
            "fixed": [{"eps": e, "recall": r, "kbar": k} for e, r, k in sweep]}


def test_learned_eps_beats_fixed_eps_on_held_out_pairs():
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    out = train_and_compare(48, 12, 300, torch, dev)
    log(str(out))
    assert out["loss_last"] < 0.7 * out["loss_first"]
    rl, kl = out["learned"]["recall"], out["learned"]["kbar"]
    fx = out["fixed"]
    ks = np.array([f["kbar"] for f in fx])
    rs = np.array([f["recall"] for f in fx])
    assert np.all(np.diff(ks) > 0) and np.all(np.diff(rs) >= 0)
    # the fixed-tolerance curve at the learned candidate count
    r_at = float(np.interp(kl, ks, rs))
    assert rl > r_at + 0.005, (rl, r_at, kl)
