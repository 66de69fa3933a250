"""The seeded generator: geometry of each workload, reproducibility and the
descriptor storage formats."""

import numpy as np
import pytest

import synth


def test_epipolar_constraint_on_noiseless_points():
    """Eq. 2 holds for the noiseless projections (up to FP32 storage)."""
    p = synth.cfg1_pair("sideways", n_kp=2000)
    t = p.gt12 >= 0
    x1 = np.c_[p.clean1[t].astype(np.float64), np.ones(t.sum())]
    x2 = np.c_[p.clean2[p.gt12[t]].astype(np.float64), np.ones(t.sum())]
    l = x1 @ p.F.T
    r = np.abs((l * x2).sum(1)) / np.hypot(l[:, 0], l[:, 1])
    assert r.max() < 1e-3


def test_epipole_classes():
    s = synth.cfg1_pair("sideways", n_kp=1000)
    e = s.e2[:2] / s.e2[2]
    assert e[0] < -10000  # far outside the image (yaw 10 deg)
    f = synth.cfg1_pair("forward", n_kp=1000)
    e = f.e2[:2] / f.e2[2]
    assert e[0] == 3024.0 and e[1] == 2016.0  # exactly the image centre
    inf = synth.cfg3_pair(0)
    assert inf.e2[2] == 0.0  # exactly infinite epipole
    far = synth.cfg3_pair(3)
    assert abs(far.e2[0] / far.e2[2]) > 1e5
    # F^T e2 = 0 and F e1 = 0
    for p in (s, f, inf, far):
        assert np.abs(p.F.T @ (p.e2 / np.linalg.norm(p.e2))).max() < 1e-12 * np.abs(p.F).max() * 1e4
        assert np.abs(p.F @ (p.e1 / np.linalg.norm(p.e1))).max() < 1e-12 * np.abs(p.F).max() * 1e4


def test_seed_reproducible_and_shapes():
    a = synth.cfg0_pair(5)
    b = synth.cfg0_pair(5)
    assert np.array_equal(a.kp1, b.kp1) and np.array_equal(a.desc2, b.desc2)
    assert a.m == 1000 and a.n == 1000 and (a.gt12 >= 0).sum() == 800
    assert a.kp1.dtype == np.float32 and a.desc1.dtype == np.float32
    assert np.allclose(np.linalg.norm(a.desc1, axis=1), 1.0, atol=1e-5)
    c = synth.cfg0_pair(6)
    assert not np.array_equal(a.kp1, c.kp1)


def test_ground_truth_map_is_a_partial_bijection():
    p = synth.cfg1_pair("forward", n_kp=3000)
    g = p.gt12[p.gt12 >= 0]
    assert len(np.unique(g)) == len(g) == 2100


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-8, 8, 100000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(synth.f32_to_bf16(x), ref)
    assert np.array_equal(synth.bf16_to_f32(ref), torch.from_numpy(ref.view(np.int16)).view(
        torch.bfloat16).float().numpy())


def test_fp8_e4m3_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    d = synth.pairs._unit_rows(rng.standard_normal((2000, 128)))
    codes, scale = synth.f32_to_fp8_e4m3(d)
    scaled = torch.from_numpy(d) / torch.from_numpy(scale)[:, None]
    ref = scaled.to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(codes, ref)
    back = synth.fp8_e4m3_to_f32(codes)
    ref_back = torch.from_numpy(ref).view(torch.float8_e4m3fn).float().numpy()
    assert np.array_equal(back, ref_back)
    assert np.abs(back).max() <= 448.0 and (np.abs(back).max(axis=1) == 448.0).all()
    # all 256 codes decode like torch (NaN codes aside)
    allc = np.arange(256, dtype=np.uint8)
    a = synth.fp8_e4m3_to_f32(allc)
    b = torch.from_numpy(allc).view(torch.float8_e4m3fn).float().numpy()
    ok = ~np.isnan(b)
    assert np.array_equal(a[ok], b[ok]) and np.isnan(a[~ok]).all()


def test_binary_flip_rate():
    p = synth.cfg0_pair(2, binary=True)
    t = p.gt12 >= 0
    h = np.bitwise_count(p.bin1[t] ^ p.bin2[p.gt12[t]]).sum(1)
    assert abs(h.mean() / 256 - 0.08) < 0.01


def test_batch_concatenation():
    pairs = [synth.cfg3_pair(r, max_kp=2000) for r in range(4)]
    b = synth.batch_pairs(pairs)
    assert b.kp1.shape[0] == sum(p.m for p in pairs)
    for k, p in enumerate(pairs):
        assert np.array_equal(b.kp2[b.k_begin[k]:b.k_begin[k] + p.n], p.kp2)


def test_fp8_rounding_error_bounds_hold():
    """The FP8 rows' rounding-error bounds that the fused FP8 tests pass in
    (tests.gpu_util.fp8_rows) are not below the FP64 error of any row and
    exceed it by no more than their rounding up."""
    from tests.gpu_util import fp8_rows
    p = synth.cfg0_pair(0)
    codes, scale, err = fp8_rows(p.desc2)
    deq = synth.fp8_e4m3_to_f32(codes).astype(np.float64) * scale[:, None]
    exact = np.sqrt(((p.desc2.astype(np.float64) - deq) ** 2).sum(axis=1))
    assert err.dtype == np.float32 and codes.dtype == np.uint8
    assert np.all(err.astype(np.float64) >= exact)
    assert np.all(err.astype(np.float64) <= exact * (1 + 1e-5) + 1e-30)
