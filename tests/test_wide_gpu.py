"""Wide rows: queries with more than 128 candidates, as at the tolerances of
the paper's experiments (25-100 px).  The wide-row pass writes their CSR rows
in ascending j from a bitmap of the tile window and selects their FP32
matches through a BF16 MFMA bound with a certified re-rank; everything is
compared with the oracle bit for bit."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _oracle(p, eps, ratio=0.0, desc2=None):
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, eps)
    d2 = p.desc2 if desc2 is None else desc2
    rb, rbd, rsd = oracle.match(p.desc1, d2, ro, rc, ratio=ratio)
    return ro, rc, rb, rbd, rsd


def _same_matches(got, ref, what):
    bi, bd, sd = got
    rb, rbd, rsd = ref
    bad = np.nonzero(bi != rb)[0]
    assert len(bad) == 0, f"{what}: best index differs at {bad[:8]} (of {len(bad)})"
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32)), what
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32)), what


def _run(p, eps, ratio=0.0, desc2=None):
    """idx.query (CSR only), then query_match (CSR + fused FP32 matches)."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    k1, k2 = _dev(torch, p.kp1), _dev(torch, p.kp2)
    d1 = _dev(torch, p.desc1)
    d2 = _dev(torch, p.desc2 if desc2 is None else desc2)
    idx = E.Index(specs_of([p]), k2, eps=eps)
    o, c = idx.query(k1)
    q = (o.cpu().numpy(), c.cpu().numpy())
    res = [x.cpu().numpy() for x in idx.query_match(k1, d1, d2, ratio=ratio)]
    torch.cuda.synchronize()
    return q, res, idx


@pytest.mark.parametrize("motion", ["sideways", "forward"])
@pytest.mark.parametrize("eps", [25.0, 50.0])
def test_paper_regime_pair(motion, eps):
    p = synth.cfg1_pair(motion, n_kp=25000)
    log(f"wide rows: {motion}, 25000 keypoints, eps {eps}")
    ref = _oracle(p, eps, ratio=0.8)
    q, res, idx = _run(p, eps, ratio=0.8)
    lens = np.diff(ref[0])
    assert np.median(lens) > 128, "the case must exercise wide rows"
    assert_csr_equal(q, ref[:2], "query")
    assert_csr_equal(res[:2], ref[:2], "query_match CSR")
    _same_matches(res[2:], ref[2:], "query_match")
    st = idx.match_stats()
    # every wide row is ranked on MFMA and nearly all are certified there
    assert st["reranked_rows"] == int((lens > 128).sum())
    assert st["fallback_rows"] < 0.1 * st["reranked_rows"]


def test_equal_descriptors_fall_back_to_the_exact_match():
    """Image-2 rows repeat four prototypes: every wide row has many candidates
    at the same distance, no bound can certify, and the exact listed match
    decides (ties to the lowest j)."""
    p = synth.cfg0_pair(2)
    rng = np.random.default_rng(3)
    protos = rng.standard_normal((4, 128)).astype(np.float32)
    d2 = protos[rng.integers(0, 4, p.n)]
    log("wide rows with repeated descriptors, cfg0 eps 60")
    ref = _oracle(p, 60.0, desc2=d2)
    assert (np.diff(ref[0]) > 128).sum() > 100
    q, res, idx = _run(p, 60.0, desc2=d2)
    assert_csr_equal(res[:2], ref[:2], "CSR")
    _same_matches(res[2:], ref[2:], "ties")
    assert idx.match_stats()["fallback_rows"] > 0


def test_image2_larger_than_one_bitmap_slab():
    """More than 65536 image-2 keypoints: the window is enumerated slab by
    slab, still in ascending j."""
    yaw = synth.pairs.rot_axis_angle([0.0, 1.0, 0.0], np.deg2rad(10.0))
    p = synth.make_pair(6048, 4032, 3400.0, yaw, [1.0, 0.0, 0.0], 3000, 500, 67000, 4242)
    assert p.n > 65536
    log(f"wide rows over {p.n} image-2 keypoints, eps 12")
    ref = _oracle(p, 12.0)
    assert (np.diff(ref[0]) > 128).sum() > 1000
    q, res, _ = _run(p, 12.0)
    assert_csr_equal(q, ref[:2], "query")
    assert_csr_equal(res[:2], ref[:2], "query_match CSR")
    _same_matches(res[2:], ref[2:], "matches")


def test_full_rank_f_scans_and_long_rows():
    """F off rank 2: query lines miss the epipole, those queries scan the
    whole pair; their long rows are rebuilt and matched outside the tile
    passes, next to the wide rows of the normal queries."""
    p = synth.cfg0_pair(1)
    rng = np.random.default_rng(11)
    F = p.F.copy()
    F = F + 1e-3 * np.abs(F).max() * rng.standard_normal((3, 3))
    p.F = F
    log("full-rank F, cfg0 eps 40")
    ref = _oracle(p, 40.0)
    q, res, idx = _run(p, 40.0)
    assert idx.stats()["scanned_queries"] > 0
    assert (np.diff(ref[0]) > 128).sum() > 0
    assert_csr_equal(q, ref[:2], "query")
    assert_csr_equal(res[:2], ref[:2], "query_match CSR")
    _same_matches(res[2:], ref[2:], "matches")


def test_wide_rows_capacity_without_host_check():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(0)
    ref = _oracle(p, 50.0)
    nnz = int(ref[0][-1])
    k1, k2 = _dev(torch, p.kp1), _dev(torch, p.kp2)
    d1, d2 = _dev(torch, p.desc1), _dev(torch, p.desc2)
    idx = E.Index(specs_of([p]), k2, eps=50.0)
    cap = nnz // 3
    offs = torch.empty(p.m + 1, dtype=torch.int64, device=k1.device)
    cols = torch.full((cap,), -7, dtype=torch.int32, device=k1.device)
    log(f"wide rows, capacity {cap} of {nnz}")
    idx.query(k1, row_offsets=offs, col_indices=cols, sync=False)
    torch.cuda.synchronize()
    assert np.array_equal(offs.cpu().numpy(), ref[0])
    assert np.array_equal(cols.cpu().numpy(), ref[1][:cap])
    cols.fill_(-7)
    idx.query_match(k1, d1, d2, row_offsets=offs, col_indices=cols, sync=False)
    torch.cuda.synchronize()
    assert np.array_equal(offs.cpu().numpy(), ref[0])
    assert np.array_equal(cols.cpu().numpy(), ref[1][:cap])


def _match_inputs(torch, p, dtype):
    d1, d2 = _dev(torch, p.desc1), _dev(torch, p.desc2)
    if dtype == "f32":
        return dict(desc1=d1, desc2=d2, dtype="f32")
    if dtype == "bf16":
        return dict(desc1=_dev(torch, synth.f32_to_bf16(p.desc1).view(np.int16)),
                    desc2=_dev(torch, synth.f32_to_bf16(p.desc2).view(np.int16)), dtype="bf16",
                    desc1_f32=d1, desc2_f32=d2)
    c1, s1 = synth.f32_to_fp8_e4m3(p.desc1)
    c2, s2 = synth.f32_to_fp8_e4m3(p.desc2)
    return dict(desc1=_dev(torch, c1), desc2=_dev(torch, c2), dtype="fp8",
                scale1=_dev(torch, s1), scale2=_dev(torch, s2), desc1_f32=d1, desc2_f32=d2)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_separate_match_on_wide_rows(dtype):
    """epm_match over the query's CSR at eps 50 px: the flagged tiles go to
    the wide-row pass (FP32 and BF16), FP8 stays on the window kernel."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg1_pair("forward", n_kp=25000)
    log(f"separate match on wide rows, {dtype}")
    ref = _oracle(p, 50.0, ratio=0.8)
    idx = E.Index(specs_of([p]), _dev(torch, p.kp2), eps=50.0)
    o, c = idx.query(_dev(torch, p.kp1))
    got = [x.cpu().numpy() for x in idx.match(o, c, ratio=0.8, algo="tiled",
                                              **_match_inputs(torch, p, dtype))]
    _same_matches(got, ref[2:], dtype)
    if dtype != "fp8":
        st = idx.match_stats()
        assert st["reranked_rows"] > 0.9 * p.m
        assert st["fallback_rows"] < 0.1 * st["reranked_rows"]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_foreign_csr_on_wide_tiles(dtype):
    """A CSR from a different tolerance on an index whose last query flagged
    its tiles as wide: rows that differ from the tile's candidate sets are
    matched exactly, so the result is the oracle's over the given CSR."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(3)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 45.0)
    rows = np.repeat(np.arange(p.m), np.diff(ro))
    keep = (rows % 3 != 0) | (np.arange(len(rc)) % 5 != 0)  # and thin some rows out
    ro2 = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=p.m))]).astype(np.int64)
    rc2 = rc[keep]
    ref = oracle.match(p.desc1, p.desc2, ro2, rc2, ratio=0.0)
    log(f"foreign CSR on wide tiles, {dtype}")
    idx = E.Index(specs_of([p]), _dev(torch, p.kp2), eps=50.0)
    o, _ = idx.query(_dev(torch, p.kp1))
    assert (np.diff(o.cpu().numpy()) > 128).sum() > 0
    got = [x.cpu().numpy() for x in idx.match(_dev(torch, ro2), _dev(torch, rc2), algo="tiled",
                                              **_match_inputs(torch, p, dtype))]
    _same_matches(got, ref, "foreign")


def _uneven_pair(m, n, seed, motion="sideways"):
    """A 6048x4032 pair with m queries and n image-2 keypoints (most of the
    surplus on either side outliers)."""
    yaw = synth.pairs.rot_axis_angle([0.0, 1.0, 0.0], np.deg2rad(10.0 if motion == "sideways" else 3.0))
    c2 = [1.0, 0.0, 0.0] if motion == "sideways" else [0.0, 0.0, 1.0]
    t = min(m, n) * 4 // 5
    return synth.make_pair(6048, 4032, 3400.0, yaw, c2, t, m - t, n - t, seed)


def _batch_against_oracle(pairs, eps_list, what):
    """Fused query + FP32 match and separate query + tiled match of one batch,
    every pair compared with the oracle (CSR and matches)."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    kp1 = np.concatenate([p.kp1 for p in pairs])
    kp2 = np.concatenate([p.kp2 for p in pairs])
    eps2 = np.concatenate([np.full(p.n, e, np.float32) for p, e in zip(pairs, eps_list)])
    d1 = np.concatenate([p.desc1 for p in pairs])
    d2 = np.concatenate([p.desc2 for p in pairs])
    idx = E.Index(specs_of(pairs), _dev(torch, kp2), eps2=_dev(torch, eps2))
    fused = [x.cpu().numpy() for x in idx.query_match(_dev(torch, kp1), _dev(torch, d1), _dev(torch, d2))]
    o, c = idx.query(_dev(torch, kp1))
    sep = [x.cpu().numpy() for x in idx.match(o, c, _dev(torch, d1), _dev(torch, d2), dtype="f32",
                                              algo="tiled")]
    torch.cuda.synchronize()
    q0 = k0 = 0
    wide = []
    for pi, (p, e) in enumerate(zip(pairs, eps_list)):
        ref = _oracle(p, e)
        wide.append(int((np.diff(ref[0]) > 128).sum()))
        lo, hi = fused[0][q0], fused[0][q0 + p.m]
        rows = (fused[0][q0:q0 + p.m + 1] - lo, fused[1][lo:hi])
        assert_csr_equal(rows, ref[:2], f"{what}: pair {pi} CSR")
        _same_matches([a[q0:q0 + p.m] for a in fused[2:]], ref[2:], f"{what}: pair {pi} fused")
        _same_matches([a[q0:q0 + p.m] for a in sep], ref[2:], f"{what}: pair {pi} separate")
        q0 += p.m
        k0 += p.n
    log(f"{what}: rows over 128 candidates per pair {wide}")
    return wide


def test_copies_and_on_chip_rows_in_one_launch():
    """Below 2048 tiles one wide-row launch decides per tile: a pair with a
    wide tile per 256 image-2 rows or more stages BF16 copies of its rows, a
    pair with few queries against many image-2 keypoints (wide rows, but too
    few tiles for copies) rounds on chip."""
    a = _uneven_pair(30000, 12000, 5151)  # 469 wide tiles x 256 >= 12000: copies
    b = _uneven_pair(2000, 40000, 5152, "forward")  # 32 x 256 < 40000: on chip
    log(f"copies and on-chip rounding in one launch: {a.m}/{a.n} + {b.m}/{b.n} keypoints, eps 50")
    wide = _batch_against_oracle([a, b], [50.0, 50.0], "mixed launch")
    assert wide[0] > 0.9 * a.m and wide[1] > 0.9 * b.m


def test_copies_and_on_chip_rows_in_two_launches():
    """Between 2048 and 16384 tiles the tiles of pairs with copies and the
    others go to two launches; a narrow pair adds tiles without wide rows."""
    a = _uneven_pair(70000, 15000, 6161)   # 1094 tiles, copies
    b = _uneven_pair(3000, 50000, 6162, "forward")  # 47 wide tiles, on chip
    c = _uneven_pair(60000, 8000, 6163)    # 938 tiles, eps 2 px: no wide row
    assert sum((p.m + 63) // 64 for p in (a, b, c)) > 2048
    log("copies and on-chip rounding in two launches: 2079 tiles")
    wide = _batch_against_oracle([a, b, c], [50.0, 50.0, 2.0], "split launches")
    assert wide[0] > 0.9 * a.m and wide[1] > 0.9 * b.m and wide[2] == 0
