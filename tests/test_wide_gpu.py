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
