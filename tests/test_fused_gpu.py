"""epm_query_match: candidate CSR and FP32 matches in one pass, against the
oracle and against the separate query + match calls, bit for bit."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, oracle_batch, specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _fused(pairs, eps, ratio=0.0, eps2=None, kp1=None):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    b = synth.batch_pairs(pairs)
    k1 = _dev(torch, b.kp1 if kp1 is None else kp1)
    e2 = None if eps2 is None else _dev(torch, eps2)
    idx = E.Index(specs_of(pairs), _dev(torch, b.kp2), eps2=e2, eps=eps)
    o, c, bi, bd, sd = idx.query_match(k1, _dev(torch, b.desc1), _dev(torch, b.desc2),
                                       ratio=ratio)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (o, c, bi, bd, sd)], idx


def _oracle(pairs, eps, ratio=0.0, kp1=None):
    b = synth.batch_pairs(pairs)
    ro, rc, _ = oracle_batch(pairs, eps, kp1=kp1)
    rows = np.repeat(np.arange(len(pairs)), [p.m for p in pairs])
    rb, rbd, rsd = oracle.match(b.desc1, b.desc2, ro, rc, ratio=ratio, col_base=b.k_begin[rows])
    return ro, rc, rb, rbd, rsd


def _same(got, ref, what):
    o, c, bi, bd, sd = got
    ro, rc, rb, rbd, rsd = ref
    assert_csr_equal((o, c), (ro, rc), what)
    assert np.array_equal(bi, rb), what
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32)), what
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32)), what


@pytest.mark.parametrize("ratio", [0.0, 0.8])
def test_cfg0_fused_equals_oracle(ratio):
    for r in range(3):
        p = synth.cfg0_pair(r)
        log(f"fused cfg0 r={r} ratio={ratio}")
        got, _ = _fused([p], 2.0, ratio)
        _same(got, _oracle([p], 2.0, ratio), f"cfg0 {r}")


@pytest.mark.parametrize("motion", ["sideways", "forward", "forward_yaw"])
@pytest.mark.parametrize("eps", [1.0, 4.0])
def test_cfg1_fused_equals_oracle(motion, eps):
    p = synth.cfg1_pair(motion)
    log(f"fused cfg1 {motion} eps={eps}")
    got, idx = _fused([p], eps)
    _same(got, _oracle([p], eps), f"{motion} {eps}")
    assert idx.stats()["candidates"] == int(got[0][-1])


def test_counters_of_the_fused_and_plain_query_agree():
    """The tile pass leaves its counters per tile whether or not it also
    matches: both calls report the same scan, angle hits and candidates, and
    the brute-force queries of an off-rank F are counted."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(1)
    F = p.F + 1e-3 * np.abs(p.F).max() * np.random.default_rng(11).standard_normal((3, 3))
    p.F = F
    log("counters: query vs query_match, full-rank F")
    k1, k2 = _dev(torch, p.kp1), _dev(torch, p.kp2)
    idx = E.Index(specs_of([p]), k2, eps=3.0)
    o, _ = idx.query(k1)
    st_q = idx.stats()
    idx.query_match(k1, _dev(torch, p.desc1), _dev(torch, p.desc2))
    st_m = idx.stats()
    assert st_q == st_m
    assert st_q["candidates"] == int(o.cpu().numpy()[-1])
    assert st_q["scanned_queries"] > 0
    assert st_q["candidates"] <= st_q["angle_hits"] <= st_q["records_scanned"]


def test_long_rows_take_the_wide_row_pass():
    """A wide tolerance gives rows beyond the on-chip list (more than 128
    candidates); the wide-row pass writes and matches them."""
    p = synth.cfg0_pair(1)
    log("fused cfg0 with eps 30")
    got, _ = _fused([p], 30.0)
    lens = np.diff(got[0])
    assert lens.max() > 128 and (lens <= 128).sum() > 0
    _same(got, _oracle([p], 30.0), "wide rows")


@pytest.mark.parametrize("eps", [1.5, 4.0])
def test_sparse_queries_over_a_dense_image(eps):
    """100 queries against 8040 image-2 keypoints: each tile spans a wide
    angle range, its window holds thousands of records (more than the pass
    keeps the j of), so its short rows are rebuilt by the fill pass and
    matched from the list."""
    yaw = synth.pairs.rot_axis_angle([0.0, 1.0, 0.0], np.deg2rad(8.0))
    p = synth.make_pair(6048, 4032, 3400.0, yaw, [1.0, 0.0, 0.0], 40, 60, 8000, 777)
    log(f"fused, sparse queries over {p.n} keypoints, eps {eps}")
    got, idx = _fused([p], eps, 0.8)
    lens = np.diff(got[0])
    assert lens.max() <= 128
    st = idx.stats()
    # each group of 16 queries spans a wide angle range: hundreds of the
    # window's records meet its key span and are tested per query
    assert st["records_scanned"] > 256 * (st["queries"] - st["empty_queries"])
    _same(got, _oracle([p], eps, 0.8), f"sparse queries eps {eps}")


def test_mixed_batch_fused_equals_oracle():
    pairs = [synth.cfg3_pair(r, max_kp=4000) for r in range(24)]
    log("fused cfg3 mixed batch of 24")
    got, idx = _fused(pairs, 2.0, 0.8)
    _same(got, _oracle(pairs, 2.0, 0.8), "cfg3")


def test_zero_line_query_gets_the_empty_match():
    # pure forward motion with K = I: the query at the origin is e1 (a = b = 0)
    rng = np.random.default_rng(5)
    F = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    p = synth.cfg0_pair(0)
    p.F = F
    p.kp1 = p.kp1.copy()
    p.kp1[:5] = 0.0
    p.kp2 = rng.uniform(-300, 300, p.kp2.shape).astype(np.float32)
    p.kp1[5:] = rng.uniform(-300, 300, p.kp1[5:].shape).astype(np.float32)
    got, _ = _fused([p], 2.0)
    assert np.all(got[2][:5] == -1) and np.all(np.isinf(got[3][:5]))
    _same(got, _oracle([p], 2.0), "zero lines")


def test_fused_equals_separate_calls_on_the_bench_step():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    pairs, eps_list = [], []
    for motion in ("sideways", "forward"):
        base = synth.cfg1_pair(motion)
        for e in (1.0, 2.0, 4.0):
            pairs.append(base)
            eps_list.append(e)
    log("fused vs separate on the six-pair step")
    b = synth.batch_pairs(pairs)
    eps2 = np.concatenate([np.full(p.n, e, np.float32) for p, e in zip(pairs, eps_list)])
    d1, d2 = _dev(torch, b.desc1), _dev(torch, b.desc2)
    k1, k2, e2 = _dev(torch, b.kp1), _dev(torch, b.kp2), _dev(torch, eps2)
    idx = E.Index(specs_of(pairs), k2, eps2=e2)
    fused = [x.cpu().numpy() for x in idx.query_match(k1, d1, d2)]
    o, c = idx.query(k1)
    sep = [x.cpu().numpy() for x in (o, c) + tuple(idx.match(o, c, d1, d2, algo="tiled"))]
    for a, r in zip(fused, sep):
        assert np.array_equal(a.view(np.uint8), r.view(np.uint8))


def test_capacity_contract():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(2)
    ref = _oracle([p], 2.0)
    k1, k2 = _dev(torch, p.kp1), _dev(torch, p.kp2)
    d1, d2 = _dev(torch, p.desc1), _dev(torch, p.desc2)
    idx = E.Index(specs_of([p]), k2, eps=2.0)
    # a too-small first buffer is grown and the call repeated (host check)
    got = [x.cpu().numpy() for x in idx.query_match(k1, d1, d2, capacity=16)]
    _same(got, ref, "retry")
    # no host check: rows written up to the capacity, row_offsets complete
    offs = torch.empty(p.m + 1, dtype=torch.int64, device=k1.device)
    cols = torch.empty(64, dtype=torch.int32, device=k1.device)
    idx.query_match(k1, d1, d2, row_offsets=offs, col_indices=cols, sync=False)
    torch.cuda.synchronize()
    assert np.array_equal(offs.cpu().numpy(), ref[0])
