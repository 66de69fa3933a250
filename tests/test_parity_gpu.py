"""GPU parity: candidate CSR and matches through the C ABI against the CPU
oracle, element by element."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, oracle_batch, run_candidates, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_fp64_terms_bit_exact():
    """Both sides of the Eq. 3 comparison (including the device sqrt) are
    bit-identical to the oracle's on many random lines and points."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    rng = np.random.default_rng(0)
    dev = torch.device("cuda:0")
    for trial in range(4):
        p = [synth.cfg0_pair(trial), synth.cfg1_pair("forward_yaw", n_kp=3000),
             synth.cfg3_pair(3, max_kp=3000), synth.cfg3_pair(0, max_kp=3000)][trial]
        K = 200_000
        qi = rng.integers(0, p.m, K)
        kj = rng.integers(0, p.n, K)
        eps = rng.uniform(1e-3, 50.0, p.n).astype(np.float32)
        num, rhs = E.point_line_terms(
            p.F, torch.from_numpy(p.kp1).to(dev), torch.from_numpy(p.kp2).to(dev),
            torch.from_numpy(qi).to(dev), torch.from_numpy(kj).to(dev),
            eps2=torch.from_numpy(eps).to(dev))
        rn, rr = oracle.candidate_terms(p.F, p.kp1, p.kp2, eps, qi, kj)
        assert np.array_equal(num.cpu().numpy().view(np.uint64), rn.view(np.uint64)), p.tag
        assert np.array_equal(rhs.cpu().numpy().view(np.uint64), rr.view(np.uint64)), p.tag


@pytest.mark.parametrize("r", [0, 1, 2])
def test_cfg0_candidates(r):
    p = synth.cfg0_pair(r)
    log(f"cfg0 r={r} {p.tag}")
    o, c, _ = run_candidates([p], 2.0)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 2.0)
    assert_csr_equal((o, c), (ro, rc), p.tag)


@pytest.mark.parametrize("motion", ["sideways", "forward", "forward_yaw"])
@pytest.mark.parametrize("eps", [1.0, 2.0, 4.0])
def test_cfg1_candidates_full_size(motion, eps):
    """6048x4032, 20000 keypoints per image (the at-scale workload)."""
    p = synth.cfg1_pair(motion)
    log(f"cfg1 {motion} eps={eps}")
    o, c, idx = run_candidates([p], eps)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, eps)
    assert_csr_equal((o, c), (ro, rc), f"{motion} eps={eps}")
    kbar = len(rc) / p.m
    assert kbar > 5
    st = idx.stats()
    log(f"  stats {st}")
    # the angular index is used for every query (no whole-pair scans) and its
    # hits are a superset of the exact set
    assert st["scanned_queries"] == 0
    assert st["candidates"] == len(rc) <= st["angle_hits"] <= st["records_scanned"]
    assert st["angle_hits"] <= 1.2 * st["candidates"] + p.m


def test_cfg1_batched_equals_per_pair():
    """All six at-scale variants in one batch give the per-pair results."""
    pairs = [synth.cfg1_pair(mo) for mo in ("sideways", "forward")]
    log("cfg1 batch")
    o, c, _ = run_candidates(pairs, 2.0)
    ro, rc, _ = oracle_batch(pairs, 2.0)
    assert_csr_equal((o, c), (ro, rc), "batched")


def test_cfg3_mixed_batch():
    """Uneven pairs with far, infinite, inside and general epipoles."""
    pairs = [synth.cfg3_pair(r, max_kp=4000) for r in range(24)]
    log("cfg3 mixed batch of 24")
    o, c, idx = run_candidates(pairs, 2.0)
    ro, rc, _ = oracle_batch(pairs, 2.0)
    assert_csr_equal((o, c), (ro, rc), "cfg3 mixed")
    st = idx.stats()
    log(f"  stats {st}")
    assert st["scanned_queries"] == 0


def test_per_keypoint_eps_and_invalid_values():
    p = synth.cfg1_pair("forward_yaw", n_kp=6000)
    rng = np.random.default_rng(3)
    eps = rng.uniform(0.25, 12.0, p.n).astype(np.float32)
    eps[:7] = [0.0, -1.0, np.nan, np.inf, 1e-3, 5000.0, -0.0]
    log("per-keypoint eps")
    o, c, _ = run_candidates([p], 0.0, eps2=eps)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, eps)
    assert_csr_equal((o, c), (ro, rc), "eps2")


def _match_parity(p, eps, ratio, binary=False, algo="plain"):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    k1 = torch.from_numpy(p.kp1).to(dev)
    k2 = torch.from_numpy(p.kp2).to(dev)
    idx = E.Index([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], k2, eps=eps)
    offs, cols = idx.query(k1)
    if binary:
        d1, d2 = torch.from_numpy(p.bin1).to(dev), torch.from_numpy(p.bin2).to(dev)
        bi, bd, sd = idx.match(offs, cols, d1, d2, dtype="bin256", ratio=ratio, algo=algo)
    else:
        d1, d2 = torch.from_numpy(p.desc1).to(dev), torch.from_numpy(p.desc2).to(dev)
        bi, bd, sd = idx.match(offs, cols, d1, d2, dtype="f32", ratio=ratio, algo=algo)
    torch.cuda.synchronize()
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, eps)
    assert_csr_equal((offs.cpu().numpy(), cols.cpu().numpy()), (ro, rc), "csr")
    if binary:
        rb, rbd, rsd = oracle.match(p.bin1, p.bin2, ro, rc, ratio=ratio, binary=True)
    else:
        rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc, ratio=ratio)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy().view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), rsd.view(np.uint32))
    return rb


@pytest.mark.parametrize("algo", ["plain", "tiled"])
@pytest.mark.parametrize("ratio", [0.0, 0.8])
def test_match_f32_bit_exact(ratio, algo):
    p = synth.cfg1_pair("sideways", n_kp=8000)
    log(f"match f32 ratio={ratio} algo={algo}")
    rb = _match_parity(p, 2.0, ratio, algo=algo)
    ok = (p.gt12 >= 0) & (rb >= 0)
    assert (rb[ok] == p.gt12[ok]).mean() > 0.9


@pytest.mark.parametrize("algo", ["plain", "tiled"])
def test_match_binary_exact(algo):
    p = synth.cfg0_pair(4, binary=True)
    log(f"match binary {algo}")
    _match_parity(p, 3.0, 0.0, binary=True, algo=algo)
    _match_parity(p, 3.0, 0.8, binary=True, algo=algo)


def test_match_f32_forward_wide_rows():
    """Forward motion at eps 4: long rows and circles around the epipole."""
    p = synth.cfg1_pair("forward", n_kp=12000)
    log("match forward eps=4")
    _match_parity(p, 4.0, 0.0, algo="tiled")


def test_repeat_runs_identical():
    p = synth.cfg1_pair("forward", n_kp=8000)
    log("determinism")
    a = run_candidates([p], 2.0)
    b = run_candidates([p], 2.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_match_window_with_foreign_csr():
    """A CSR that is not the index's own (extra candidates far from the line)
    still matches exactly: entries outside the tile windows are gathered."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    p = synth.cfg1_pair("forward_yaw", n_kp=6000)
    log("foreign csr")
    k1, k2 = torch.from_numpy(p.kp1).to(dev), torch.from_numpy(p.kp2).to(dev)
    idx = E.Index([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], k2, eps=2.0)
    offs, cols = idx.query(k1)
    o, c = offs.cpu().numpy(), cols.cpu().numpy()
    rng = np.random.default_rng(11)
    rows = []
    for i in range(p.m):
        r = set(c[o[i]:o[i + 1]].tolist())
        if i % 3 == 0:
            r.add(int(rng.integers(0, p.n)))
        if i % 7 == 0:
            r = set()
        rows.append(sorted(r))
    no = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    nc = np.array([j for r in rows for j in r], np.int32)
    d1, d2 = torch.from_numpy(p.desc1).to(dev), torch.from_numpy(p.desc2).to(dev)
    bi, bd, sd = idx.match(torch.from_numpy(no).to(dev), torch.from_numpy(nc).to(dev), d1, d2,
                           dtype="f32", algo="auto")
    torch.cuda.synchronize()
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, no, nc)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy().view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), rsd.view(np.uint32))
