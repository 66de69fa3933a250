"""Reduced-precision matching (BF16 / FP8-E4M3 on MFMA with FP32 re-rank)
and binary matching at the 60000-keypoint precision workload: final matches
must equal the FP32 oracle's bit for bit, Hamming exactly."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cfg2():
    p = synth.cfg2_pair(0)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 2.0)
    return p, ro, rc


def _index(p, eps=2.0):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    idx = E.Index([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], torch.from_numpy(p.kp2).to(dev), eps=eps)
    offs, cols = idx.query(torch.from_numpy(p.kp1).to(dev))
    return idx, offs, cols, dev


@pytest.mark.parametrize("measured", [False, True])
@pytest.mark.parametrize("ratio", [0.0, 0.8])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_reduced_precision_matches_equal_fp32(cfg2, fmt, ratio, measured):
    torch = torch_gpu()
    p, ro, rc = cfg2
    log(f"precision {fmt} ratio={ratio}")
    idx, offs, cols, dev = _index(p)
    assert_csr_equal((offs.cpu().numpy(), cols.cpu().numpy()), (ro, rc), "cfg2 csr")
    m1 = torch.from_numpy(p.desc1).to(dev)
    m2 = torch.from_numpy(p.desc2).to(dev)
    if fmt == "bf16":
        q1 = torch.from_numpy(synth.f32_to_bf16(p.desc1).view(np.int16)).to(dev)
        q2 = torch.from_numpy(synth.f32_to_bf16(p.desc2).view(np.int16)).to(dev)
        s1 = s2 = None
    else:
        c1, sc1 = synth.f32_to_fp8_e4m3(p.desc1)
        c2, sc2 = synth.f32_to_fp8_e4m3(p.desc2)
        q1, q2 = torch.from_numpy(c1).to(dev), torch.from_numpy(c2).to(dev)
        s1, s2 = torch.from_numpy(sc1).to(dev), torch.from_numpy(sc2).to(dev)
    e1 = e2 = None
    if measured:  # bounds from the rows' measured rounding errors
        import paper_2603_18401_amd as E
        e1 = E.rounding_error(m1, q1, fmt, scale=s1)
        e2 = E.rounding_error(m2, q2, fmt, scale=s2)
    bi, bd, sd = idx.match(offs, cols, q1, q2, dtype=fmt, scale1=s1, scale2=s2, desc1_f32=m1,
                           desc2_f32=m2, ratio=ratio, qerr1=e1, qerr2=e2)
    torch.cuda.synchronize()
    st = idx.match_stats()
    log(f"  match stats {st} (measured errors: {measured})")
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc, ratio=ratio)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy().view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), rsd.view(np.uint32))
    assert st["reranked_rows"] + st["long_rows"] > 0.9 * p.m
    # the bounds leave a fraction of the candidates to evaluate exactly
    # (k = 61 on average): BF16 about 3 per row, FP8 with its measured
    # errors under a third
    if fmt == "bf16":
        assert st["exact_distances"] < 0.1 * len(rc)
    elif measured:
        assert st["exact_distances"] < 0.35 * len(rc)


def test_binary_hamming_full_size(cfg2):
    torch = torch_gpu()
    p, ro, rc = cfg2
    log("binary 60k")
    idx, offs, cols, dev = _index(p)
    bi, bd, sd = idx.match(offs, cols, torch.from_numpy(p.bin1).to(dev),
                           torch.from_numpy(p.bin2).to(dev), dtype="bin256")
    torch.cuda.synchronize()
    rb, rbd, rsd = oracle.match(p.bin1, p.bin2, ro, rc, binary=True)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy(), rbd) and np.array_equal(sd.cpu().numpy(), rsd)


def test_reduced_precision_without_query_uses_masters():
    """No angle tiles (CSR not produced by this index's query): exact FP32 on
    the masters, same results."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(5)
    dev = torch.device("cuda:0")
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 2.0)
    idx = E.Index([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], torch.from_numpy(p.kp2).to(dev), eps=2.0)
    m1, m2 = torch.from_numpy(p.desc1).to(dev), torch.from_numpy(p.desc2).to(dev)
    q1 = torch.from_numpy(synth.f32_to_bf16(p.desc1).view(np.int16)).to(dev)
    q2 = torch.from_numpy(synth.f32_to_bf16(p.desc2).view(np.int16)).to(dev)
    bi, bd, sd = idx.match(torch.from_numpy(ro).to(dev), torch.from_numpy(rc).to(dev), q1, q2,
                           dtype="bf16", desc1_f32=m1, desc2_f32=m2)
    torch.cuda.synchronize()
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy().view(np.uint32), rbd.view(np.uint32))


def test_descriptor_distance_error_against_fp64(cfg2):
    """The distances the matching kernels compute (epm_descriptor_distances)
    against the FP64 squared distance of the FP32 masters, on candidate
    pairs of the 60000-keypoint pair: the canonical FP32 chain equals the
    oracle's bit for bit and lies within 130 * 2^-24 (relative) of FP64; the
    BF16 and FP8 MFMA approximations lie within their certified envelopes
    (rounding bound of each format per row, FP32 accumulation bound)."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p, ro, rc = cfg2
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31)
    rows = np.repeat(np.arange(p.m), np.diff(ro))
    pick = rng.choice(len(rc), 20000, replace=False)
    qi, kj = rows[pick].astype(np.int64), rc[pick].astype(np.int64)
    d64 = oracle.desc_dist_f64(p.desc1, p.desc2, qi, kj)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    tq, tk = g(qi), g(kj)
    f32 = E.descriptor_distances(g(p.desc1), g(p.desc2), tq, tk, dtype="f32").cpu().numpy()
    b1, b2 = synth.f32_to_bf16(p.desc1), synth.f32_to_bf16(p.desc2)
    bf = E.descriptor_distances(g(b1.view(np.int16)), g(b2.view(np.int16)), tq, tk,
                                dtype="bf16").cpu().numpy()
    c1, s1 = synth.f32_to_fp8_e4m3(p.desc1)
    c2, s2 = synth.f32_to_fp8_e4m3(p.desc2)
    f8 = E.descriptor_distances(g(c1), g(c2), tq, tk, dtype="fp8", scale1=g(s1),
                                scale2=g(s2)).cpu().numpy()
    ref32 = np.array([oracle.desc_dist_f32(p.desc1[i], p.desc2[j]) for i, j in zip(qi, kj)],
                     np.float32)
    assert np.array_equal(f32.view(np.uint32), ref32.view(np.uint32))
    rel = lambda a: np.abs(a.astype(np.float64) - d64) / d64  # noqa: E731
    log(f"  rel. error vs FP64 (max / median): f32 {rel(f32).max():.2e} / "
        f"{np.median(rel(f32)):.2e}, bf16 {rel(bf).max():.2e} / {np.median(rel(bf)):.2e}, "
        f"fp8 {rel(f8).max():.2e} / {np.median(rel(f8)):.2e}")
    assert rel(f32).max() <= 130 * 2.0 ** -24
    # envelopes: |approx - exact| <= 2 sqrt(exact) (dq + dw) + (dq + dw)^2 + em
    # (FP8 adds half its subnormal spacing, 2^-10 scale, per element)
    one = np.ones(p.m, np.float32), np.ones(p.n, np.float32)
    for name, approx, u, a, deq1, deq2, sc1, sc2 in (
            ("bf16", bf, 2.0 ** -8, 0.0, synth.bf16_to_f32(b1), synth.bf16_to_f32(b2), *one),
            ("fp8", f8, 2.0 ** -4, 2.0 ** -10, synth.fp8_e4m3_to_f32(c1) * s1[:, None],
             synth.fp8_e4m3_to_f32(c2) * s2[:, None], s1, s2)):
        nq = np.linalg.norm(deq1[qi].astype(np.float64), axis=1)
        nw = np.linalg.norm(deq2[kj].astype(np.float64), axis=1)
        dq = (u * nq + a * sc1[qi] * np.sqrt(128)) / (1 - u)
        dw = (u * nw + a * sc2[kj] * np.sqrt(128)) / (1 - u)
        em = 3e-5 * (nq + nw) ** 2
        env = 2 * np.sqrt(d64) * (dq + dw) + (dq + dw) ** 2 + em
        assert (np.abs(approx.astype(np.float64) - d64) <= env).all(), name


@pytest.mark.parametrize("ratio", [0.0, 0.8])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_fused_reduced_precision_full_size(cfg2, fmt, ratio):
    """The BF16 and FP8 selections fused into the stabbing pass at the
    60000-keypoint pair: CSR and matches equal the oracle's, and at least
    90 % of the rows are certified by their bounds (FP8 with the rows'
    measured rounding errors, computed here in NumPy)."""
    import paper_2603_18401_amd as E
    from tests.gpu_util import fp8_rows
    torch = torch_gpu()
    p, ro, rc = cfg2
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    idx = E.Index([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], g(p.kp2), eps=2.0)
    m1, m2 = g(p.desc1), g(p.desc2)
    log(f"fused {fmt} at 60000 keypoints, ratio={ratio}")
    if fmt == "bf16":
        res = idx.query_match_bf16(g(p.kp1), g(synth.f32_to_bf16(p.desc1).view(np.int16)),
                                   g(synth.f32_to_bf16(p.desc2).view(np.int16)), m1, m2,
                                   ratio=ratio)
    else:
        c2, s2, e2 = fp8_rows(p.desc2)
        res = idx.query_match_fp8(g(p.kp1), g(c2), g(s2), g(e2), m1, m2, ratio=ratio)
    torch.cuda.synchronize()
    offs, cols, bi, bd, sd = [x.cpu().numpy() for x in res]
    st = idx.match_stats()
    log(f"  match stats {st}")
    assert_csr_equal((offs, cols), (ro, rc), f"{fmt} csr")
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc, ratio=ratio)
    assert np.array_equal(bi, rb)
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32))
    assert st["reranked_rows"] > 0.9 * p.m
    assert st["fallback_rows"] < 0.1 * st["reranked_rows"]
    assert st["exact_distances"] < (0.1 if fmt == "bf16" else 0.2) * len(rc)
