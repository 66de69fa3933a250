"""epm_query_match_fp8: the candidate CSR and the matches of the FP32
masters, selected through MFMA bounds over FP8 (E4M3FN) image-2 rows fused
into the stabbing pass, must equal the oracle (brute-force candidates of
Eq. 3-4, canonical FP32 selection of Sec. 4.3 on the masters) element for
element, on every path a row can take: certified by its bounds, left
uncertified (exact listed match), rows wider than the on-chip lists (the
wide-row pass), brute-force queries of an off-rank F.  The per-row rounding
errors the bounds take are computed here in FP64 from the masters and the
codes (NumPy), not by the library."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, fp8_rows, oracle_batch, specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _fused_fp8(pairs, eps, ratio=0.0, desc=None, err_scale=1.0):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    b = synth.batch_pairs(pairs)
    d1, d2 = (b.desc1, b.desc2) if desc is None else desc
    codes, scale, err = fp8_rows(d2)
    idx = E.Index(specs_of(pairs), _dev(torch, b.kp2), eps=eps)
    o, c, bi, bd, sd = idx.query_match_fp8(_dev(torch, b.kp1), _dev(torch, codes),
                                           _dev(torch, scale),
                                           _dev(torch, (err * err_scale).astype(np.float32)),
                                           _dev(torch, d1), _dev(torch, d2), ratio=ratio)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (o, c, bi, bd, sd)], idx


def _oracle(pairs, eps, ratio=0.0, desc=None):
    b = synth.batch_pairs(pairs)
    d1, d2 = (b.desc1, b.desc2) if desc is None else desc
    ro, rc, _ = oracle_batch(pairs, eps)
    rows = np.repeat(np.arange(len(pairs)), [p.m for p in pairs])
    rb, rbd, rsd = oracle.match(d1, d2, ro, rc, ratio=ratio, col_base=b.k_begin[rows])
    return ro, rc, rb, rbd, rsd


def _same(got, ref, what):
    o, c, bi, bd, sd = got
    ro, rc, rb, rbd, rsd = ref
    assert_csr_equal((o, c), (ro, rc), what)
    assert np.array_equal(bi, rb), what
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32)), what
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32)), what


@pytest.mark.parametrize("ratio", [0.0, 0.8])
def test_cfg0_fp8_fused_equals_oracle(ratio):
    for r in range(3):
        p = synth.cfg0_pair(r)
        log(f"fp8 fused cfg0 r={r} ratio={ratio}")
        got, _ = _fused_fp8([p], 2.0, ratio)
        _same(got, _oracle([p], 2.0, ratio), f"cfg0 {r}")


@pytest.mark.parametrize("motion", ["sideways", "forward", "forward_yaw"])
@pytest.mark.parametrize("eps", [1.0, 4.0])
def test_cfg1_fp8_fused_equals_oracle(motion, eps):
    p = synth.cfg1_pair(motion)
    log(f"fp8 fused cfg1 {motion} eps={eps}")
    got, idx = _fused_fp8([p], eps)
    _same(got, _oracle([p], eps), f"{motion} {eps}")
    ms = idx.match_stats()
    kbar = got[0][-1] / p.m
    log(f"  match stats {ms}, kbar {kbar:.2f}")
    # most rows are certified by their bounds, with fewer exact distances
    # than candidates
    assert ms["reranked_rows"] > 0.9 * p.m
    assert ms["fallback_rows"] < 0.25 * ms["reranked_rows"]
    assert ms["exact_distances"] < kbar * p.m


def test_looser_error_bounds_still_exact():
    """Error bounds four times the measured ones: wider bounds, more exact
    distances or uncertified rows, the same matches."""
    p = synth.cfg1_pair("sideways")
    log("fp8 fused with error bounds x4")
    got, idx = _fused_fp8([p], 2.0, err_scale=4.0)
    _same(got, _oracle([p], 2.0), "err x4")


def test_uncertified_rows_take_the_exact_path():
    """Descriptors with many exact duplicates: the bounds of equal candidates
    coincide and cannot separate them, so rows are left to the exact listed
    match; ties go to the lowest j as in the oracle."""
    p = synth.cfg0_pair(5)
    rng = np.random.default_rng(3)
    base = synth.pairs._unit_rows(rng.standard_normal((4, 128)))
    d1 = base[rng.integers(0, 4, p.m)]
    d2 = base[rng.integers(0, 4, p.n)]
    log("fp8 fused with duplicated descriptors, eps 20")
    got, idx = _fused_fp8([p], 20.0, desc=(d1, d2))
    _same(got, _oracle([p], 20.0, desc=(d1, d2)), "duplicates")
    assert idx.match_stats()["fallback_rows"] > 0


def test_zero_and_tiny_rows():
    """All-zero image-2 rows (scale 1, every code 0) and rows with values in
    E4M3's subnormal range."""
    p = synth.cfg0_pair(2)
    rng = np.random.default_rng(17)
    d2 = p.desc2.copy()
    d2[rng.choice(p.n, p.n // 20, replace=False)] = 0.0
    tiny = rng.choice(p.n, p.n // 20, replace=False)
    d2[tiny[:, None], rng.integers(0, 128, (len(tiny), 64))] *= 1e-4
    log("fp8 fused with zero and tiny rows, eps 6")
    got, _ = _fused_fp8([p], 6.0, desc=(p.desc1, d2))
    _same(got, _oracle([p], 6.0, desc=(p.desc1, d2)), "zero/tiny rows")


def test_mixed_batch_and_wide_rows():
    """A cfg3-mix batch plus a pair whose rows exceed the on-chip lists
    (eps 60 px: rows of hundreds of candidates go through the wide-row pass
    on the masters)."""
    pairs = [synth.cfg3_pair(r, max_kp=4000) for r in range(12)]
    pairs.append(synth.cfg1_pair("sideways", n_kp=8000))
    log("fp8 fused: 12 cfg3 pairs + one 8000-keypoint pair, eps 2")
    got, _ = _fused_fp8(pairs, 2.0)
    _same(got, _oracle(pairs, 2.0), "mixed batch")
    wide = [synth.cfg1_pair("forward", n_kp=6000)]
    log("fp8 fused: wide rows, eps 60")
    got, idx = _fused_fp8(wide, 60.0)
    _same(got, _oracle(wide, 60.0), "wide rows")
    assert int(np.diff(got[0]).max()) > 128


def test_off_rank_F_brute_force_queries():
    p = synth.cfg0_pair(1)
    p.F = p.F + 1e-3 * np.abs(p.F).max() * np.random.default_rng(11).standard_normal((3, 3))
    log("fp8 fused: full-rank F (brute-force queries)")
    got, idx = _fused_fp8([p], 3.0)
    _same(got, _oracle([p], 3.0), "off-rank F")
    assert idx.stats()["scanned_queries"] > 0


def test_fp8_entry_rejects_missing_error_bounds():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(0)
    codes, scale, err = fp8_rows(p.desc2)
    idx = E.Index(specs_of([p]), _dev(torch, p.kp2), eps=2.0)
    with pytest.raises(ValueError):
        idx.query_match_fp8(_dev(torch, p.kp1), _dev(torch, codes), _dev(torch, scale),
                            _dev(torch, err[:-1]), _dev(torch, p.desc1), _dev(torch, p.desc2))


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_graph_fp8_fused(persistent):
    """The fused FP8 pass recorded in a batch graph (epm_batch_desc.err2),
    replayed three times: every replay equals the oracle."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    pairs = [synth.cfg3_pair(r, max_kp=3000) for r in range(16)]
    b = synth.batch_pairs(pairs)
    ref = _oracle(pairs, 2.0)
    codes, scale, err = fp8_rows(b.desc2)
    sched = E.Sched(64, 64, 1) if persistent else E.Sched()
    log(f"fp8 fused graph, persistent={persistent}")
    bt = E.Batch(specs_of(pairs), _dev(torch, b.kp1), _dev(torch, b.kp2), None,
                 _dev(torch, codes), len(ref[1]) + 16, eps=2.0, dtype="fp8",
                 scale2=_dev(torch, scale), desc1_f32=_dev(torch, b.desc1),
                 desc2_f32=_dev(torch, b.desc2), err2=_dev(torch, err), sched=sched)
    for rep in range(3):
        bt.launch()
        got = [x.cpu().numpy() for x in bt.outputs()]
        _same(got, ref, f"replay {rep}")
    ms = bt.match_stats()
    log(f"  match stats {ms}")
    assert ms["reranked_rows"] > 0.9 * len(ref[2])
    bt.close()
