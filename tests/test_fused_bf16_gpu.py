"""epm_query_match_bf16: the candidate CSR and the matches of the FP32
masters, selected through BF16 MFMA bounds fused into the stabbing pass, must
equal the oracle (brute-force candidates of Eq. 3-4, canonical FP32 selection
of Sec. 4.3 on the masters) element for element, on every path a row can
take: certified by its bounds, left uncertified (exact listed match), rows
wider than the on-chip lists (the wide-row pass), brute-force queries of an
off-rank F, and the graph replay of a batch."""

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


def _codes(d):
    return synth.f32_to_bf16(d).view(np.int16)


def _fused_bf16(pairs, eps, ratio=0.0, desc=None):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    b = synth.batch_pairs(pairs)
    d1, d2 = (b.desc1, b.desc2) if desc is None else desc
    idx = E.Index(specs_of(pairs), _dev(torch, b.kp2), eps=eps)
    o, c, bi, bd, sd = idx.query_match_bf16(_dev(torch, b.kp1), _dev(torch, _codes(d1)),
                                            _dev(torch, _codes(d2)), _dev(torch, d1),
                                            _dev(torch, d2), ratio=ratio)
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
def test_cfg0_bf16_fused_equals_oracle(ratio):
    for r in range(3):
        p = synth.cfg0_pair(r)
        log(f"bf16 fused cfg0 r={r} ratio={ratio}")
        got, _ = _fused_bf16([p], 2.0, ratio)
        _same(got, _oracle([p], 2.0, ratio), f"cfg0 {r}")


@pytest.mark.parametrize("motion", ["sideways", "forward", "forward_yaw"])
@pytest.mark.parametrize("eps", [1.0, 4.0])
def test_cfg1_bf16_fused_equals_oracle(motion, eps):
    p = synth.cfg1_pair(motion)
    log(f"bf16 fused cfg1 {motion} eps={eps}")
    got, idx = _fused_bf16([p], eps)
    _same(got, _oracle([p], eps), f"{motion} {eps}")
    ms = idx.match_stats()
    log(f"  match stats {ms}")
    # nearly every row is certified by its bounds, with few exact distances
    assert ms["reranked_rows"] > 0.9 * p.m
    assert ms["fallback_rows"] < 0.05 * ms["reranked_rows"]
    kbar = got[0][-1] / p.m
    assert ms["exact_distances"] < 0.5 * kbar * p.m


def test_uncertified_rows_take_the_exact_path():
    """Descriptors with many exact duplicates: the bounds of equal candidates
    coincide and cannot separate them, so rows are left to the exact listed
    match; ties go to the lowest j as in the oracle."""
    p = synth.cfg0_pair(5)
    rng = np.random.default_rng(3)
    base = synth.pairs._unit_rows(rng.standard_normal((4, 128)))
    d1 = base[rng.integers(0, 4, p.m)]
    d2 = base[rng.integers(0, 4, p.n)]
    log("bf16 fused with duplicated descriptors, eps 20")
    got, idx = _fused_bf16([p], 20.0, desc=(d1, d2))
    _same(got, _oracle([p], 20.0, desc=(d1, d2)), "duplicates")
    assert idx.match_stats()["fallback_rows"] > 0


def test_mixed_batch_and_wide_rows():
    """A cfg3-mix batch plus a pair whose rows exceed the on-chip lists
    (eps 60 px: rows of hundreds of candidates go through the wide-row pass
    on the masters)."""
    pairs = [synth.cfg3_pair(r, max_kp=4000) for r in range(12)]
    pairs.append(synth.cfg1_pair("sideways", n_kp=8000))
    log("bf16 fused: 12 cfg3 pairs + one 8000-keypoint pair, eps 2")
    got, _ = _fused_bf16(pairs, 2.0)
    _same(got, _oracle(pairs, 2.0), "mixed batch")
    wide = [synth.cfg1_pair("forward", n_kp=6000)]
    log("bf16 fused: wide rows, eps 60")
    got, idx = _fused_bf16(wide, 60.0)
    _same(got, _oracle(wide, 60.0), "wide rows")
    assert int(np.diff(got[0]).max()) > 128


def test_off_rank_F_brute_force_queries():
    p = synth.cfg0_pair(1)
    p.F = p.F + 1e-3 * np.abs(p.F).max() * np.random.default_rng(11).standard_normal((3, 3))
    log("bf16 fused: full-rank F (brute-force queries)")
    got, idx = _fused_bf16([p], 3.0)
    _same(got, _oracle([p], 3.0), "off-rank F")
    assert idx.stats()["scanned_queries"] > 0


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_graph_bf16_fused(persistent):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    pairs = [synth.cfg3_pair(r, max_kp=3000) for r in range(16)]
    b = synth.batch_pairs(pairs)
    ref = _oracle(pairs, 2.0)
    sched = E.Sched(64, 64, 1) if persistent else E.Sched()
    log(f"bf16 fused graph, persistent={persistent}")
    bt = E.Batch(specs_of(pairs), _dev(torch, b.kp1), _dev(torch, b.kp2),
                 _dev(torch, _codes(b.desc1)), _dev(torch, _codes(b.desc2)),
                 len(ref[1]) + 16, eps=2.0, dtype="bf16", desc1_f32=_dev(torch, b.desc1),
                 desc2_f32=_dev(torch, b.desc2), sched=sched)
    for rep in range(3):
        bt.launch()
        got = [x.cpu().numpy() for x in bt.outputs()]
        _same(got, ref, f"replay {rep}")
    assert bt.match_stats()["reranked_rows"] > 0
    bt.close()
