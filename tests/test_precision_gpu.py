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


@pytest.mark.parametrize("ratio", [0.0, 0.8])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_reduced_precision_matches_equal_fp32(cfg2, fmt, ratio):
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
    bi, bd, sd = idx.match(offs, cols, q1, q2, dtype=fmt, scale1=s1, scale2=s2, desc1_f32=m1,
                           desc2_f32=m2, ratio=ratio)
    torch.cuda.synchronize()
    st = idx.match_stats()
    log(f"  match stats {st}")
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc, ratio=ratio)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy().view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), rsd.view(np.uint32))
    assert st["reranked_rows"] + st["long_rows"] > 0.9 * p.m
    if fmt == "bf16":
        assert st["fallback_rows"] < 0.5 * st["reranked_rows"]


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
