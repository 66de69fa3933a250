"""Batch graphs whose pair setup runs on the device (epm_batch_desc.F_dev):
every replay recomputes the epipole and pencil basis (Algorithm 1,
preprocessing) from F in device memory, so new F written between replays are
matched exactly -- against the oracle's brute-force candidates (Eq. 3-4) and
canonical FP32 matches (Sec. 4.3) for each F -- including F without a pencil
(zero, rank 1, non-finite), whose pairs are scanned exhaustively."""

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


def _oracle(pairs, Fs, b, eps):
    offs = [np.zeros(1, np.int64)]
    cols = []
    base = 0
    for p, F, qb, kb in zip(pairs, Fs, b.q_begin, b.k_begin):
        o, c, _ = oracle.candidates(F, p.kp1, p.kp2, eps)
        offs.append(o[1:] + base)
        base += int(o[-1])
        cols.append(c)
    ro = np.concatenate(offs)
    rc = np.concatenate(cols)
    col_base = np.repeat(b.k_begin, [p.m for p in pairs])
    rb, rbd, rsd = oracle.match(b.desc1, b.desc2, ro, rc, col_base=col_base)
    return ro, rc, rb, rbd, rsd


def _same(bt, ref, what):
    o, c, bi, bd, sd = [x.cpu().numpy() for x in bt.outputs()]
    ro, rc, rb, rbd, rsd = ref
    assert_csr_equal((o, c), (ro, rc), what)
    assert np.array_equal(bi, rb), what
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32)), what
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32)), what


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_new_F_between_replays(dtype):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    dev = torch.device("cuda:0")
    pairs = [synth.cfg3_pair(r, max_kp=3000) for r in range(12)]
    b = synth.batch_pairs(pairs)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    F0 = np.stack([p.F.reshape(9) for p in pairs])
    Fd = g(F0)
    if dtype == "f32":
        d1, d2, m1, m2 = g(b.desc1), g(b.desc2), None, None
    else:
        d1 = g(synth.f32_to_bf16(b.desc1).view(np.int16))
        d2 = g(synth.f32_to_bf16(b.desc2).view(np.int16))
        m1, m2 = g(b.desc1), g(b.desc2)
    # F of the same scenes seen from perturbed poses (level 2: rotations up
    # to 2 degrees, translations up to 0.5 m), and F without a pencil
    F1 = np.stack([synth.perturbed_F(p, 2, 7000 + i).reshape(9) for i, p in enumerate(pairs)])
    F2 = F1.copy()
    F2[0] = 0.0                                         # zero: empty rows
    u = np.array([1.0, 2.0, -1.0])
    F2[1] = np.outer(u, [0.001, -0.002, 1.0]).reshape(9)  # rank 1: scanned
    F2[2, 4] = np.nan                                   # non-finite: no candidates
    refs = [_oracle(pairs, [f.reshape(3, 3) for f in F], b, 4.0) for F in (F0, F1, F2)]
    cap = max(len(r[1]) for r in refs) + 64
    bt = E.Batch(specs_of(pairs), g(b.kp1), g(b.kp2), d1, d2, cap, eps=4.0, dtype=dtype,
                 desc1_f32=m1, desc2_f32=m2, F_dev=Fd)
    for k, (F, ref) in enumerate(zip((F0, F1, F2, F0), refs + [refs[0]])):
        log(f"device pair setup, {dtype}, F set {k}")
        Fd.copy_(g(F))
        bt.launch()
        _same(bt, ref, f"{dtype} F set {k}")
        if k == 2:
            assert bt.stats()["scanned_queries"] >= pairs[1].m
    bt.close()
