"""The batching workload at its full size, against the oracle: 512 pairs of
1920x1080 / 4032x3024 / 6048x4032 images with 500-30000 keypoints per image
(near-pure sideways motion with the epipole 1e6-1e9 px away plus one exactly
infinite epipole, forward motion, general motion), BF16 descriptors with FP32
masters, eps = 2 px.  The recorded graph (persistent longest-first schedule)
and the eager calls (one workgroup per tile) must both return the oracle's
CSR (Eq. 3-4, brute force in FP64) and the oracle's FP32 matches (Sec. 4.3),
element for element; so must the fused BF16 call (epm_query_match_bf16).  The
graph uses the fused BF16 pass, the eager calls the separate query and
window-kernel match."""

import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import specs_of, torch_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

NUM_PAIRS = 512
EPS = 2.0


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 8


@pytest.fixture(scope="module")
def cfg3():
    print(f"cfg3: generating {NUM_PAIRS} pairs", flush=True)
    pairs = synth.cfg3_batch(NUM_PAIRS, workers=_threads())
    b = synth.batch_pairs(pairs)
    m = np.array([p.m for p in pairs], np.int64)
    n = np.array([p.n for p in pairs], np.int64)
    print(f"cfg3: oracle over {int(m.sum())} queries x {int(n.sum())} keypoints", flush=True)
    ro, rc, _ = oracle.candidates_batch([p.F for p in pairs], b.kp1, b.kp2, EPS, b.q_begin, m,
                                        b.k_begin, n, nthreads=_threads())
    col_base = np.repeat(b.k_begin, m)
    rb, rbd, rsd = oracle.match(b.desc1, b.desc2, ro, rc, col_base=col_base,
                                nthreads=_threads())
    print(f"cfg3: oracle done, {len(rc)} candidates", flush=True)
    return pairs, b, (ro, rc, rb, rbd, rsd)


def _assert_same(got, ref, what):
    names = ("row_offsets", "col_indices", "best_idx", "best_dist", "second_dist")
    for name, g, r in zip(names, got, ref):
        assert g.shape == r.shape, (what, name, g.shape, r.shape)
        if r.dtype == np.float32:
            g, r = g.view(np.uint32), r.view(np.uint32)
        if not np.array_equal(g, r):
            bad = np.nonzero(g != r)[0]
            raise AssertionError(f"{what}: {name} differs at {bad[:8]} ({len(bad)} entries)")


def test_cfg3_full_batch_equals_oracle(cfg3):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    pairs, b, ref = cfg3
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    kp1, kp2, m1, m2 = g(b.kp1), g(b.kp2), g(b.desc1), g(b.desc2)
    q1 = g(synth.f32_to_bf16(b.desc1).view(np.int16))
    q2 = g(synth.f32_to_bf16(b.desc2).view(np.int16))
    specs = specs_of(pairs)
    nnz = len(ref[1])
    cap = nnz + 4096

    # eager: build + query + BF16 match (one workgroup per tile)
    print("cfg3: eager calls", flush=True)
    idx = E.Index(specs, kp2, eps=EPS)
    offs, cols = idx.query(kp1, capacity=cap)
    best, bd, sd = idx.match(offs, cols, q1, q2, dtype="bf16", desc1_f32=m1, desc2_f32=m2)
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in (offs, cols, best, bd, sd)]
    idx.close()
    _assert_same(got, ref, "eager")

    # eager, BF16 selection fused into the stabbing pass
    print("cfg3: eager fused BF16 call", flush=True)
    idx = E.Index(specs, kp2, eps=EPS)
    got = idx.query_match_bf16(kp1, q1, q2, m1, m2, capacity=cap)
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in got]
    ms = idx.match_stats()
    idx.close()
    _assert_same(got, ref, "eager fused BF16")
    print(f"cfg3: fused BF16 match stats {ms}", flush=True)

    # graph: persistent longest-first schedule, replayed twice
    print("cfg3: graph replays", flush=True)
    bt = E.Batch(specs, kp1, kp2, q1, q2, cap, eps=EPS, dtype="bf16", desc1_f32=m1,
                 desc2_f32=m2, sched=E.Sched(768, 512, 1))
    for rep in range(2):
        bt.launch()
        got = [t.cpu().numpy() for t in bt.outputs()]
        _assert_same(got, ref, f"graph replay {rep}")
    bt.close()
