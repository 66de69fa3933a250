"""Batched execution: the whole build / query / match pipeline of a batch of
uneven pairs recorded as one HIP graph and replayed, and the persistent and
longest-first tile schedules.  Every replay and every schedule must give the
oracle's candidate sets and matches bit for bit."""

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, oracle_batch, specs_of, torch_gpu

pytestmark = pytest.mark.gpu

# (stabbing workgroups, matching workgroups, longest first, records per round)
SCHEDS = [(0, 0, 0, 0), (0, 0, 0, 256), (0, 0, 0, 1024), (768, 512, 0, 0), (768, 512, 1, 1024),
          (256, 256, 1, 256), (7, 5, 1, 0)]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class _Case:
    """A mixed batch (far, infinite, forward and general epipoles; 500-3000
    keypoints per image) on the device, with its oracle results."""

    def __init__(self, torch, npairs=16, max_kp=3000, seed0=0):
        self.pairs = [synth.cfg3_pair(r, max_kp=max_kp) for r in range(seed0, seed0 + npairs)]
        b = synth.batch_pairs(self.pairs)
        dev = torch.device("cuda:0")
        g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        self.b = b
        self.kp1, self.kp2 = g(b.kp1), g(b.kp2)
        self.m1, self.m2 = g(b.desc1), g(b.desc2)
        self.q1 = g(synth.f32_to_bf16(b.desc1).view(np.int16))
        self.q2 = g(synth.f32_to_bf16(b.desc2).view(np.int16))
        self.specs = specs_of(self.pairs)
        self.reference(b.kp1)

    def reference(self, kp1):
        ro, rc, _ = oracle_batch(self.pairs, 2.0, kp1=kp1)
        rows = np.repeat(np.arange(len(self.pairs)), [p.m for p in self.pairs])
        col_base = self.b.k_begin[rows]
        rb, rbd, rsd = oracle.match(self.b.desc1, self.b.desc2, ro, rc, col_base=col_base)
        self.ref = (ro, rc, rb, rbd, rsd)
        return self.ref


def _check(outs, ref, what):
    offs, cols, bi, bd, sd = [x.cpu().numpy() for x in outs]
    ro, rc, rb, rbd, rsd = ref
    assert_csr_equal((offs, cols), (ro, rc), what)
    assert np.array_equal(bi, rb), what
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32)), what
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32)), what


@pytest.fixture(scope="module")
def case():
    return _Case(torch_gpu())


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("sched", SCHEDS)
def test_graph_replays_equal_oracle(case, dtype, sched):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    log(f"batch graph {dtype} sched {sched}: {len(case.pairs)} pairs")
    nnz = int(case.ref[0][-1])
    d1, d2 = (case.m1, case.m2) if dtype == "f32" else (case.q1, case.q2)
    b = E.Batch(case.specs, case.kp1, case.kp2, d1, d2, nnz + 100, eps=2.0, dtype=dtype,
                desc1_f32=case.m1, desc2_f32=case.m2, sched=E.Sched(*sched))
    for rep in range(3):
        b.launch()
        _check(b.outputs(), case.ref, f"replay {rep}")
        # eager work on the same device between replays
        idx = E.Index(case.specs[:2], case.kp2[: case.pairs[0].n + case.pairs[1].n], eps=4.0)
        idx.query(case.kp1[: case.pairs[0].m + case.pairs[1].m])
        torch.cuda.synchronize()
    st = b.stats()
    assert st["candidates"] == nnz and st["scanned_queries"] >= 0
    if dtype == "bf16":
        ms = b.match_stats()
        assert ms["reranked_rows"] + ms["long_rows"] > 0
    b.close()


def test_graph_replay_reads_new_inputs(case):
    """New keypoints written into the same buffers between replays."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    log("batch graph with new query keypoints")
    nnz0 = int(case.ref[0][-1])
    b = E.Batch(case.specs, case.kp1, case.kp2, case.m1, case.m2, 4 * nnz0 + 1000, eps=2.0,
                sched=E.Sched(768, 512, 1))
    b.launch()
    _check(b.outputs(), case.ref, "first inputs")
    rng = np.random.default_rng(7)
    kp1_new = (case.b.kp1 + rng.normal(0, 3.0, case.b.kp1.shape)).astype(np.float32)
    saved = case.kp1.clone()
    case.kp1.copy_(torch.from_numpy(kp1_new).to(case.kp1.device))
    try:
        b.launch()
        ref_new = case.reference(kp1_new)
        _check(b.outputs(), ref_new, "new inputs")
    finally:
        case.kp1.copy_(saved)
        case.reference(case.b.kp1)
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_graph_capacity_overflow_is_reported(case, dtype):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    log(f"batch graph {dtype} with a too-small CSR buffer")
    nnz = int(case.ref[0][-1])
    d1, d2 = (case.m1, case.m2) if dtype == "f32" else (case.q1, case.q2)
    b = E.Batch(case.specs, case.kp1, case.kp2, d1, d2, nnz // 2, eps=2.0, dtype=dtype,
                desc1_f32=case.m1, desc2_f32=case.m2)
    b.best_idx.fill_(-7)
    b.launch()
    with pytest.raises(E.EpmError) as ei:
        b.nnz()
    assert ei.value.status == 3
    torch.cuda.synchronize()
    assert np.array_equal(b.row_offsets.cpu().numpy(), case.ref[0])
    # the columns that fit are the leading ones of the full CSR; both dtypes
    # match in the fused pass, whose outputs are then incomplete (reported)
    assert np.array_equal(b.col_indices.cpu().numpy(), case.ref[1][: nnz // 2])
    b.close()


@pytest.mark.parametrize("sched", SCHEDS[1:])
def test_eager_index_schedules(sched):
    """The same schedules through the eager calls, full-size single pair."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg1_pair("forward")
    log(f"eager schedule {sched}: cfg1 forward")
    dev = torch.device("cuda:0")
    k1, k2 = torch.from_numpy(p.kp1).to(dev), torch.from_numpy(p.kp2).to(dev)
    d1, d2 = torch.from_numpy(p.desc1).to(dev), torch.from_numpy(p.desc2).to(dev)
    idx = E.Index(specs_of([p]), k2, eps=2.0)
    idx.set_sched(E.Sched(*sched))
    offs, cols = idx.query(k1)
    bi, bd, sd = idx.match(offs, cols, d1, d2, algo="tiled")
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 2.0)
    assert_csr_equal((offs.cpu().numpy(), cols.cpu().numpy()), (ro, rc), "csr")
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc)
    assert np.array_equal(bi.cpu().numpy(), rb)
    assert np.array_equal(bd.cpu().numpy().view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), rsd.view(np.uint32))


def test_match_skips_truncated_csr():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(0)
    log("eager match with check_capacity on a truncated CSR")
    dev = torch.device("cuda:0")
    k1, k2 = torch.from_numpy(p.kp1).to(dev), torch.from_numpy(p.kp2).to(dev)
    d1, d2 = torch.from_numpy(p.desc1).to(dev), torch.from_numpy(p.desc2).to(dev)
    idx = E.Index(specs_of([p]), k2, eps=2.0)
    offs = torch.empty(p.m + 1, dtype=torch.int64, device=dev)
    cols = torch.empty(100, dtype=torch.int32, device=dev)
    idx.query(k1, row_offsets=offs, col_indices=cols, sync=False)
    out = tuple(torch.full((p.m,), v, dtype=t, device=dev)
                for v, t in ((-7, torch.int32), (-1.0, torch.float32), (-1.0, torch.float32)))
    idx.match(offs, cols, d1, d2, out=out, check_capacity=True)
    torch.cuda.synchronize()
    assert int(offs[-1].item()) > 100
    assert bool((out[0] == -7).all()) and bool((out[1] == -1.0).all())


def test_autotune_picks_and_caches(case, tmp_path):
    import paper_2603_18401_amd as E
    from paper_2603_18401_amd import autotune
    torch = torch_gpu()
    log("autotune on the mixed batch")
    nnz = int(case.ref[0][-1])
    cache = str(tmp_path / "tune.json")
    cand = [E.Sched(0, 0, 0), E.Sched(256, 256, 0, 1024), E.Sched(768, 512, 1, 256)]
    best, info = autotune.tune(case.specs, case.kp1, case.kp2, case.q1, case.q2, nnz + 10,
                               dtype="bf16", eps=2.0, desc1_f32=case.m1, desc2_f32=case.m2,
                               cache=cache, sched_list=cand, steps=2, warmup=1, log=log)
    assert not info["cached"] and len(info["candidates"]) == 3
    assert best.as_dict() in [c.as_dict() for c in cand]
    again, info2 = autotune.tune(case.specs, case.kp1, case.kp2, case.q1, case.q2, nnz + 10,
                                 dtype="bf16", eps=2.0, desc1_f32=case.m1, desc2_f32=case.m2,
                                 cache=cache, sched_list=cand)
    assert info2["cached"] and again.as_dict() == best.as_dict()
    b = E.Batch(case.specs, case.kp1, case.kp2, case.q1, case.q2, nnz + 10, eps=2.0,
                dtype="bf16", desc1_f32=case.m1, desc2_f32=case.m2, sched=best)
    b.launch()
    _check(b.outputs(), case.ref, "tuned")
    torch.cuda.synchronize()


def test_bad_tile_shape_is_refused():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(0)
    idx = E.Index(specs_of([p]), torch.from_numpy(p.kp2).to(torch.device("cuda:0")), eps=2.0)
    for bad in (E.Sched(0, 0, 0, 300), E.Sched(0, 0, 2, 0), E.Sched(-1, 0, 0, 0)):
        with pytest.raises(RuntimeError):
            idx.set_sched(bad)
    idx.set_sched(E.Sched(0, 0, 0, 1024))
    idx.close()
