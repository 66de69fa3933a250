"""The allocation-free entry point (epm_query_match_noalloc, index in the
library's fixed device array) against the workspace entry points
(epm_build_intervals + epm_query_match) on the same inputs, on two calls in a
row whose second input is smaller: CSR and matches must be identical."""

import numpy as np
import pytest

import synth
from tests.gpu_util import specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _both(pairs, eps, ratio):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    b = synth.batch_pairs(pairs)
    k1, k2 = _dev(torch, b.kp1), _dev(torch, b.kp2)
    d1, d2 = _dev(torch, b.desc1), _dev(torch, b.desc2)
    specs = specs_of(pairs)
    idx = E.Index(specs, k2, eps=eps)
    ref = idx.query_match(k1, d1, d2, ratio=ratio)
    torch.cuda.synchronize()
    ref = [t.cpu().numpy() for t in ref]
    idx.close()
    got = E.query_match_noalloc(specs, k1, k2, d1, d2, eps=eps, ratio=ratio)
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in got]
    return ref, got


def _assert_same(ref, got, what):
    names = ("row_offsets", "col_indices", "best_idx", "best_dist", "second_dist")
    for name, r, g in zip(names, ref, got):
        assert r.shape == g.shape, (what, name)
        if r.dtype == np.float32:
            r, g = r.view(np.uint32), g.view(np.uint32)
        assert np.array_equal(r, g), (what, name)


def test_noalloc_matches_workspace_path_on_two_calls():
    # first call: three 6048x4032 pairs of 6000 keypoints (several tiles,
    # ragged tails); second call: one small 640x480 pair
    first = [synth.cfg1_pair(m, n_kp=6000) for m in ("sideways", "forward", "forward_yaw")]
    print("noalloc call 1: 3 pairs x 6000 keypoints", flush=True)
    ref, got = _both(first, 2.0, 0.0)
    _assert_same(ref, got, "call 1")
    assert len(ref[1]) > 0
    second = [synth.cfg0_pair(3)]
    print("noalloc call 2: 1 pair x 1000 keypoints", flush=True)
    ref, got = _both(second, 2.0, 0.8)
    _assert_same(ref, got, "call 2")
    assert (ref[2] >= 0).any()
