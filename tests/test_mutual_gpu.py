"""Mutual guided matching through the library (both directions on the GPU,
the transposed matrix guiding image 2 against image 1, and the cross-check
kernel) against the oracle, bit for bit."""

import sys

import numpy as np
import pytest

import synth
from oracle.mutual import mutual_match as oracle_mutual
from tests.gpu_util import specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _run(pairs, eps, ratio):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    b = synth.batch_pairs(pairs)
    out = E.mutual_match(specs_of(pairs), [(p.W, p.H) for p in pairs], _dev(torch, b.kp1),
                         _dev(torch, b.kp2), _dev(torch, b.desc1), _dev(torch, b.desc2), eps=eps,
                         ratio=ratio)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in out]


def _check(pairs, eps, ratio):
    b12, b21, mu = _run(pairs, eps, ratio)
    q0 = k0 = 0
    for p in pairs:
        r12, r21, rmu = oracle_mutual(p.F, p.kp1, p.kp2, p.desc1, p.desc2, eps, eps, ratio=ratio)
        assert np.array_equal(b12[q0:q0 + p.m], r12)
        assert np.array_equal(b21[k0:k0 + p.n], r21)
        assert np.array_equal(mu[q0:q0 + p.m], rmu)
        q0 += p.m
        k0 += p.n
    return mu


@pytest.mark.parametrize("ratio", [0.0, 0.8])
def test_mutual_cfg0_batch(ratio):
    pairs = [synth.cfg0_pair(r) for r in range(4)]
    print(f"mutual cfg0 x4 ratio {ratio}", flush=True)
    mu = _check(pairs, 2.0, ratio)
    assert (mu >= 0).sum() > 0


@pytest.mark.parametrize("motion", ["sideways", "forward"])
def test_mutual_cfg1(motion):
    print(f"mutual cfg1 {motion} eps 4", flush=True)
    _check([synth.cfg1_pair(motion)], 4.0, 0.8)


def test_mutual_wide_rows():
    print("mutual 25000 keypoints eps 25", flush=True)
    sys.stdout.flush()
    _check([synth.cfg1_pair("forward", n_kp=25000)], 25.0, 0.0)
