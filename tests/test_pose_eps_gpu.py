"""Pose-uncertainty tolerance on the GPU (epm_pose_eps) against the oracle
(oracle/pose_eps.py, derivatives by central differences in FP64), and the
exact candidate sets and matches at the derived per-keypoint tolerances."""

import numpy as np
import pytest

import oracle
import synth
from oracle import pose_eps as PE
from tests.gpu_util import assert_csr_equal, specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _case(kind):
    if kind == "sideways":
        p = synth.cfg1_pair("sideways", n_kp=4000)
        R, t = synth.perturbed_pose(p, 1.0, 4242)
        cov = synth.noise_covariance(1.0)
    elif kind == "forward_yaw":
        p = synth.cfg1_pair("forward_yaw", n_kp=4000)
        R, t = synth.perturbed_pose(p, 2.0, 4243)
        cov = synth.noise_covariance(2.0)
    else:  # a general pose with a correlated covariance
        p = synth.cfg3_pair(2, max_kp=3000)
        R, t = synth.perturbed_pose(p, 0.5, 4244)
        A = np.random.default_rng(9).standard_normal((6, 6)) * np.array([2e-3] * 3 + [3e-2] * 3)
        cov = A @ A.T
    p.F = synth.fundamental_from_cameras(p.K1, p.K2, R, t)
    return p, R, t, cov


@pytest.mark.parametrize("depth", [(0.0, np.inf), (4.0, 16.0), (3.0, np.inf)])
@pytest.mark.parametrize("kind", ["sideways", "forward_yaw", "general"])
def test_pose_eps_equals_oracle_and_matching_is_exact(kind, depth):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p, R, t, cov = _case(kind)
    zmin, zmax = depth
    print(f"pose eps {kind} depth {depth}", flush=True)
    prior = E.PosePrior(p.K1, p.K2, R, t, cov, p.W, p.H, zmin, zmax)
    eps0, k, emax = 2.0, 3.0, 400.0
    e_gpu = E.pose_eps([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], [prior], _dev(torch, p.kp2), eps0,
                       k, emax).cpu().numpy()
    sample = np.random.default_rng(1).choice(p.n, 150, replace=False)
    e_ref = PE.pose_eps(p.kp2[sample], p.K1, p.K2, R, t, cov, p.W, p.H, eps0, k, emax, zmin,
                        zmax)
    assert np.allclose(e_gpu[sample], e_ref, rtol=1e-5, atol=1e-5), \
        np.abs(e_gpu[sample] - e_ref).max()
    assert e_gpu.min() >= eps0 and e_gpu.max() <= emax
    assert e_gpu.max() > 2 * eps0  # the covariance widens some tolerances
    # candidates and matches at the derived tolerances: exact
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, e_gpu)
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc)
    idx = E.Index(specs_of([p]), _dev(torch, p.kp2), eps2=_dev(torch, e_gpu))
    o, c, b, bd, sd = [x.cpu().numpy() for x in idx.query_match(
        _dev(torch, p.kp1), _dev(torch, p.desc1), _dev(torch, p.desc2))]
    assert_csr_equal((o, c), (ro, rc), kind)
    assert np.array_equal(b, rb)
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32))


def test_zero_covariance_is_the_base_tolerance():
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(1)
    prior = E.PosePrior(p.K1, p.K2, p.R, p.t, np.zeros((6, 6)), p.W, p.H)
    e = E.pose_eps([E.PairSpec(p.F, p.W, p.H, p.m, p.n)], [prior], _dev(torch, p.kp2), 1.5, 3.0,
                   10.0).cpu().numpy()
    assert (e == np.float32(1.5)).all()


def test_back_to_back_calls_keep_their_tables():
    """Twelve calls in a row without waiting (more than the eight upload slots
    of the library, so some calls reuse a slot) equal the same calls made one
    at a time."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg0_pair(2)
    R, t = synth.perturbed_pose(p, 1.0, 77)
    spec = [E.PairSpec(synth.fundamental_from_cameras(p.K1, p.K2, R, t), p.W, p.H, p.m, p.n)]
    kp2 = _dev(torch, p.kp2)
    covs = [synth.noise_covariance(0.1 * (k + 1)) for k in range(12)]
    burst = [E.pose_eps(spec, [E.PosePrior(p.K1, p.K2, R, t, c, p.W, p.H, 4.0, 16.0)], kp2, 1.0,
                        2.0, 1e4) for c in covs]
    torch.cuda.synchronize()
    for c, got in zip(covs, burst):
        one = E.pose_eps(spec, [E.PosePrior(p.K1, p.K2, R, t, c, p.W, p.H, 4.0, 16.0)], kp2, 1.0,
                         2.0, 1e4)
        torch.cuda.synchronize()
        assert torch.equal(got, one)
    assert not torch.equal(burst[0], burst[-1])
