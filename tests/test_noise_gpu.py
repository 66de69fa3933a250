"""Pose noise (the paper's noise-sensitivity setting): F from a perturbed
relative pose, tolerance 200 px.  Candidates and matches against the oracle,
bit for bit, and the recall the sweep reports."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_csr_equal, specs_of, torch_gpu

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


@pytest.mark.parametrize("motion,level", [("sideways", 1.0), ("forward", 3.3)])
def test_perturbed_pose_eps_200(motion, level):
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    p = synth.cfg1_pair(motion, n_kp=8000)
    p.F = synth.perturbed_F(p, level, 777)
    print(f"noise {motion} level {level}", flush=True)
    ro, rc, _ = oracle.candidates(p.F, p.kp1, p.kp2, 200.0)
    rb, rbd, rsd = oracle.match(p.desc1, p.desc2, ro, rc)
    idx = E.Index(specs_of([p]), _dev(torch, p.kp2), eps=200.0)
    o, c, b, bd, sd = [x.cpu().numpy() for x in idx.query_match(
        _dev(torch, p.kp1), _dev(torch, p.desc1), _dev(torch, p.desc2))]
    assert_csr_equal((o, c), (ro, rc), "noisy F")
    assert np.array_equal(b, rb)
    assert np.array_equal(bd.view(np.uint32), rbd.view(np.uint32))
    assert np.array_equal(sd.view(np.uint32), rsd.view(np.uint32))
    assert np.median(np.diff(ro)) > 128  # the wide-row regime


def test_noise_sweep_bench_line(monkeypatch, capsys):
    import json
    import sys

    import bench
    torch_gpu()
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "noise", "--steps", "1",
                                      "--warmup", "0"])
    bench.main()
    line = json.loads([x for x in capsys.readouterr().out.splitlines() if x.startswith("{")][-1])
    per = {r["level"]: r for r in line["recall_by_level"]}
    assert per[0.0]["candidate_recall"] == 1.0
    assert all(0.0 <= r["match_recall"] <= r["candidate_recall"] for r in per.values())
