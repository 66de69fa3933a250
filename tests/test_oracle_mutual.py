"""Pins of the mutual-matching oracle (CPU)."""

import numpy as np

import synth
from oracle import candidates
from oracle.mutual import mutual_check, mutual_match


def _true_pairs(p):
    i = np.nonzero(p.gt12 >= 0)[0]
    return i, p.gt12[i]


def _has(o, c, i, j):
    return np.array([j[k] in set(c[o[i[k]]:o[i[k] + 1]]) for k in range(len(i))])


def test_noiseless_true_matches_are_candidates_both_ways():
    """On the noiseless keypoints every true match lies on the other's
    epipolar line in both images: with F forward and F^T backward it is a
    candidate at a tolerance far below a pixel."""
    p = synth.cfg0_pair(1)
    i, j = _true_pairs(p)
    o12, c12, _ = candidates(p.F, p.clean1, p.clean2, 1e-3)
    o21, c21, _ = candidates(p.F.T, p.clean2, p.clean1, 1e-3)
    assert _has(o12, c12, i, j).all()
    assert _has(o21, c21, j, i).all()


def test_reverse_direction_needs_the_transposed_matrix():
    """The mutant that guides image 2 with F itself loses the true matches."""
    p = synth.cfg0_pair(1)
    i, j = _true_pairs(p)
    o21, c21, _ = candidates(p.F, p.clean2, p.clean1, 1e-3)
    assert _has(o21, c21, j, i).mean() < 0.1


def test_cross_check_hand_case():
    best12 = np.array([2, -1, 0, 1])
    best21 = np.array([2, 0, 0])  # keypoint 0 -> query 2, 1 -> 0, 2 -> 0
    assert mutual_check(best12, best21).tolist() == [2, -1, 0, -1]


def test_mutual_keeps_most_true_matches_and_rejects_outliers():
    p = synth.cfg0_pair(2)
    b12, b21, mu = mutual_match(p.F, p.kp1, p.kp2, p.desc1, p.desc2, 2.0, 2.0)
    true = p.gt12 >= 0
    assert (mu[true] == p.gt12[true]).mean() > 0.9
    # outlier queries (no true match) keep far fewer matches than one-way matching
    assert (mu[~true] >= 0).sum() < 0.5 * (b12[~true] >= 0).sum()
    # every mutual match is a forward match
    assert np.all((mu == -1) | (mu == b12))
