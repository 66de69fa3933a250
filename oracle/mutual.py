"""Mutual guided matching, the plain definition -- TEST INFRASTRUCTURE ONLY.

Guided matching combines with the standard matching strategies (Sec. 4.3);
the cross-check keeps a correspondence (i, j) only when j is the match of
query i in image 2 and i is the match of query j in image 1, the second
direction being guided by the transposed fundamental matrix (Eq. 1 with the
cameras exchanged, x1^T F^T x2 = 0).

Parity: pinned in tests/test_oracle_mutual.py (noiseless true matches are
candidates in both directions only with the transposed matrix; the check
on a hand-made example).
"""

import numpy as np

from . import candidates, match


def mutual_check(best12, best21):
    """mutual[i] = best12[i] if best21[best12[i]] == i, else -1 (one pair,
    local indices, -1 for no match)."""
    best12 = np.asarray(best12)
    best21 = np.asarray(best21)
    out = np.full(len(best12), -1, dtype=np.int32)
    for i, j in enumerate(best12):
        if j >= 0 and best21[j] == i:
            out[i] = j
    return out


def mutual_match(F, kp1, kp2, desc1, desc2, eps2, eps1, ratio=0.0):
    """Both guided directions on one pair and the cross-check: returns
    (best12, best21, mutual) with local indices."""
    o12, c12, _ = candidates(F, kp1, kp2, eps2)
    b12, _, _ = match(desc1, desc2, o12, c12, ratio=ratio)
    o21, c21, _ = candidates(np.asarray(F, dtype=np.float64).reshape(3, 3).T, kp2, kp1, eps1)
    b21, _, _ = match(desc2, desc1, o21, c21, ratio=ratio)
    return b12, b21, mutual_check(b12, b21)
