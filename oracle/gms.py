"""GMS validation of guided matches -- TEST INFRASTRUCTURE ONLY.

The paper's experiments filter every method's matches with GMS (grid-based
motion statistics, Bian et al., cited in Sec. 4.3) with the threshold fixed
to 6 (experimental setup, Sec. 5).  GMS rests on motion smoothness: a true
match has, in the neighbourhood of its cell in image 1, many other matches
that land in the matching neighbourhood in image 2.  Restated from the
published method, in its single-grid form:

  * both images are divided into G x G cells (G = 20);
  * for every image-1 cell a, the image-2 cell b receiving most of a's
    matches is its motion;
  * the score of (a, b) sums the matches from each cell of the 3 x 3
    neighbourhood of a to the cell at the same offset around b;
  * (a, b) passes when score > alpha sqrt(n), n the mean number of matches
    per cell of that neighbourhood of a (alpha = 6);
  * a match is kept when it goes from a to b and (a, b) passes.

Readings where the paper (which only cites GMS) is silent:
  G1 cell of a point: floor(x G / W) in FP64, clamped to [0, G - 1] (points
     off the image fall in the border cells); index row-major (cy G + cx);
  G2 the "features" of the threshold are the putative matches (queries with
     a match), as in GMS where every feature carries one putative match;
  G3 neighbour cells outside a grid contribute nothing, and cells outside
     image 1's grid are left out of the mean;
  G4 the motion of a cell is its most frequent image-2 cell, ties to the
     lowest cell index;
  G5 the test is strict and taken exactly: S^2 * cells > alpha^2 * total
     (FP64, exact for integer alpha^2);
  G6 one grid only: no half-cell shifts and no rotation or scale variants.

Parity: pinned in tests/test_oracle_gms.py (hand-built motions, the
threshold boundary at a corner cell, the tie rule, invariance under the
query order).
"""

import numpy as np


def cells(xy, w, h, grid):
    """Row-major cell index of each point (G1)."""
    xy = np.asarray(xy, dtype=np.float32).reshape(-1, 2)
    cx = np.floor(xy[:, 0].astype(np.float64) * grid / float(w))
    cy = np.floor(xy[:, 1].astype(np.float64) * grid / float(h))
    cx = np.clip(cx, 0, grid - 1).astype(np.int64)
    cy = np.clip(cy, 0, grid - 1).astype(np.int64)
    return cy * grid + cx


def gms(kp1, kp2, best, w1, h1, w2, h2, grid=20, alpha=6.0):
    """best [m] image-2 indices or -1 -> the kept matches (-1 elsewhere)."""
    best = np.asarray(best)
    out = np.full(len(best), -1, dtype=np.int32)
    q = np.nonzero(best >= 0)[0]
    if len(q) == 0:
        return out
    G = int(grid)
    a = cells(np.asarray(kp1)[q], w1, h1, G)
    b = cells(np.asarray(kp2)[best[q]], w2, h2, G)
    N = np.zeros((G * G, G * G), dtype=np.int64)
    np.add.at(N, (a, b), 1)
    count = N.sum(axis=1)
    a2 = float(np.float64(np.float32(alpha))) ** 2
    for ac in np.nonzero(count)[0]:
        bd = int(np.argmax(N[ac]))  # first maximum: the lowest cell index (G4)
        ax, ay, bx, by = ac % G, ac // G, bd % G, bd // G
        score = total = ncell = 0
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                x1, y1 = ax + dx, ay + dy
                if not (0 <= x1 < G and 0 <= y1 < G):
                    continue
                ak = y1 * G + x1
                total += int(count[ak])
                ncell += 1
                x2, y2 = bx + dx, by + dy
                if 0 <= x2 < G and 0 <= y2 < G:
                    score += int(N[ak, y2 * G + x2])
        if float(score * score * ncell) > a2 * float(total):
            sel = (a == ac) & (b == bd)
            out[q[sel]] = best[q[sel]]
    return out
