"""Pins of the GMS oracle (CPU): hand-built motion fields whose outcome
follows from the definition by hand."""

import numpy as np

from oracle.gms import cells, gms

W = H = 200.0  # 20 x 20 cells of 10 px


def _pt(cx, cy, k=0):
    # a point inside cell (cx, cy), spread a little so points are distinct
    return [cx * 10.0 + 1.0 + (k % 8), cy * 10.0 + 1.0 + (k // 8) % 8]


def _field(moves):
    """moves: list of (cell1, cell2, count) -> kp1, kp2, best (match i -> i)."""
    kp1, kp2 = [], []
    for (c1, c2, n) in moves:
        for k in range(n):
            kp1.append(_pt(*c1, k))
            kp2.append(_pt(*c2, k))
    kp1 = np.array(kp1, np.float32)
    kp2 = np.array(kp2, np.float32)
    return kp1, kp2, np.arange(len(kp1), dtype=np.int32)


def test_cells_floor_and_clamp():
    xy = np.array([[0, 0], [9.999, 0], [10, 0], [199.99, 199.99], [-5, 250]], np.float32)
    assert cells(xy, W, H, 20).tolist() == [0, 0, 1, 19 * 20 + 19, 19 * 20 + 0]


def test_coherent_neighbourhood_kept_isolated_match_rejected():
    # cell (5,5) -> (7,5) with 20 matches, its 8 neighbours move the same way
    moves = [((5, 5), (7, 5), 20)]
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx or dy:
                moves.append(((5 + dx, 5 + dy), (7 + dx, 5 + dy), 10))
    moves.append(((15, 15), (2, 2), 1))  # isolated: S = 1, n = 1/9 -> 9 > 36 fails
    kp1, kp2, best = _field(moves)
    out = gms(kp1, kp2, best, W, H, W, H)
    assert np.all(out[:-1] == best[:-1])
    assert out[-1] == -1


def test_threshold_boundary_at_a_corner_cell():
    # corner cell (0,0): 4 cells in its neighbourhood; k coherent matches give
    # S = k, total = k, so S^2 * 4 > 36 k  <=>  k > 9
    for k, kept in ((9, False), (10, True)):
        kp1, kp2, best = _field([((0, 0), (3, 0), k)])
        out = gms(kp1, kp2, best, W, H, W, H)
        assert bool(np.all(out == best)) == kept and bool(np.all(out == -1)) == (not kept)


def test_dominant_cell_ties_go_to_the_lowest_index():
    # 15 matches (0,0) -> (3,0) and 15 -> (5,0): cell 3 < cell 5 wins,
    # S = 15, total = 30: 225 * 4 = 900 > 1080 fails ... so add support
    moves = [((0, 0), (3, 0), 15), ((0, 0), (5, 0), 15), ((1, 0), (4, 0), 20)]
    kp1, kp2, best = _field(moves)
    out = gms(kp1, kp2, best, W, H, W, H)
    # cell (0,0): S = 15 + 20 = 35, total = 30 + 20 = 50 -> 1225 * 4 > 1800: kept for b = (3,0)
    assert np.all(out[:15] == best[:15])
    assert np.all(out[15:30] == -1)
    # cell (1,0): S = 20 + 15 (from (0,0) to (3,0)) = 35, total = 50, 6 cells
    assert np.all(out[30:] == best[30:])


def test_invariant_under_query_order():
    rng = np.random.default_rng(0)
    n = 4000
    kp1 = rng.uniform(0, 160, (n, 2)).astype(np.float32)
    kp2 = (kp1 + 30.0 + rng.normal(0, 0.5, kp1.shape)).astype(np.float32)
    best = np.arange(n, dtype=np.int32)
    wrong = rng.random(n) < 0.3  # random outlier matches
    best[wrong] = rng.integers(0, n, int(wrong.sum()))
    best[rng.random(n) < 0.1] = -1  # and some queries without a match
    out = gms(kp1, kp2, best, W, H, W, H)
    perm = rng.permutation(n)
    out_p = gms(kp1[perm], kp2, best[perm], W, H, W, H)
    assert np.array_equal(out_p, out[perm])
    # the coherent shift survives, the random matches mostly do not
    good = (best >= 0) & ~wrong
    assert (out[good] >= 0).mean() > 0.7 and (out[wrong] >= 0).mean() < 0.1
