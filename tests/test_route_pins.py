"""CPU pins of the route-stage reference (grid geodesics and the tour).

Geodesics: in an empty grid they equal the octile closed form
cell (max - min + sqrt(2) min) of the cell offsets; a wall with one gap
forces the detour through the gap (sum of the two octile legs); the
triangle inequality holds.  Tours: on small instances the local search
never beats brute force, finds the brute-force optimum for points in
convex position, and leaves no improving 2-opt or Or-opt move."""
import itertools
import math

import numpy as np
import pytest

from oracle import route


def _octile(a, b, cell):
    dr, dc = abs(a[0] - b[0]), abs(a[1] - b[1])
    return cell * ((max(dr, dc) - min(dr, dc)) + math.sqrt(2.0) * min(dr, dc))


def test_empty_grid_is_octile():
    free = np.ones((30, 40), np.uint8)
    rng = np.random.default_rng(0)
    cells = rng.integers(0, [30, 40], size=(12, 2))
    stops = np.stack([(cells[:, 1] + 0.5) * 0.25, (cells[:, 0] + 0.5) * 0.25], 1)
    D = route.geodesic_matrix(free, 0.0, 0.0, 0.25, stops)
    for a, b in itertools.combinations(range(12), 2):
        assert D[a, b] == pytest.approx(_octile(cells[a], cells[b], 0.25), rel=1e-12, abs=1e-12)
    assert np.all(np.diag(D) == 0)


def test_wall_with_gap_and_triangle_inequality():
    free = np.ones((20, 21), np.uint8)
    free[:, 10] = 0
    free[15, 10] = 1  # the gap
    a, b, g = (2, 3), (4, 17), (15, 10)
    stops = np.array([[a[1] + 0.5, a[0] + 0.5], [b[1] + 0.5, b[0] + 0.5]], np.float64)
    D = route.geodesic_matrix(free, 0.0, 0.0, 1.0, stops)
    # through the gap: no corner cutting, so the gap cell is entered and left
    # straight from its two free neighbours (15, 9) and (15, 11)
    expect = _octile(a, (15, 9), 1.0) + 2.0 + _octile((15, 11), b, 1.0)
    assert D[0, 1] == pytest.approx(expect, rel=1e-12)
    rng = np.random.default_rng(1)
    fr = np.argwhere(free)
    pick = fr[rng.choice(len(fr), 9, replace=False)]
    st = np.stack([pick[:, 1] + 0.5, pick[:, 0] + 0.5], 1)
    D = route.geodesic_matrix(free, 0.0, 0.0, 1.0, st)
    for i, j, k in itertools.permutations(range(9), 3):
        assert D[i, j] <= D[i, k] + D[k, j] + 1e-12


def test_blocked_stop_rejected():
    free = np.ones((5, 5), np.uint8)
    free[2, 2] = 0
    with pytest.raises(ValueError):
        route.geodesic_matrix(free, 0.0, 0.0, 1.0, np.array([[2.5, 2.5]]))


@pytest.mark.parametrize("seed", range(6))
def test_local_search_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    m = 8
    P = rng.uniform(0, 10, size=(m, 2))
    D = np.sqrt(((P[:, None] - P[None]) ** 2).sum(-1))
    t, _ = route.local_search(D)
    assert sorted(t.tolist()) == list(range(m)) and t[0] == 0
    bt, best = route.brute_force_tour(D)
    L = route.tour_length(D, t)
    assert L >= best - 1e-12
    # local optimality: no improving 2-opt or Or-opt move is left
    d2, _, _ = route._best_two_opt(D, t)
    do = route._best_or_opt(D, t)[0]
    assert d2 >= -1e-12 * L and do >= -1e-12 * L


def test_convex_position_reaches_the_optimum():
    m = 9
    ang = np.sort(np.random.default_rng(3).uniform(0, 2 * np.pi, m))
    P = np.stack([np.cos(ang), np.sin(ang)], 1)[np.random.default_rng(4).permutation(m)]
    D = np.sqrt(((P[:, None] - P[None]) ** 2).sum(-1))
    t, _ = route.local_search(D)
    bt, best = route.brute_force_tour(D)
    assert route.tour_length(D, t) == pytest.approx(best, rel=1e-12)


def test_plan_time():
    assert route.plan_time([10.0, 20.0], 15.0, v_max=0.5) == 60.0
