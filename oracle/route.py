"""Route stage reference -- TEST INFRASTRUCTURE ONLY.

The second stage of the paper's two-stage plan (Sec. IV-D): after the LP
fixes the dwell times, the robot visits the poses with t_k > 0 along a
closed tour (the paper solves this TSP with LKH over roadmap distances,
Sec. IV-B/IV-D); plan time = sum t + tour length / v_max (v_max = 0.5 m/s,
Sec. V).  Readings (the paper is silent): distances are grid geodesics
through free space (8-connected cells, step costs cell and cell*sqrt(2),
diagonal steps only between two free orthogonal neighbours), and the tour
comes from a deterministic local search (nearest neighbour from the first
stop, then best-improvement 2-opt, then best-improvement Or-opt of
segments of 1-3 stops when 2-opt finds nothing), not from LKH.

Plain NumPy/SciPy: SciPy's Dijkstra gives the geodesics; the local search
evaluates every move of a pass in FP64 with the delta written out in the
same operation order as the definition below, and takes the smallest delta
(ties: the lowest move index).  Brute force over permutations serves as the
pin for small tours.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

SQRT2 = math.sqrt(2.0)


def stop_cells(stops, x0, y0, cell):
    """Grid cell (row, col) of each stop: floor((p - origin) / cell) in FP64."""
    st = np.asarray(stops, np.float32).astype(np.float64)
    col = np.floor((st[:, 0] - np.float64(np.float32(x0))) / np.float64(np.float32(cell))).astype(np.int64)
    row = np.floor((st[:, 1] - np.float64(np.float32(y0))) / np.float64(np.float32(cell))).astype(np.int64)
    return row, col


def grid_graph(free, cell):
    """Sparse FP64 adjacency of the free cells (8-connected, no corner
    cutting)."""
    free = np.asarray(free, bool)
    H, W = free.shape
    w_o = np.float64(np.float32(cell))
    w_d = w_o * SQRT2
    idx = np.arange(H * W).reshape(H, W)
    rows, cols, vals = [], [], []
    for dr, dc in ((0, 1), (1, 0), (0, -1), (-1, 0), (1, 1), (1, -1), (-1, 1), (-1, -1)):
        r0, r1 = max(0, -dr), H - max(0, dr)
        c0, c1 = max(0, -dc), W - max(0, dc)
        a = free[r0:r1, c0:c1] & free[r0 + dr:r1 + dr, c0 + dc:c1 + dc]
        if dr != 0 and dc != 0:
            a &= free[r0 + dr:r1 + dr, c0:c1] & free[r0:r1, c0 + dc:c1 + dc]
        src = idx[r0:r1, c0:c1][a]
        dst = idx[r0 + dr:r1 + dr, c0 + dc:c1 + dc][a]
        rows.append(src)
        cols.append(dst)
        vals.append(np.full(src.size, w_d if (dr and dc) else w_o))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(H * W, H * W))


def geodesic_matrix(free, x0, y0, cell, stops):
    """m x m geodesic distances between the stops' cells; symmetrised as
    min(d(a, b), d(b, a)) (the two directions sum the same steps in
    opposite orders).  inf where no free path exists."""
    free = np.asarray(free, bool)
    H, W = free.shape
    row, col = stop_cells(stops, x0, y0, cell)
    if np.any((row < 0) | (row >= H) | (col < 0) | (col >= W)) or not np.all(free[row, col]):
        raise ValueError("a stop lies outside the grid or in a blocked cell")
    G = grid_graph(free, cell)
    src = row * W + col
    D = dijkstra(G, directed=True, indices=src)[:, src]
    return np.minimum(D, D.T)


def tour_length(D, tour):
    L = 0.0
    m = len(tour)
    for q in range(m):
        L = L + D[tour[q], tour[(q + 1) % m]]
    return L


def nearest_neighbour(D):
    m = D.shape[0]
    tour = [0]
    used = np.zeros(m, bool)
    used[0] = True
    for _ in range(m - 1):
        d = np.where(used, np.inf, D[tour[-1]])
        nxt = int(np.argmin(d))  # first index of the minimum
        tour.append(nxt)
        used[nxt] = True
    return np.array(tour, np.int64)


def _best_two_opt(D, t):
    """Moves (i, j), 0 <= i <= m-3, i+2 <= j <= m-1, not (0, m-1): replace
    edges (t_i, t_i+1), (t_j, t_j+1) by (t_i, t_j), (t_i+1, t_j+1);
    delta = (D[a,c] + D[b,e]) - (D[a,b] + D[c,e]).  Move index q = i m + j."""
    m = len(t)
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    ok = (i <= m - 3) & (j >= i + 2) & ~((i == 0) & (j == m - 1))
    a, b, c, e = t[i], t[(i + 1) % m], t[j], t[(j + 1) % m]
    delta = (D[a, c] + D[b, e]) - (D[a, b] + D[c, e])
    delta = np.where(ok, delta, np.inf).ravel()
    q = int(np.argmin(delta))
    return float(delta[q]), q // m, q % m


def _best_or_opt(D, t):
    """Moves (s, i, p): the segment t_i .. t_i+s-1 (1 <= s <= 3,
    1 <= i <= m-s) leaves its place and is inserted, same orientation,
    between t_p and t_p+1 (p outside [i-1, i+s-1]);
    delta = ((D[prev,next] + D[u,f]) + D[l,v]) - ((D[prev,f] + D[l,next]) + D[u,v]).
    Move index q = ((s - 1) m + i) m + p."""
    m = len(t)
    best = (math.inf, -1, 0, 0, 0)
    for s in (1, 2, 3):
        i, p = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        ok = (i >= 1) & (i <= m - s) & ~((p >= i - 1) & (p <= i + s - 1))
        if m - s < 1:
            continue
        f, l = t[i], t[np.minimum(i + s - 1, m - 1)]
        prev, nxt = t[i - 1], t[(i + s) % m]
        u, v = t[p], t[(p + 1) % m]
        delta = ((D[prev, nxt] + D[u, f]) + D[l, v]) - ((D[prev, f] + D[l, nxt]) + D[u, v])
        delta = np.where(ok, delta, np.inf).ravel()
        q = int(np.argmin(delta))
        qq = ((s - 1) * m) * m + q
        if delta[q] < best[0]:
            best = (float(delta[q]), qq, s, q // m, q % m)
    return best


def _apply_or_opt(t, s, i, p):
    seg = list(t[i:i + s])
    rest = list(t[:i]) + list(t[i + s:])
    u = t[p]
    at = rest.index(u) + 1
    return np.array(rest[:at] + seg + rest[at:], np.int64)


def local_search(D, max_moves: int | None = None):
    """Nearest-neighbour tour from stop 0, then best-improvement 2-opt;
    when no 2-opt move improves, the best Or-opt move; until neither
    improves by more than 1e-12 of the tour length.  Returns (tour, moves)."""
    D = np.asarray(D, np.float64)
    m = D.shape[0]
    t = nearest_neighbour(D)
    if m < 4:
        return t, 0
    cap = 100 * m if max_moves is None else max_moves
    moves = 0
    while moves < cap:
        eps = 1e-12 * tour_length(D, t)
        d2, i, j = _best_two_opt(D, t)
        if d2 < -eps:
            t = np.concatenate([t[:i + 1], t[i + 1:j + 1][::-1], t[j + 1:]])
            moves += 1
            continue
        do, _, s, i, p = _best_or_opt(D, t)
        if do < -eps:
            t = _apply_or_opt(t, s, i, p)
            moves += 1
            continue
        break
    return t, moves


def brute_force_tour(D):
    """Optimal closed tour by enumerating every order of stops 1..m-1."""
    D = np.asarray(D, np.float64)
    m = D.shape[0]
    best, bt = math.inf, None
    for perm in itertools.permutations(range(1, m)):
        t = (0,) + perm
        L = tour_length(D, t)
        if L < best:
            best, bt = L, t
    return np.array(bt, np.int64), best


def plan_time(t_dwell, length, v_max: float = 0.5):
    return float(np.sum(t_dwell)) + length / v_max
