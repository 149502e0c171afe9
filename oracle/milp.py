"""Joint dwell-time and tour MILP (Appendix I) -- TEST INFRASTRUCTURE ONLY.

The paper's exact formulation of the discrete plan: dwell times t_k >= 0,
binary edge choices z_kl (k != l), single-commodity flows g_kl >= 0;

    minimise   sum_k t_k + (1 / v_max) sum_kl d_kl z_kl
    subject to sum_k E[k, i] t_k >= mu_min          (every visible element)
               t_k <= M sum_l (z_kl + z_lk)          (dwell only on the loop)
               sum_k z_kl <= 1  (l >= 1),  sum_k z_k0 = 1   (pose 0 on the loop)
               sum_k z_kl = sum_k z_lk               (as many edges in as out)
               sum_k g_kl - sum_k g_lk = sum_k z_kl  (l >= 1: one unit unloaded)
               0 <= g_kl <= K z_kl,  g_kl <= sum_ab z_ab - 1

(0-based indices; pose 0 plays the paper's first configuration).  The last
line is written with one extra variable s = sum_ab z_ab, which keeps the
matrix at O(K^2) nonzeros.  Readings: elements that no pose sees are
dropped (as in the relaxed LP); M is an upper bound on the optimum, so it
never cuts an optimal t_k.  Solved by SciPy's milp (HiGHS branch and
bound).  Brute force over visited subsets and tours pins it on tiny cases.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp
from scipy.optimize import Bounds, LinearConstraint, linprog, milp


def _lp_min_time(E, mu, idx):
    """min sum t over the poses idx (all visible elements covered); inf if
    some visible element cannot be covered by them."""
    Ev = E[:, E.max(0) > 0]
    sub = Ev[list(idx)]
    if np.any(sub.max(0) <= 0):
        return math.inf
    res = linprog(np.ones(len(idx)), A_ub=-sub.T, b_ub=np.full(sub.shape[1], -mu), bounds=(0, None),
                  method="highs")
    return res.fun if res.status == 0 else math.inf


def solve(E, d, mu_min: float = 280.0, v_max: float = 0.5, M: float | None = None, time_limit: float = 300.0):
    """Returns dict(objective, t [K], tour edges z [K, K] (0/1), status)."""
    E = np.asarray(E, np.float64)
    d = np.asarray(d, np.float64)
    K, N = E.shape
    vis = E.max(0) > 0
    Ev = E[:, vis]
    nv = Ev.shape[1]
    if M is None:
        # an upper bound on the optimum: every pose dwelling as the full LP
        # says, plus a nearest-neighbour loop through all poses
        t_all = _lp_min_time(E, mu_min, range(K))
        tour = [0]
        left = set(range(1, K))
        while left:
            nxt = min(left, key=lambda q: (d[tour[-1], q], q))
            tour.append(nxt)
            left.remove(nxt)
        loop = sum(d[tour[q], tour[(q + 1) % K]] for q in range(K))
        M = t_all + loop / v_max
    nz = K * K
    it, iz, ig, isv = 0, K, K + nz, K + 2 * nz  # variable blocks: t, z, g, s
    nvar = K + 2 * nz + 1
    zi = lambda k, l: iz + k * K + l  # noqa: E731
    gi = lambda k, l: ig + k * K + l  # noqa: E731
    c = np.zeros(nvar)
    c[it:it + K] = 1.0
    for k in range(K):
        for l in range(K):
            c[zi(k, l)] = d[k, l] / v_max
    rows, cols, vals, lo, hi = [], [], [], [], []
    r = 0

    def add(entries, lb, ub):
        nonlocal r
        for col, v in entries:
            rows.append(r)
            cols.append(col)
            vals.append(v)
        lo.append(lb)
        hi.append(ub)
        r += 1

    for i in range(nv):  # coverage
        add([(it + k, Ev[k, i]) for k in range(K) if Ev[k, i] != 0.0], mu_min, np.inf)
    for k in range(K):  # big M
        add([(it + k, 1.0)] + [(zi(k, l), -M) for l in range(K) if l != k] + [(zi(l, k), -M) for l in range(K)
                                                                             if l != k], -np.inf, 0.0)
    for l in range(K):  # at most one incoming edge; exactly one into pose 0
        add([(zi(k, l), 1.0) for k in range(K) if k != l], 1.0 if l == 0 else -np.inf, 1.0)
    for l in range(K):  # as many edges in as out
        add([(zi(k, l), 1.0) for k in range(K) if k != l] + [(zi(l, k), -1.0) for k in range(K) if k != l], 0.0, 0.0)
    for l in range(1, K):  # single-commodity flow: one unit unloaded at every visited pose
        add([(gi(k, l), 1.0) for k in range(K) if k != l] + [(gi(l, k), -1.0) for k in range(K) if k != l]
            + [(zi(k, l), -1.0) for k in range(K) if k != l], 0.0, 0.0)
    for k in range(K):
        for l in range(K):
            if k == l:
                continue
            add([(gi(k, l), 1.0), (zi(k, l), -float(K))], -np.inf, 0.0)
            add([(gi(k, l), 1.0), (isv, -1.0)], -np.inf, -1.0)
    add([(isv, 1.0)] + [(zi(a, b), -1.0) for a in range(K) for b in range(K) if a != b], 0.0, 0.0)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(r, nvar))
    lb = np.zeros(nvar)
    ub = np.full(nvar, np.inf)
    integrality = np.zeros(nvar)
    for k in range(K):
        for l in range(K):
            ub[zi(k, l)] = 0.0 if k == l else 1.0
            ub[gi(k, l)] = 0.0 if k == l else np.inf
            integrality[zi(k, l)] = 1
    res = milp(c, constraints=LinearConstraint(A, lo, hi), integrality=integrality, bounds=Bounds(lb, ub),
               options={"time_limit": time_limit, "mip_rel_gap": 1e-9})
    if res.x is None:
        raise RuntimeError(f"MILP failed: {res.message}")
    x = res.x
    z = np.rint(x[iz:iz + nz]).reshape(K, K)
    return {"objective": float(res.fun), "t": x[it:it + K], "z": z, "status": int(res.status),
            "optimal": res.status == 0, "M": M}


def brute_force(E, d, mu_min: float = 280.0, v_max: float = 0.5):
    """Optimum by enumeration for tiny K: every visited set containing pose
    0 and at least one other pose, the LP's least dwell time on it plus its
    shortest closed tour."""
    E = np.asarray(E, np.float64)
    d = np.asarray(d, np.float64)
    K = E.shape[0]
    best = math.inf
    for r in range(1, K):
        for rest in itertools.combinations(range(1, K), r):
            S = (0,) + rest
            tt = _lp_min_time(E, mu_min, S)
            if not math.isfinite(tt):
                continue
            L = min(sum(d[p[q], p[(q + 1) % len(p)]] for q in range(len(p)))
                    for p in ((0,) + perm for perm in itertools.permutations(rest)))
            best = min(best, tt + L / v_max)
    return best
