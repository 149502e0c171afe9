"""Relaxed dosage LP reference -- TEST INFRASTRUCTURE ONLY.

The relaxed LP of Sec. IV-D (equation "simple LP"):

    minimise   sum_k t_k + sum_i p_i sigma_i
    subject to sum_k I_i(x_k) t_k + sigma_i >= mu_min   for every element i
               sum_k t_k <= T_max,   t >= 0,  sigma >= 0

with E[k, i] = I_i(x_k) (pose-major).  Readings: elements that no pose sees
(max_k E[k, i] = 0) are dropped, their sigma_i = mu_min fixed, and the
reported objective excludes their constant p_i mu_min; the default penalty is
p_i = 1.001 * ||E||_F (the paper asks for p_i > ||I||_F).  Solved with SciPy's
HiGHS (dual simplex), which returns a vertex solution and duals.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def default_penalty(E: np.ndarray) -> float:
    return 1.001 * float(np.sqrt((np.asarray(E, np.float64) ** 2).sum()))


def solve(E, mu_min: float = 280.0, t_max: float = 3.6e5, penalty=None, method: str = "highs-ds"):
    """Returns dict(t [K], sigma [N], objective, visible mask, duals, status)."""
    E = np.asarray(E, np.float64)
    K, N = E.shape
    vis = E.max(axis=0) > 0.0
    if penalty is None:
        p = np.full(N, default_penalty(E))
    else:
        p = np.broadcast_to(np.asarray(penalty, np.float64), (N,)).copy()
    Ev = E[:, vis]
    Nv = int(vis.sum())
    c = np.concatenate([np.ones(K), p[vis]])
    # -(E^T t + sigma) <= -mu ;  sum t <= T_max
    A1 = sp.hstack([sp.csr_matrix(-Ev.T), -sp.identity(Nv, format="csr")])
    A2 = sp.hstack([sp.csr_matrix(np.ones((1, K))), sp.csr_matrix((1, Nv))])
    A = sp.vstack([A1, A2]).tocsr()
    b = np.concatenate([np.full(Nv, -mu_min), [t_max]])
    res = linprog(c, A_ub=A, b_ub=b, bounds=(0, None), method=method)
    if res.status != 0:
        raise RuntimeError(f"HiGHS failed: {res.message}")
    t = res.x[:K]
    sigma = np.full(N, float(mu_min))
    sigma[vis] = res.x[K:]
    return {"t": t, "sigma": sigma, "objective": float(res.fun), "visible": vis,
            "duals": -res.ineqlin.marginals, "penalty": p, "status": res.status}


def kkt_residuals(E, sol, mu_min: float = 280.0, t_max: float = 3.6e5):
    """Primal feasibility, dual feasibility and relative gap of (t, sigma, duals)
    for the visible-element LP: a certificate independent of the solver."""
    E = np.asarray(E, np.float64)
    vis = sol["visible"]
    Ev = E[:, vis]
    t, s = sol["t"], sol["sigma"][vis]
    p = sol["penalty"][vis]
    y = sol["duals"]          # >= 0: N_vis coverage rows, then the time-budget row
    yc, yt = y[:-1], y[-1]
    prim = max(0.0, float(np.max(mu_min - (Ev.T @ t + s), initial=0.0)), float(t.sum() - t_max),
               float(-t.min(initial=0.0)), float(-s.min(initial=0.0)))
    # reduced costs: for t: 1 - E yc + yt >= 0 ; for sigma: p - yc >= 0
    rt = 1.0 - Ev @ yc + yt
    rs = p - yc
    dual = max(0.0, float(-rt.min(initial=0.0)), float(-rs.min(initial=0.0)), float(-y.min(initial=0.0)))
    pobj = t.sum() + p @ s
    dobj = mu_min * yc.sum() - t_max * yt
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return prim, dual, gap


def relative_objective_gap(obj, ref) -> float:
    return abs(obj - ref) / max(1.0, abs(ref))
