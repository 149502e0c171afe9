"""Pins of the LP reference (relaxed dosage LP, Sec. IV-D) against facts
that do not depend on the solver: KKT certificates, a one-element closed
form, the infeasible-element reading, and brute-force vertex enumeration on
tiny instances."""
import itertools

import numpy as np
import pytest

from oracle import lp, ref
from paper_2103_14137_amd import workloads as wl


def test_single_element_closed_form():
    """One element: min sum t s.t. sum_k E_k t_k >= mu is solved by dwelling
    only at the best pose, t = mu / max_k E_k."""
    E = np.array([[0.5], [2.0], [1.25]])
    sol = lp.solve(E, mu_min=280.0, t_max=1e9, penalty=1e6)
    assert abs(sol["objective"] - 280.0 / 2.0) <= 1e-9 * 140.0
    assert abs(sol["t"][1] - 140.0) <= 1e-7 and np.all(np.abs(sol["t"][[0, 2]]) <= 1e-9)


def test_never_visible_elements_are_dropped():
    E = np.array([[1.0, 0.0, 2.0], [0.5, 0.0, 0.0]])
    sol = lp.solve(E, mu_min=10.0, t_max=1e6)
    assert not sol["visible"][1] and sol["sigma"][1] == 10.0
    assert abs(sol["objective"] - 10.0) <= 1e-9  # t_0 = 10 covers both visible elements


def test_time_budget_binds_and_penalty_is_paid():
    E = np.array([[1.0, 1.0]])
    sol = lp.solve(E, mu_min=100.0, t_max=40.0, penalty=3.0)
    # t = 40 (budget), sigma = 60 each: 40 + 3 * 60 * 2 = 400
    assert abs(sol["objective"] - 400.0) <= 1e-8


def _vertex_enumeration(E, mu, t_max, p):
    """Brute force: the optimum of an LP with a bounded feasible region is at
    a vertex; enumerate every basis of the inequality system."""
    K, N = E.shape
    n = K + N
    c = np.concatenate([np.ones(K), p])
    A = [np.concatenate([E[:, i], np.eye(N)[i]]) for i in range(N)]      # >= mu
    b = [mu] * N
    A.append(-np.concatenate([np.ones(K), np.zeros(N)]))                 # -sum t >= -T
    b.append(-t_max)
    for j in range(n):
        A.append(np.eye(n)[j])                                             # x >= 0
        b.append(0.0)
    A = np.array(A)
    b = np.array(b)
    best = np.inf
    for rows in itertools.combinations(range(len(b)), n):
        M = A[list(rows)]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, b[list(rows)])
        if np.all(A @ x >= b - 1e-9):
            best = min(best, float(c @ x))
    return best


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_matches_vertex_enumeration(seed):
    rng = np.random.default_rng(seed)
    E = rng.uniform(0.0, 3.0, size=(3, 3)) * (rng.uniform(size=(3, 3)) > 0.25)
    E[:, E.max(0) == 0] = 0.5
    mu, T, p = 10.0, float(rng.uniform(3, 30)), rng.uniform(0.5, 5.0, size=3)
    sol = lp.solve(E, mu_min=mu, t_max=T, penalty=p)
    assert abs(sol["objective"] - _vertex_enumeration(E, mu, T, p)) <= 1e-7 * max(1.0, sol["objective"])


def test_kkt_certificate_on_box_room():
    w = wl.box_room()
    E, _ = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power)
    for t_max in (3.6e5, 1800.0):
        sol = lp.solve(E, mu_min=280.0, t_max=t_max)
        prim, dual, gap = lp.kkt_residuals(E, sol, 280.0, t_max)
        assert prim <= 1e-6 and dual <= 1e-6 and gap <= 1e-9, (prim, dual, gap)


# ---------------------------------------------------------------------------
# The KKT checker itself, fed points whose residuals are known in closed form
# (Sec. IV-D relaxed LP).  A checker that clipped a residual the wrong way,
# dropped the budget term from the dual objective or ignored a sign would
# fail one of these.

def _cert(E, t, sigma, y_cov, y_budget, p):
    E = np.asarray(E, np.float64)
    return {"t": np.asarray(t, np.float64), "sigma": np.asarray(sigma, np.float64),
            "visible": E.max(0) > 0, "penalty": np.broadcast_to(np.asarray(p, np.float64), (E.shape[1],)).copy(),
            "duals": np.concatenate([np.asarray(y_cov, np.float64), [float(y_budget)]])}


def test_kkt_exact_certificate_budget_binding():
    """E = [[1, 1]], mu = 100, T = 40, p = 3: the budget binds, t = 40,
    sigma = (60, 60); sigma > 0 forces y_i = p = 3 and t > 0 forces
    1 - (3 + 3) + y_b = 0, so y_b = 5.  Primal 40 + 3 * 120 = 400 equals the
    dual 100 * 6 - 40 * 5 = 400: every residual is zero.  Without the budget
    term the dual objective would be 600 and the gap 200 / 1001."""
    E = [[1.0, 1.0]]
    prim, dual, gap = lp.kkt_residuals(E, _cert(E, [40.0], [60.0, 60.0], [3.0, 3.0], 5.0, 3.0), 100.0, 40.0)
    assert prim == 0.0 and dual == 0.0 and gap == 0.0


def test_kkt_exact_certificate_overcovered_element():
    """E = [[1, 2]], mu = 100, T large: t = 100 covers element 0 exactly and
    element 1 twice over (coverage 200 > mu must not count as a violation);
    y = (1, 0), y_b = 0: reduced cost of t is 1 - 1 = 0, of sigma p - y >= 0,
    primal 100 = dual 100 * 1."""
    E = [[1.0, 2.0]]
    prim, dual, gap = lp.kkt_residuals(E, _cert(E, [100.0], [0.0, 0.0], [1.0, 0.0], 0.0, 5.0), 100.0, 1e6)
    assert prim == 0.0 and dual == 0.0 and gap == 0.0


def test_kkt_detects_a_short_coverage_row():
    """Element 0 covered 1 % short: the primal residual is that shortfall."""
    E = [[1.0, 2.0]]
    prim, _, _ = lp.kkt_residuals(E, _cert(E, [99.0], [0.0, 0.0], [1.0, 0.0], 0.0, 5.0), 100.0, 1e6)
    assert abs(prim - 1.0) <= 1e-12 and prim > 1e-3


def test_kkt_detects_an_exceeded_budget():
    E = [[1.0, 1.0]]
    prim, _, _ = lp.kkt_residuals(E, _cert(E, [40.5], [59.5, 59.5], [3.0, 3.0], 5.0, 3.0), 100.0, 40.0)
    assert abs(prim - 0.5) <= 1e-12 and prim > 1e-3


def test_kkt_detects_a_budget_dual_with_the_wrong_sign():
    """y_b = -5 instead of 5: dual infeasible (y >= 0 and the reduced cost of
    t, 1 - 6 - 5 = -10) and the dual objective 800 no longer meets 400."""
    E = [[1.0, 1.0]]
    prim, dual, gap = lp.kkt_residuals(E, _cert(E, [40.0], [60.0, 60.0], [3.0, 3.0], -5.0, 3.0), 100.0, 40.0)
    assert prim == 0.0
    assert abs(dual - 10.0) <= 1e-12 and abs(gap - 400.0 / 1201.0) <= 1e-12


def test_kkt_detects_a_dual_above_the_penalty():
    """y_0 = 4 > p = 3 makes the reduced cost of sigma_0 negative."""
    E = [[1.0, 1.0]]
    _, dual, _ = lp.kkt_residuals(E, _cert(E, [40.0], [60.0, 60.0], [4.0, 3.0], 5.0, 3.0), 100.0, 40.0)
    assert abs(dual - 1.0) <= 1e-12


def test_kkt_detects_a_suboptimal_feasible_point():
    """A feasible but wasteful plan (t = 150 where 100 suffices) with the
    optimal duals: feasible on both sides, but the gap is 50 / 251."""
    E = [[1.0, 2.0]]
    prim, dual, gap = lp.kkt_residuals(E, _cert(E, [150.0], [0.0, 0.0], [1.0, 0.0], 0.0, 5.0), 100.0, 1e6)
    assert prim == 0.0 and dual == 0.0 and abs(gap - 50.0 / 251.0) <= 1e-12


def test_kkt_detects_perturbed_highs_solutions():
    """HiGHS' optimum on the box room certifies; the same point with one
    coverage row 1 % short, with the budget dual's sign flipped, or with
    dwell times past T_max does not (each residual > 1e-3)."""
    w = wl.box_room()
    E, _ = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power)
    # half the unconstrained plan's total time: the budget binds, y_b > 0
    t_max = 0.5 * float(lp.solve(E, mu_min=280.0, t_max=3.6e5)["t"].sum())
    sol = lp.solve(E, mu_min=280.0, t_max=t_max)
    assert max(lp.kkt_residuals(E, sol, 280.0, t_max)) <= 1e-6
    assert sol["duals"][-1] > 1e-3
    vis = sol["visible"]
    # one covered (sigma = 0) row 1 % short: lower sigma of an element whose
    # coverage comes from t, by reducing the dwell time of its best pose
    bad = {**sol, "t": sol["t"].copy(), "sigma": sol["sigma"].copy()}
    cov = E[:, vis].T @ sol["t"] + sol["sigma"][vis]
    i = int(np.flatnonzero(vis)[np.argmax((sol["sigma"][vis] == 0.0) & (cov <= 280.0 * (1 + 1e-9)))])
    bad["sigma"][i] -= 0.01 * 280.0 if bad["sigma"][i] >= 2.8 else 0.0
    if bad["sigma"][i] == sol["sigma"][i]:
        k = int(np.argmax(E[:, i] * (sol["t"] > 0)))
        bad["t"][k] -= 0.01 * 280.0 / E[k, i]
    assert lp.kkt_residuals(E, bad, 280.0, t_max)[0] > 1e-3
    flipped = {**sol, "duals": sol["duals"].copy()}
    flipped["duals"][-1] = -flipped["duals"][-1]
    r = lp.kkt_residuals(E, flipped, 280.0, t_max)
    assert r[1] > 1e-3 and r[2] > 1e-3
    over = {**sol, "t": sol["t"] * (1.0 + 1e-3) + 1.0 / len(sol["t"])}
    assert lp.kkt_residuals(E, over, 280.0, t_max)[0] > 1e-3
