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
