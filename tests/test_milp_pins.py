"""CPU pins of the MILP reference (Appendix I): on tiny instances its
optimum equals brute-force enumeration of visited sets and tours; with no
travel cost it equals the dwell-time LP plus nothing; its edges form one
loop through pose 0 that contains every pose with a dwell time."""
import numpy as np
import pytest

from oracle import milp


def _instance(seed, K, N):
    rng = np.random.default_rng(seed)
    E = rng.lognormal(0.0, 0.7, size=(K, N)) * (rng.uniform(size=(K, N)) < 0.5)
    E[:, E.max(0) == 0] = 0.0
    P = rng.uniform(0, 6, size=(K, 2))
    d = np.sqrt(((P[:, None] - P[None]) ** 2).sum(-1))
    return E, d


def _loop_ok(z, t):
    K = z.shape[0]
    succ = {k: int(np.argmax(z[k])) for k in range(K) if z[k].sum() > 0}
    assert 0 in succ
    seen, k = [0], succ[0]
    while k != 0:
        seen.append(k)
        k = succ[k]
    assert sorted(seen) == sorted(succ)  # one loop, no other cycles
    assert all(t[k] <= 1e-7 * max(1.0, t.sum()) or k in succ for k in range(K))


@pytest.mark.parametrize("seed", range(4))
def test_milp_equals_brute_force(seed):
    E, d = _instance(seed, 6, 12)
    sol = milp.solve(E, d, mu_min=10.0, v_max=0.5)
    bf = milp.brute_force(E, d, mu_min=10.0, v_max=0.5)
    assert sol["optimal"]
    assert sol["objective"] == pytest.approx(bf, rel=1e-7)
    _loop_ok(sol["z"], sol["t"])


def test_no_travel_cost_is_the_lp():
    E, d = _instance(7, 7, 15)
    sol = milp.solve(E, np.zeros_like(d), mu_min=10.0)
    lp = milp._lp_min_time(E, 10.0, range(7))
    assert sol["objective"] == pytest.approx(lp, rel=1e-7)
