"""Pins of the ranker reference (oracle/ranker.py) against facts that do not
come from it: an analytic empty-box answer, finite differences, closed forms
of the loss and of Adam's first step, and hand-rounded bfloat16 values."""
import math

import numpy as np
import pytest

from oracle import ranker as R
from paper_2103_14137_amd import workloads as W


def test_directions_equal_area_and_unit():
    U = R.directions()
    assert U.shape == (256, 3)
    assert np.allclose(np.linalg.norm(U, axis=1), 1.0, atol=1e-15)
    # 16 bands of equal height 1/8 in the vertical cosine, 16 rays each: by
    # Archimedes' hat-box theorem every cell covers 4 pi / 256 steradians
    z, counts = np.unique(np.round(U[:, 2], 12), return_counts=True)
    assert np.allclose(z, -1.0 + (np.arange(16) + 0.5) / 8.0, atol=1e-12)
    assert np.all(counts == 16)
    assert abs(U.sum(axis=0)).max() < 1e-12


@pytest.mark.parametrize("q", [(1.3, 0.7, 0.9), (0.4, 3.1, 1.7), (2.2, 2.9, 0.31)])
def test_features_empty_box_match_wall_planes(q):
    """Closest hits against the triangulated empty box equal the first wall
    plane each ray reaches (computed without any triangle)."""
    lo, hi = (0.0, 0.0, 0.0), (3.0, 4.0, 2.5)
    verts, tris = W.box_surface(lo, hi, (6, 8, 5), inward=True)
    F = R.features(verts, tris, np.array([[q[0], q[1]]]), h=q[2])
    A = R.box_features_analytic(lo, hi, q)
    assert np.allclose(F[0], A, rtol=1e-12, atol=1e-12)
    assert F[0].max() > 0


def test_features_single_facing_triangle():
    """One big triangle z = 2 above the origin: only upward rays hit it, at
    r = 2 / u_z with |cos| = u_z."""
    verts = np.array([[-100.0, -100.0, 2.0], [100.0, -100.0, 2.0], [0.0, 100.0, 2.0]])
    tris = np.array([[0, 1, 2]])
    F = R.features(verts, tris, np.array([[0.0, 0.0]]), h=0.0)
    U = R.directions()
    sums = np.zeros(64)
    for u in U:
        if u[2] > 0:
            r = 2.0 / u[2]
            x, y = r * u[0], r * u[1]
            # inside the triangle (it covers a 100 m region around the axis)
            assert abs(x) < 60 and abs(y) < 60 or r > 6
            d = int(np.sum(np.array([0.5, 1, 1.5, 2, 3, 4, 6]) <= r))
            c = min(7, int(8 * u[2]))
            sums[8 * d + c] += 4 * math.pi / 256 * r * r / max(u[2], 0.05)
    assert np.allclose(F[0], np.log1p(sums), rtol=1e-12, atol=1e-12)


def test_features_nothing_to_hit():
    verts = np.array([[0.0, 0.0, -1.0], [1.0, 0.0, -1.0], [0.0, 1.0, -1.0]]) + np.array([50.0, 50.0, 0.0])
    F = R.features(verts, np.array([[0, 1, 2]]), np.array([[0.0, 0.0]]), h=0.5)
    assert np.all(F == 0)


def test_feature_ambiguity_flags_edge_rays():
    """A ray aimed at the vertical corner edge between two walls is flagged;
    a generic pose has no flagged rays."""
    lo, hi = (0.0, 0.0, 0.0), (2.0, 2.0, 2.0)
    verts, tris = W.box_surface(lo, hi, (2, 2, 2), inward=True)
    _, amb = R.features(verts, tris, np.array([[0.713, 1.291]]), h=0.937, with_ambiguity=True)
    assert amb[0] == 0
    U = R.directions()
    j = 16 * 8 + 1                       # azimuth 3 pi / 16 (x, y > 0), slightly upward
    u = U[j]
    corner = np.array([2.0, 2.0, 1.3])
    r = 1.1
    q = corner - r * u                   # the ray from q along u meets the edge x = y = 2
    assert np.all(q > 0) and np.all(q < 2)
    _, amb = R.features(verts, tris, np.array([[q[0], q[1]]]), h=q[2], with_ambiguity=True)
    assert amb[0] >= 1


def _finite_diff(f, p, h=1e-6):
    g = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        g[i] = (f(p + e) - f(p - e)) / (2 * h)
    return g


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    sizes = (4, 3, 3)
    n = R.param_count(*sizes)
    p = rng.normal(size=n)
    X = rng.normal(size=(7, 4))
    y = (rng.uniform(size=7) > 0.5).astype(float)
    loss, g = R.mlp_loss_grad(p, X, y, sizes)
    fd = _finite_diff(lambda q: R.mlp_loss_grad(q, X, y, sizes)[0], p)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))
    assert np.all(np.isfinite(g)) and loss > 0


def test_mlp_layout_by_hand():
    """Hand-computed forward pass of a 2 -> 2 -> 1 -> 1 network."""
    sizes = (2, 2, 1)
    # W1 = [[1, 2], [3, 4]], b1 = [0.5, -100], W2 = [[2, 1]], b2 = [1], W3 = [3], b3 = 0.25
    p = np.array([1, 2, 3, 4, 0.5, -100, 2, 1, 1, 3, 0.25], float)
    assert p.size == R.param_count(*sizes)
    s, _ = R.mlp_forward(p, np.array([[1.0, 1.0]]), sizes)
    # z1 = [3.5, -93] -> h1 = [3.5, 0]; z2 = 8 -> h2 = 8; s = 24.25
    assert s[0] == 24.25


def test_bce_closed_forms():
    n = R.param_count()
    X = np.random.default_rng(1).normal(size=(10, 64))
    y = np.array([1, 0, 1, 1, 0, 0, 0, 1, 0, 0], float)
    loss, g = R.mlp_loss_grad(np.zeros(n), X, y)
    assert loss == pytest.approx(math.log(2.0), rel=1e-15)
    assert g[-1] == pytest.approx(np.mean(0.5 - y), rel=1e-15)
    assert np.all(g[:-1] == 0.0)   # every hidden unit is dead at zero weights
    assert R.bce_with_logits(np.array([40.0]), np.array([1.0]))[0] == pytest.approx(math.exp(-40.0), rel=1e-12)
    assert R.bce_with_logits(np.array([-40.0]), np.array([1.0]))[0] == pytest.approx(40.0 + math.exp(-40.0))


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = R.adam_step(np.ones(4), np.zeros(4), np.zeros(4), g, lr=0.01, step=1)
    expect = 1.0 - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, expect, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_by_hand():
    one = 1.0
    ulp = 2.0 ** -7
    vals = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + 0.75 * ulp, -3.0, 0.0, 2.0 ** -130])
    r = R.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                  # tie -> even mantissa
    assert r[2] == one + 2 * ulp        # tie -> even mantissa
    assert r[3] == one + ulp            # above the tie
    assert r[4] == -3.0 and r[5] == 0.0
    assert r[6] == 2.0 ** -130          # an FP32 subnormal whose low half is already zero
