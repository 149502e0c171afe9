"""CPU pins of the oracle's area-integrated irradiance (Sec. IV-C, the
visibility-cube procedure: per cube-map pixel the closest triangle collects
the pixel's power; the entry is collected power over triangle area).

Pins: power is conserved in closed scenes (every pixel lands on a front
face); an unoccluded triangle collects P Omega / (4 pi) with Omega from the
Van Oosterom-Strackee formula, with an error that falls as the cube
resolution grows; a small far triangle tends to the centroid entry
P cos / (4 pi r^2); a triangle in the shadow of an opaque square collects
nothing, one facing away from the source collects nothing; sources add; a
constant emission table scales exactly."""
import math

import numpy as np
import pytest

from oracle import ref
from paper_2103_14137_amd import workloads as wl


def _solid_angle(O, a, b, c):
    """Van Oosterom-Strackee: solid angle of triangle abc seen from O."""
    a, b, c = (np.asarray(x, np.float64) - np.asarray(O, np.float64) for x in (a, b, c))
    la, lb, lc = (np.linalg.norm(x) for x in (a, b, c))
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * math.atan2(num, den)


def _tri_mesh(*tris):
    v = np.asarray([p for t in tris for p in t], np.float32)
    t = np.arange(len(v), dtype=np.int32).reshape(-1, 3)
    return v, t


@pytest.mark.parametrize("R", [8, 16])
def test_power_is_conserved_in_closed_rooms(R):
    w = wl.box_room()
    _, _, area, _ = ref.elements(w.mesh.verts, w.mesh.tris)
    E, amb, landed = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:3], w.lamp.dz, w.lamp.power, R)
    assert np.allclose(landed, 80.0, rtol=1e-12, atol=0)
    assert np.allclose((E * area).sum(1), 80.0, rtol=1e-12, atol=0)
    lamp = wl.tower_lamp()
    E, amb, landed = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[3:5] * 0.9 + 0.2, lamp.dz, lamp.power,
                                         R)
    assert np.allclose(landed, 160.0, rtol=1e-12, atol=0)


def test_unoccluded_triangle_collects_its_solid_angle():
    """Source at (0, 0, 1) (a 2-D pose at the origin, dz = 1), one large
    triangle below it facing up: F A -> P Omega / (4 pi), error shrinking
    with the resolution."""
    tri = [(-1.3, -0.7, 0.0), (1.6, -0.9, 0.0), (0.2, 1.4, 0.0)]
    v, t = _tri_mesh(tri)
    _, _, area, _ = ref.elements(v, t)
    om = _solid_angle((0.0, 0.0, 1.0), *[np.asarray(p, np.float32) for p in tri])
    expect = 80.0 * om / (4 * math.pi)
    errs = []
    for R in (16, 64, 256):
        E, _, landed = ref.area_irradiance(v, t, np.zeros((1, 2), np.float32), [1.0], [80.0], R)
        got = E[0, 0] * area[0]
        assert got == pytest.approx(landed[0], rel=1e-12)
        errs.append(abs(got - expect) / expect)
    assert errs[2] < 0.01 and errs[2] < errs[1] < errs[0], errs


def test_small_far_triangle_tends_to_the_centroid_entry():
    h = 0.05
    c0 = np.array([1.2, 0.7, 0.0])
    tri = [c0 + (-h, -h, 0), c0 + (h, -h * 0.5, 0), c0 + (0, h, 0)]
    v, t = _tri_mesh(tri)
    E, _, _ = ref.area_irradiance(v, t, np.zeros((1, 2), np.float32), [2.0], [80.0], 512)
    Ec, vis = ref.irradiance_pairs(v, t, np.zeros((1, 2), np.float32), [2.0], [80.0], [0], [0])
    assert vis[0] == 1
    assert E[0, 0] == pytest.approx(Ec[0], rel=0.03)


def test_shadow_back_side_and_superposition():
    # receiver below an opaque square (two triangles) that covers its whole solid angle
    rec = [(-0.2, -0.2, 0.0), (0.2, -0.2, 0.0), (0.0, 0.25, 0.0)]
    sq = [[(-1, -1, 0.5), (1, -1, 0.5), (1, 1, 0.5)], [(-1, -1, 0.5), (1, 1, 0.5), (-1, 1, 0.5)]]  # facing up
    v, t = _tri_mesh(rec, *sq)
    E, _, landed = ref.area_irradiance(v, t, np.zeros((1, 2), np.float32), [1.0], [80.0], 32)
    assert E[0, 0] == 0.0 and E[0, 1] > 0 and E[0, 2] > 0
    # a triangle wound to face away from the source collects nothing
    back = [(-1.3, -0.7, 0.0), (0.2, 1.4, 0.0), (1.6, -0.9, 0.0)]
    vb, tb = _tri_mesh(back)
    E, _, landed = ref.area_irradiance(vb, tb, np.zeros((1, 2), np.float32), [1.0], [80.0], 32)
    assert E[0, 0] == 0.0 and landed[0] == 0.0
    # two sources add (sums in a different order: rounding only)
    w = wl.box_room()
    E2, _, _ = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [0.6, 1.4], [30.0, 50.0], 8)
    Ea, _, _ = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [0.6], [30.0], 8)
    Eb, _, _ = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [1.4], [50.0], 8)
    assert np.allclose(E2, Ea + Eb, rtol=1e-12, atol=1e-300)


def test_constant_table_scales_exactly_and_shield_halves():
    w = wl.box_room()
    E0, a0, l0 = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [1.0], [80.0], 8)
    E1, a1, l1 = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [1.0], [80.0], 8, profile=[0.5, 0.5])
    assert np.array_equal(E1, 0.5 * E0) and np.array_equal(a0, a1)
    # an upward-only and a downward-only source split the cube (R even: no pixel centre at d_z = 0)
    Eu, _, lu = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [1.0], [80.0], 8, up_mask=1)
    Ed, _, ld = ref.area_irradiance(w.mesh.verts, w.mesh.tris, w.poses[:2], [1.0], [80.0], 8, down_mask=1)
    assert np.allclose(lu + ld, 80.0, rtol=1e-12) and np.allclose(lu, 40.0, rtol=1e-12)
    assert np.allclose(Eu + Ed, E0, rtol=1e-12, atol=1e-300)
