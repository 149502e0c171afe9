"""CPU pins of the oracle's lamp variants (Sec. IV-C: a lamp as point
sources; each source may carry its own emission pattern): an angular
emission table over cos(theta) (theta from the upward vertical through the
source, linear interpolation between equally spaced nodes) and hemisphere
masks (a source that emits only above or only below its own height).

Pins: the uniform table reduces to the plain oracle bit for bit; a constant
table scales it exactly; closed forms directly below and above a source and
for a linear table at a lateral offset; in an empty convex box (every
front-facing element visible) the weight equals NumPy's linear interpolation
of the table; the entry is linear in the table; the two hemisphere masks
split the plain result."""
import math

import numpy as np
import pytest

from oracle import ref
from paper_2103_14137_amd import workloads as wl


def _empty_box(cell=0.4, L=(4.0, 4.0, 3.0)):
    mb = wl.MeshBuilder()
    mb.add(*wl.box_surface((0, 0, 0), L, [wl._ncells(x, cell) for x in L], inward=True))
    return mb.mesh()


@pytest.fixture(scope="module")
def box():
    mesh = _empty_box()
    rng = np.random.default_rng(3)
    poses = np.stack([rng.uniform(0.5, 3.5, 6), rng.uniform(0.5, 3.5, 6)], 1).astype(np.float32)
    return mesh, poses


def test_uniform_and_constant_tables(box):
    mesh, poses = box
    lamp = wl.tower_lamp()
    E0, v0 = ref.irradiance_dense(mesh.verts, mesh.tris, poses, lamp.dz, lamp.power)
    E1, v1 = ref.irradiance_dense(mesh.verts, mesh.tris, poses, lamp.dz, lamp.power, profile=[1.0, 1.0, 1.0])
    assert np.array_equal(E0, E1) and np.array_equal(v0, v1)
    Eh, vh = ref.irradiance_dense(mesh.verts, mesh.tris, poses, lamp.dz, lamp.power, profile=[0.5] * 5)
    assert np.array_equal(vh, v0)
    assert np.array_equal(Eh, 0.5 * E0)


def test_closed_forms_below_above_and_linear_table(box):
    mesh, _ = box
    c, _, _, _ = ref.elements(mesh.verts, mesh.tris)
    prof = [0.25, 0.6, 0.9, 0.4, 0.75]
    h = 1.25
    fl = int(np.argmin(np.abs(c[:, 2]) + np.abs(c[:, 0] - 1.7) + np.abs(c[:, 1] - 2.2)))
    ce = int(np.argmin(np.abs(c[:, 2] - 3.0) + np.abs(c[:, 0] - 1.7) + np.abs(c[:, 1] - 2.2)))
    assert c[fl, 2] == 0.0 and c[ce, 2] == 3.0 and c[ce, 0] == c[fl, 0] and c[ce, 1] == c[fl, 1]
    pose = np.array([[c[fl, 0], c[fl, 1]]], np.float32)
    E, vis = ref.irradiance_pairs(mesh.verts, mesh.tris, pose, [h], [80.0], [0, 0], [fl, ce], profile=prof)
    assert vis.tolist() == [1, 1]
    assert abs(E[0] - 80.0 * prof[0] / (4 * math.pi * h * h)) <= 1e-13 * E[0]          # straight down
    d = 3.0 - h
    assert abs(E[1] - 80.0 * prof[-1] / (4 * math.pi * d * d)) <= 1e-13 * E[1]          # straight up
    # linear table [0, 1]: w = (1 + cos theta) / 2 with cos theta = -h / r on the floor
    floor = np.nonzero(c[:, 2] == 0.0)[0]
    i = int(floor[np.argmin(np.abs(c[floor, 0] - 0.7) + np.abs(c[floor, 1] - 0.9))])
    pxy = np.array([[float(c[i, 0]) + 0.66, float(c[i, 1]) + 0.88]], np.float32)
    E, vis = ref.irradiance_pairs(mesh.verts, mesh.tris, pxy, [1.0], [80.0], [0], [i], profile=[0.0, 1.0])
    dx, dy = float(pxy[0, 0]) - float(c[i, 0]), float(pxy[0, 1]) - float(c[i, 1])
    r = math.sqrt(dx * dx + dy * dy + 1.0)
    expect = 80.0 * 0.5 * (1.0 - 1.0 / r) * (1.0 / r) / (4 * math.pi * r * r)
    assert vis[0] == 1 and abs(E[0] - expect) <= 1e-12 * expect


def test_weight_is_linear_interpolation_in_empty_box(box):
    """One source in an empty convex box: every front-facing element is
    visible, and the entry is the uniform entry times the table interpolated
    at cos(theta) (NumPy's np.interp on the node grid)."""
    mesh, poses = box
    c, _, _, _ = ref.elements(mesh.verts, mesh.tris)
    rng = np.random.default_rng(8)
    prof = rng.uniform(0.1, 2.0, 9)
    dz = np.array([1.1], np.float32)
    E0, v0 = ref.irradiance_dense(mesh.verts, mesh.tris, poses, dz, [80.0])
    E1, v1 = ref.irradiance_dense(mesh.verts, mesh.tris, poses, dz, [80.0], profile=prof)
    assert np.array_equal(v0, v1) and v0.sum() > 0.4 * v0.size
    src = np.concatenate([poses.astype(np.float64), np.full((len(poses), 1), float(dz[0]))], 1)
    d = c.astype(np.float64)[None] - src[:, None]
    cos_t = d[..., 2] / np.linalg.norm(d, axis=-1)
    w = np.interp(cos_t, np.linspace(-1.0, 1.0, prof.size), prof.astype(np.float32).astype(np.float64))
    on = v0 != 0
    assert np.allclose(E1[on], w[on] * E0[on], rtol=1e-12, atol=0)
    assert np.all(E1[~on] == 0)


def test_linear_in_the_table(box):
    """Tables on a 1/64 grid, so that t1 + 2 t2 is exact in FP32: the
    entries combine the same way."""
    mesh, poses = box
    lamp = wl.tower_lamp()
    rng = np.random.default_rng(4)
    t1 = (rng.integers(0, 64, 7) / 64.0).astype(np.float32)
    t2 = (rng.integers(1, 64, 7) / 64.0).astype(np.float32)
    t3 = (t1 + 2 * t2).astype(np.float32)
    E1, _ = ref.irradiance_dense(mesh.verts, mesh.tris, poses, lamp.dz, lamp.power, profile=t1)
    E2, _ = ref.irradiance_dense(mesh.verts, mesh.tris, poses, lamp.dz, lamp.power, profile=t2)
    E3, _ = ref.irradiance_dense(mesh.verts, mesh.tris, poses, lamp.dz, lamp.power, profile=t3)
    assert np.allclose(E3, E1 + 2 * E2, rtol=1e-12, atol=0)


def test_hemisphere_masks_split_the_plain_result():
    w = wl.box_room()
    lamp = wl.tower_lamp(n=3, spacing=0.5)
    poses = w.poses[:5]
    E0, v0 = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, poses, lamp.dz, lamp.power)
    Eu, vu = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, poses, lamp.dz, lamp.power, up_mask=0b111)
    Ed, vd = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, poses, lamp.dz, lamp.power, down_mask=0b111)
    c, _, _, _ = ref.elements(w.mesh.verts, w.mesh.tris)
    at_height = np.isin(c[:, 2], np.asarray(lamp.dz, np.float32))[None].repeat(len(poses), 0)
    assert not np.any(vu & vd)
    ok = ~at_height
    assert np.array_equal((vu | vd)[ok], v0[ok])
    assert np.allclose((Eu + Ed)[ok], E0[ok], rtol=1e-15, atol=0)
    # one source masked, the others untouched
    E1, v1 = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, poses, lamp.dz, lamp.power, up_mask=0b010)
    assert np.array_equal(v1 & 0b101, v0 & 0b101)
    assert np.all(((v1 >> 1) & 1) <= ((v0 >> 1) & 1))


def test_invalid_lamp_variants_rejected(box):
    mesh, poses = box
    with pytest.raises(ValueError):
        ref.irradiance_pairs(mesh.verts, mesh.tris, poses, [1.0], [80.0], [0], [0], profile=[1.0])
    with pytest.raises(ValueError):
        ref.irradiance_pairs(mesh.verts, mesh.tris, poses, [1.0], [80.0], [0], [0], up_mask=1, down_mask=1)
