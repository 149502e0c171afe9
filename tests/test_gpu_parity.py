"""Parity of the HIP irradiance path with the CPU oracle (run on an MI355X).

Bars: visibility bits identical; E within |E32 - E64| <= 1e-5 * E64 +
1e-5 * sum_j V_j P_j / (4 pi r_j^2) (FP32 storage and arithmetic against the
FP64 oracle; the second term covers grazing cosines); centroids bit-exact;
CSR identical to the dense path bit for bit.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2103_14137_amd import workloads as wl  # noqa: E402


@pytest.fixture(scope="module")
def uvc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_14137_amd import uvc as U
    return U


_cache = {}


def _workload(name):
    if name not in _cache:
        _cache[name] = wl.CONFIGS[name]()
    return _cache[name]


def _check_entries(E32, vis32, E64, vis64, tol_abs, what=""):
    vis32 = np.asarray(vis32).astype(np.uint32)
    bad = np.nonzero(vis32 != vis64)[0]
    assert bad.size == 0, f"{what}: {bad.size} visibility mismatches, first at {bad[:5]}"
    err = np.abs(E32.astype(np.float64) - E64)
    lim = 1e-5 * E64 + tol_abs
    worst = int(np.argmax(err - lim))
    assert np.all(err <= lim), f"{what}: E error {err[worst]} > {lim[worst]} at {worst}"
    assert np.array_equal(E32 != 0, vis64 != 0), f"{what}: nonzero pattern differs from visibility"


def test_elements_match_oracle(uvc):
    for name in ("box_room", "ward"):
        w = _workload(name)
        sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
        c, n, a = (t.cpu().numpy() for t in sc.elements())
        c64, n64, a64, _ = ref.elements(w.mesh.verts, w.mesh.tris)
        assert np.array_equal(c.view(np.uint32), c64.view(np.uint32)), name
        assert np.allclose(n, n64, atol=2e-7, rtol=0), name
        assert np.allclose(a, a64, rtol=2e-7, atol=0), name
        sc.close()


@pytest.mark.parametrize("path", ["brute", "lbvh"])
def test_box_room_full_parity(uvc, path):
    """The whole 200 x 1,052 matrix against the oracle."""
    w = _workload("box_room")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses).cuda()
    E, vis = uvc.irradiance_dense(sc, poses, w.lamp, path=path, want_vis=True)
    torch.cuda.synchronize()
    E64, vis64 = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power)
    tol = ref.entry_tolerance(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, vis64)
    _check_entries(E.cpu().numpy().ravel(), vis.cpu().numpy().ravel(), E64.ravel(), vis64.ravel(), tol, path)
    sc.close()


def test_paths_bit_identical_and_band_independent(uvc):
    """Brute force and hierarchy, and every decision band (including all
    decisions in FP64), produce the same bits and the same values."""
    w = _workload("ward")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses[::250].copy()).cuda()
    E1, v1 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True)
    E2, v2 = uvc.irradiance_dense(sc, poses, w.lamp, path="brute", want_vis=True)
    E3, v3 = uvc.irradiance_dense(sc, poses[:4].contiguous(), w.lamp, path="lbvh", want_vis=True,
                                  band_scale=float("inf"))
    E4, v4 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2) and torch.equal(E1, E2)
    assert torch.equal(v1[:4], v3) and torch.equal(E1[:4], E3)
    assert torch.equal(v1, v4) and torch.equal(E1, E4)  # deterministic
    for tp in (1, 4, 16, 64):  # packet shapes: same bits, same values
        E5, v5 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True, packet_poses=tp)
        assert torch.equal(v1, v5) and torch.equal(E1, E5), tp
    for wv in (5, 6, 8):  # occupancy variants of the same kernel
        E7, v7 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True, waves=wv)
        assert torch.equal(v1, v7) and torch.equal(E1, E7), wv
    # walking every segment to its target instead of using the near lists
    E6, v6 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True, flags=uvc.FLAG_NO_NEAR)
    assert torch.equal(v1, v6) and torch.equal(E1, E6)
    # without the per-lane last-occluder test, and without both shortcuts
    for fl in (uvc.FLAG_NO_CACHE, uvc.FLAG_NO_CACHE | uvc.FLAG_NO_NEAR):
        E8, v8 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True, flags=fl)
        assert torch.equal(v1, v8) and torch.equal(E1, E8), fl
    sc.close()


def test_last_occluder_test_is_used_and_exact(uvc):
    """On a room with obstacles the last-occluder test fires and finds
    blocked segments; with it off no such test is counted and every bit of
    the result is unchanged (the test is the predicate on one triangle)."""
    w = _workload("ward")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses[::50].copy()).cuda()
    s_on, s_off = uvc.new_stats(), uvc.new_stats()
    E1, v1 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True, stats=s_on)
    E2, v2 = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True, stats=s_off,
                                  flags=uvc.FLAG_NO_CACHE)
    torch.cuda.synchronize()
    on, off = uvc.stats_dict(s_on), uvc.stats_dict(s_off)
    assert torch.equal(v1, v2) and torch.equal(E1, E2)
    assert on["cache"] > 0 and 0 < on["cache_hit"] <= on["cache"]
    assert off["cache"] == 0 and off["cache_hit"] == 0
    assert on["visible"] == off["visible"] and on["rays"] == off["rays"]
    # a lane found blocked by its last occluder skips the walk
    assert on["nodes"] < off["nodes"]
    sc.close()


def test_ward_sampled_parity_full_launch(uvc):
    """Full 5,000 x ~52k ward matrix from exactly the launch the benchmark
    times (hierarchy path, default packet shape and occupancy, no visibility
    output, no counters): sampled blocks and random entries against the
    oracle.  A second launch with the visibility output must write the same
    E and the oracle's bits; the work counters come from a third, separate
    instrumented launch."""
    w = _workload("ward")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses).cuda()
    E = torch.empty((w.K, w.N), dtype=torch.float32, device="cuda")
    uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", out=E)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1234)
    ks = np.sort(rng.choice(w.K, 8, replace=False))
    i0 = rng.integers(0, w.N - 256)
    kk, ii = np.meshgrid(ks, np.arange(i0, i0 + 256), indexing="ij")
    pk = np.concatenate([kk.ravel(), rng.integers(0, w.K, 1500)])
    pi = np.concatenate([ii.ravel(), rng.integers(0, w.N, 1500)])
    E64, vis64 = ref.irradiance_pairs(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, pk, pi)
    tol = ref.entry_tolerance(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, vis64, pk, pi)
    Eg = E.cpu().numpy()[pk, pi]
    err = np.abs(Eg.astype(np.float64) - E64)
    assert np.all(err <= 1e-5 * E64 + tol), float(np.max(err - (1e-5 * E64 + tol)))
    assert np.array_equal(Eg != 0, vis64 != 0), int(np.sum((Eg != 0) != (vis64 != 0)))
    # the same launch with the visibility output: identical E, the oracle's bits
    E2, vis = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", want_vis=True)
    torch.cuda.synchronize()
    assert torch.equal(E, E2)
    del E2
    _check_entries(Eg, vis.cpu().numpy()[pk, pi], E64, vis64, tol, "ward")
    # work counters from a separate instrumented launch
    stats = uvc.new_stats()
    E3, _ = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh", stats=stats)
    torch.cuda.synchronize()
    assert torch.equal(E, E3)
    del E3
    st = uvc.stats_dict(stats)
    assert st["rays"] > 0 and st["nodes"] > 0 and st["tris"] > 0
    vall = vis.cpu().numpy().astype(np.uint32)
    popc = np.unpackbits(vall.view(np.uint8)).sum()
    assert st["visible"] == popc
    sc.close()


def test_translated_room_far_from_origin(uvc):
    """The box room moved far from the origin (+1,000 m in x, -1,000 m in y,
    +500 m in z; FP32 spacing there is 6e-5 m), with 3-D poses lifted by the
    same amount: every bit and every entry still matches the oracle on both
    paths.  Far from the origin the box padding and the decision bands are
    relative to coordinates ~1e3 times larger than the room."""
    w = _workload("box_room")
    off = np.array([1000.0, -1000.0, 500.0], np.float32)
    verts = (w.mesh.verts + off).astype(np.float32)
    p3 = np.concatenate([w.poses + off[:2], np.full((w.K, 1), off[2], np.float32)], 1).astype(np.float32)
    E64, vis64 = ref.irradiance_dense(verts, w.mesh.tris, p3, w.lamp.dz, w.lamp.power)
    tol = ref.entry_tolerance(verts, w.mesh.tris, p3, w.lamp.dz, w.lamp.power, vis64)
    assert int((vis64 != 0).sum()) > 0.2 * vis64.size
    sc = uvc.Scene(verts, w.mesh.tris)
    for path in ("lbvh", "brute"):
        E, vis = uvc.irradiance_dense(sc, torch.from_numpy(p3).cuda(), w.lamp, path=path, want_vis=True)
        torch.cuda.synchronize()
        _check_entries(E.cpu().numpy().ravel(), vis.cpu().numpy().ravel(), E64.ravel(), vis64.ravel(), tol,
                       f"translated {path}")
    sc.close()


def test_ragged_sizes_and_tiny_meshes(uvc):
    """Meshes of 1, 2, 3, 65 and 130 triangles (partial tiles and packets)."""
    w = _workload("box_room")
    rng = np.random.default_rng(9)
    for n in (1, 2, 3, 65, 130):
        sel = np.sort(rng.choice(w.N, n, replace=False))
        tris = w.mesh.tris[sel]
        poses = w.poses[:7]
        for path in ("brute", "lbvh"):
            sc = uvc.Scene(w.mesh.verts, tris)
            E, vis = uvc.irradiance_dense(sc, torch.from_numpy(poses).cuda(), w.lamp, path=path, want_vis=True)
            E64, vis64 = ref.irradiance_dense(w.mesh.verts, tris, poses, w.lamp.dz, w.lamp.power)
            tol = ref.entry_tolerance(w.mesh.verts, tris, poses, w.lamp.dz, w.lamp.power, vis64)
            _check_entries(E.cpu().numpy().ravel(), vis.cpu().numpy().ravel(), E64.ravel(), vis64.ravel(), tol,
                           f"n={n} {path}")
            sc.close()


def test_pose_dim3_and_empty_inputs(uvc):
    w = _workload("box_room")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    p3 = np.concatenate([w.poses[:5], np.full((5, 1), 0.25, np.float32)], 1)
    E, vis = uvc.irradiance_dense(sc, torch.from_numpy(p3).cuda(), w.lamp, want_vis=True)
    E64, vis64 = ref.irradiance_dense(w.mesh.verts, w.mesh.tris, p3, w.lamp.dz, w.lamp.power)
    tol = ref.entry_tolerance(w.mesh.verts, w.mesh.tris, p3, w.lamp.dz, w.lamp.power, vis64)
    _check_entries(E.cpu().numpy().ravel(), vis.cpu().numpy().ravel(), E64.ravel(), vis64.ravel(), tol, "pose3")
    E0, _ = uvc.irradiance_dense(sc, torch.zeros((0, 2), dtype=torch.float32, device="cuda"), w.lamp)
    assert E0.shape == (0, w.N)
    rp, col, val = uvc.irradiance_csr(sc, torch.zeros((0, 2), dtype=torch.float32, device="cuda"), w.lamp)
    assert rp.cpu().tolist() == [0] and col.numel() == 0
    sc.close()
    empty = uvc.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    E, _ = uvc.irradiance_dense(empty, torch.from_numpy(w.poses[:3]).cuda(), w.lamp)
    assert E.shape == (3, 0)
    empty.close()


def test_invalid_inputs_rejected(uvc):
    w = _workload("box_room")
    v = w.mesh.verts.copy()
    v[3, 1] = np.nan
    with pytest.raises(uvc.UvcError, match="non-finite"):
        uvc.Scene(v, w.mesh.tris)
    v = w.mesh.verts.copy()
    v[3, 0] = 1e8
    with pytest.raises(uvc.UvcError, match="2\\^26"):
        uvc.Scene(v, w.mesh.tris)
    t = w.mesh.tris.copy()
    t[5, 2] = len(w.mesh.verts)
    with pytest.raises(uvc.UvcError, match="outside"):
        uvc.Scene(w.mesh.verts, t)
    t = w.mesh.tris.copy()
    t[7] = [t[7, 0], t[7, 0], t[7, 1]]
    with pytest.raises(uvc.UvcError, match="zero area"):
        uvc.Scene(w.mesh.verts, t)
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses[:4]).cuda()
    with pytest.raises(uvc.UvcError, match="1..32"):
        uvc.irradiance_dense(sc, poses, uvc.Lamp(np.zeros(0, np.float32), np.zeros(0, np.float32)))
    with pytest.raises(uvc.UvcError, match="positive"):
        uvc.irradiance_dense(sc, poses, uvc.Lamp([1.0], [-5.0]))
    bad = poses.clone()
    bad[2, 0] = float("inf")
    with pytest.raises(uvc.UvcError, match="not finite"):
        uvc.irradiance_dense(sc, bad, w.lamp)
    far = poses.clone()
    far[1, 1] = 1e4
    with pytest.raises(uvc.UvcError, match="farther"):
        uvc.irradiance_dense(sc, far, w.lamp)
    sc.close()


@pytest.mark.parametrize("name,stride", [("box_room", 1), ("ward", 100)])
def test_csr_matches_dense(uvc, name, stride):
    w = _workload(name)
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses[::stride].copy()).cuda()
    E, vis = uvc.irradiance_dense(sc, poses, w.lamp, want_vis=True)
    rp, col, val = uvc.irradiance_csr(sc, poses, w.lamp)
    torch.cuda.synchronize()
    K, N = E.shape
    dense = torch.zeros((K, N), dtype=torch.float32, device="cuda")
    rows = torch.repeat_interleave(torch.arange(K, device="cuda"), rp[1:] - rp[:-1])
    dense[rows, col.long()] = val
    assert torch.equal(dense, E)
    assert int(rp[-1]) == int((vis != 0).sum())
    # ascending columns within rows
    c = col.cpu().numpy()
    r = rp.cpu().numpy()
    for k in range(0, K, max(1, K // 16)):
        assert np.all(np.diff(c[r[k]:r[k + 1]]) > 0)
    sc.close()


def test_hierarchy_invariants(uvc):
    w = _workload("ward")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    nodes, perm, codes = sc.export_bvh()
    N = w.N
    assert np.all(np.diff(codes.astype(np.int64)) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(N))
    refs = nodes[:, 12:14].view(np.int32).ravel()
    leaves = np.sort(~refs[refs < 0])
    internal = np.sort(refs[refs >= 0])
    assert np.array_equal(leaves, np.arange(N))
    assert np.array_equal(internal, np.arange(1, N - 1))
    # every child box contains its subtree: leaf boxes contain their triangle
    V = w.mesh.verts[w.mesh.tris[perm]]  # [N,3,3] in slot order
    tlo, thi = V.min(1), V.max(1)
    for side, off in ((0, 0), (1, 6)):
        ref_ = nodes[:, 12 + side].view(np.int32)
        lo, hi = nodes[:, off:off + 3], nodes[:, off + 3:off + 6]
        leaf = ref_ < 0
        slot = ~ref_[leaf]
        assert np.all(lo[leaf] <= tlo[slot]) and np.all(hi[leaf] >= thi[slot])
        inn = ~leaf
        child = ref_[inn]
        clo = np.minimum(nodes[child, 0:3], nodes[child, 6:9])
        chi = np.maximum(nodes[child, 3:6], nodes[child, 9:12])
        assert np.all(lo[inn] <= clo) and np.all(hi[inn] >= chi)
    info = sc.info()
    assert 2 <= info["bvh_depth"] <= 64
    sc.close()


def test_power_of_two_scaling(uvc):
    w = _workload("box_room")
    s = np.float32(0.25)
    sc0 = uvc.Scene(w.mesh.verts, w.mesh.tris)
    sc1 = uvc.Scene(w.mesh.verts * s, w.mesh.tris)
    E0, v0 = uvc.irradiance_dense(sc0, torch.from_numpy(w.poses).cuda(), w.lamp, want_vis=True)
    lamp1 = uvc.Lamp(w.lamp.dz * s, w.lamp.power)
    E1, v1 = uvc.irradiance_dense(sc1, torch.from_numpy(w.poses * s).cuda(), lamp1, want_vis=True)
    torch.cuda.synchronize()
    assert torch.equal(v0, v1)
    # every operation of the path scales exactly by powers of two (no
    # subnormals here): lengths by 1/4, the cosine numerator by 1/4, the
    # inverse cube of the distance by 64, so E by exactly 16
    assert torch.equal(E1 * 0.0625, E0)
    sc0.close()
    sc1.close()


def test_floorplan_csr_sampled_parity_full_size(uvc):
    """The ~488k-triangle, 20,000-pose floor plan as CSR, in the benchmark's
    launch configuration: sampled rows (a contiguous block, nonzeros drawn
    from each row, uniform columns) against the oracle entry by entry.  The
    CSR stores an entry exactly when some source sees the element, so the
    nonzero pattern is checked against the oracle's visibility."""
    w = _workload("floorplan")
    print(f"floorplan N={w.N} K={w.K}", flush=True)
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses).cuda()
    rp, col, val = uvc.irradiance_csr(sc, poses, w.lamp, path="lbvh")
    torch.cuda.synchronize()
    r = rp.cpu().numpy()
    nnz = int(r[-1])
    assert nnz == col.numel() and nnz > 0 and np.all(np.diff(r) >= 0)
    rng = np.random.default_rng(77)
    rows = np.sort(rng.choice(w.K, 48, replace=False))
    pk, pi, got = [], [], []
    for q, k in enumerate(rows):
        c = col[r[k]:r[k + 1]].cpu().numpy()
        v = val[r[k]:r[k + 1]].cpu().numpy()
        assert np.all(np.diff(c) > 0) and np.all(v > 0)
        picks = [rng.integers(0, w.N, 16)]
        if c.size:
            picks.append(c[rng.integers(0, c.size, 16)])
        if q < 2:
            i0 = int(rng.integers(0, w.N - 512))
            picks.append(np.arange(i0, i0 + 512))
        ii = np.concatenate(picks)
        at = np.searchsorted(c, ii)
        hit = (at < c.size) & (c[np.minimum(at, max(c.size - 1, 0))] == ii) if c.size else np.zeros(ii.size, bool)
        got.append(np.where(hit, v[np.minimum(at, max(c.size - 1, 0))] if c.size else 0.0, 0.0))
        pk.append(np.full(ii.size, k))
        pi.append(ii)
    pk, pi, got = np.concatenate(pk), np.concatenate(pi), np.concatenate(got).astype(np.float32)
    E64, vis64 = ref.irradiance_pairs(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, pk, pi)
    tol = ref.entry_tolerance(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, vis64, pk, pi)
    assert np.array_equal(got != 0, vis64 != 0), int(np.sum((got != 0) != (vis64 != 0)))
    err = np.abs(got.astype(np.float64) - E64)
    assert np.all(err <= 1e-5 * E64 + tol), float(np.max(err - (1e-5 * E64 + tol)))
    assert int((vis64 != 0).sum()) > 500
    sc.close()
