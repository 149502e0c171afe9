"""Many rooms in one persistent launch (and from a hipGraph) produce exactly
the per-room results, which match the oracle."""
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


@pytest.fixture(scope="module")
def rooms():
    return [wl.batch_room(3 + r, n_range=(1500, 9000), k_range=(60, 400)) for r in range(7)]


def test_batched_equals_per_room_and_oracle(uvc, rooms):
    scenes = [uvc.Scene(w.mesh.verts, w.mesh.tris) for w in rooms]
    poses = [torch.from_numpy(w.poses).cuda() for w in rooms]
    lamp = rooms[0].lamp
    single = [uvc.irradiance_dense(sc, p, lamp, path="lbvh")[0] for sc, p in zip(scenes, poses)]
    b = uvc.Batch(scenes, poses, lamp)
    for mode in ("per_room", "persistent", "graph", "graph", "graph"):
        for e in b.E:
            e.fill_(-1.0)
        torch.cuda.synchronize()
        b.run(mode)
        torch.cuda.synchronize()
        x = torch.zeros(1000, device="cuda").sum()  # eager work between graph replays
        for r, (e, s1) in enumerate(zip(b.E, single)):
            assert torch.equal(e, s1), (mode, r)
    # oracle spot check on two rooms
    rng = np.random.default_rng(5)
    for r in (0, 4):
        w = rooms[r]
        pk = rng.integers(0, w.K, 300)
        pi = rng.integers(0, w.N, 300)
        E64, vis64 = ref.irradiance_pairs(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, pk, pi)
        tol = ref.entry_tolerance(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, vis64, pk, pi)
        Eg = b.E[r].cpu().numpy()[pk, pi].astype(np.float64)
        assert np.array_equal(Eg != 0, vis64 != 0)
        assert np.all(np.abs(Eg - E64) <= 1e-5 * E64 + tol)
    b.close()
    for sc in scenes:
        sc.close()


def test_full_size_batch_equals_per_room_and_oracle(uvc):
    """The full 64-room batched workload (rooms seeded 3..66, 2k-80k
    triangles and 500-8,000 poses each, log-uniform; ~1.2 M triangles and
    ~150 k poses in all, ~10.8 GB of E): one persistent launch and three
    hipGraph replays write exactly the bits of one launch per room, and
    sampled entries of the largest and the smallest room match the oracle."""
    rooms = wl.batch(3, 64)
    print(f"64 rooms: sum N={sum(w.N for w in rooms)} sum K={sum(w.K for w in rooms)}", flush=True)
    scenes = [uvc.Scene(w.mesh.verts, w.mesh.tris) for w in rooms]
    poses = [torch.from_numpy(w.poses).cuda() for w in rooms]
    b = uvc.Batch(scenes, poses, rooms[0].lamp)
    b.run("per_room")
    torch.cuda.synchronize()
    ref_E = [e.clone() for e in b.E]
    for mode in ("persistent", "graph", "graph", "graph"):
        for e in b.E:
            e.fill_(-1.0)
        b.run(mode)
        torch.cuda.synchronize()
        x = torch.zeros(1000, device="cuda").sum()  # eager work between graph replays
        for r, (e, s1) in enumerate(zip(b.E, ref_E)):
            assert torch.equal(e, s1), (mode, r)
        print(mode, "equal", flush=True)
    rng = np.random.default_rng(11)
    big = int(np.argmax([w.N for w in rooms]))
    small = int(np.argmin([w.N for w in rooms]))
    for r in (big, small):
        w = rooms[r]
        pk = np.concatenate([rng.integers(0, w.K, 400), np.full(128, rng.integers(0, w.K))])
        i0 = int(rng.integers(0, w.N - 128))
        pi = np.concatenate([rng.integers(0, w.N, 400), np.arange(i0, i0 + 128)])
        E64, vis64 = ref.irradiance_pairs(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, pk, pi)
        tol = ref.entry_tolerance(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, vis64, pk, pi)
        Eg = ref_E[r].cpu().numpy()[pk, pi].astype(np.float64)
        assert np.array_equal(Eg != 0, vis64 != 0), (r, int(np.sum((Eg != 0) != (vis64 != 0))))
        assert np.all(np.abs(Eg - E64) <= 1e-5 * E64 + tol), r
        assert int((vis64 != 0).sum()) > 20
    b.close()
    del ref_E
    for sc in scenes:
        sc.close()


def _table(entries):
    """A tuning table in the layout uvc_autotune writes."""
    import json
    return json.dumps({k: {"path": p, "packet_poses": tp, "waves": wv, "tile_tris": 512, "rays_per_s": 1.0}
                       for k, (p, tp, wv) in entries.items()})


def test_tuned_batch_equals_per_room(uvc, rooms):
    """A batch driven by a tuning table (a different packet shape and
    occupancy per size class) writes the bits of the untuned batch in every
    mode; the table is also honoured when registered and the batch asks for
    UVC_PATH_AUTO."""
    scenes = [uvc.Scene(w.mesh.verts, w.mesh.tris) for w in rooms]
    poses = [torch.from_numpy(w.poses).cuda() for w in rooms]
    lamp = rooms[0].lamp
    b0 = uvc.Batch(scenes, poses, lamp)
    b0.run("persistent")
    torch.cuda.synchronize()
    ref_E = [e.clone() for e in b0.E]
    b0.close()
    buckets = sorted({int(np.floor(np.log2(w.N))) for w in rooms})
    shapes = [(1, 4, 5), (1, 64, 8), (1, 32, 6), (1, 8, 5), (1, 1, 6)]
    table = _table({f"n{bk}_s8": shapes[q % len(shapes)] for q, bk in enumerate(buckets)})
    for how in ("argument", "registered"):
        if how == "argument":
            b = uvc.Batch(scenes, poses, lamp, tune_table=table)
        else:
            uvc.set_tune_table(table)
            b = uvc.Batch(scenes, poses, lamp, path="auto")
        for mode in ("persistent", "graph", "per_room"):
            for e in b.E:
                e.fill_(-1.0)
            b.run(mode)
            torch.cuda.synchronize()
            for r, (e, s1) in enumerate(zip(b.E, ref_E)):
                assert torch.equal(e, s1), (how, mode, r)
        b.close()
    uvc.set_tune_table(None)
    for sc in scenes:
        sc.close()


def test_registered_table_drives_auto_path(uvc):
    """With a registered table, UVC_PATH_AUTO takes the table's path for the
    scene's size class: the box room (1,052 triangles) goes to the hierarchy
    instead of the built-in brute-force rule (the counters show node
    visits), with the same bits; clearing the table restores the rule."""
    w = wl.box_room()
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(w.poses[:20].copy()).cuda()
    s0 = uvc.new_stats()
    E0, _ = uvc.irradiance_dense(sc, poses, w.lamp, path="auto", stats=s0)
    uvc.set_tune_table(_table({"n10_s1": (1, 16, 6)}))
    s1 = uvc.new_stats()
    E1, _ = uvc.irradiance_dense(sc, poses, w.lamp, path="auto", stats=s1)
    uvc.set_tune_table(None)
    s2 = uvc.new_stats()
    E2, _ = uvc.irradiance_dense(sc, poses, w.lamp, path="auto", stats=s2)
    torch.cuda.synchronize()
    assert uvc.stats_dict(s0)["nodes"] == 0 and uvc.stats_dict(s1)["nodes"] > 0 and uvc.stats_dict(s2)["nodes"] == 0
    assert torch.equal(E0, E1) and torch.equal(E0, E2)
    with pytest.raises(uvc.UvcError, match="invalid options"):
        uvc.set_tune_table(_table({"n10_s1": (1, 3, 6)}))
    sc.close()
