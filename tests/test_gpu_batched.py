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
