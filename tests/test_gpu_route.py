"""Route stage on the GPU against the route reference: geodesic matrices
equal bit for bit (both take the smallest FP64 path sum), tours equal move
for move (same start, same moves, same tie rule), and the LP -> route plan
of the box room and the ward equals the reference on the same dwell
times."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import route as RT  # noqa: E402
from paper_2103_14137_amd import workloads as wl  # noqa: E402


@pytest.fixture(scope="module")
def uvc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_14137_amd import uvc as U
    return U


CELL = 0.05


@pytest.mark.parametrize("name,m", [("box_room", 40), ("ward", 120)])
def test_geodesics_and_tour_equal_reference(uvc, name, m):
    w = wl.CONFIGS[name]()
    free, x0, y0 = wl.occupancy(w, CELL)
    rng = np.random.default_rng(5)
    stops = w.poses[np.sort(rng.choice(w.K, m, replace=False))]
    D = uvc.route_geodesics(torch.from_numpy(free).cuda(), x0, y0, CELL, torch.from_numpy(stops).cuda())
    torch.cuda.synchronize()
    Dref = RT.geodesic_matrix(free, x0, y0, CELL, stops)
    Dg = D.cpu().numpy()
    assert np.array_equal(Dg, Dref), float(np.max(np.abs(Dg - Dref)))
    tour, L, moves = uvc.route_tour(D)
    tref, mref = RT.local_search(Dref)
    print(name, m, "moves", moves, mref, "length", L, flush=True)
    assert np.array_equal(tour, tref) and moves == mref
    assert L == RT.tour_length(Dref, tref)


def test_plan_after_lp_equals_reference(uvc):
    for name in ("box_room", "ward"):
        w = wl.CONFIGS[name]()
        sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
        poses = torch.from_numpy(w.poses).cuda()
        E, _ = uvc.irradiance_dense(sc, poses, w.lamp)
        sol = uvc.solve_lp(E, t_max=3.6e5, max_iter=300)
        free, x0, y0 = wl.occupancy(w, CELL)
        r = uvc.plan_route(poses, sol["t"], torch.from_numpy(free).cuda(), x0, y0, CELL, rel_threshold=1e-5)
        t = sol["t"].cpu().numpy()
        sel = np.nonzero(t > 1e-5 * t.sum())[0]
        Dref = RT.geodesic_matrix(free, x0, y0, CELL, w.poses[sel])
        tref, _ = RT.local_search(Dref)
        Lref = RT.tour_length(Dref, tref)
        print(name, "stops", len(sel), "tour", Lref, "m; plan", r["plan_time"], "s", flush=True)
        assert np.array_equal(r["stops"], sel[tref])
        assert r["length"] == Lref
        assert r["plan_time"] == pytest.approx(RT.plan_time(t, Lref), rel=1e-12)
        sc.close()


def test_route_errors(uvc):
    free = torch.ones((10, 10), dtype=torch.uint8, device="cuda")
    free[:, 5] = 0  # two disconnected halves
    st = torch.tensor([[1.5, 1.5], [8.5, 1.5]], dtype=torch.float32, device="cuda")
    with pytest.raises(uvc.UvcError, match="not connected"):
        uvc.route_geodesics(free, 0.0, 0.0, 1.0, st)
    st2 = torch.tensor([[5.5, 1.5]], dtype=torch.float32, device="cuda")
    with pytest.raises(uvc.UvcError, match="blocked"):
        uvc.route_geodesics(free, 0.0, 0.0, 1.0, st2)
    tour, L, mv = uvc.route_tour(torch.zeros((1, 1), dtype=torch.float64, device="cuda"))
    assert tour.tolist() == [0] and L == 0.0
