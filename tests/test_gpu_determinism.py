"""Every kernel family run twice on the same inputs gives the same bits
(fixed-order reductions, no atomics in any value path)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_repeated_runs_are_bit_identical():
    from paper_2103_14137_amd import ranker as RK
    from paper_2103_14137_amd import uvc
    from paper_2103_14137_amd import workloads as W
    w = W.batch_room(31, n_range=(3000, 4000), k_range=(100, 140))
    runs = []
    for _ in range(2):
        sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
        P = torch.from_numpy(np.ascontiguousarray(w.poses)).cuda()
        E, vis = uvc.irradiance_dense(sc, P, w.lamp, want_vis=True)
        rp, col, val = uvc.irradiance_csr(sc, P, w.lamp)
        feat = uvc.ranker_features(sc, P)
        lp = uvc.solve_lp(E)
        params = torch.from_numpy(RK.init_params(3)).cuda()
        m = torch.zeros_like(params)
        v = torch.zeros_like(params)
        y = torch.from_numpy((np.arange(w.K) % 7 == 0).astype(np.float32)).cuda()
        loss = uvc.ranker_train_step(params, m, v, feat, y, None, 1e-3, 1)
        plan = uvc.plan_ranked(sc, P, w.lamp, mode="mlp", params=params, keep_frac=0.2)
        runs.append([E, vis, rp, col, val, feat, lp["t"], lp["sigma"], lp["y"], params, m, v,
                     torch.tensor([loss]), plan["t"]])
        sc.close()
    for a, b in zip(*runs):
        assert torch.equal(a.cpu(), b.cpu())
