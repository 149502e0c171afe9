"""Target-subset irradiance and the autotuner, through the C ABI."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2103_14137_amd import uvc
from paper_2103_14137_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def room():
    w = W.batch_room(11, n_range=(4000, 6000), k_range=(90, 110))
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    poses = torch.from_numpy(np.ascontiguousarray(w.poses, np.float32)).cuda()
    yield w, sc, poses
    sc.close()


@pytest.mark.parametrize("path", ["lbvh", "brute"])
def test_target_columns_equal_dense_columns(room, path):
    w, sc, poses = room
    print(f"targets: N={w.N} K={w.K} path={path}", flush=True)
    E, vis = uvc.irradiance_dense(sc, poses, w.lamp, path=path, want_vis=True)
    rng = np.random.default_rng(4)
    for n in (1, 63, 64, 65, 1000, w.N):
        tg = rng.integers(0, w.N, size=n).astype(np.int32)
        if n > 2:
            tg[1] = tg[0]                     # a repeated element
        T = torch.from_numpy(tg).cuda()
        Et, vt = uvc.irradiance_targets(sc, poses, w.lamp, T, path=path, want_vis=True)
        assert torch.equal(Et, E[:, T.long()]), n
        assert torch.equal(vt, vis[:, T.long()]), n
    # every element in input order reproduces the whole matrix
    Et, _ = uvc.irradiance_targets(sc, poses, w.lamp, torch.arange(w.N, dtype=torch.int32, device="cuda"),
                                   path=path)
    assert torch.equal(Et, E)


def test_targets_reject_bad_indices(room):
    w, sc, poses = room
    for bad in (-1, w.N):
        T = torch.tensor([0, bad], dtype=torch.int32, device="cuda")
        with pytest.raises(uvc.UvcError):
            uvc.irradiance_targets(sc, poses, w.lamp, T)
    Et, _ = uvc.irradiance_targets(sc, poses, w.lamp, torch.empty(0, dtype=torch.int32, device="cuda"))
    assert Et.shape == (w.K, 0)


def test_autotune_table_roundtrip(room, tmp_path):
    w, sc, poses = room
    table = str(tmp_path / "tune.json")
    best = uvc.autotune(sc, poses, w.lamp, probe_poses=48, table_path=table)
    print("autotune:", best, flush=True)
    assert os.path.exists(table)
    with open(table) as f:
        tab = json.load(f)
    key = f"n{int(np.floor(np.log2(w.N)))}_s{w.lamp.n_src}"
    assert key in tab
    again = uvc.autotune(sc, poses, w.lamp, probe_poses=48, table_path=table)
    assert again == best
    E0, _ = uvc.irradiance_dense(sc, poses, w.lamp)
    E1, _ = uvc.irradiance_dense(sc, poses, w.lamp, path=best["path"], packet_poses=best["packet_poses"],
                                 waves=best["waves"], tile_tris=best["tile_tris"])
    assert torch.equal(E0, E1)
