"""Adversarial segments through the GPU path: every pose's segments cross an
occluder quad exactly at its shared diagonal, its edges or its vertices (up
to FP32 rounding of the targets), where FP32 decisions are least reliable.
The visibility bits must equal the oracle's; with the decision bands set to
zero (pure FP32 decisions) they must not, which shows the bands matter."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402


def _scene(seed, n_poses=48, per_pose=8):
    rng = np.random.default_rng(seed)
    quad = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], np.float64) * 2.0 - 1.0
    quad[:, 2] = 0.0
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    quad = quad @ q.T
    nrm = np.cross(quad[1] - quad[0], quad[3] - quad[0])
    nrm /= np.linalg.norm(nrm)
    verts = [quad.astype(np.float32)]
    tris = [np.array([[0, 1, 2], [0, 2, 3]], np.int32)]
    poses = []
    nv = 4
    for k in range(n_poses):
        O = 0.3 * rng.normal(size=3) + nrm * rng.uniform(1.0, 3.0)
        O = O.astype(np.float32).astype(np.float64)
        poses.append(O)
        for _ in range(per_pose):
            kind = rng.integers(4)
            if kind == 0:
                s = rng.uniform(0.05, 0.95)
                P = (1 - s) * quad[0] + s * quad[2]
            elif kind == 1:
                e = rng.integers(4)
                s = rng.uniform(0.0, 1.0)
                P = (1 - s) * quad[e] + s * quad[(e + 1) % 4]
            elif kind == 2:
                P = quad[rng.integers(4)]
            else:
                P = quad[0] + rng.uniform(-0.1, 1.1) * (quad[1] - quad[0]) + rng.uniform(-0.1, 1.1) * (quad[3] - quad[0])
            T = P - (O - P) * rng.uniform(0.2, 1.0)
            d = O - T
            d /= np.linalg.norm(d)
            e1 = np.cross(d, [0.0, 0.0, 1.0] if abs(d[2]) < 0.9 else [1.0, 0.0, 0.0])
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(d, e1)
            u = 1e-3
            a, b, c = T + u * e1, T + u * e2, T - u * (e1 + e2)
            if np.dot(np.cross(b - a, c - a), d) < 0:  # face the pose
                b, c = c, b
            verts.append(np.array([a, b, c], np.float32))
            tris.append(np.array([[nv, nv + 1, nv + 2]], np.int32))
            nv += 3
    V = np.concatenate(verts).astype(np.float32)
    T_ = np.concatenate(tris).astype(np.int32)
    return V, T_, np.array(poses, np.float32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adversarial_segments_match_oracle(seed):
    from paper_2103_14137_amd import uvc
    V, T, poses = _scene(seed)
    dz = np.zeros(1, np.float32)
    pw = np.full(1, 80.0, np.float32)
    lamp = uvc.Lamp(dz, pw)
    sc = uvc.Scene(V, T)
    P = torch.from_numpy(poses).cuda()
    E64, vis64 = ref.irradiance_dense(V, T, poses, dz, pw)
    assert (vis64 != 0).sum() > 0 and (vis64 == 0).sum() > 0
    mism0 = 0
    for path in ("lbvh", "brute"):
        E, vis = uvc.irradiance_dense(sc, P, lamp, path=path, want_vis=True)
        v = vis.cpu().numpy().astype(np.uint32)
        assert np.array_equal(v, vis64), (path, int((v != vis64).sum()))
        E0, vis0 = uvc.irradiance_dense(sc, P, lamp, path=path, want_vis=True, band_scale=0.0)
        mism0 += int((vis0.cpu().numpy().astype(np.uint32) != vis64).sum())
    print(f"seed {seed}: band-0 mismatches {mism0}", flush=True)
    sc.close()
    test_adversarial_segments_match_oracle.mismatches = getattr(test_adversarial_segments_match_oracle,
                                                                "mismatches", 0) + mism0


def test_zero_band_shows_mismatches():
    """Summed over more seeds: pure FP32 decisions disagree with the oracle on
    these segments somewhere, so the FP64 bands are doing real work."""
    from paper_2103_14137_amd import uvc
    dz = np.zeros(1, np.float32)
    pw = np.full(1, 80.0, np.float32)
    lamp = uvc.Lamp(dz, pw)
    total = 0
    for seed in range(3, 9):
        V, T, poses = _scene(seed)
        sc = uvc.Scene(V, T)
        P = torch.from_numpy(poses).cuda()
        _, vis64 = ref.irradiance_dense(V, T, poses, dz, pw)
        _, vis0 = uvc.irradiance_dense(sc, P, lamp, path="lbvh", want_vis=True, band_scale=0.0)
        total += int((vis0.cpu().numpy().astype(np.uint32) != vis64).sum())
        sc.close()
    print("band-0 mismatches over 6 scenes:", total, flush=True)
    assert total > 0
