"""Pose-ranker reference -- TEST INFRASTRUCTURE ONLY.

The ranker is not part of the paper; it prunes candidate poses before the
irradiance matrix of Sec. III-B / IV-C is assembled, and the relaxed LP of
Sec. IV-D on the full candidate set is the reference for it.  This module restates its
definition plainly, in FP64, so that the GPU kernels can be checked:

features(verts, tris, poses, h)
    From q = (x, y, z + h) (z = 0 for 2-D poses) cast 256 rays along the
    equal-area direction set: direction j = 16 b + a has azimuth
    2 pi (a + 1/2) / 16 and vertical cosine -1 + 2 (b + 1/2) / 16.  Each ray
    takes its closest triangle hit (brute force over every triangle,
    Moller-Trumbore); a hit at distance r whose triangle normal makes cosine
    cos with the ray adds (4 pi / 256) r^2 / max(|cos|, 0.05) to bin
    8 d + c, d = number of distance edges (0.5, 1, 1.5, 2, 3, 4, 6 m) not
    above r, c = min(7, floor(8 |cos|)).  Features = log1p(bin sums).

mlp_forward / mlp_loss_grad / adam_step
    A ReLU MLP 64 -> 128 -> 128 -> 1 whose parameters are one flat vector
    W1[h1][d], b1[h1], W2[h2][h1], b2[h2], W3[h2], b3; the loss is the mean
    binary cross-entropy with logits; Adam with bias correction.  The layer
    sizes are arguments so that finite differences can pin the gradient on
    a tiny network.
"""
from __future__ import annotations

import math

import numpy as np

DIST_EDGES = np.array([0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0])
N_RAYS = 256


def directions() -> np.ndarray:
    """The 256 unit ray directions, row j = 16 b + a."""
    j = np.arange(N_RAYS)
    a, b = j % 16, j // 16
    phi = 2.0 * math.pi * (a + 0.5) / 16.0
    cz = -1.0 + 2.0 * (b + 0.5) / 16.0
    r = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([r * np.cos(phi), r * np.sin(phi), cz], axis=1)


def unit_normals(verts, tris) -> np.ndarray:
    V = np.asarray(verts, np.float64)
    T = np.asarray(tris, np.int64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    m = np.cross(b - a, c - a)
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def closest_hits(verts, tris, q, dirs, eps_bary: float = 0.0):
    """Closest hit of each ray q + r u (r > 0) with the triangles.

    Returns (r [R], index [R], r_all [R, N]) where index = -1 for a miss and
    r_all holds every hit distance (inf for misses).  eps_bary > 0 widens the
    inside test (used to find rays that pass within that margin of an edge).
    """
    V = np.asarray(verts, np.float64)
    T = np.asarray(tris, np.int64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    e1, e2 = b - a, c - a                                    # [N, 3]
    u = np.asarray(dirs, np.float64)                         # [R, 3]
    p = np.cross(u[:, None, :], e2[None, :, :])              # [R, N, 3]
    det = np.einsum("rnk,nk->rn", p, e1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = np.asarray(q, np.float64)[None, :] - a           # [N, 3]
        bu = np.einsum("rnk,nk->rn", p, s) * inv
        qv = np.cross(s, e1)                                 # [N, 3]
        bv = np.einsum("rk,nk->rn", u, qv) * inv
        t = np.einsum("nk,nk->n", e2, qv)[None, :] * inv
    ok = (det != 0.0) & (bu >= -eps_bary) & (bv >= -eps_bary) & (bu + bv <= 1.0 + eps_bary) & (t > 0.0)
    r_all = np.where(ok, t, np.inf)
    idx = np.argmin(r_all, axis=1)
    r = r_all[np.arange(len(u)), idx]
    idx = np.where(np.isfinite(r), idx, -1)
    return r, idx, r_all


def _bin_and_weight(r, cosv):
    d = np.searchsorted(DIST_EDGES, r, side="right")
    c = np.minimum(7, np.floor(8.0 * cosv).astype(np.int64))
    w = (4.0 * math.pi / N_RAYS) * r * r / np.maximum(cosv, 0.05)
    return 8 * d + c, w


def features(verts, tris, poses, h: float = 0.9, with_ambiguity: bool = False, rel: float = 1e-5):
    """K x 64 features (FP64).  With with_ambiguity, also a [K] count of rays
    whose bin an FP32 evaluation could legitimately change: the ray passes
    within rel (barycentric) of a triangle edge, a second hit lies within a
    relative distance rel of the closest one with another bin, or the hit
    sits within rel of a distance or cosine bin edge."""
    P = np.asarray(poses, np.float64)
    K = P.shape[0]
    nrm = unit_normals(verts, tris)
    U = directions()
    F = np.zeros((K, 64))
    amb = np.zeros(K, np.int64)
    for k in range(K):
        z = P[k, 2] if P.shape[1] == 3 else 0.0
        q = np.array([P[k, 0], P[k, 1], z + h])
        r, idx, r_all = closest_hits(verts, tris, q, U)
        sums = np.zeros(64)
        hit = idx >= 0
        cosv = np.abs(np.einsum("rk,rk->r", U[hit], nrm[idx[hit]]))
        bins, w = _bin_and_weight(r[hit], cosv)
        for jj, (bb, ww) in zip(np.nonzero(hit)[0], zip(bins, w)):
            sums[bb] += ww
        F[k] = np.log1p(sums)
        if with_ambiguity:
            r2, idx2, r_all2 = closest_hits(verts, tris, q, U, eps_bary=rel)
            n_amb = 0
            for j in range(N_RAYS):
                if idx[j] != idx2[j] and (idx[j] < 0 or idx2[j] < 0 or not np.isclose(r[j], r2[j], rtol=rel)):
                    n_amb += 1
                    continue
                if idx[j] < 0:
                    continue
                cj = abs(U[j] @ nrm[idx[j]])
                bj, _ = _bin_and_weight(np.array([r[j]]), np.array([cj]))
                close = np.nonzero(np.abs(r_all2[j] - r[j]) <= rel * r[j])[0]
                for m in close:
                    cm = abs(U[j] @ nrm[m])
                    bm, _ = _bin_and_weight(np.array([r_all2[j][m]]), np.array([cm]))
                    if bm[0] != bj[0]:
                        n_amb += 1
                        break
                else:
                    if (np.min(np.abs(r[j] - DIST_EDGES)) <= rel * max(r[j], 1.0)
                            or abs(8.0 * cj - round(8.0 * cj)) <= 8.0 * rel):
                        n_amb += 1
        amb[k] = n_amb if with_ambiguity else 0
    return (F, amb) if with_ambiguity else F


def box_features_analytic(lo, hi, q) -> np.ndarray:
    """Features seen from q inside the empty axis-aligned box [lo, hi]: each
    ray's closest hit is the first wall plane it reaches, whose normal is that
    wall's axis (no triangles involved)."""
    lo, hi, q = (np.asarray(x, np.float64) for x in (lo, hi, q))
    U = directions()
    sums = np.zeros(64)
    for u in U:
        best, axis = np.inf, -1
        for ax in range(3):
            if u[ax] > 0:
                t = (hi[ax] - q[ax]) / u[ax]
            elif u[ax] < 0:
                t = (lo[ax] - q[ax]) / u[ax]
            else:
                continue
            if t < best:
                best, axis = t, ax
        b, w = _bin_and_weight(np.array([best]), np.array([abs(u[axis])]))
        sums[b[0]] += w[0]
    return np.log1p(sums)


# ------------------------------------------------------------------- MLP
def sizes_default():
    return (64, 128, 128)


def param_count(d=64, h1=128, h2=128) -> int:
    return h1 * d + h1 + h2 * h1 + h2 + h2 + 1


def unpack(params, d=64, h1=128, h2=128):
    p = np.asarray(params, np.float64)
    if p.size != param_count(d, h1, h2):
        raise ValueError("parameter vector has the wrong size")
    o = 0
    W1 = p[o:o + h1 * d].reshape(h1, d); o += h1 * d
    b1 = p[o:o + h1]; o += h1
    W2 = p[o:o + h2 * h1].reshape(h2, h1); o += h2 * h1
    b2 = p[o:o + h2]; o += h2
    W3 = p[o:o + h2]; o += h2
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), as FP64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(params, X, sizes=None, bf16: bool = False):
    """Scores [B] and the cache (z1, h1, z2, h2) of the forward pass."""
    d, h1n, h2n = sizes or sizes_default()
    W1, b1, W2, b2, W3, b3 = unpack(params, d, h1n, h2n)
    X = np.asarray(X, np.float64)
    rnd = (lambda a: bf16_round(a)) if bf16 else (lambda a: a)
    if bf16:
        W1, W2, W3 = bf16_round(W1), bf16_round(W2), bf16_round(W3)
    z1 = rnd(X) @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = rnd(h1) @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    s = rnd(h2) @ W3 + b3
    return s, (X, z1, h1, z2, h2)


def bce_with_logits(s, y) -> np.ndarray:
    s = np.asarray(s, np.float64)
    y = np.asarray(y, np.float64)
    return np.maximum(s, 0.0) - s * y + np.log1p(np.exp(-np.abs(s)))


def mlp_loss_grad(params, X, y, sizes=None):
    """Mean BCE-with-logits loss and its gradient (flat, parameter layout)."""
    d, h1n, h2n = sizes or sizes_default()
    W1, b1, W2, b2, W3, b3 = unpack(params, d, h1n, h2n)
    s, (X, z1, h1, z2, h2) = mlp_forward(params, X, (d, h1n, h2n))
    y = np.asarray(y, np.float64)
    B = X.shape[0]
    loss = float(bce_with_logits(s, y).mean())
    ds = (1.0 / (1.0 + np.exp(-s)) - y) / B          # dL/ds
    gW3 = h2.T @ ds
    gb3 = ds.sum()
    dz2 = np.outer(ds, W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, g


def adam_step(params, m, v, grad, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected, 1-based step); returns new (p, m, v)."""
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * grad
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
