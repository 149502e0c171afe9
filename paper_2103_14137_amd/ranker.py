"""Learned pose ranker: training, checkpoints and held-out evaluation.

Host orchestration only.  Features, labels (the irradiance matrix and the
relaxed dosage LP of Sec. IV-D), the forward and backward passes, Adam and
the ranked plan all run in libuvc kernels through the binding; this module
draws seeded rooms, shuffles sample indices, and reads and writes files.

Labels: a pose is positive when the full-candidate LP gives it a dwell time
above LABEL_REL times the plan's total dwell time.  The LP solver is an
interior point method, so poses outside the optimal support keep dwell
times near the solver tolerance instead of exact zeros; the relative
threshold separates the two.

Checkpoint format: one JSON header line (magic, parameter count, Adam step,
metadata), then the parameters, and optionally Adam's m and v, as raw
little-endian float32.

    python -m paper_2103_14137_amd.ranker train --out ranker.bin
    python -m paper_2103_14137_amd.ranker eval --weights ranker.bin
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import uvc, workloads

MAGIC = "uvc-ranker-v1"
LABEL_REL = 1e-5
FEATURE_HEIGHT = 0.9
# training / held-out rooms: the batched-room generator at reduced sizes
TRAIN_N_RANGE = (2000, 20000)
TRAIN_K_RANGE = (200, 1000)
TRAIN_SEED0 = 100_000
HELDOUT_SEED0 = 900_000


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights for the ReLU layers, small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    w1 = rng.normal(0.0, math.sqrt(2.0 / 64), size=(128, 64))
    w2 = rng.normal(0.0, math.sqrt(2.0 / 128), size=(128, 128))
    w3 = rng.normal(0.0, math.sqrt(1.0 / 128), size=128)
    p = np.concatenate([w1.ravel(), np.zeros(128), w2.ravel(), np.zeros(128), w3, [0.0]]).astype(np.float32)
    assert p.size == uvc.ranker_param_count()
    return p


def save_checkpoint(path: str, params, m=None, v=None, step: int = 0, meta: dict | None = None) -> None:
    arrs = [np.asarray(a, np.float32).reshape(-1) for a in (params, m, v) if a is not None]
    n = arrs[0].size
    if any(a.size != n for a in arrs):
        raise ValueError("params, m and v must have the same size")
    head = {"magic": MAGIC, "n_params": int(n), "has_adam": len(arrs) == 3, "step": int(step), "meta": meta or {}}
    with open(path, "wb") as f:
        f.write((json.dumps(head, sort_keys=True) + "\n").encode())
        for a in arrs:
            f.write(a.astype("<f4").tobytes())


def load_checkpoint(path: str) -> dict:
    with open(path, "rb") as f:
        head = json.loads(f.readline().decode())
        if head.get("magic") != MAGIC:
            raise ValueError(f"{path}: not a ranker checkpoint")
        n = int(head["n_params"])
        body = np.frombuffer(f.read(), dtype="<f4")
    k = 3 if head["has_adam"] else 1
    if body.size != k * n:
        raise ValueError(f"{path}: truncated checkpoint")
    out = {"params": body[:n].copy(), "step": int(head["step"]), "meta": head["meta"], "m": None, "v": None}
    if k == 3:
        out["m"], out["v"] = body[n:2 * n].copy(), body[2 * n:].copy()
    return out


def room(seed: int, n_range=TRAIN_N_RANGE, k_range=TRAIN_K_RANGE) -> workloads.Workload:
    return workloads.batch_room(seed, n_range=n_range, k_range=k_range)


def room_samples(w: workloads.Workload, mu_min: float = 280.0, t_max: float = 3.6e5, tol: float = 1e-9) -> dict:
    """Features and LP labels of one room (full candidate set)."""
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    try:
        poses = torch.from_numpy(np.ascontiguousarray(w.poses, np.float32)).cuda()
        feat = uvc.ranker_features(sc, poses, FEATURE_HEIGHT)
        E, _ = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh")
        lp = uvc.solve_lp(E, mu_min=mu_min, t_max=t_max, tol=tol, allow_notconv=True)
        t = lp["t"].cpu().numpy()
        y = (t > LABEL_REL * t.sum()).astype(np.float32)
        return {"feat": feat.cpu(), "y": y, "objective": lp["objective"], "converged": lp["converged"],
                "K": w.K, "N": w.N}
    finally:
        sc.close()


# ------------------------------------------------------------ label cache
# One JSON line per labelled room: how to regenerate it (seed and size
# ranges), a hash of the generated scene (mesh, poses, lamp) so that a
# regenerated room is checked to be the one that was labelled, and the
# label: the poses with a dwell time in the full-candidate LP.  Labels thus
# survive across runs; features are recomputed (one cheap kernel per room).
def scene_key(w: workloads.Workload) -> str:
    h = hashlib.sha1()
    for a in (w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:20]


def read_cache(path: str) -> dict:
    out = {}
    if path and os.path.exists(path):
        with open(path) as f:
            for line in f:
                line = line.strip()
                if line:
                    rec = json.loads(line)
                    out[(rec["seed"], tuple(rec["n_range"]), tuple(rec["k_range"]))] = rec
    return out


def label_record(seed: int, n_range, k_range, mu_min: float = 280.0, t_max: float = 3.6e5,
                 tol: float = 1e-9) -> dict:
    w = room(seed, tuple(n_range), tuple(k_range))
    t0 = time.time()
    d = room_samples(w, mu_min, t_max, tol)
    return {"seed": int(seed), "n_range": list(n_range), "k_range": list(k_range), "key": scene_key(w),
            "K": w.K, "N": w.N, "positives": np.nonzero(d["y"])[0].astype(int).tolist(),
            "objective": d["objective"], "converged": bool(d["converged"]), "seconds": time.time() - t0}


def cached_samples(rec: dict) -> tuple:
    """Features (recomputed) and labels of a cached room, after checking
    that the regenerated scene is the labelled one."""
    w = room(rec["seed"], tuple(rec["n_range"]), tuple(rec["k_range"]))
    if scene_key(w) != rec["key"]:
        raise ValueError(f"room {rec['seed']}: regenerated scene differs from the labelled one")
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    try:
        poses = torch.from_numpy(np.ascontiguousarray(w.poses, np.float32)).cuda()
        feat = uvc.ranker_features(sc, poses, FEATURE_HEIGHT).cpu()
    finally:
        sc.close()
    y = np.zeros(w.K, np.float32)
    y[np.asarray(rec["positives"], np.int64)] = 1.0
    return feat, y


def train(feat: torch.Tensor, y: np.ndarray, params=None, m=None, v=None, step0: int = 0, epochs: int = 30,
          batch: int = 1024, lr: float = 1e-3, seed: int = 0, log=None):
    """Adam on mean BCE; feat [S, 64] (any device), y [S].  Returns
    (params, m, v, step, epoch losses) as NumPy arrays / ints."""
    n = uvc.ranker_param_count()
    dev = torch.device("cuda")
    P = torch.from_numpy(np.asarray(params if params is not None else init_params(seed), np.float32)).to(dev)
    M = torch.from_numpy(np.asarray(m, np.float32)).to(dev) if m is not None else torch.zeros(n, device=dev)
    V = torch.from_numpy(np.asarray(v, np.float32)).to(dev) if v is not None else torch.zeros(n, device=dev)
    X = feat.to(dev, torch.float32).contiguous()
    Y = torch.from_numpy(np.asarray(y, np.float32)).to(dev)
    S = X.shape[0]
    rng = np.random.default_rng(seed)
    step = step0
    losses = []
    for ep in range(epochs):
        perm = rng.permutation(S).astype(np.int32)
        tot, cnt = 0.0, 0
        for b0 in range(0, S, batch):
            idx = torch.from_numpy(perm[b0:b0 + batch]).to(dev)
            step += 1
            loss = uvc.ranker_train_step(P, M, V, X, Y, idx, lr, step)
            tot += loss * idx.numel()
            cnt += idx.numel()
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {losses[-1]:.5f}")
    return P.cpu().numpy(), M.cpu().numpy(), V.cpu().numpy(), step, losses


def evaluate_room(w: workloads.Workload, params: np.ndarray, keep_frac: float = 0.1, bf16: bool = False,
                  modes=("mlp", "area"), mu_min: float = 280.0, t_max: float = 3.6e5, tol: float = 1e-9,
                  max_rounds: int = 20) -> dict:
    """Full-candidate plan vs pruned plans of one room.  Every LP uses the
    full matrix's default penalty p = 1.001 ||E||_F, and every plan is scored
    on the full E with it (uvc_plan_evaluate)."""
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    try:
        poses = torch.from_numpy(np.ascontiguousarray(w.poses, np.float32)).cuda()
        P = torch.from_numpy(np.asarray(params, np.float32)).cuda()
        full = uvc.plan_ranked(sc, poses, w.lamp, mode="none", mu_min=mu_min, t_max=t_max, tol=tol)
        p = full["penalty"]
        E, _ = uvc.irradiance_dense(sc, poses, w.lamp, path="lbvh")
        ref = uvc.plan_evaluate(E, full["t"], mu_min, penalty=p)
        out = {"room": w.name, "K": w.K, "N": w.N, "penalty": p, "full_objective": ref["objective"],
               "full_ms": full["ms_total"], "full_lp_iterations": full["lp_iterations"],
               "support": int(np.sum(full["t"].cpu().numpy() > LABEL_REL * float(full["t"].sum())))}
        for mode in modes:
            r = uvc.plan_ranked(sc, poses, w.lamp, mode=mode, params=P, bf16=bf16, keep_frac=keep_frac,
                                penalty=p, mu_min=mu_min, t_max=t_max, tol=tol, max_rounds=max_rounds)
            ev = uvc.plan_evaluate(E, r["t"], mu_min, penalty=p)
            out[mode] = {"objective": ev["objective"],
                         "gap": (ev["objective"] - ref["objective"]) / ref["objective"],
                         "fell_back": r["fell_back"], "n_kept": r["n_kept"], "n_added": r["n_added"],
                         "rounds": r["rounds"], "rounds_added": r["rounds_added"], "n_priced": r["n_priced"],
                         "n_dropped": r["n_dropped"],
                         "ms": r["ms_total"],
                         "lp_iterations": r["lp_iterations"],
                         "ms_parts": {k: r[k] for k in ("ms_features", "ms_score", "ms_E", "ms_lp", "ms_price",
                                                        "ms_fallback")}}
        del E
        return out
    finally:
        sc.close()


def summarize(results: list, modes=("mlp", "area")) -> dict:
    s = {"rooms": len(results)}
    full_ms = np.array([r["full_ms"] for r in results])
    for mode in modes:
        g = np.array([r[mode]["gap"] for r in results])
        fb = np.array([r[mode]["fell_back"] for r in results])
        ms = np.array([r[mode]["ms"] for r in results])
        rounds = np.array([r[mode]["rounds"] for r in results])
        added = np.array([r[mode]["n_added"] for r in results])
        s[mode] = {"gap_mean": float(g.mean()), "gap_max": float(g.max()),
                   "gap_le_2pct": float(np.mean(g <= 0.02)), "fallback_rate": float(fb.mean()),
                   "rounds_mean": float(rounds.mean()), "added_mean": float(added.mean()),
                   "ms_total": float(ms.sum()), "speedup_vs_full": float(full_ms.sum() / max(ms.sum(), 1e-9))}
    s["full_ms_total"] = float(full_ms.sum())
    return s


def _main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2103_14137_amd.ranker")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train", help="generate labelled rooms and train")
    t.add_argument("--rooms", type=int, default=256)
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=1024)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--resume", default=None, help="checkpoint with Adam state to continue from")
    t.add_argument("--out", required=True)
    g = sub.add_parser("labels", help="label rooms into a cache (resumable)")
    g.add_argument("--cache", required=True)
    g.add_argument("--seed0", type=int, default=TRAIN_SEED0)
    g.add_argument("--rooms", type=int, default=256)
    g.add_argument("--n-range", type=int, nargs=2, default=list(TRAIN_N_RANGE))
    g.add_argument("--k-range", type=int, nargs=2, default=list(TRAIN_K_RANGE))
    g.add_argument("--time-limit", type=float, default=0.0, help="stop starting rooms after this many seconds")
    tc = sub.add_parser("train-cached", help="train on the rooms of label caches")
    tc.add_argument("--cache", nargs="+", required=True)
    tc.add_argument("--epochs", type=int, default=40)
    tc.add_argument("--batch", type=int, default=1024)
    tc.add_argument("--lr", type=float, default=1e-3)
    tc.add_argument("--seed", type=int, default=0)
    tc.add_argument("--out", required=True)
    e = sub.add_parser("eval", help="held-out evaluation of a checkpoint")
    e.add_argument("--results", default=None, help="JSON lines of per-room results (resumable)")
    e.add_argument("--modes", nargs="+", default=["mlp", "area"])
    e.add_argument("--time-limit", type=float, default=0.0)
    e.add_argument("--weights", required=True)
    e.add_argument("--rooms", type=int, default=64)
    e.add_argument("--keep", type=float, default=0.1)
    e.add_argument("--bf16", action="store_true")
    e.add_argument("--json", default=None)
    e.add_argument("--n-range", type=int, nargs=2, default=list(TRAIN_N_RANGE))
    e.add_argument("--k-range", type=int, nargs=2, default=list(TRAIN_K_RANGE))
    e.add_argument("--seed0", type=int, default=HELDOUT_SEED0)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if a.cmd == "labels":
        have = read_cache(a.cache)
        t0 = time.time()
        done = 0
        with open(a.cache, "a") as f:
            for r in range(a.rooms):
                key = (a.seed0 + r, tuple(a.n_range), tuple(a.k_range))
                if key in have:
                    continue
                if a.time_limit and time.time() - t0 > a.time_limit:
                    log(f"time limit: stopping after {done} new rooms")
                    break
                rec = label_record(a.seed0 + r, a.n_range, a.k_range)
                f.write(json.dumps(rec) + "\n")
                f.flush()
                done += 1
                log(f"room {a.seed0 + r}: K={rec['K']} N={rec['N']} positives {len(rec['positives'])} "
                    f"({rec['seconds']:.1f} s)")
        log(f"labelled {done} new rooms in {time.time() - t0:.1f} s; cache has {len(read_cache(a.cache))}")
        return 0
    if a.cmd == "train-cached":
        feats, ys, rooms, skipped = [], [], 0, 0
        for path in a.cache:
            for rec in read_cache(path).values():
                if not rec["converged"]:  # labels of an LP that hit its iteration limit are left out
                    skipped += 1
                    continue
                fx, yy = cached_samples(rec)
                feats.append(fx)
                ys.append(yy)
                rooms += 1
        X = torch.cat(feats)
        Y = np.concatenate(ys)
        log(f"{rooms} rooms ({skipped} unconverged left out), {X.shape[0]} poses, positives {Y.mean():.4f}")
        p, m, v, step, losses = train(X, Y, None, None, None, 0, a.epochs, a.batch, a.lr, a.seed, log)
        meta = {"rooms": rooms, "skipped_unconverged": skipped, "samples": int(X.shape[0]),
                "positives": float(Y.mean()), "epochs": a.epochs, "batch": a.batch, "lr": a.lr,
                "final_loss": losses[-1], "label_rel": LABEL_REL, "feature_height": FEATURE_HEIGHT,
                "caches": [os.path.basename(c) for c in a.cache]}
        save_checkpoint(a.out, p, m, v, step, meta)
        log(json.dumps(meta))
        return 0
    if a.cmd == "train":
        feats, ys = [], []
        t0 = time.time()
        for r in range(a.rooms):
            d = room_samples(room(TRAIN_SEED0 + r))
            feats.append(d["feat"])
            ys.append(d["y"])
            if (r + 1) % 16 == 0:
                log(f"labelled {r + 1}/{a.rooms} rooms ({time.time() - t0:.1f} s), "
                    f"positives {np.concatenate(ys).mean():.4f}")
        X = torch.cat(feats)
        Y = np.concatenate(ys)
        ck = load_checkpoint(a.resume) if a.resume else None
        p, m, v, step, losses = train(X, Y, ck["params"] if ck else None, ck["m"] if ck else None,
                                      ck["v"] if ck else None, ck["step"] if ck else 0, a.epochs, a.batch, a.lr,
                                      a.seed, log)
        meta = {"rooms": a.rooms, "samples": int(X.shape[0]), "positives": float(Y.mean()), "epochs": a.epochs,
                "batch": a.batch, "lr": a.lr, "final_loss": losses[-1], "label_rel": LABEL_REL,
                "feature_height": FEATURE_HEIGHT, "n_range": TRAIN_N_RANGE, "k_range": TRAIN_K_RANGE,
                "seed0": TRAIN_SEED0}
        save_checkpoint(a.out, p, m, v, step, meta)
        log(json.dumps(meta))
        return 0
    ck = load_checkpoint(a.weights)
    modes = tuple(a.modes)
    res = []
    if a.results and os.path.exists(a.results):
        with open(a.results) as f:
            res = [json.loads(line) for line in f if line.strip()]
    done = {x["room"] for x in res}
    t0 = time.time()
    for r in range(a.rooms):
        w = room(a.seed0 + r, tuple(a.n_range), tuple(a.k_range))
        if w.name in done:
            continue
        if a.time_limit and time.time() - t0 > a.time_limit:
            log(f"time limit: {len(res)} rooms evaluated")
            break
        x = evaluate_room(w, ck["params"], a.keep, a.bf16, modes=modes)
        res.append(x)
        if a.results:
            with open(a.results, "a") as f:
                f.write(json.dumps(x) + "\n")
        log(f"room {r}: K={x['K']} N={x['N']} full {x['full_ms']:.0f} ms | " +
            " | ".join(f"{m} gap {x[m]['gap']:.1e} rounds {x[m]['rounds']} kept {x[m]['n_kept']} {x[m]['ms']:.0f} ms"
                       for m in modes))
    s = summarize(res, modes)
    log(json.dumps(s))
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"summary": s, "rooms": res}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(_main())
