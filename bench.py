#!/usr/bin/env python3
"""Irradiance-matrix assembly throughput on one MI355X.

One step = one pass of the whole hot path over the ward workload (8 x 6 x 3 m
room, 6 beds + 10 cuboids, 52,488 triangles, 5,000 lamp poses, tower lamp of
8 point sources x 20 W), inputs already resident in HBM:
  build the scene from the device-resident mesh (surface elements, Morton
  codes, radix sort, hierarchy, refit) and assemble the dense 5,000 x 52,488
  FP32 irradiance matrix (front-facing test, occlusion segment per front-facing
  (pose, source, element) triple, inverse-square cosine term, sum over the 8
  sources).

Prints one JSON line.  value = occlusion rays per second (rays = front-facing
triples, each of which casts one occlusion segment); entries/s is reported
beside it.  roofline: algorithmic FLOPs of the dominant kernel per launch
(24 per hierarchy node visit, 40 per segment/triangle test, 20 per evaluated
(pose, source, element) entry term; counts from an instrumented launch)
divided by its HIP-event-timed duration.  cpu_baseline: the FP64 CPU oracle
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "occlusion rays/s + E entries/s (fraction of FP32 peak); ranked vs full plan time @≤2% gap"
PEAK_FP32 = 157.3          # TFLOP/s, MI355X vector FP32 (packed)
PEAK_FP32_UNPACKED = 78.6  # TFLOP/s, without packed FP32
PEAK_HBM = 8000.0          # GB/s
FLOP_NODE, FLOP_TRI, FLOP_ENTRY = 24, 40, 20
KERNEL = "k_irr_lbvh"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("irradiance.hip", "scene.hip", "uvc_common.hpp"):
        with open(os.path.join(ROOT, "paper_2103_14137_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_launch_bytes_unused=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "k_irr_lbvh_ward_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, n_poses=32, n_elems=1024, seed=2024):
    """The oracle (FP64 brute force, all host threads) on a seeded sample of
    n_poses poses x n_elems contiguous elements x all sources."""
    import numpy as np
    from oracle import ref

    rng = np.random.default_rng(seed)
    ks = np.sort(rng.choice(w.K, n_poses, replace=False))
    i0 = int(rng.integers(0, w.N - n_elems))
    kk, ii = np.meshgrid(ks, np.arange(i0, i0 + n_elems), indexing="ij")
    pk, pi = kk.ravel(), ii.ravel()
    c32, _, _, m64 = ref.elements(w.mesh.verts, w.mesh.tris)
    rays = 0
    for j in range(w.lamp.n_src):
        p = np.stack([w.poses[pk, 0], w.poses[pk, 1], np.full(len(pk), w.lamp.dz[j], np.float32)], -1)
        d = p.astype(np.float64) - c32[pi].astype(np.float64)
        rays += int(((d * m64[pi]).sum(-1) > 0).sum())
    ref.lib()
    t0 = time.perf_counter()
    ref.irradiance_pairs(w.mesh.verts, w.mesh.tris, w.poses, w.lamp.dz, w.lamp.power, pk, pi)
    dt = time.perf_counter() - t0
    return {"value": rays / dt, "unit": "rays/s", "cores": ref.max_threads(), "kind": "oracle",
            "sample": f"{n_poses} seeded poses x {n_elems} contiguous elements x {w.lamp.n_src} sources "
                      f"({len(pk)} entries, {rays} occlusion rays) of the same ward workload",
            "seconds": dt, "entries_per_s": len(pk) / dt}


def extras(uvc, workloads, dev, log, floorplan_lp=False):
    """The additions around the hot path, each timed once: the 64-room
    batched launch (persistent, hipGraph replay, one launch per room), the
    floor plan as CSR and its dosage LP (column generation), the area-integrated
    matrix, the route stage, the dosage LP on one room, and the ranked plan
    (learned ranker + column generation) against the full-candidate LP on
    one larger room."""
    import numpy as np
    import torch

    out = {}
    # batched: 64 rooms, 2k-80k triangles and 500-8000 poses each
    t0 = time.perf_counter()
    rooms = workloads.batch(seed=3, n_rooms=64)
    gen_s = time.perf_counter() - t0
    scenes = [uvc.Scene(torch.from_numpy(r.mesh.verts).to(dev), torch.from_numpy(r.mesh.tris).to(dev))
              for r in rooms]
    poses = [torch.from_numpy(np.ascontiguousarray(r.poses)).to(dev) for r in rooms]
    lamp = uvc.Lamp(rooms[0].lamp.dz, rooms[0].lamp.power)
    b = uvc.Batch(scenes, poses, lamp)
    entries = sum(r.K * r.N for r in rooms)
    modes = {}
    for mode in ("persistent", "graph", "per_room"):
        b.run(mode, timing=True)
        ms = b.run(mode, timing=True)
        modes[mode] = {"ms": ms, "entries_per_s": entries / (ms * 1e-3)}
    # the autotuner on the largest room of every size class, then the batch
    # driven by that table (per-room packet shapes; one launch per room also
    # per-room occupancy)
    import tempfile
    t0 = time.perf_counter()
    rep = {}
    for q, r in enumerate(rooms):
        key = int(np.floor(np.log2(r.N)))
        if key not in rep or r.N > rooms[rep[key]].N:
            rep[key] = q
    with tempfile.TemporaryDirectory() as td:
        tpath = os.path.join(td, "tune.json")
        tuned = {}
        for key, q in sorted(rep.items()):
            tuned[f"n{key}"] = uvc.autotune(scenes[q], poses[q], lamp, probe_poses=256, table_path=tpath)
        table = open(tpath).read()
    tune_s = time.perf_counter() - t0
    b.close()
    b = uvc.Batch(scenes, poses, lamp, tune_table=table)
    for mode in ("persistent", "per_room"):
        b.run(mode, timing=True)
        ms = b.run(mode, timing=True)
        modes["tuned_" + mode] = {"ms": ms, "entries_per_s": entries / (ms * 1e-3)}
    out["batched"] = {"rooms": len(rooms), "N_total": sum(r.N for r in rooms), "K_total": sum(r.K for r in rooms),
                      "entries": entries, "E_GB": entries * 4 / 1e9, "generate_s": gen_s, "modes": modes,
                      "autotune_s": tune_s, "tuned_options": tuned}
    log(f"batched {out['batched']}")
    b.close()
    for sc in scenes:
        sc.close()
    del b, poses
    torch.cuda.empty_cache()
    # CSR at the floor-plan size (~488k triangles, 20,000 poses)
    fp = workloads.floorplan()
    sc = uvc.Scene(torch.from_numpy(fp.mesh.verts).to(dev), torch.from_numpy(fp.mesh.tris).to(dev))
    P = torch.from_numpy(np.ascontiguousarray(fp.poses)).to(dev)
    flamp = uvc.Lamp(fp.lamp.dz, fp.lamp.power)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp, col, val = uvc.irradiance_csr(sc, P, flamp, path="lbvh")
    torch.cuda.synchronize()
    csr_s = time.perf_counter() - t0
    nnz = int(rp[-1])
    out["floorplan_csr"] = {"K": fp.K, "N": fp.N, "seconds": csr_s, "nnz": nnz, "csr_GB": nnz * 8 / 1e9,
                            "entries_per_s": fp.K * fp.N / csr_s}
    log(f"floorplan csr {out['floorplan_csr']}")
    if floorplan_lp:
        # the floor plan's dosage LP straight from the CSR (column generation;
        # progress per round on stderr)
        os.environ["UVC_VERBOSE"] = "1"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flp = uvc.solve_lp(val, csr=(rp, col, fp.N), allow_notconv=True, max_iter=300)
        torch.cuda.synchronize()
        out["floorplan_lp"] = {"seconds": time.perf_counter() - t0, "objective": flp["objective"],
                               "converged": flp["converged"], "working_poses": flp["working_poses"],
                               "rounds": flp["rounds"], "iterations": flp["iterations"],
                               "primal_residual": flp["primal_residual"], "dual_residual": flp["dual_residual"],
                               "gap": flp["gap"], "n_visible": flp["n_visible"], "dwell_s": float(flp["t"].sum()),
                               "stops": int((flp["t"] > 1e-5 * flp["t"].sum()).sum())}
        log(f"floorplan lp {out['floorplan_lp']}")
        del flp
        os.environ.pop("UVC_VERBOSE", None)
    del rp, col, val
    sc.close()
    torch.cuda.empty_cache()
    # area-integrated irradiance (visibility cube at the paper's 512 x 512
    # per face) on 64 ward poses
    w = workloads.ward()
    sc = uvc.Scene(torch.from_numpy(w.mesh.verts).to(dev), torch.from_numpy(w.mesh.tris).to(dev))
    P = torch.from_numpy(np.ascontiguousarray(w.poses[:: max(1, w.K // 64)][:64])).to(dev)
    uvc.irradiance_area(sc, P[:2].contiguous(), lamp, face_res=512)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ea, Pw = uvc.irradiance_area(sc, P, lamp, face_res=512)
    torch.cuda.synchronize()
    area_s = time.perf_counter() - t0
    nray = P.shape[0] * lamp.n_src * 6 * 512 * 512
    out["area_irradiance"] = {"poses": int(P.shape[0]), "N": w.N, "face_res": 512, "rays": nray,
                              "seconds": area_s, "rays_per_s": nray / area_s,
                              "power_collected_W": float(Pw.mean())}
    log(f"area {out['area_irradiance']}")
    del Ea
    # the ward's full plan: dense E, LP, then the route over the dwell poses
    E, _ = uvc.irradiance_dense(sc, torch.from_numpy(w.poses).to(dev), lamp, path="lbvh")
    sol = uvc.solve_lp(E, allow_notconv=True, max_iter=300)
    free, x0, y0 = workloads.occupancy(w, 0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rt = uvc.plan_route(torch.from_numpy(w.poses).to(dev), sol["t"], torch.from_numpy(free).to(dev), x0, y0, 0.05)
    route_s = time.perf_counter() - t0
    out["route"] = {"workload": "ward LP solution, 0.05 m grid", "stops": int(len(rt["stops"])),
                    "tour_m": rt["length"], "plan_time_s": rt["plan_time"], "seconds": route_s}
    log(f"route {out['route']}")
    del E
    sc.close()
    torch.cuda.empty_cache()
    # dosage LP on one room (2k-20k triangles, 200-1000 poses family)
    from paper_2103_14137_amd import ranker
    w = ranker.room(ranker.TRAIN_SEED0)
    sc = uvc.Scene(w.mesh.verts, w.mesh.tris)
    P = torch.from_numpy(np.ascontiguousarray(w.poses)).to(dev)
    E, _ = uvc.irradiance_dense(sc, P, lamp, path="lbvh")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lp = uvc.solve_lp(E, allow_notconv=True)
    out["lp"] = {"K": w.K, "N": w.N, "ms": 1e3 * (time.perf_counter() - t0), "iterations": lp["iterations"],
                 "converged": lp["converged"], "objective": lp["objective"]}
    log(f"lp {out['lp']}")
    sc.close()
    del E
    # ranked plan vs full: the committed summary over the 200 held-out rooms
    # at the batched-room sizes, and one of those rooms (the one whose full
    # LP takes longest) run live
    wdir = os.path.join(ROOT, "paper_2103_14137_amd", "weights")
    wpath = os.path.join(wdir, "ranker_tower8_batchrooms.bin")
    if os.path.exists(wpath):
        ck = ranker.load_checkpoint(wpath)
        w = ranker.room(200006, (2000, 80000), (500, 8000))
        r = ranker.evaluate_room(w, ck["params"], keep_frac=0.1, modes=("mlp", "area"))
        out["ranked_plan"] = {"room": "held-out batch room 200006", "K": r["K"], "N": r["N"], "full_ms": r["full_ms"],
                              **{m: {k: r[m][k] for k in ("gap", "ms", "rounds", "n_kept", "fell_back")}
                                 for m in ("mlp", "area")}}
        sp = os.path.join(wdir, "ranker_tower8_batchrooms_eval_heldout200.json")
        if os.path.exists(sp):
            summ = json.load(open(sp))["summary"]
            out["ranked_plan"]["heldout200_recorded"] = {
                "rooms": summ["rooms"], "full_ms_total": summ["full_ms_total"],
                **{m: {k: summ[m][k] for k in ("gap_max", "gap_le_2pct", "fallback_rate", "ms_total",
                                              "speedup_vs_full")} for m in ("mlp", "area")}}
        log(f"ranked plan {out['ranked_plan']}")
    return out


def floorplan_run(uvc, workloads, dev, log):
    """The floor plan (12 rooms, ~488k triangles, 20,000 poses): CSR matrix
    timed, the same launch again with counters (occlusion rays), then the
    dosage LP straight from the CSR by column generation, with its KKT
    residuals."""
    import numpy as np
    import torch

    fp = workloads.floorplan()
    sc = uvc.Scene(torch.from_numpy(fp.mesh.verts).to(dev), torch.from_numpy(fp.mesh.tris).to(dev))
    P = torch.from_numpy(np.ascontiguousarray(fp.poses)).to(dev)
    flamp = uvc.Lamp(fp.lamp.dz, fp.lamp.power)
    log(f"floor plan: K={fp.K} N={fp.N} S={flamp.n_src}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp, col, val = uvc.irradiance_csr(sc, P, flamp, path="lbvh")
    torch.cuda.synchronize()
    csr_s = time.perf_counter() - t0
    nnz = int(rp[-1])
    log(f"csr {csr_s:.2f} s, nnz {nnz}")
    st = uvc.new_stats()
    rp2, col2, val2 = uvc.irradiance_csr(sc, P, flamp, path="lbvh", stats=st)
    torch.cuda.synchronize()
    same = bool(torch.equal(rp, rp2) and torch.equal(col, col2) and torch.equal(val, val2))
    del rp2, col2, val2
    counts = uvc.stats_dict(st)
    log(f"counted launch: {counts['rays']} rays, identical CSR: {same}")
    out = {"mode": "floorplan", "workload": "floor plan 12 rooms, N=%d triangles, K=%d poses, tower lamp 8 x 20 W"
           % (fp.N, fp.K),
           "csr": {"K": fp.K, "N": fp.N, "seconds": csr_s, "entries_per_s": fp.K * fp.N / csr_s,
                   "rays": counts["rays"], "rays_per_s": counts["rays"] / csr_s, "nnz": nnz, "nnz_per_s": nnz / csr_s,
                   "csr_GB": nnz * 8 / 1e9, "counted_launch_identical": same}}
    os.environ["UVC_VERBOSE"] = "1"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flp = uvc.solve_lp(val, csr=(rp, col, fp.N), allow_notconv=True, max_iter=300)
    torch.cuda.synchronize()
    out["lp"] = {"seconds": time.perf_counter() - t0, "objective": flp["objective"], "converged": flp["converged"],
                 "working_poses": flp["working_poses"], "rounds": flp["rounds"], "iterations": flp["iterations"],
                 "primal_residual": flp["primal_residual"], "dual_residual": flp["dual_residual"], "gap": flp["gap"],
                 "n_visible": flp["n_visible"], "penalty": flp["penalty"], "dwell_s": float(flp["t"].sum()),
                 "stops": int((flp["t"] > 1e-5 * flp["t"].sum()).sum())}
    log(f"lp {out['lp']}")
    sc.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the brute-force path comparison")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched / LP / ranked-plan sections")
    ap.add_argument("--no-floorplan-lp", action="store_true",
                    help="skip the floor plan's dosage LP (column generation from its CSR; ~30 s)")
    ap.add_argument("--mode", choices=["bench", "kernel", "copy", "floorplan"], default="bench",
                    help="kernel: only two launches of the irradiance kernel (for counter runs); "
                         "copy: a plain 1 GiB device copy (counter calibration); "
                         "floorplan: the floor plan's CSR matrix (timed, then counted) and its dosage LP "
                         "by column generation (about a minute)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: the irradiance path runs on a single GPU in this build "
              "(multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2103_14137_amd import uvc, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "copy":
        nbytes = 1 << 30
        x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                          "copies": 3}), flush=True)
        return
    if args.mode == "floorplan":
        print(json.dumps(floorplan_run(uvc, workloads, dev, log)), flush=True)
        return
    w = workloads.ward()
    K, N, S = w.K, w.N, w.lamp.n_src
    verts = torch.from_numpy(w.mesh.verts).to(dev)
    tris = torch.from_numpy(w.mesh.tris).to(dev)
    poses = torch.from_numpy(w.poses).to(dev)
    lamp = uvc.Lamp(w.lamp.dz, w.lamp.power)
    E = torch.empty((K, N), dtype=torch.float32, device=dev)
    log(f"ward: K={K} N={N} S={S}")
    if args.mode == "kernel":
        sc = uvc.Scene(verts, tris)
        for _ in range(2):
            uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E)
        torch.cuda.synchronize()
        sc.close()
        print(json.dumps({"mode": "kernel", "launches": 2, "K": K, "N": N, "S": S,
                          "source_hash": source_hash()}), flush=True)
        return

    def step():
        sc = uvc.Scene(verts, tris)
        uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E)
        sc.close()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / max(args.steps, 1)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    # instrumented launch: algorithmic work counts (outside the timed region)
    sc = uvc.Scene(verts, tris)
    stats = uvc.new_stats(dev)
    uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E, stats=stats)
    st = uvc.stats_dict(stats)
    rays = st["rays"]
    flops = FLOP_NODE * st["nodes"] + FLOP_TRI * (st["tris"] + st["near"] + st["cache"]) + FLOP_ENTRY * K * N * S
    # live HIP-event timing of the dominant kernel on the stream it runs on
    kms = []
    for _ in range(3):
        t = ctypes.c_float(0.0)
        uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E, timing=t)
        kms.append(t.value)
    kernel_ms = float(np.mean(kms))
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    log(f"stats {st}; kernel {kernel_ms:.3f} ms; {achieved:.2f} TFLOP/s algorithmic")

    paths = {"lbvh": {"kernel_ms": kernel_ms, "rays_per_s": rays / (kernel_ms * 1e-3)}}
    if not args.no_compare:
        for tp in (1, 4, 16, 64):
            t = ctypes.c_float(0.0)
            uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E, timing=t, packet_poses=tp)
            paths[f"lbvh_tp{tp}"] = {"kernel_ms": t.value, "rays_per_s": rays / (t.value * 1e-3)}
        for wv in (5, 6, 8):
            t = ctypes.c_float(0.0)
            uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E, timing=t, waves=wv)
            paths[f"lbvh_waves{wv}"] = {"kernel_ms": t.value, "rays_per_s": rays / (t.value * 1e-3)}
        t = ctypes.c_float(0.0)
        uvc.irradiance_dense(sc, poses, lamp, path="lbvh", out=E, timing=t, flags=uvc.FLAG_NO_NEAR)
        paths["lbvh_no_near"] = {"kernel_ms": t.value, "rays_per_s": rays / (t.value * 1e-3)}

        sub = poses[:: max(1, K // 16)][:16].contiguous()
        for pth in ("lbvh", "brute"):
            sst = uvc.new_stats(dev)
            uvc.irradiance_dense(sc, sub, lamp, path=pth, stats=sst)
            t = ctypes.c_float(0.0)
            uvc.irradiance_dense(sc, sub, lamp, path=pth, timing=t)
            r = uvc.stats_dict(sst)["rays"]
            paths[pth + "_16poses"] = {"kernel_ms": t.value, "rays_per_s": r / (t.value * 1e-3)}
        log(f"paths {paths}")
    sc.close()

    value = rays / (ms_per_step * 1e-3)
    traffic = traffic_from_profile()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ward 8x6x3 m, 6 beds + 10 cuboids, N={N} triangles, K={K} poses, "
                               f"tower lamp {S} x 20 W; step = scene build + dense E",
                   "K": K, "N": N, "S": S, "path": "lbvh"},
        "entries_per_s": K * N / (ms_per_step * 1e-3),
        "rays_per_step": rays,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": traffic, "kernel": KERNEL,
                     "kernel_ms": kernel_ms, "algorithmic_flops_per_launch": flops,
                     "peak_unpacked": PEAK_FP32_UNPACKED, "frac_unpacked": achieved / PEAK_FP32_UNPACKED,
                     "e_write_GBps": K * N * 4 / (kernel_ms * 1e-3) / 1e9,
                     "counts": st, "source_hash": source_hash()},
        "paths": paths,
    }
    del E
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["extras"] = extras(uvc, workloads, dev, log, floorplan_lp=not args.no_floorplan_lp)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
