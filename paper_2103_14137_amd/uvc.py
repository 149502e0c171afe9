"""Thin Python binding of the libuvc C ABI (include/uvc.h).

Argument marshalling only: every step of the irradiance path runs in the HIP
library.  PyTorch provides device memory and the current stream.  There is
no fallback: if the library cannot be loaded or no GPU is present, the calls
raise.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch  # imported before the library so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("UVC_LIB_PATH") or os.path.join(_HERE, "libuvc.so")

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32

PATHS = {"auto": 0, "lbvh": 1, "brute": 2}
STAT_NAMES = ["rays", "nodes", "tris", "recheck", "front64", "visible", "steps", "near", "cache", "cache_hit", "leaf_steps"]
FLAG_NO_NEAR = 1
FLAG_NO_CACHE = 2
STAT_N = 11


class UvcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"uvc status {status}: {msg}")
        self.status = status


class LampC(ctypes.Structure):
    _fields_ = [("n_src", _I32), ("dz", _P), ("power_w", _P), ("n_prof", _I32), ("profile", _P),
                ("up_mask", ctypes.c_uint32), ("down_mask", ctypes.c_uint32)]


class LpInfoC(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("primal_residual", ctypes.c_double),
                ("dual_residual", ctypes.c_double), ("gap", ctypes.c_double), ("iterations", _I32),
                ("n_visible", _I64), ("penalty", ctypes.c_double), ("working_poses", _I64), ("rounds", _I32)]


class OptsC(ctypes.Structure):
    _fields_ = [("path", _I32), ("packet_poses", _I32), ("band_scale", ctypes.c_float), ("tile_tris", _I32),
                ("flags", _I32), ("waves", _I32), ("stats_dev", _P),
                ("kernel_ms", ctypes.POINTER(ctypes.c_float))]


class PlanInfoC(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("penalty", ctypes.c_double), ("min_reduced_cost", ctypes.c_double),
                ("n_kept", _I64), ("n_added", _I64), ("n_priced", _I64), ("rounds", _I32), ("rounds_added", _I32),
                ("fell_back", _I32),
                ("lp_iterations", _I32), ("lp_converged", _I32),
                ("ms_features", ctypes.c_float), ("ms_score", ctypes.c_float), ("ms_E", ctypes.c_float),
                ("ms_lp", ctypes.c_float), ("ms_price", ctypes.c_float), ("ms_fallback", ctypes.c_float),
                ("ms_total", ctypes.c_float), ("n_dropped", _I64)]


_lib = None


def lib():
    """Load libuvc.so (building it first only if no build exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build
        build.build()
    L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    sig = {
        "uvc_last_error": ([], ctypes.c_char_p),
        "uvc_version": ([], _I32),
        "uvc_build_scene": ([_P, _I64, _P, _I64, _I32, _P, ctypes.POINTER(_P)], _I32),
        "uvc_scene_info": ([_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)], _I32),
        "uvc_scene_elements": ([_P, _P, _P, _P, _P], _I32),
        "uvc_scene_export_bvh": ([_P, _P, _P, _P, _P], _I32),
        "uvc_destroy_scene": ([_P], None),
        "uvc_compute_irradiance_dense": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), ctypes.POINTER(OptsC), _P, _P,
                                          _P], _I32),
        "uvc_compute_irradiance_dense_noalloc": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), ctypes.POINTER(OptsC),
                                                  _P, _P, _P], _I32),
        "uvc_compute_irradiance_area": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), _I32, _P, _P, _P], _I32),
        "uvc_compute_irradiance_targets": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), ctypes.POINTER(OptsC), _P,
                                            _I64, _P, _P, _P], _I32),
        "uvc_compute_irradiance_csr_begin": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), ctypes.POINTER(OptsC), _P,
                                              ctypes.POINTER(_P), ctypes.POINTER(_I64)], _I32),
        "uvc_compute_irradiance_csr_finish": ([_P, _P, _P, _P, _P], _I32),
        "uvc_csr_job_destroy": ([_P], None),
        "uvc_batch_create": ([ctypes.POINTER(_P), _I32, ctypes.POINTER(_P), ctypes.POINTER(_I64), _I32,
                              ctypes.POINTER(LampC), ctypes.POINTER(OptsC), ctypes.c_char_p, ctypes.POINTER(_P), _P,
                              ctypes.POINTER(_P)], _I32),
        "uvc_set_tune_table": ([ctypes.c_char_p], _I32),
        "uvc_batch_run": ([_P, _I32, ctypes.POINTER(ctypes.c_float), _P], _I32),
        "uvc_batch_destroy": ([_P], None),
        "uvc_autotune": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), _I32, ctypes.c_char_p, _I32,
                          ctypes.POINTER(OptsC), _P], _I32),
        "uvc_solve_dosage_lp": ([_P, _P, _P, _I64, _I64, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _I32, _P, _P,
                                 _P, ctypes.POINTER(LpInfoC), _P], _I32),
        "uvc_route_geodesics": ([_P, _I32, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P, _I32, _P, _P],
                                _I32),
        "uvc_route_tour": ([_P, _I32, _I32, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32), _P], _I32),
        "uvc_plan_route": ([_P, _I64, _I32, _P, ctypes.c_double, _P, _I32, _I32, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, ctypes.c_double, _P, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), _P], _I32),
        "uvc_ranker_param_count": ([], _I64),
        "uvc_ranker_features": ([_P, _P, _I64, _I32, ctypes.c_float, _P, _P], _I32),
        "uvc_ranker_forward": ([_P, _P, _I64, _I32, _P, _P], _I32),
        "uvc_ranker_area_score": ([_P, _I64, _P, _P], _I32),
        "uvc_ranker_train_step": ([_P, _P, _P, _P, _P, _P, _I64, ctypes.c_float, _I64, _P,
                                   ctypes.POINTER(ctypes.c_float), _P], _I32),
        "uvc_plan_ranked": ([_P, _P, _I64, _I32, ctypes.POINTER(LampC), ctypes.POINTER(OptsC), _I32, _P, _I32,
                             ctypes.c_float, ctypes.c_float, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, _I32, _I32, _P, _P, _P, ctypes.POINTER(PlanInfoC), _P], _I32),
        "uvc_plan_evaluate": ([_P, _I64, _I64, _P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), ctypes.POINTER(_I64), _P], _I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int) -> None:
    if status != 0:
        raise UvcError(status, lib().uvc_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _require_cuda(t: torch.Tensor, name: str, dtype) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    return t.contiguous()


class Lamp:
    """Point sources dz[j] metres above the pose base, power[j] watts each;
    optionally an emission table over cos(theta) (profile) and hemisphere
    masks (sources that emit only above / below their own height)."""

    def __init__(self, dz, power, profile=None, up_mask: int = 0, down_mask: int = 0):
        self.dz = np.ascontiguousarray(dz, np.float32).reshape(-1)
        self.power = np.ascontiguousarray(power, np.float32).reshape(-1)
        if self.dz.shape != self.power.shape:
            raise ValueError("dz and power must have the same length")
        self.profile = None if profile is None else np.ascontiguousarray(profile, np.float32).reshape(-1)
        self.up_mask, self.down_mask = int(up_mask), int(down_mask)
        np_ = 0 if self.profile is None else int(self.profile.shape[0])
        pp = None if self.profile is None else self.profile.ctypes.data_as(_P)
        self._c = LampC(int(self.dz.shape[0]), self.dz.ctypes.data_as(_P), self.power.ctypes.data_as(_P), np_, pp,
                        self.up_mask, self.down_mask)

    @property
    def n_src(self) -> int:
        return int(self.dz.shape[0])


def as_lamp(lamp) -> Lamp:
    if isinstance(lamp, Lamp):
        return lamp
    return Lamp(lamp.dz, lamp.power)


def make_opts(path="auto", band_scale: float = 1.0, tile_tris: int = 0, stats: torch.Tensor | None = None,
              timing: ctypes.c_float | None = None, packet_poses: int = 0, flags: int = 0,
              waves: int = 0) -> OptsC:
    if stats is not None:
        stats = _require_cuda(stats, "stats", torch.int64)
        if stats.numel() < STAT_N:
            raise ValueError(f"stats needs {STAT_N} counters")
    return OptsC(PATHS[path] if isinstance(path, str) else int(path), int(packet_poses), float(band_scale),
                 int(tile_tris), int(flags), int(waves),
                 stats.data_ptr() if stats is not None else None,
                 ctypes.pointer(timing) if timing is not None else None)


class Scene:
    """A mesh with its surface elements and hierarchy, resident on the GPU."""

    def __init__(self, verts, tris, stream=None):
        """verts [V,3] float32 and tris [N,3] int32, as NumPy arrays (host) or
        as CUDA tensors (device-resident inputs)."""
        self._h = None
        h = _P()
        if isinstance(verts, torch.Tensor):
            v = _require_cuda(verts, "verts", torch.float32)
            t = _require_cuda(tris, "tris", torch.int32)
            if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
                raise ValueError("verts must be [V,3] and tris [N,3]")
            check(lib().uvc_build_scene(v.data_ptr(), v.shape[0], t.data_ptr(), t.shape[0], 1, _stream(stream),
                                        ctypes.byref(h)))
        else:
            v = np.ascontiguousarray(verts, np.float32)
            t = np.ascontiguousarray(tris, np.int32)
            if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
                raise ValueError("verts must be [V,3] and tris [N,3]")
            check(lib().uvc_build_scene(v.ctypes.data_as(_P), v.shape[0], t.ctypes.data_as(_P), t.shape[0], 0,
                                        _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n = int(t.shape[0])

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("scene is closed")
        return self._h

    def info(self):
        n, d, m = _I64(), _I32(), ctypes.c_float()
        check(lib().uvc_scene_info(self.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(m)))
        return {"n_tris": n.value, "bvh_depth": d.value, "max_abs_coord": m.value}

    def elements(self, stream=None):
        c = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        nrm = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        a = torch.empty((self.n,), dtype=torch.float32, device="cuda")
        check(lib().uvc_scene_elements(self.handle, c.data_ptr(), nrm.data_ptr(), a.data_ptr(), _stream(stream)))
        return c, nrm, a

    def export_bvh(self, stream=None):
        nodes = np.zeros((max(self.n - 1, 0), 16), np.float32)
        perm = np.zeros(self.n, np.int32)
        codes = np.zeros(self.n, np.uint32)
        check(lib().uvc_scene_export_bvh(self.handle, nodes.ctypes.data_as(_P) if nodes.size else None,
                                         perm.ctypes.data_as(_P), codes.ctypes.data_as(_P), _stream(stream)))
        return nodes, perm, codes

    def close(self):
        if self._h is not None:
            lib().uvc_destroy_scene(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def irradiance_dense(scene: Scene, poses: torch.Tensor, lamp, path="auto", band_scale: float = 1.0,
                     want_vis: bool = False, stats: torch.Tensor | None = None, out: torch.Tensor | None = None,
                     tile_tris: int = 0, stream=None, timing: ctypes.c_float | None = None,
                     packet_poses: int = 0, flags: int = 0, waves: int = 0):
    """Dense K x N irradiance matrix (and optional visibility bits).  With a
    ctypes.c_float passed as timing, the call synchronises and stores the
    irradiance kernel's duration in milliseconds (HIP events)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    lamp = as_lamp(lamp)
    N = scene.n
    if out is None:
        out = torch.empty((K, N), dtype=torch.float32, device=poses.device)
    else:
        out = _require_cuda(out, "out", torch.float32)
        if out.numel() != K * N:
            raise ValueError("out must hold K*N floats")
    vis = torch.empty((K, N), dtype=torch.int32, device=poses.device) if want_vis else None
    opts = make_opts(path, band_scale, tile_tris, stats, timing, packet_poses, flags, waves)
    check(lib().uvc_compute_irradiance_dense(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c),
                                             ctypes.byref(opts), out.data_ptr(),
                                             vis.data_ptr() if vis is not None else None, _stream(stream)))
    return out, vis


def irradiance_dense_noalloc(scene: Scene, poses: torch.Tensor, lamp, out: torch.Tensor,
                             vis: torch.Tensor | None = None, path="auto", band_scale: float = 1.0,
                             stats: torch.Tensor | None = None, stream=None, packet_poses: int = 0, flags: int = 0,
                             waves: int = 0, tile_tris: int = 0):
    """The dense matrix into caller-provided out (K x N float32) and
    optional vis (K x N int32) through the entry point that allocates no
    device memory (its scratch is a fixed device array; K <= 2^20)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    lamp = as_lamp(lamp)
    out = _require_cuda(out, "out", torch.float32)
    if out.numel() != K * scene.n:
        raise ValueError("out must hold K*N floats")
    if vis is not None:
        vis = _require_cuda(vis, "vis", torch.int32)
        if vis.numel() != K * scene.n:
            raise ValueError("vis must hold K*N ints")
    opts = make_opts(path, band_scale, tile_tris, stats, None, packet_poses, flags, waves)
    check(lib().uvc_compute_irradiance_dense_noalloc(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c),
                                                     ctypes.byref(opts), out.data_ptr(),
                                                     vis.data_ptr() if vis is not None else None, _stream(stream)))
    return out, vis


def irradiance_area(scene: Scene, poses: torch.Tensor, lamp, face_res: int = 0, stream=None):
    """Area-integrated irradiance by the visibility-cube procedure (see
    uvc_compute_irradiance_area): E (K x N float32) and the power collected
    per pose (K float64)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    lamp = as_lamp(lamp)
    E = torch.empty((K, scene.n), dtype=torch.float32, device=poses.device)
    pw = torch.empty(K, dtype=torch.float64, device=poses.device)
    check(lib().uvc_compute_irradiance_area(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c),
                                            int(face_res), E.data_ptr(), pw.data_ptr(), _stream(stream)))
    return E, pw


def irradiance_targets(scene: Scene, poses: torch.Tensor, lamp, targets: torch.Tensor, path="auto",
                       band_scale: float = 1.0, want_vis: bool = False, stream=None, packet_poses: int = 0,
                       flags: int = 0, waves: int = 0, tile_tris: int = 0):
    """K x len(targets) irradiance of the listed input elements (column j =
    element targets[j])."""
    poses = _require_cuda(poses, "poses", torch.float32)
    targets = _require_cuda(targets, "targets", torch.int32)
    K, pd = poses.shape
    n = targets.numel()
    lamp = as_lamp(lamp)
    out = torch.empty((K, n), dtype=torch.float32, device=poses.device)
    vis = torch.empty((K, n), dtype=torch.int32, device=poses.device) if want_vis else None
    opts = make_opts(path, band_scale, tile_tris, None, None, packet_poses, flags, waves)
    check(lib().uvc_compute_irradiance_targets(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c),
                                               ctypes.byref(opts), targets.data_ptr(), n, out.data_ptr(),
                                               vis.data_ptr() if vis is not None else None, _stream(stream)))
    return out, vis


def irradiance_csr(scene: Scene, poses: torch.Tensor, lamp, path="auto", band_scale: float = 1.0,
                   stats: torch.Tensor | None = None, tile_tris: int = 0, stream=None, packet_poses: int = 0,
                   flags: int = 0):
    """CSR irradiance matrix: (row_ptr int64 [K+1], col int32 [nnz], val float32 [nnz])."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    lamp = as_lamp(lamp)
    opts = make_opts(path, band_scale, tile_tris, stats, None, packet_poses, flags)
    job = _P()
    nnz = _I64()
    s = _stream(stream)
    check(lib().uvc_compute_irradiance_csr_begin(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c),
                                                 ctypes.byref(opts), s, ctypes.byref(job), ctypes.byref(nnz)))
    row_ptr = torch.empty(K + 1, dtype=torch.int64, device=poses.device)
    col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=poses.device)
    val = torch.empty(max(nnz.value, 1), dtype=torch.float32, device=poses.device)
    check(lib().uvc_compute_irradiance_csr_finish(job, row_ptr.data_ptr(), col.data_ptr(), val.data_ptr(), s))
    return row_ptr, col[:nnz.value], val[:nnz.value]


def new_stats(device="cuda") -> torch.Tensor:
    return torch.zeros(STAT_N, dtype=torch.int64, device=device)


def stats_dict(stats: torch.Tensor) -> dict:
    v = stats.cpu().numpy().astype(np.uint64)
    return {k: int(v[i]) for i, k in enumerate(STAT_NAMES)}


def solve_lp(E: torch.Tensor, mu_min: float = 280.0, t_max: float = 3.6e5, penalty: torch.Tensor | None = None,
             tol: float = 1e-9, max_iter: int = 200, stream=None, allow_notconv: bool = False,
             csr: tuple | None = None):
    """Relaxed dosage LP on the pose-major E: dense (E is K x N float32,
    device), or CSR when csr = (row_ptr int64 [K+1], col int32 [nnz], N) is
    given (E then holds the nnz float32 values).  Returns dict(t [K] float64,
    sigma [N] float64, y [N+1] float64, objective, residuals, ...)."""
    E = _require_cuda(E, "E", torch.float32)
    if csr is None:
        K, N = E.shape
        rp_ptr = col_ptr = None
    else:
        rp, col, N = csr
        rp = _require_cuda(rp, "row_ptr", torch.int64)
        col = _require_cuda(col, "col", torch.int32)
        K = rp.numel() - 1
        if K < 0 or col.numel() != E.numel():
            raise ValueError("CSR: row_ptr needs K+1 entries and col one per value")
        rp_ptr, col_ptr = rp.data_ptr(), col.data_ptr()
    dev = E.device
    t = torch.empty(K, dtype=torch.float64, device=dev)
    sg = torch.empty(N, dtype=torch.float64, device=dev)
    y = torch.empty(N + 1, dtype=torch.float64, device=dev)
    if penalty is not None:
        penalty = _require_cuda(penalty, "penalty", torch.float64)
    info = LpInfoC()
    st = lib().uvc_solve_dosage_lp(E.data_ptr(), rp_ptr, col_ptr, K, N,
                                   penalty.data_ptr() if penalty is not None else None,
                                   float(mu_min), float(t_max), float(tol), int(max_iter), t.data_ptr(),
                                   sg.data_ptr(), y.data_ptr(), ctypes.byref(info), _stream(stream))
    if st != 0 and not (allow_notconv and st == -4):
        check(st)
    return {"t": t, "sigma": sg, "y": y, "objective": info.objective, "primal_residual": info.primal_residual,
            "dual_residual": info.dual_residual, "gap": info.gap, "iterations": info.iterations,
            "n_visible": info.n_visible, "penalty": info.penalty, "working_poses": info.working_poses,
            "rounds": info.rounds, "converged": st == 0}


BATCH_MODES = {"persistent": 0, "graph": 1, "per_room": 2}


class Batch:
    """Dense irradiance matrices of many rooms, computed by one persistent
    launch (optionally replayed from a hipGraph).  Keeps references to the
    scenes, poses and outputs it was created with."""

    def __init__(self, scenes, poses_list, lamp, packet_poses: int = 0, waves: int = 0, stream=None,
                 tune_table: str | None = None, path: str = "lbvh"):
        self.scenes = list(scenes)
        self.poses = [_require_cuda(p, "poses", torch.float32) for p in poses_list]
        if len(self.poses) != len(self.scenes):
            raise ValueError("one pose tensor per scene")
        pd = self.poses[0].shape[1] if self.poses else 2
        self.lamp = as_lamp(lamp)
        self.E = [torch.empty((p.shape[0], sc.n), dtype=torch.float32, device=p.device)
                  for p, sc in zip(self.poses, self.scenes)]
        n = len(self.scenes)
        SA = _P * max(n, 1)
        KA = _I64 * max(n, 1)
        self._sc = SA(*[sc.handle for sc in self.scenes])
        self._ps = SA(*[p.data_ptr() for p in self.poses])
        self._ks = KA(*[p.shape[0] for p in self.poses])
        self._es = SA(*[e.data_ptr() for e in self.E])
        self._opts = make_opts(path, packet_poses=packet_poses, waves=waves)
        h = _P()
        self._h = None
        tt = tune_table.encode() if tune_table is not None else None
        check(lib().uvc_batch_create(self._sc, n, self._ps, self._ks, pd, ctypes.byref(self.lamp._c),
                                     ctypes.byref(self._opts), tt, self._es, _stream(stream), ctypes.byref(h)))
        self._h = h

    def run(self, mode: str = "graph", timing: bool = False, stream=None):
        t = ctypes.c_float(0.0)
        check(lib().uvc_batch_run(self._h, BATCH_MODES[mode], ctypes.byref(t) if timing else None,
                                  _stream(stream)))
        return t.value if timing else None

    def close(self):
        if self._h is not None:
            lib().uvc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_tune_table(json_text: str | None) -> None:
    """Register a tuning table (its JSON text) for UVC_PATH_AUTO calls; None
    clears it (see uvc_set_tune_table)."""
    check(lib().uvc_set_tune_table(json_text.encode() if json_text is not None else None))


def autotune(scene: Scene, poses: torch.Tensor, lamp, probe_poses: int = 256, table_path: str | None = None,
             force: bool = False, stream=None) -> dict:
    """Fastest launch options for this scene size class (see uvc_autotune)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    lamp = as_lamp(lamp)
    best = OptsC()
    check(lib().uvc_autotune(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c), int(probe_poses),
                             table_path.encode() if table_path else None, int(force), ctypes.byref(best),
                             _stream(stream)))
    return {"path": {0: "auto", 1: "lbvh", 2: "brute"}[best.path], "packet_poses": best.packet_poses,
            "waves": best.waves, "tile_tris": best.tile_tris}


# ------------------------------------------------------------------ ranker
RANK_MODES = {"mlp": 0, "area": 1, "none": 2}
FEATURES = 64


def ranker_param_count() -> int:
    return int(lib().uvc_ranker_param_count())


def ranker_features(scene: Scene, poses: torch.Tensor, src_height: float = 0.9, stream=None) -> torch.Tensor:
    """K x 64 visibility features of the poses (see uvc_ranker_features)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    feat = torch.empty((K, FEATURES), dtype=torch.float32, device=poses.device)
    check(lib().uvc_ranker_features(scene.handle, poses.data_ptr(), K, pd, float(src_height), feat.data_ptr(),
                                    _stream(stream)))
    return feat


def ranker_forward(params: torch.Tensor, feat: torch.Tensor, bf16: bool = False, stream=None) -> torch.Tensor:
    params = _require_cuda(params, "params", torch.float32)
    feat = _require_cuda(feat, "feat", torch.float32)
    if params.numel() != ranker_param_count() or feat.ndim != 2 or feat.shape[1] != FEATURES:
        raise ValueError("params must hold ranker_param_count() floats and feat be [B, 64]")
    B = feat.shape[0]
    score = torch.empty(B, dtype=torch.float32, device=feat.device)
    check(lib().uvc_ranker_forward(params.data_ptr(), feat.data_ptr(), B, int(bool(bf16)), score.data_ptr(),
                                   _stream(stream)))
    return score


def ranker_area_score(feat: torch.Tensor, stream=None) -> torch.Tensor:
    feat = _require_cuda(feat, "feat", torch.float32)
    if feat.ndim != 2 or feat.shape[1] != FEATURES:
        raise ValueError("feat must be [K, 64]")
    score = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
    check(lib().uvc_ranker_area_score(feat.data_ptr(), feat.shape[0], score.data_ptr(), _stream(stream)))
    return score


def ranker_train_step(params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, feat: torch.Tensor,
                      labels: torch.Tensor, idx: torch.Tensor | None, lr: float, step: int,
                      grad_out: torch.Tensor | None = None, stream=None) -> float:
    """One Adam step in place on params / m / v; returns the batch loss."""
    n = ranker_param_count()
    for name, t in (("params", params), ("m", m), ("v", v)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and t.numel() == n):
            raise ValueError(f"{name} must be a contiguous CUDA float32 tensor of {n} values")
    feat = _require_cuda(feat, "feat", torch.float32)
    labels = _require_cuda(labels, "labels", torch.float32)
    if idx is not None:
        idx = _require_cuda(idx, "idx", torch.int32)
        B = idx.numel()
    else:
        B = feat.shape[0]
    if grad_out is not None and not (grad_out.is_cuda and grad_out.dtype == torch.float32 and grad_out.numel() == n):
        raise ValueError("grad_out must be a CUDA float32 tensor of the parameter count")
    loss = ctypes.c_float(0.0)
    check(lib().uvc_ranker_train_step(params.data_ptr(), m.data_ptr(), v.data_ptr(), feat.data_ptr(),
                                      labels.data_ptr(), idx.data_ptr() if idx is not None else None, B, float(lr),
                                      int(step), grad_out.data_ptr() if grad_out is not None else None,
                                      ctypes.byref(loss), _stream(stream)))
    return float(loss.value)


def plan_ranked(scene: Scene, poses: torch.Tensor, lamp, mode: str = "mlp", params: torch.Tensor | None = None,
                bf16: bool = False, keep_frac: float = 0.1, feature_height: float = 0.9, penalty: float = 0.0,
                mu_min: float = 280.0, t_max: float = 3.6e5, tol: float = 1e-9, max_iter: int = 200,
                max_rounds: int = 20, path="lbvh", packet_poses: int = 0, waves: int = 0, stream=None) -> dict:
    """Dwell-time plan with pose pruning and column generation (see
    uvc_plan_ranked)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    K, pd = poses.shape
    lamp = as_lamp(lamp)
    if params is not None:
        params = _require_cuda(params, "params", torch.float32)
    t = torch.empty(K, dtype=torch.float64, device=poses.device)
    sg = torch.empty(scene.n, dtype=torch.float64, device=poses.device)
    kept = np.zeros(K, np.int32)
    info = PlanInfoC()
    opts = make_opts(path, packet_poses=packet_poses, waves=waves)
    check(lib().uvc_plan_ranked(scene.handle, poses.data_ptr(), K, pd, ctypes.byref(lamp._c), ctypes.byref(opts),
                                RANK_MODES[mode], params.data_ptr() if params is not None else None, int(bool(bf16)),
                                float(keep_frac), float(feature_height), float(penalty), float(mu_min), float(t_max),
                                float(tol), int(max_iter), int(max_rounds), t.data_ptr(), sg.data_ptr(),
                                kept.ctypes.data_as(_P), ctypes.byref(info), _stream(stream)))
    out = {f: getattr(info, f) for f, _ in PlanInfoC._fields_}
    out.update(t=t, sigma=sg, kept=kept[:info.n_kept].copy())
    return out


def plan_evaluate(E: torch.Tensor, t: torch.Tensor, mu_min: float = 280.0, penalty: float = 0.0,
                  stream=None) -> dict:
    """Objective of dwell times t on E with sigma at its smallest feasible
    value (see uvc_plan_evaluate)."""
    E = _require_cuda(E, "E", torch.float32)
    t = _require_cuda(t, "t", torch.float64)
    K, N = E.shape
    if t.numel() != K:
        raise ValueError("t must hold one value per row of E")
    obj, sh = ctypes.c_double(), ctypes.c_double()
    ns, nv = _I64(), _I64()
    check(lib().uvc_plan_evaluate(E.data_ptr(), K, N, t.data_ptr(), float(mu_min), float(penalty), ctypes.byref(obj),
                                  ctypes.byref(sh), ctypes.byref(ns), ctypes.byref(nv), _stream(stream)))
    return {"objective": obj.value, "shortfall": sh.value, "n_short": ns.value, "n_visible": nv.value}


def route_geodesics(free: torch.Tensor, x0: float, y0: float, cell: float, stops: torch.Tensor, stream=None):
    """m x m grid-geodesic distances between the stops (see
    uvc_route_geodesics); free is an H x W uint8 device grid."""
    free = _require_cuda(free, "free", torch.uint8)
    stops = _require_cuda(stops, "stops", torch.float32)
    H, W = free.shape
    m = stops.shape[0]
    D = torch.empty((m, m), dtype=torch.float64, device=stops.device)
    check(lib().uvc_route_geodesics(free.data_ptr(), H, W, float(x0), float(y0), float(cell), stops.data_ptr(), m,
                                    D.data_ptr(), _stream(stream)))
    return D


def route_tour(D: torch.Tensor, max_moves: int = 0, stream=None):
    """Closed tour over the stops of distance matrix D (see uvc_route_tour):
    (tour int32 numpy array, length, moves)."""
    D = _require_cuda(D, "D", torch.float64)
    m = D.shape[0]
    tour = np.zeros(max(m, 1), np.int32)
    L, mv = ctypes.c_double(), _I32()
    check(lib().uvc_route_tour(D.data_ptr(), m, int(max_moves), tour.ctypes.data_as(_P), ctypes.byref(L),
                               ctypes.byref(mv), _stream(stream)))
    return tour[:m].copy(), L.value, mv.value


def plan_route(poses: torch.Tensor, t: torch.Tensor, free: torch.Tensor, x0: float, y0: float, cell: float,
               rel_threshold: float = 1e-5, v_max: float = 0.5, stream=None) -> dict:
    """Tour over the poses with a dwell time (see uvc_plan_route)."""
    poses = _require_cuda(poses, "poses", torch.float32)
    t = _require_cuda(t, "t", torch.float64)
    free = _require_cuda(free, "free", torch.uint8)
    K, pd = poses.shape
    H, W = free.shape
    stops = np.zeros(max(K, 1), np.int32)
    m, L, T = _I32(), ctypes.c_double(), ctypes.c_double()
    check(lib().uvc_plan_route(poses.data_ptr(), K, pd, t.data_ptr(), float(rel_threshold), free.data_ptr(), H, W,
                               float(x0), float(y0), float(cell), float(v_max), stops.ctypes.data_as(_P),
                               ctypes.byref(m), ctypes.byref(L), ctypes.byref(T), _stream(stream)))
    return {"stops": stops[:m.value].copy(), "length": L.value, "plan_time": T.value}
