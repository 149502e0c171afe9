"""Python front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loads (building on demand) the plain-C FP64 brute force in uvc_oracle.c and
exposes it with NumPy arrays.  Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uvc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FP contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c11", "-D_DEFAULT_SOURCE", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_elements.argtypes = [_P, _P, _I64, _P, _P, _P, _P]
        L.oracle_elements.restype = None
        L.oracle_hit.argtypes = [_P, _P, _P, _P, _P]
        L.oracle_hit.restype = ctypes.c_int
        L.oracle_segment_blocked.argtypes = [_P, _P, _I64, _P, _P, _I64]
        L.oracle_segment_blocked.restype = ctypes.c_int
        L.oracle_irradiance_pairs.argtypes = [_P, _P, _I64, _P, _I64, _I32, _I32, _P, _P,
                                              _P, _P, _I64, _P, _P, _I32]
        L.oracle_irradiance_pairs.restype = ctypes.c_int
        L.oracle_irradiance_pairs_lamp.argtypes = [_P, _P, _I64, _P, _I64, _I32, _I32, _P, _P, _I32, _P,
                                                   ctypes.c_uint32, ctypes.c_uint32, _P, _P, _I64, _P, _P, _I32]
        L.oracle_irradiance_pairs_lamp.restype = ctypes.c_int
        L.oracle_area_irradiance.argtypes = [_P, _P, _I64, _P, _I64, _I32, _I32, _P, _P, _I32, _P,
                                             ctypes.c_uint32, ctypes.c_uint32, _I32, _P, _P, _P, _I32]
        L.oracle_area_irradiance.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def elements(verts: np.ndarray, tris: np.ndarray):
    """(centroid FP32 [N,3], unit normal FP64 [N,3], area FP64 [N], m FP64 [N,3])."""
    v = _c(verts, np.float32)
    t = _c(tris, np.int32)
    n = t.shape[0]
    c32 = np.empty((n, 3), np.float32)
    n64 = np.empty((n, 3), np.float64)
    a64 = np.empty(n, np.float64)
    m64 = np.empty((n, 3), np.float64)
    lib().oracle_elements(_ptr(v), _ptr(t), n, _ptr(c32), _ptr(n64), _ptr(a64), _ptr(m64))
    return c32, n64, a64, m64


def hit(O, T, v0, v1, v2) -> int:
    """The FP64 segment/triangle predicate on FP32 inputs."""
    arrs = [_c(x, np.float32).reshape(3) for x in (O, T, v0, v1, v2)]
    return int(lib().oracle_hit(*[_ptr(a) for a in arrs]))


def segment_blocked(verts, tris, O, T, skip: int = -1) -> int:
    v = _c(verts, np.float32)
    t = _c(tris, np.int32)
    o = _c(O, np.float32).reshape(3)
    tt = _c(T, np.float32).reshape(3)
    return int(lib().oracle_segment_blocked(_ptr(v), _ptr(t), t.shape[0], _ptr(o), _ptr(tt), int(skip)))


def irradiance_pairs(verts, tris, poses, dz, power, pk, pi, threads: int = 0, profile=None, up_mask: int = 0,
                     down_mask: int = 0):
    """E (FP64) and visibility bits (uint32, bit j = source j) for the pairs
    (pose pk[q], element pi[q]).  profile: None (uniform emission) or the
    emission-pattern table over cos(theta) in [-1, 1]; up_mask / down_mask:
    sources that emit only above / below their own height."""
    if profile is not None or up_mask or down_mask:
        return _irradiance_pairs_lamp(verts, tris, poses, dz, power, pk, pi, threads, profile, up_mask, down_mask)
    v = _c(verts, np.float32)
    t = _c(tris, np.int32)
    p = _c(poses, np.float32)
    K, pdim = p.shape
    dzf = _c(dz, np.float32)
    pw = _c(power, np.float32)
    pk = _c(pk, np.int64)
    pi = _c(pi, np.int64)
    npairs = pk.shape[0]
    E = np.empty(npairs, np.float64)
    vis = np.empty(npairs, np.uint32)
    rc = lib().oracle_irradiance_pairs(_ptr(v), _ptr(t), t.shape[0], _ptr(p), K, pdim, dzf.shape[0],
                                       _ptr(dzf), _ptr(pw), _ptr(pk), _ptr(pi), npairs,
                                       _ptr(E), _ptr(vis), int(threads))
    if rc != 0:
        raise ValueError("oracle_irradiance_pairs: invalid arguments")
    return E, vis


def _irradiance_pairs_lamp(verts, tris, poses, dz, power, pk, pi, threads, profile, up_mask, down_mask):
    v = _c(verts, np.float32)
    t = _c(tris, np.int32)
    p = _c(poses, np.float32)
    K, pdim = p.shape
    dzf = _c(dz, np.float32)
    pw = _c(power, np.float32)
    prof = _c(profile if profile is not None else np.zeros(0), np.float32)
    pk = _c(pk, np.int64)
    pi = _c(pi, np.int64)
    npairs = pk.shape[0]
    E = np.empty(npairs, np.float64)
    vis = np.empty(npairs, np.uint32)
    rc = lib().oracle_irradiance_pairs_lamp(_ptr(v), _ptr(t), t.shape[0], _ptr(p), K, pdim, dzf.shape[0],
                                            _ptr(dzf), _ptr(pw), prof.shape[0], _ptr(prof) if prof.size else None,
                                            int(up_mask), int(down_mask), _ptr(pk), _ptr(pi), npairs,
                                            _ptr(E), _ptr(vis), int(threads))
    if rc != 0:
        raise ValueError("oracle_irradiance_pairs_lamp: invalid arguments")
    return E, vis


def irradiance_dense(verts, tris, poses, dz, power, threads: int = 0, profile=None, up_mask: int = 0,
                     down_mask: int = 0):
    """Full K x N matrices (E FP64, vis uint32)."""
    K = np.asarray(poses).shape[0]
    N = np.asarray(tris).shape[0]
    kk, ii = np.meshgrid(np.arange(K), np.arange(N), indexing="ij")
    E, vis = irradiance_pairs(verts, tris, poses, dz, power, kk.ravel(), ii.ravel(), threads, profile, up_mask,
                              down_mask)
    return E.reshape(K, N), vis.reshape(K, N)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def entry_tolerance(verts, tris, poses, dz, power, vis, pk=None, pi=None, profile=None):
    """Absolute tolerance per entry for comparing an FP32 irradiance with the
    FP64 oracle: 1e-5 * E64 is added by the caller; this returns the grazing
    term 1e-5 * sum_j V_j P_j W / (4 pi r_j^2), which bounds the FP32 error of
    the cosine factor when the cosine itself is small.  W = 1 for uniform
    emission; with an emission table W = max(largest table value, largest
    table step x (n - 1) / 2), which also bounds the interpolated weight's
    FP32 error (a few ulps of cos(theta) times the table's slope)."""
    W = 1.0
    if profile is not None:
        pr = np.asarray(profile, np.float64)
        W = max(float(pr.max()), float(np.abs(np.diff(pr)).max()) * (pr.size - 1) / 2.0)
    c32, _, _, _ = elements(verts, tris)
    p = np.asarray(poses, np.float32)
    pdim = p.shape[1]
    K, N = p.shape[0], c32.shape[0]
    if pk is None:
        kk, ii = np.meshgrid(np.arange(K), np.arange(N), indexing="ij")
        pk, pi = kk.ravel(), ii.ravel()
    pk = np.asarray(pk)
    pi = np.asarray(pi)
    vis = np.asarray(vis).ravel()
    zb = p[pk, 2] if pdim == 3 else np.zeros(len(pk), np.float32)
    tol = np.zeros(len(pk), np.float64)
    for j, (h, pw) in enumerate(zip(np.asarray(dz, np.float32), np.asarray(power, np.float32))):
        pz = (zb + h).astype(np.float32)
        d = np.stack([p[pk, 0], p[pk, 1], pz], -1).astype(np.float64) - c32[pi].astype(np.float64)
        r2 = (d * d).sum(-1)
        on = ((vis >> j) & 1).astype(bool)
        tol += np.where(on, float(pw) * W / (4.0 * np.pi * r2), 0.0)
    return 1e-5 * tol


def area_irradiance(verts, tris, poses, dz, power, face_res: int, profile=None, up_mask: int = 0,
                    down_mask: int = 0, threads: int = 0):
    """Area-integrated irradiance by the visibility-cube procedure (closest
    hit per cube-map pixel, pixel power to the hit triangle, collected power
    over triangle area): E (K x N FP64), the near-tie pixel counts (K x N
    int32) and the power collected per pose (K)."""
    v = _c(verts, np.float32)
    t = _c(tris, np.int32)
    p = _c(poses, np.float32)
    K, pdim = p.shape
    N = t.shape[0]
    dzf = _c(dz, np.float32)
    pw = _c(power, np.float32)
    prof = _c(profile if profile is not None else np.zeros(0), np.float32)
    E = np.empty((K, N), np.float64)
    amb = np.empty((K, N), np.int32)
    landed = np.empty(K, np.float64)
    rc = lib().oracle_area_irradiance(_ptr(v), _ptr(t), N, _ptr(p), K, pdim, dzf.shape[0], _ptr(dzf), _ptr(pw),
                                      prof.shape[0], _ptr(prof) if prof.size else None, int(up_mask),
                                      int(down_mask), int(face_res), _ptr(E), _ptr(amb), _ptr(landed), int(threads))
    if rc != 0:
        raise ValueError("oracle_area_irradiance: invalid arguments")
    return E, amb, landed


def cube_pixel_power_max(power, face_res: int, profile=None) -> float:
    """An upper bound on the power one cube-map pixel carries for these
    sources: pixels shrink away from a face's centre, and none subtends more
    than the square [-1/R, 1/R]^2 at unit distance, 4 atan(h^2 / sqrt(1 +
    2 h^2)) with h = 1/R."""
    h = 1.0 / face_res
    dom = 4.0 * np.arctan(h * h / np.sqrt(1.0 + 2.0 * h * h))
    wmax = 1.0 if profile is None else float(np.max(np.asarray(profile, np.float64)))
    return float(np.max(np.asarray(power, np.float64))) * wmax * dom / (4.0 * np.pi)
