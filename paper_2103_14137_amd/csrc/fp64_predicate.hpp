// FP64 decisions of the irradiance path (GPU side), shared by the scene
// build and the irradiance kernels.  Each evaluates its definition with the
// same operations in the same order, without contraction, on the FP32 inputs
// promoted to FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace uvc {

// Plane side of point T for triangle v0 v1 v2: (T - v0) . ((v1-v0) x (v2-v0)).
__device__ __forceinline__ double plane_side_fp64(float ftx, float fty, float ftz, float f0x, float f0y, float f0z,
                                                  float f1x, float f1y, float f1z, float f2x, float f2y, float f2z) {
#pragma clang fp contract(off)
    const double v0x = f0x, v0y = f0y, v0z = f0z;
    const double e1x = (double)f1x - v0x, e1y = (double)f1y - v0y, e1z = (double)f1z - v0z;
    const double e2x = (double)f2x - v0x, e2y = (double)f2y - v0y, e2z = (double)f2z - v0z;
    const double mx = e1y * e2z - e1z * e2y;
    const double my = e1z * e2x - e1x * e2z;
    const double mz = e1x * e2y - e1y * e2x;
    return (((double)ftx - v0x) * mx + ((double)fty - v0y) * my) + ((double)ftz - v0z) * mz;
}

// The segment/triangle predicate, evaluated in FP64 on the FP32 inputs:
// open segment O->T, closed triangle v0 v1 v2.  Same operations and order as
// its definition: m = (v1-v0) x (v2-v0); the plane sides (O-v0).m and
// (T-v0).m must be strictly opposite; with D = T-O and a, b, c = v0-O,
// v1-O, v2-O the edge orientations D.(b x c), D.(c x a), D.(a x b) must not
// be of mixed strict sign.  Dot products are ((x x' + y y') + z z').
static __device__ __noinline__ bool seg_tri_fp64(float fox, float foy, float foz, float ftx, float fty, float ftz,
                                          float f0x, float f0y, float f0z, float f1x, float f1y, float f1z,
                                          float f2x, float f2y, float f2z) {
#pragma clang fp contract(off)
    const double ox = fox, oy = foy, oz = foz, tx = ftx, ty = fty, tz = ftz;
    const double v0x = f0x, v0y = f0y, v0z = f0z, v1x = f1x, v1y = f1y, v1z = f1z, v2x = f2x, v2y = f2y, v2z = f2z;
    const double e1x = v1x - v0x, e1y = v1y - v0y, e1z = v1z - v0z;
    const double e2x = v2x - v0x, e2y = v2y - v0y, e2z = v2z - v0z;
    const double mx = e1y * e2z - e1z * e2y;
    const double my = e1z * e2x - e1x * e2z;
    const double mz = e1x * e2y - e1y * e2x;
    const double sO = ((ox - v0x) * mx + (oy - v0y) * my) + (oz - v0z) * mz;
    const double sT = ((tx - v0x) * mx + (ty - v0y) * my) + (tz - v0z) * mz;
    if (!((sO > 0.0 && sT < 0.0) || (sO < 0.0 && sT > 0.0))) return false;
    const double Dx = tx - ox, Dy = ty - oy, Dz = tz - oz;
    const double ax = v0x - ox, ay = v0y - oy, az = v0z - oz;
    const double bx = v1x - ox, by = v1y - oy, bz = v1z - oz;
    const double cx = v2x - ox, cy = v2y - oy, cz = v2z - oz;
    const double bcx = by * cz - bz * cy, bcy = bz * cx - bx * cz, bcz = bx * cy - by * cx;
    const double cax = cy * az - cz * ay, cay = cz * ax - cx * az, caz = cx * ay - cy * ax;
    const double abx = ay * bz - az * by, aby = az * bx - ax * bz, abz = ax * by - ay * bx;
    const double U = (Dx * bcx + Dy * bcy) + Dz * bcz;
    const double V = (Dx * cax + Dy * cay) + Dz * caz;
    const double W = (Dx * abx + Dy * aby) + Dz * abz;
    const bool neg = (U < 0.0) || (V < 0.0) || (W < 0.0);
    const bool pos = (U > 0.0) || (V > 0.0) || (W > 0.0);
    return !(neg && pos);
}

// Front-facing test in FP64: (p - c) . ((v1-v0) x (v2-v0)) > 0, strict.
static __device__ __noinline__ bool front_fp64(float fpx, float fpy, float fpz, float fcx, float fcy, float fcz,
                                        float f0x, float f0y, float f0z, float f1x, float f1y, float f1z,
                                        float f2x, float f2y, float f2z) {
#pragma clang fp contract(off)
    const double v0x = f0x, v0y = f0y, v0z = f0z;
    const double e1x = (double)f1x - v0x, e1y = (double)f1y - v0y, e1z = (double)f1z - v0z;
    const double e2x = (double)f2x - v0x, e2y = (double)f2y - v0y, e2z = (double)f2z - v0z;
    const double mx = e1y * e2z - e1z * e2y;
    const double my = e1z * e2x - e1x * e2z;
    const double mz = e1x * e2y - e1y * e2x;
    const double dx = (double)fpx - (double)fcx, dy = (double)fpy - (double)fcy, dz = (double)fpz - (double)fcz;
    return ((dx * mx + dy * my) + dz * mz) > 0.0;
}

}  // namespace uvc
