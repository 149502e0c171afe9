// Closest-hit ray traversal of the scene hierarchy (FP32, no exact
// decisions): used by the ranker's feature rays and by the cube-map rays of
// the area-integrated irradiance.  A wavefront walks the hierarchy as one
// packet; every lane keeps its own closest hit (parameter tbest in units of
// its direction vector, and the leaf slot of the triangle); there is no
// early exit.
#pragma once
#include "uvc_common.hpp"

namespace uvc {

__device__ __forceinline__ float max3r(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }
__device__ __forceinline__ float min3r(float a, float b, float c) { return fminf(fminf(a, b), c); }

struct CRay {
    float ox, oy, oz, dx, dy, dz, ix, iy, iz, nx, ny, nz;
    float tbest;
    int best;
};

__device__ __forceinline__ bool cslab(const CRay& r, float lx, float ly, float lz, float hx, float hy, float hz) {
    const float t0x = fmaf(lx, r.ix, r.nx), t1x = fmaf(hx, r.ix, r.nx);
    const float t0y = fmaf(ly, r.iy, r.ny), t1y = fmaf(hy, r.iy, r.ny);
    const float t0z = fmaf(lz, r.iz, r.nz), t1z = fmaf(hz, r.iz, r.nz);
    const float tn = fmaxf(max3r(fminf(t0x, t1x), fminf(t0y, t1y), fminf(t0z, t1z)), 0.0f);
    const float tf = fminf(min3r(fmaxf(t0x, t1x), fmaxf(t0y, t1y), fmaxf(t0z, t1z)), r.tbest);
    return tn <= tf;
}

// Closest hit of the ray with one triangle record (FP32, no exact
// decisions).  Updates tbest / best.  WIDE: a ray within a small band of an
// edge counts as inside (band 2^-20 |D|_1 G L, G the largest |coordinate|
// of the vertices relative to the origin, L the largest edge component:
// about twice the rounding error of the orientations), so that no ray slips
// between two triangles that share an edge; both then report the hit and
// the smaller parameter wins.
template <bool WIDE>
__device__ __forceinline__ void ctri(CRay& r, const float* __restrict__ t, int slot) {
    const float v0x = t[0], v0y = t[1], v0z = t[2];
    const float e01x = t[TRI_E01], e01y = t[TRI_E01 + 1], e01z = t[TRI_E01 + 2];
    const float e12x = t[TRI_E12], e12y = t[TRI_E12 + 1], e12z = t[TRI_E12 + 2];
    const float e20x = t[TRI_E20], e20y = t[TRI_E20 + 1], e20z = t[TRI_E20 + 2];
    const float ax = v0x - r.ox, ay = v0y - r.oy, az = v0z - r.oz;
    const float bx = t[3] - r.ox, by = t[4] - r.oy, bz = t[5] - r.oz;
    const float cx = t[6] - r.ox, cy = t[7] - r.oy, cz = t[8] - r.oz;
    const float U = r.dx * fmaf(by, e12z, -bz * e12y) + r.dy * fmaf(bz, e12x, -bx * e12z) + r.dz * fmaf(bx, e12y, -by * e12x);
    const float V = r.dx * fmaf(cy, e20z, -cz * e20y) + r.dy * fmaf(cz, e20x, -cx * e20z) + r.dz * fmaf(cx, e20y, -cy * e20x);
    const float W = r.dx * fmaf(ay, e01z, -az * e01y) + r.dy * fmaf(az, e01x, -ax * e01z) + r.dz * fmaf(ax, e01y, -ay * e01x);
    bool in;
    if (WIDE) {
        const float G = max3r(max3r(fabsf(ax), fabsf(ay), fabsf(az)), max3r(fabsf(bx), fabsf(by), fabsf(bz)),
                              max3r(fabsf(cx), fabsf(cy), fabsf(cz)));
        const float band = 0x1p-20f * (fabsf(r.dx) + fabsf(r.dy) + fabsf(r.dz)) * G * t[TRI_L];
        in = (U >= -band && V >= -band && W >= -band) || (U <= band && V <= band && W <= band);
    } else {
        in = ((U >= 0.f && V >= 0.f && W >= 0.f) || (U <= 0.f && V <= 0.f && W <= 0.f)) && (U + V + W) != 0.f;
    }
    if (!in) return;
    // plane crossing: t = ((v0 - O) . m) / (D . m), m = e01 x (v2 - v0) = e20 x e01
    const float mx = fmaf(e20y, e01z, -e20z * e01y), my = fmaf(e20z, e01x, -e20x * e01z),
                mz = fmaf(e20x, e01y, -e20y * e01x);
    const float den = r.dx * mx + r.dy * my + r.dz * mz;
    if (den == 0.f) return;
    const float tt = (ax * mx + ay * my + az * mz) / den;
    if (tt > 0.f && tt < r.tbest) {
        r.tbest = tt;
        r.best = slot;
    }
}

// Walks the hierarchy of an N-triangle scene for the wave's rays; r.tbest
// must start at the largest parameter of interest and r.best at -1.
template <bool WIDE>
__device__ __forceinline__ void closest_hit_walk(CRay& r, const float* __restrict__ tri,
                                                 const float* __restrict__ nodes, int64_t N, int lane) {
    if (N == 1) {
        ctri<WIDE>(r, tri, 0);
    } else if (N > 1) {
        // packet walk: every lane keeps its own closest hit; no early exit
        unsigned long long m = ~0ull;
        int node = 0, sp = 0, sn = 0, slo = 0, shi = 0;
        while (true) {
            const float4* q = reinterpret_cast<const float4*>(nodes + (int64_t)node * NODE_WORDS);
            const float4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
            unsigned long long mL = __ballot(cslab(r, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y)) & m;
            unsigned long long mR = __ballot(cslab(r, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w)) & m;
            const int cl = __float_as_int(q3.x), cr = __float_as_int(q3.y);
            if (cl < 0 && mL) {
                if ((mL >> lane) & 1ull) ctri<WIDE>(r, tri + (int64_t)(~cl) * TRI_WORDS, ~cl);
                mL = 0;
            }
            if (cr < 0 && mR) {
                if ((mR >> lane) & 1ull) ctri<WIDE>(r, tri + (int64_t)(~cr) * TRI_WORDS, ~cr);
                mR = 0;
            }
            if (mL && mR) {
                const bool here = lane == sp;
                sn = here ? cr : sn;
                slo = here ? (int)(unsigned)mR : slo;
                shi = here ? (int)(unsigned)(mR >> 32) : shi;
                ++sp;
                node = cl;
                m = mL;
            } else if (mL) {
                node = cl;
                m = mL;
            } else if (mR) {
                node = cr;
                m = mR;
            } else {
                if (sp == 0) break;
                --sp;
                node = __builtin_amdgcn_readlane(sn, sp);
                const unsigned lo = (unsigned)__builtin_amdgcn_readlane(slo, sp);
                const unsigned hi = (unsigned)__builtin_amdgcn_readlane(shi, sp);
                m = ((unsigned long long)hi << 32) | lo;
            }
        }
    }
}

}  // namespace uvc
