// Irradiance matrix assembly (Sec. IV-C): per (pose k, source j, element i)
// the inverse-square, cosine-weighted point-source irradiance, counted when
// the element faces the source and no other triangle meets the segment from
// the source to the element's centroid.
//
// Work decomposition: one wavefront = one packet of 64 elements (consecutive
// leaf slots, i.e. a compact patch in Morton order) for one pose; the wave
// loops over the lamp's sources in ascending order, so all 64 occlusion
// segments of a source share their origin.  Both occlusion paths keep the
// control flow uniform across the wave:
//  - hierarchy path: the packet walks the LBVH together; every node carries
//    the 64-bit mask of lanes whose segment entered it, the stack of deferred
//    (node, mask) pairs lives in three VGPRs indexed by lane, node and
//    triangle records are read with uniform (scalar) loads;
//  - brute-force path: the workgroup (4 packets, one pose) stages per-source
//    triangle data -- the three edge cross products relative to the shared
//    origin -- in LDS tiles, after which each segment/triangle edge test is
//    three dot products per lane.
// Every decision is taken in FP32 only when the FP32 value is provably on
// the same side of zero as the exact one; otherwise the FP64 predicate is
// evaluated with the same operations in the same order as its definition.
#include "uvc_common.hpp"
#include "fp64_predicate.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

namespace uvc {

constexpr float INV_4PI = 0.0795774715459476678844f;  // 1 / (4 pi)


struct IrrParams {
    const float* tri;
    const float* elem;
    const float* nodes;
    const int32_t* near_off;
    const int32_t* near;
    const float* poses;        // poses of this launch (row k = pose k of the launch)
    const int32_t* pose_order; // hierarchy path: packet position -> pose row
    const int32_t* targets;    // NULL (every element, columns = input index) or
                               // leaf slots of the target elements (column = list position)
    int64_t K;                 // poses in this launch
    int64_t N;                 // triangles in the scene
    int64_t ntargets;          // elements computed (N, or the length of targets)
    int64_t ld;                // row stride of E and vis
    int64_t ntiles;            // element tiles per pose tile
    int64_t nquads;            // ceil(ntiles / 4)
    int64_t kgroups;           // pose tiles (hierarchy) or poses (brute force)
    int32_t pose_dim;
    int32_t tile_tris;         // brute-force LDS tile
    int32_t tk_log2;           // hierarchy path: log2 of the poses per packet (0..6)
    int32_t use_near;          // hierarchy path: stop segments short and test near lists
    int32_t use_cache;         // hierarchy path: test each lane's last occluder first
    int32_t waves;             // hierarchy path: occupancy target of the kernel variant (0, 6, 8)
    float tau_f, tau_e, tau_p;
    float* E;                  // rows of this launch, K x N
    uint32_t* vis;             // NULL or K x N
    unsigned long long* stats;
    LampArgs lamp;
};

// Scene arrays are read-only while a kernel runs; records addressed by a
// uniform index (hierarchy nodes, leaf triangles) are read through the
// constant address space so that they become scalar loads.
typedef __attribute__((address_space(4))) const float cfloat;

// ------------------------------------------------------------------ FP32
struct Ray {
    float ox, oy, oz;     // origin: the source (uniform across the packet)
    float dx, dy, dz;     // D = T - O
    float ix, iy, iz;     // 1 / D, zero components replaced by +-1e-30
    float nx, ny, nz;     // -O / D
    float l1;             // |D|_1
    float tmax;           // hierarchy culling covers t in [0, tmax]
    float tx, ty, tz;     // target: the element centroid
    int self;             // input index of the target's own triangle
};

__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }
__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }
__device__ __forceinline__ float amax3(float a, float b, float c) { return max3f(fabsf(a), fabsf(b), fabsf(c)); }

__device__ __forceinline__ float guard_inv(float d) {
    const float g = (fabsf(d) < 1e-30f) ? copysignf(1e-30f, d) : d;
    return 1.0f / g;
}

__device__ __forceinline__ void make_ray(Ray& r, float ox, float oy, float oz, float tx, float ty, float tz,
                                         int self) {
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.tx = tx; r.ty = ty; r.tz = tz;
    r.dx = tx - ox; r.dy = ty - oy; r.dz = tz - oz;
    r.ix = guard_inv(r.dx); r.iy = guard_inv(r.dy); r.iz = guard_inv(r.dz);
    r.nx = -ox * r.ix; r.ny = -oy * r.iy; r.nz = -oz * r.iz;
    r.l1 = fabsf(r.dx) + fabsf(r.dy) + fabsf(r.dz);
    r.tmax = 1.0f;
    r.self = self;
}

// make_ray with the x and y reciprocals and offsets already formed (the same
// arithmetic, so the same bits).
__device__ __forceinline__ void make_ray_z(Ray& r, float ox, float oy, float oz, float tx, float ty, float tz,
                                           int self, float ix, float iy, float nx, float ny) {
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.tx = tx; r.ty = ty; r.tz = tz;
    r.dx = tx - ox; r.dy = ty - oy; r.dz = tz - oz;
    r.ix = ix; r.iy = iy; r.iz = guard_inv(r.dz);
    r.nx = nx; r.ny = ny; r.nz = -oz * r.iz;
    r.l1 = fabsf(r.dx) + fabsf(r.dy) + fabsf(r.dz);
    r.tmax = 1.0f;
    r.self = self;
}

// Does the segment's parameter interval [0, tmax] meet the (padded) box?
__device__ __forceinline__ bool slab(const Ray& r, float lx, float ly, float lz, float hx, float hy, float hz) {
    const float t0x = fmaf(lx, r.ix, r.nx), t1x = fmaf(hx, r.ix, r.nx);
    const float t0y = fmaf(ly, r.iy, r.ny), t1y = fmaf(hy, r.iy, r.ny);
    const float t0z = fmaf(lz, r.iz, r.nz), t1z = fmaf(hz, r.iz, r.nz);
    const float tn = fmaxf(max3f(fminf(t0x, t1x), fminf(t0y, t1y), fminf(t0z, t1z)), 0.0f);
    const float tf = fminf(min3f(fmaxf(t0x, t1x), fmaxf(t0y, t1y), fmaxf(t0z, t1z)), r.tmax);
    return tn <= tf;
}

// Slow part of the triangle decision, reached when the edge orientations do
// not already prove a miss: certain "inside" edges go on to the FP32 plane
// test; any decision within its band is re-taken in FP64.
// Returns bit 0 = hit, bit 1 = the decision was re-taken in FP64.
__device__ __forceinline__ int tri_rare(float rox, float roy, float roz, float rtx, float rty, float rtz, float v0x,
                                     float v0y, float v0z, float v1x, float v1y, float v1z, float v2x, float v2y,
                                     float v2z, float mn, float mx, float be, float tau_p) {
    const bool inside = (mn > be) || (mx < -be);
    if (inside) {
        const float e1x = v1x - v0x, e1y = v1y - v0y, e1z = v1z - v0z;
        const float e2x = v2x - v0x, e2y = v2y - v0y, e2z = v2z - v0z;
        const float mx_ = fmaf(e1y, e2z, -e1z * e2y);
        const float my_ = fmaf(e1z, e2x, -e1x * e2z);
        const float mz_ = fmaf(e1x, e2y, -e1y * e2x);
        const float gm = amax3(e1x, e1y, e1z) * amax3(e2x, e2y, e2z);
        const float wox = rox - v0x, woy = roy - v0y, woz = roz - v0z;
        const float wtx = rtx - v0x, wty = rty - v0y, wtz = rtz - v0z;
        const float sO = fmaf(woz, mz_, fmaf(woy, my_, wox * mx_));
        const float sT = fmaf(wtz, mz_, fmaf(wty, my_, wtx * mx_));
        const float bO = tau_p * amax3(wox, woy, woz) * gm;
        const float bT = tau_p * amax3(wtx, wty, wtz) * gm;
        if (fabsf(sO) > bO && fabsf(sT) > bT) return ((sO > 0.0f) != (sT > 0.0f)) ? 1 : 0;
    }
    return 2 | (seg_tri_fp64(rox, roy, roz, rtx, rty, rtz, v0x, v0y, v0z, v1x, v1y, v1z, v2x, v2y, v2z) ? 1 : 0);
}

// Full per-lane triangle decision for the hierarchy path.  t is the
// triangle record (uniform across the wave).  The edge cross products
// (vi - O) x (vj - vi) are the same for every lane (shared origin); only the
// three dot products with D are per lane.  Forming them from the short edge
// vector keeps their FP32 error proportional to |vi - O| |vj - vi|, the
// scale of the edge orientation itself.
template <class TP>
__device__ __forceinline__ bool tri_hit(const Ray& r, TP t, float tau_e, float tau_p, int* rechecks) {
    const float v0x = t[0], v0y = t[1], v0z = t[2], v1x = t[3], v1y = t[4], v1z = t[5];
    const float v2x = t[6], v2y = t[7], v2z = t[8];
    const float e01x = t[TRI_E01], e01y = t[TRI_E01 + 1], e01z = t[TRI_E01 + 2];
    const float e12x = t[TRI_E12], e12y = t[TRI_E12 + 1], e12z = t[TRI_E12 + 2];
    const float e20x = t[TRI_E20], e20y = t[TRI_E20 + 1], e20z = t[TRI_E20 + 2];
    const float L = t[TRI_L];
    const float ax = v0x - r.ox, ay = v0y - r.oy, az = v0z - r.oz;
    const float bx = v1x - r.ox, by = v1y - r.oy, bz = v1z - r.oz;
    const float cx = v2x - r.ox, cy = v2y - r.oy, cz = v2z - r.oz;
    const float ux = fmaf(by, e12z, -bz * e12y), uy = fmaf(bz, e12x, -bx * e12z), uz = fmaf(bx, e12y, -by * e12x);
    const float vx = fmaf(cy, e20z, -cz * e20y), vy = fmaf(cz, e20x, -cx * e20z), vz = fmaf(cx, e20y, -cy * e20x);
    const float wx = fmaf(ay, e01z, -az * e01y), wy = fmaf(az, e01x, -ax * e01z), wz = fmaf(ax, e01y, -ay * e01x);
    const float g = max3f(amax3(ax, ay, az), amax3(bx, by, bz), amax3(cx, cy, cz));
    const float kap = tau_e * g * fmaf(0x1p-28f, g, L);
    const float U = fmaf(r.dz, uz, fmaf(r.dy, uy, r.dx * ux));
    const float V = fmaf(r.dz, vz, fmaf(r.dy, vy, r.dx * vx));
    const float W = fmaf(r.dz, wz, fmaf(r.dy, wy, r.dx * wx));
    const float be = kap * r.l1;
    const float mn = min3f(U, V, W), mx = max3f(U, V, W);
    if (mn < -be && mx > be) return false;
    const int q = tri_rare(r.ox, r.oy, r.oz, r.tx, r.ty, r.tz, v0x, v0y, v0z, v1x, v1y, v1z, v2x, v2y, v2z, mn, mx,
                           be, tau_p);
    if (rechecks) *rechecks += q >> 1;
    return (q & 1) != 0;
}

// Irradiance term of one visible source: P_j/(4 pi) * <d, n> / |d|^3, never
// below FLT_MIN (the exact term of a visible source is positive).  Written
// with explicit FMAs and no contraction so that every kernel produces the
// same bits.
__device__ __forceinline__ float entry_term(float dx, float dy, float dz, float s, float pw) {
#pragma clang fp contract(off)
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float w = (pw * fmaxf(s, 0.0f)) * ((ri * ri) * ri);
    return fmaxf(w, FLT_MIN);
}

// The same term times the source's emission weight: the lamp's table
// interpolated at cos(theta) = -dz / |d| (d = source - element, so -dz is
// the element's height above the source).
__device__ __forceinline__ float entry_term_weighted(float dx, float dy, float dz, float s, float pw,
                                                     const LampArgs& L) {
#pragma clang fp contract(off)
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float wgt = (L.nprof > 0) ? table_weight(L, -dz * ri) : 1.0f;
    const float w = ((pw * fmaxf(s, 0.0f)) * ((ri * ri) * ri)) * wgt;
    return fmaxf(w, FLT_MIN);
}

// Does source j emit towards a point at height cz (source height oz)?
__device__ __forceinline__ bool lamp_emits(const LampArgs& L, int j, float cz, float oz) {
    if ((L.up >> j) & 1u) return cz > oz;
    if ((L.down >> j) & 1u) return cz < oz;
    return true;
}

__device__ __forceinline__ float cos_numerator(float dx, float dy, float dz, float nx, float ny, float nz) {
#pragma clang fp contract(off)
    return __builtin_fmaf(dz, nz, __builtin_fmaf(dy, ny, dx * nx));
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ unsigned long long wave_sum_u32(unsigned v) {
    unsigned long long s = v;
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// Workgroup (4 packets) -> (pose group, quad of element tiles), spreading
// consecutive logical workgroups over the 8 XCDs in contiguous ranges so
// that each XCD's L2 serves a compact region of the element space.
__device__ __forceinline__ void block_coords(const IrrParams& P, int64_t& kg, int64_t& quad) {
    const uint64_t B = gridDim.x, b = blockIdx.x;
    const uint64_t xcd = b & 7u, loc = b >> 3, per = B >> 3, rem = B & 7u;
    const uint64_t logical = xcd * per + (xcd < rem ? xcd : rem) + loc;
    kg = (int64_t)(logical % (uint64_t)P.kgroups);
    quad = (int64_t)(logical / (uint64_t)P.kgroups);
}

struct ElemLane {
    float cx, cy, cz, nx, ny, nz;
    float rho_t;
    int self;
    bool valid;
};

// Element record of leaf slot `slot` (valid lanes only).
template <class PT>
__device__ __forceinline__ ElemLane elem_record(PT& P, int32_t slot, bool valid) {
    ElemLane e;
    e.valid = valid;
    if (valid) {
        const float4* q = reinterpret_cast<const float4*>(P.elem + (int64_t)slot * ELEM_WORDS);
        const float4 a = q[0], b = q[1];
        e.cx = a.x; e.cy = a.y; e.cz = a.z; e.nx = a.w; e.ny = b.x; e.nz = b.y;
        e.self = __float_as_int(b.z);
        e.rho_t = b.w;
    } else {
        e.cx = e.cy = e.cz = e.nx = e.ny = e.nz = e.rho_t = 0.f;
        e.self = -1;
    }
    return e;
}

// Maps a lane's list position to its leaf slot and output column (the
// input element index, or the position in the target list).
template <class PT>
__device__ __forceinline__ ElemLane load_elem(PT& P, int32_t& slot, int32_t& col) {
    const bool valid = slot < P.ntargets;
    col = 0;
    if (valid && P.targets) {
        col = slot;
        slot = P.targets[slot];
    }
    const ElemLane e = elem_record(P, slot, valid);
    if (valid && !P.targets) col = e.self;
    return e;
}

// Front-facing decision for the lane's element: FP32 with band, FP64 inside.
template <class PT>
__device__ __forceinline__ bool front_face(PT& P, const ElemLane& e, int32_t slot, float ox, float oy,
                                           float oz, float dx, float dy, float dz, float s, int* f64) {
    const float l1 = fabsf(dx) + fabsf(dy) + fabsf(dz);
    if (fabsf(s) > P.tau_f * l1) return s > 0.0f;
    if (f64) ++*f64;
    const float* t = P.tri + (int64_t)slot * TRI_WORDS;
    return front_fp64(ox, oy, oz, e.cx, e.cy, e.cz, t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7], t[8]);
}

// ------------------------------------------------------------ hierarchy
struct NodeRec {
    float4 a, b, c, d;  // left box lo xyz hi x | hi yz, right lo xy | right lo z hi xyz | refs, hint
};

// The hierarchy is read-only while a kernel runs and the node index is
// uniform: read it through the constant address space (scalar loads).

__device__ __forceinline__ NodeRec load_node(const float* __restrict__ nodes, int node) {
    // a 32-bit byte offset lets the load take it as its scalar offset operand
    const cfloat* q = (const cfloat*)((const char*)nodes + (uint32_t)node * (uint32_t)(NODE_WORDS * 4));
    NodeRec r;
    r.a = make_float4(q[0], q[1], q[2], q[3]);
    r.b = make_float4(q[4], q[5], q[6], q[7]);
    r.c = make_float4(q[8], q[9], q[10], q[11]);
    r.d = make_float4(q[12], q[13], q[14], q[15]);
    return r;
}

// Lane `lane` of v takes the uniform value val (v_writelane; val and lane
// are scalar operands written by the scalar unit; the lane goes through M0).
__device__ __forceinline__ int write_lane(int v, int val, int lane) {
    asm("v_writelane_b32 %0, %1, m0" : "+v"(v) : "s"(val), "{m0}"(lane));
    return v;
}

// Packet traversal.  Control flow is uniform: m is the mask of lanes whose
// segment entered the current node; both child boxes are tested for every
// lane and the ballots are masked with m.  Deferred (node, mask) pairs live
// in three VGPRs, entry i in lane i (depth <= 64).  A step with two inner
// children (the common case) takes one branch on the child kinds; lanes
// found occluded leave the masks where a leaf test finds them, and popped
// masks drop them too.
template <bool STATS, class PT>
__device__ __forceinline__ unsigned long long traverse(PT& P, const Ray& r, unsigned long long live,
                                                       unsigned long long& n_nodes, unsigned long long& n_tris,
                                                       unsigned long long& n_steps, unsigned long long& n_leafw,
                                                       int* rechecks, int& last) {
    const int lane = lane_id();
    unsigned long long occl = 0;
    if (P.N < 2) return 0;
    const float* __restrict__ nodes = P.nodes;
    const float* __restrict__ tri = P.tri;
    // near-first order follows the first live lane's origin (order keys)
    const int l0 = __builtin_ctzll(live);
    const int kx = float_key(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.ox), l0)));
    const int ky = float_key(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.oy), l0)));
    const int kz = float_key(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.oz), l0)));
    unsigned long long m = live;
    int node = 0;
    int sp = 0;
    int stk_node = 0, stk_lo = 0, stk_hi = 0;
    while (true) {
        const NodeRec cur = load_node(nodes, node);
        const int cl = __float_as_int(cur.d.x), cr = __float_as_int(cur.d.y);
        const bool hL = slab(r, cur.a.x, cur.a.y, cur.a.z, cur.a.w, cur.b.x, cur.b.y);
        const bool hR = slab(r, cur.b.z, cur.b.w, cur.c.x, cur.c.y, cur.c.z, cur.c.w);
        unsigned long long mL = __ballot(hL) & m, mR = __ballot(hR) & m;
        if (STATS) {
            n_nodes += (unsigned long long)__popcll(m);
            ++n_steps;
        }
        if ((cl | cr) < 0) {
            if (cl < 0 && mL) {
                const cfloat* t = (const cfloat*)(tri + (int64_t)(~cl) * TRI_WORDS);
                const int who = __float_as_int(t[TRI_ID]);
                const bool act = ((mL >> lane) & 1ull) && r.self != who;
                bool h = false;
                if (act) h = tri_hit(r, t, P.tau_e, P.tau_p, rechecks);
                if (h) last = ~cl;
                if (STATS) {
                    n_tris += (unsigned long long)__popcll(__ballot(act));
                    ++n_leafw;
                }
                occl |= __ballot(h);
                mL = 0;
            }
            if (cr < 0 && mR) {
                const cfloat* t = (const cfloat*)(tri + (int64_t)(~cr) * TRI_WORDS);
                const int who = __float_as_int(t[TRI_ID]);
                const bool act = ((mR >> lane) & 1ull) && r.self != who;
                bool h = false;
                if (act) h = tri_hit(r, t, P.tau_e, P.tau_p, rechecks);
                if (h) last = ~cr;
                if (STATS) {
                    n_tris += (unsigned long long)__popcll(__ballot(act));
                    ++n_leafw;
                }
                occl |= __ballot(h);
                mR = 0;
            }
            if ((live & ~occl) == 0ull) break;
            mL &= ~occl;
            mR &= ~occl;
        }
        if (mL == 0ull) {
            if (mR != 0ull) {
                node = cr;
                m = mR;
                continue;
            }
        } else if (mR == 0ull) {
            node = cl;
            m = mL;
            continue;
        } else {
            const int hint = __float_as_int(cur.d.z);
            const int axis = hint & 3;
            const int ko = axis == 0 ? kx : (axis == 1 ? ky : kz);
            const bool left_first = (ko < __float_as_int(cur.d.w)) == ((hint & 4) != 0);
            const int nfar = left_first ? cr : cl;
            const unsigned long long mfar = left_first ? mR : mL;
            // the stack entry sp lives in lane sp
            stk_node = write_lane(stk_node, nfar, sp);
            stk_lo = write_lane(stk_lo, (int)(unsigned)mfar, sp);
            stk_hi = write_lane(stk_hi, (int)(unsigned)(mfar >> 32), sp);
            ++sp;
            node = left_first ? cl : cr;
            m = left_first ? mL : mR;
            continue;
        }
        // no child entered: pop the next entry that still has live lanes
        bool done = false;
        while (true) {
            if (sp == 0) {
                done = true;
                break;
            }
            --sp;
            node = __builtin_amdgcn_readlane(stk_node, sp);
            const unsigned lo = (unsigned)__builtin_amdgcn_readlane(stk_lo, sp);
            const unsigned hi = (unsigned)__builtin_amdgcn_readlane(stk_hi, sp);
            m = (((unsigned long long)hi << 32) | lo) & ~occl;
            if (m) break;
        }
        if (done) break;
    }
    return occl;
}

// Hierarchy path.  A packet is TK = 2^tk_log2 poses x TE = 64 / TK elements:
// lane = (pose kk, element ee).  Poses are visited in a compact 2D order
// (pose_order) so that a packet's origins are close together; with TK = 64
// the 64 segments of a source share their target and diverge only towards
// their nearby origins.  Each lane sums its element's terms over the sources
// in ascending order, exactly like the brute-force path.
template <bool STATS, bool LV, class PT>
__device__ __forceinline__ void irr_lbvh_packet(PT& P, const LampArgs& L, int64_t kg, int64_t quad) {
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const int tkl = P.tk_log2, tel = 6 - tkl;
    const int kk = lane >> tel, ee = lane & ((1 << tel) - 1);
    const int64_t tile = quad * 4 + w;
    if (tile >= P.ntiles) return;
    const int64_t kpos = (kg << tkl) + kk;
    const bool kok = kpos < P.K;
    const int32_t k = kok ? P.pose_order[kpos] : 0;
    int32_t slot = (int32_t)((tile << tel) + ee), col;
    bool ok;
    {
        const ElemLane e0 = load_elem(P, slot, col);
        ok = kok && e0.valid;
    }
    const float* pp = P.poses + (int64_t)k * P.pose_dim;
    const float px = kok ? pp[0] : 0.0f, py = kok ? pp[1] : 0.0f;
    const float pz0 = (kok && P.pose_dim == 3) ? pp[2] : 0.0f;
    float acc = 0.0f;
    uint32_t bits = 0;
    int rechecks = 0, f64 = 0;
    int* const rc_p = STATS ? &rechecks : nullptr;
    int* const f64_p = STATS ? &f64 : nullptr;
    unsigned n_near = 0;
    unsigned long long n_rays = 0, n_nodes = 0, n_tris = 0, n_vis = 0, n_steps = 0, n_cache = 0, n_cache_hit = 0,
                       n_leafw = 0;
    // Leaf slot of the triangle that last blocked this lane's segment (-1:
    // none yet).  The sources of a lamp are close together, so a triangle
    // that blocks one of them from an element often blocks the next one too.
    // Testing it first is exact: a segment is blocked iff some triangle's
    // predicate says so, and this is that predicate on that triangle.
    int last = -1;
    // The sources differ only in height: the horizontal parts of the
    // direction, their reciprocals and offsets are the same for every source.
    float hix, hiy, hnx, hny;
    {
        const ElemLane e = elem_record(P, slot, ok);
        hix = guard_inv(e.cx - px);
        hiy = guard_inv(e.cy - py);
        hnx = -px * hix;
        hny = -py * hiy;
    }
    for (int j = 0; j < L.S; ++j) {
        const int32_t sl = slot;
        const ElemLane e = elem_record(P, sl, ok);
        const float oz = pz0 + L.dz[j];
        const float dx = px - e.cx, dy = py - e.cy, dz = oz - e.cz;
        const float s = cos_numerator(dx, dy, dz, e.nx, e.ny, e.nz);
        bool f = false;
        if (ok && (!LV || lamp_emits(L, j, e.cz, oz))) f = front_face(P, e, sl, px, py, oz, dx, dy, dz, s, f64_p);
        const unsigned long long live = __ballot(f);
        if (!live) continue;
        Ray r;
        make_ray_z(r, px, py, oz, e.cx, e.cy, e.cz, e.self, hix, hiy, hnx, hny);
        bool trav = f;
        if (P.use_near) {
            // stop rho_t short of the target; the near list covers the rest
            const float r2 = __builtin_fmaf(r.dz, r.dz, __builtin_fmaf(r.dy, r.dy, r.dx * r.dx));
            r.tmax = 1.0f - e.rho_t * __builtin_amdgcn_rsqf(r2);
            trav = f && r.tmax > 0.0f;
        }
        unsigned long long occl = 0;
        if (P.use_cache) {
            const bool tc = f && last >= 0;
            const unsigned long long mc = __ballot(tc);
            if (mc) {
                bool h = false;
                if (tc) h = tri_hit(r, P.tri + (int64_t)last * TRI_WORDS, P.tau_e, P.tau_p, rc_p);
                occl = __ballot(h);
                if (STATS) {
                    n_cache += (unsigned long long)__popcll(mc);
                    n_cache_hit += (unsigned long long)__popcll(occl);
                }
            }
        }
        const unsigned long long tlive = __ballot(trav) & ~occl;
        if (tlive) occl |= traverse<STATS>(P, r, tlive, n_nodes, n_tris, n_steps, n_leafw, rc_p, last);
        bool vis = f && !((occl >> lane) & 1ull);
        if (P.use_near && vis) {
            const int32_t nb = P.near_off[sl], ne = P.near_off[sl + 1];
            for (int32_t q = nb; q < ne && vis; ++q) {
                const int32_t tq = P.near[q];
                if (tri_hit(r, P.tri + (int64_t)tq * TRI_WORDS, P.tau_e, P.tau_p, rc_p)) {
                    vis = false;
                    last = tq;
                }
                if (STATS) ++n_near;
            }
        }
        if (STATS) {
            n_rays += (unsigned long long)__popcll(live);
            n_vis += (unsigned long long)__popcll(__ballot(vis));
        }
        if (vis) {
            acc = acc + (LV ? entry_term_weighted(dx, dy, dz, s, L.pw[j], L) : entry_term(dx, dy, dz, s, L.pw[j]));
            bits |= 1u << j;
        }
    }
    if (ok) {
        const int64_t at = (int64_t)k * P.ld + col;
        P.E[at] = acc;
        if (P.vis) P.vis[at] = bits;
    }
    if (STATS) {
        const unsigned long long rc = wave_sum_u32((unsigned)rechecks), fc = wave_sum_u32((unsigned)f64);
        const unsigned long long nn = wave_sum_u32(n_near);
        if (lane == 0) {
            atomicAdd(P.stats + UVC_STAT_RAYS, n_rays);
            atomicAdd(P.stats + UVC_STAT_NODES, n_nodes);
            atomicAdd(P.stats + UVC_STAT_TRIS, n_tris);
            atomicAdd(P.stats + UVC_STAT_RECHECK, rc);
            atomicAdd(P.stats + UVC_STAT_FRONT64, fc);
            atomicAdd(P.stats + UVC_STAT_VISIBLE, n_vis);
            atomicAdd(P.stats + UVC_STAT_STEPS, n_steps);
            atomicAdd(P.stats + UVC_STAT_NEAR, nn);
            atomicAdd(P.stats + UVC_STAT_CACHE, n_cache);
            atomicAdd(P.stats + UVC_STAT_CACHE_HIT, n_cache_hit);
            atomicAdd(P.stats + UVC_STAT_LEAF_STEPS, n_leafw);
        }
    }
}

// Persistent work distribution.  The items (workgroup-sized pieces of
// work) are cut into 8 contiguous ranges, one per XCD (workgroups are
// dispatched to the XCDs round robin, so workgroup b runs on XCD b mod 8).
// A workgroup takes items from its own XCD's range through an atomic
// counter, which keeps each XCD's L2 on a compact part of the work, then
// takes what is left in the other ranges; it exits once all 8 are
// exhausted.  counter[x] counts the items taken from range x.
struct PersistArgs {
    unsigned long long* counter;  // 8 counters, zeroed before the launch
    int64_t range_off[9];         // range x = [range_off[x], range_off[x + 1])
};

__device__ __forceinline__ int64_t next_item(const PersistArgs& Q, int& range, long long* item_s) {
    const int home = (int)(blockIdx.x & 7u);
    while (range < 8) {
        const int x = (home + range) & 7;
        const int64_t r0 = Q.range_off[x], r1 = Q.range_off[x + 1];
        if (threadIdx.x == 0) *item_s = (long long)(r0 + (int64_t)atomicAdd(Q.counter + x, 1ull));
        __syncthreads();
        // the item is the same for the whole workgroup: make that explicit
        const long long v = *item_s;
        const int64_t item = (int64_t)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32))
                                        << 32) |
                                       (unsigned)__builtin_amdgcn_readfirstlane((int)v));
        __syncthreads();
        if (item < r1) return item;
        ++range;
    }
    return -1;
}

template <bool STATS, bool LV>
__device__ __forceinline__ void irr_lbvh_body(const IrrParams& P, const PersistArgs& Q) {
    __shared__ long long item_s;
    int range = 0;
    for (int64_t item; (item = next_item(Q, range, &item_s)) >= 0;)
        irr_lbvh_packet<STATS, LV, const IrrParams>(P, P.lamp, item % P.kgroups, item / P.kgroups);
}

// Kernel variants differ only in the occupancy the register allocator aims
// for (waves per SIMD); which one is fastest depends on the scene.  LV: the
// lamp has an emission pattern or hemisphere masks (a separate
// instantiation, so that uniform lamps run the plain code).
template <bool STATS, bool LV>
__global__ __launch_bounds__(256) void k_irr_lbvh(IrrParams P, PersistArgs Q) {
    irr_lbvh_body<STATS, LV>(P, Q);
}
template <bool STATS, bool LV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_irr_lbvh_w6(IrrParams P,
                                                                                             PersistArgs Q) {
    irr_lbvh_body<STATS, LV>(P, Q);
}
template <bool STATS, bool LV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_irr_lbvh_w8(IrrParams P,
                                                                                             PersistArgs Q) {
    irr_lbvh_body<STATS, LV>(P, Q);
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int n) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n) p[threadIdx.x] = v;
}

// ------------------------------------------------------------- batched
// Many rooms in one persistent launch.  The work queue lists the rooms in
// descending estimated cost per work item (longest first); item_off[q] is the
// first item of queue entry q and room_of[q] its room.  Each workgroup takes
// the next item from an atomic counter until the queue is drained, so every
// wave reaches the exit.  An item is one workgroup's worth of work of the
// single-room kernel (4 packets), run by the same code.
typedef __attribute__((address_space(4))) IrrParams CIrrParams;

struct BatchArgs {
    const IrrParams* rooms;   // per-room parameters (their lamp fields are not read)
    LampArgs lamp;            // the lamp shared by every room
    const int64_t* item_off;  // n_queue + 1
    const int32_t* room_of;   // n_queue
    int32_t n_queue;
    int64_t total;
    PersistArgs q;            // the item ranges and their counters
};

__device__ __forceinline__ int32_t ufl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t ufl64(int64_t v) {
    return (int64_t)(((unsigned long long)(unsigned)ufl((int32_t)(v >> 32)) << 32) | (unsigned)ufl((int32_t)v));
}
template <class T>
__device__ __forceinline__ T* uflp(T* p) {
    return reinterpret_cast<T*>(ufl64(reinterpret_cast<int64_t>(p)));
}

// A room's parameters, read by the whole workgroup at a uniform address and
// made explicitly uniform so that they live in scalar registers; the lamp is
// the batch's.
__device__ __forceinline__ IrrParams uniform_room(const IrrParams* src) {
    IrrParams P;
    P.tri = uflp(src->tri);
    P.elem = uflp(src->elem);
    P.nodes = uflp(src->nodes);
    P.near_off = uflp(src->near_off);
    P.near = uflp(src->near);
    P.poses = uflp(src->poses);
    P.pose_order = uflp(src->pose_order);
    P.targets = uflp(src->targets);
    P.K = ufl64(src->K);
    P.N = ufl64(src->N);
    P.ntargets = ufl64(src->ntargets);
    P.ld = ufl64(src->ld);
    P.ntiles = ufl64(src->ntiles);
    P.nquads = ufl64(src->nquads);
    P.kgroups = ufl64(src->kgroups);
    P.pose_dim = ufl(src->pose_dim);
    P.tile_tris = ufl(src->tile_tris);
    P.tk_log2 = ufl(src->tk_log2);
    P.use_near = ufl(src->use_near);
    P.use_cache = ufl(src->use_cache);
    P.waves = ufl(src->waves);
    P.tau_f = __int_as_float(ufl(__float_as_int(src->tau_f)));
    P.tau_e = __int_as_float(ufl(__float_as_int(src->tau_e)));
    P.tau_p = __int_as_float(ufl(__float_as_int(src->tau_p)));
    P.E = uflp(src->E);
    P.vis = uflp(src->vis);
    P.stats = uflp(src->stats);
    P.lamp.S = 0;  // the batch's lamp is passed separately
    return P;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_irr_batched(BatchArgs B) {
    __shared__ long long item_s;
    int range = 0;
    for (int64_t item; (item = next_item(B.q, range, &item_s)) >= 0;) {
        int lo = 0, hi = B.n_queue - 1;  // last q with item_off[q] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B.item_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const int32_t room = ufl(B.room_of[ufl(lo)]);
        // the rooms' parameters are never written while the kernel runs: read
        // them through the constant address space (scalar loads)
        const CIrrParams& P = ((const CIrrParams*)(B.rooms))[room];
        const int64_t local = ufl64(item - B.item_off[lo]);
        irr_lbvh_packet<false, false, const CIrrParams>(P, B.lamp, local % P.kgroups, local / P.kgroups);
    }
}

// ---------------------------------------------------------- brute force
template <bool STATS, bool LV>
__global__ __launch_bounds__(256) void k_irr_brute(IrrParams P) {
    extern __shared__ float4 lds[];  // tile_tris x 3 float4
    int64_t kk, quad;
    block_coords(P, kk, quad);  // kgroups = K: one pose per workgroup
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6), tid = (int)threadIdx.x;
    const int64_t tile = quad * 4 + w;
    int32_t slot = (int32_t)(tile * 64 + lane), col;
    const ElemLane e = load_elem(P, slot, col);  // invalid lanes (and whole waves past the end) idle
    const float* pp = P.poses + kk * P.pose_dim;
    const float px = pp[0], py = pp[1], pz0 = (P.pose_dim == 3) ? pp[2] : 0.0f;
    const int TT = P.tile_tris;
    float acc = 0.0f;
    uint32_t bits = 0;
    int rechecks = 0, f64 = 0;
    unsigned long long n_rays = 0, n_tris = 0, n_vis = 0;
    for (int j = 0; j < P.lamp.S; ++j) {
        const float oz = pz0 + P.lamp.dz[j];
        const float dx = px - e.cx, dy = py - e.cy, dz = oz - e.cz;
        const float s = cos_numerator(dx, dy, dz, e.nx, e.ny, e.nz);
        bool f = false;
        if (e.valid && (!LV || lamp_emits(P.lamp, j, e.cz, oz))) f = front_face(P, e, slot, px, py, oz, dx, dy, dz, s, &f64);
        const unsigned long long live = __ballot(f);
        Ray r;
        make_ray(r, px, py, oz, e.cx, e.cy, e.cz, e.self);
        bool occluded = false;
        const int any_live = __syncthreads_or(live != 0ull);
        if (any_live) {
            for (int64_t base = 0; base < P.N; base += TT) {
                const int cnt = (int)((P.N - base) < TT ? (P.N - base) : TT);
                __syncthreads();
                for (int t = tid; t < cnt; t += 256) {
                    const float* tp = P.tri + (base + t) * TRI_WORDS;
                    const float4* qp = reinterpret_cast<const float4*>(tp);
                    const float4 q0 = qp[0], q1 = qp[1], q2 = qp[2], q3 = qp[3], q4 = qp[4];
                    // q0 = v0xyz v1x, q1 = v1yz v2xy, q2 = v2z e01xyz, q3 = e12xyz e20x, q4 = e20yz L id
                    const float ax = q0.x - px, ay = q0.y - py, az = q0.z - oz;
                    const float bx = q0.w - px, by = q1.x - py, bz = q1.y - oz;
                    const float cx = q1.z - px, cy = q1.w - py, cz = q2.x - oz;
                    const float e01x = q2.y, e01y = q2.z, e01z = q2.w;
                    const float e12x = q3.x, e12y = q3.y, e12z = q3.z;
                    const float e20x = q3.w, e20y = q4.x, e20z = q4.y;
                    const float g = max3f(amax3(ax, ay, az), amax3(bx, by, bz), amax3(cx, cy, cz));
                    float4 o0, o1, o2;
                    o0.x = fmaf(by, e12z, -bz * e12y); o0.y = fmaf(bz, e12x, -bx * e12z); o0.z = fmaf(bx, e12y, -by * e12x);
                    o0.w = fmaf(cy, e20z, -cz * e20y); o1.x = fmaf(cz, e20x, -cx * e20z); o1.y = fmaf(cx, e20y, -cy * e20x);
                    o1.z = fmaf(ay, e01z, -az * e01y); o1.w = fmaf(az, e01x, -ax * e01z); o2.x = fmaf(ax, e01y, -ay * e01x);
                    o2.y = P.tau_e * g * fmaf(0x1p-28f, g, q4.z);
                    o2.z = q4.w;  // input index (int bits)
                    o2.w = 0.f;
                    lds[3 * t + 0] = o0;
                    lds[3 * t + 1] = o1;
                    lds[3 * t + 2] = o2;
                }
                __syncthreads();
                for (int t0 = 0; t0 < cnt; t0 += 32) {
                    const unsigned long long act = live & ~__ballot(occluded);
                    if (!act) break;
                    const int t1 = (cnt - t0) < 32 ? cnt : t0 + 32;
                    if (STATS) n_tris += (unsigned long long)__popcll(act) * (unsigned long long)(t1 - t0);
                    for (int t = t0; t < t1; ++t) {
                        const float4 o0 = lds[3 * t + 0], o1 = lds[3 * t + 1], o2 = lds[3 * t + 2];
                        const float U = fmaf(r.dz, o0.z, fmaf(r.dy, o0.y, r.dx * o0.x));
                        const float V = fmaf(r.dz, o1.y, fmaf(r.dy, o1.x, r.dx * o0.w));
                        const float W = fmaf(r.dz, o2.x, fmaf(r.dy, o1.w, r.dx * o1.z));
                        const float be = o2.y * r.l1;
                        const float mn = min3f(U, V, W), mx = max3f(U, V, W);
                        if (!(mn < -be && mx > be) && f && !occluded && __float_as_int(o2.z) != e.self) {
                            const float* tp = P.tri + (base + t) * TRI_WORDS;
                            const int q = tri_rare(r.ox, r.oy, r.oz, r.tx, r.ty, r.tz, tp[0], tp[1], tp[2], tp[3],
                                                   tp[4], tp[5], tp[6], tp[7], tp[8], mn, mx, be, P.tau_p);
                            rechecks += q >> 1;
                            occluded = (q & 1) != 0;
                        }
                    }
                }
            }
        }
        const bool vis = f && !occluded;
        if (STATS) {
            n_rays += (unsigned long long)__popcll(live);
            n_vis += (unsigned long long)__popcll(__ballot(vis));
        }
        if (vis) {
            acc = acc + (LV ? entry_term_weighted(dx, dy, dz, s, P.lamp.pw[j], P.lamp)
                            : entry_term(dx, dy, dz, s, P.lamp.pw[j]));
            bits |= 1u << j;
        }
    }
    if (e.valid) {
        P.E[kk * P.ld + col] = acc;
        if (P.vis) P.vis[kk * P.ld + col] = bits;
    }
    if (STATS) {
        const unsigned long long rc = wave_sum_u32((unsigned)rechecks), fc = wave_sum_u32((unsigned)f64);
        if (lane == 0) {
            atomicAdd(P.stats + UVC_STAT_RAYS, n_rays);
            atomicAdd(P.stats + UVC_STAT_TRIS, n_tris);
            atomicAdd(P.stats + UVC_STAT_RECHECK, rc);
            atomicAdd(P.stats + UVC_STAT_FRONT64, fc);
            atomicAdd(P.stats + UVC_STAT_VISIBLE, n_vis);
        }
    }
}

// ------------------------------------------------------------ CSR pieces
// One wave per row: number of nonzero entries.
__global__ void k_row_count(const float* __restrict__ E, int64_t rows, int64_t N, int64_t* __restrict__ counts) {
    const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (row >= rows) return;
    const float* e = E + row * N;
    unsigned long long c = 0;
    for (int64_t base = 0; base < N; base += 64) {
        const int64_t i = base + lane;
        const bool nz = i < N && e[i] != 0.0f;
        c += (unsigned long long)__popcll(__ballot(nz));
    }
    if (lane == 0) counts[row] = (int64_t)c;
}

// Exclusive scan of n int64 counts into out[0..n] (out[n] = total), plus a
// base offset; one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_i64(const int64_t* __restrict__ in, int64_t* __restrict__ out,
                                                   int64_t n, int64_t base) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = base;
    __syncthreads();
    for (int64_t b0 = 0; b0 < n; b0 += 1024) {
        const int64_t i = b0 + tid;
        const int64_t v = (i < n) ? in[i] : 0;
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t t = (tid >= off) ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += t;
            __syncthreads();
        }
        if (i < n) out[i] = carry + part[tid] - v;
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
    if (tid == 0) out[n] = carry;
}

// One wave per row: write the row's nonzeros in ascending column order.
__global__ void k_row_gather(const float* __restrict__ E, int64_t rows, int64_t N, const int64_t* __restrict__ offs,
                             int32_t* __restrict__ col, float* __restrict__ val) {
    const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (row >= rows) return;
    const float* e = E + row * N;
    int64_t pos = offs[row];
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int64_t base = 0; base < N; base += 64) {
        const int64_t i = base + lane;
        const float v = (i < N) ? e[i] : 0.0f;
        const bool nz = v != 0.0f;
        const unsigned long long mk = __ballot(nz);
        if (nz) {
            const int64_t p = pos + __popcll(mk & lt);
            col[p] = (int32_t)i;
            val[p] = v;
        }
        pos += __popcll(mk);
    }
}

// ------------------------------------------------------------------ host
// Validated device copy of a lamp (shared by every kernel that emits from
// lamp sources).
uvc_status lamp_args(const uvc_lamp* lamp, LampArgs& L) {
    if (!lamp || lamp->n_src < 1 || lamp->n_src > 32 || !lamp->dz || !lamp->power_w)
        return fail(UVC_EINVAL, "lamp must have 1..32 sources with dz and power arrays");
    std::memset(&L, 0, sizeof(L));
    L.S = lamp->n_src;
    for (int j = 0; j < lamp->n_src; ++j) {
        if (!std::isfinite(lamp->dz[j])) return fail(UVC_EINVAL, "lamp dz[" + std::to_string(j) + "] is not finite");
        if (!(lamp->power_w[j] > 0.f) || !std::isfinite(lamp->power_w[j]))
            return fail(UVC_EINVAL, "lamp power[" + std::to_string(j) + "] must be positive and finite");
        L.dz[j] = lamp->dz[j];
        L.pw[j] = (float)((double)lamp->power_w[j] / (4.0 * M_PI));
    }
    if (lamp->n_prof != 0) {
        if (lamp->n_prof < 2 || lamp->n_prof > 33 || !lamp->profile)
            return fail(UVC_EINVAL, "lamp emission table must have 2..33 entries");
        bool any = false;
        for (int q = 0; q < lamp->n_prof; ++q) {
            const float v = lamp->profile[q];
            if (!std::isfinite(v) || v < 0.f)
                return fail(UVC_EINVAL, "lamp emission table entry " + std::to_string(q) + " must be finite and >= 0");
            any = any || v > 0.f;
            L.prof[q] = v;
        }
        if (!any) return fail(UVC_EINVAL, "lamp emission table is all zero");
        L.nprof = lamp->n_prof;
        L.ph = 0.5f * (float)(lamp->n_prof - 1);
    }
    const uint32_t srcmask = lamp->n_src == 32 ? 0xffffffffu : ((1u << lamp->n_src) - 1u);
    if ((lamp->up_mask | lamp->down_mask) & ~srcmask)
        return fail(UVC_EINVAL, "lamp hemisphere masks name sources beyond n_src");
    if (lamp->up_mask & lamp->down_mask)
        return fail(UVC_EINVAL, "a source cannot emit only upwards and only downwards");
    L.up = lamp->up_mask;
    L.down = lamp->down_mask;
    return UVC_OK;
}

static bool lamp_variant(const LampArgs& L) { return L.nprof > 0 || L.up != 0u || L.down != 0u; }

static uvc_status make_params(const uvc_scene* s, const float* poses, int64_t K, int32_t pd, const uvc_lamp* lamp,
                              const uvc_opts* opts, IrrParams& P) {
    if (!s) return fail(UVC_EINVAL, "scene is NULL");
    if (K < 0) return fail(UVC_EINVAL, "K < 0");
    if (pd != 2 && pd != 3) return fail(UVC_EINVAL, "pose_dim must be 2 or 3");
    if (!lamp || lamp->n_src < 1 || lamp->n_src > 32 || !lamp->dz || !lamp->power_w)
        return fail(UVC_EINVAL, "lamp must have 1..32 sources with dz and power arrays");
    if (K > 0 && s->n > 0 && !poses) return fail(UVC_EINVAL, "poses is NULL");
    std::memset(&P, 0, sizeof(P));
    UVC_TRY(lamp_args(lamp, P.lamp));
    const float bs = opts ? opts->band_scale : 1.0f;
    if (!(bs >= 0.f)) return fail(UVC_EINVAL, "band_scale must be >= 0");
    P.tau_f = TAU_F * bs;
    P.tau_e = TAU_E * bs;
    P.tau_p = TAU_P * bs;
    P.tri = s->tri;
    P.elem = s->elem;
    P.nodes = s->nodes;
    P.near_off = s->near_off;
    P.near = s->near;
    P.use_near = (opts && (opts->flags & UVC_FLAG_NO_NEAR)) ? 0 : 1;
    P.use_cache = (opts && (opts->flags & UVC_FLAG_NO_CACHE)) ? 0 : 1;
    P.waves = (opts && opts->waves > 0) ? opts->waves : 6;
    if (P.waves != 5 && P.waves != 6 && P.waves != 8) return fail(UVC_EINVAL, "waves must be 0, 5, 6 or 8");
    P.poses = poses;
    P.K = K;
    P.N = s->n;
    P.ntargets = s->n;
    P.ld = s->n;
    P.targets = nullptr;
    P.pose_dim = pd;
    int tk = (opts && opts->packet_poses > 0) ? opts->packet_poses : 16;
    if (tk != 1 && tk != 2 && tk != 4 && tk != 8 && tk != 16 && tk != 32 && tk != 64)
        return fail(UVC_EINVAL, "packet_poses must be a power of two in [1, 64]");
    P.tk_log2 = 0;
    while ((1 << P.tk_log2) < tk) ++P.tk_log2;
    P.tile_tris = (opts && opts->tile_tris > 0) ? opts->tile_tris : 512;
    if (P.tile_tris > 2048) return fail(UVC_EINVAL, "tile_tris must be <= 2048");
    P.stats = opts ? reinterpret_cast<unsigned long long*>(opts->stats_dev) : nullptr;
    return UVC_OK;
}

// Poses are copied to the host once per call: validated there (finite, and
// every source point within 2 * max_abs_coord of the origin, which bounds the
// rounding the box padding has to absorb) and sorted into a compact order.
static uvc_status fetch_poses(const uvc_scene* s, const float* poses, int64_t K, int pd, const LampArgs& L,
                              hipStream_t st, std::vector<float>& hp) {
    hp.assign((size_t)K * pd, 0.f);
    if (K == 0) return UVC_OK;
    UVC_HIP(hipMemcpyAsync(hp.data(), poses, hp.size() * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    float dzmin = L.dz[0], dzmax = L.dz[0];
    for (int j = 1; j < L.S; ++j) {
        dzmin = std::min(dzmin, L.dz[j]);
        dzmax = std::max(dzmax, L.dz[j]);
    }
    const float lim = 2.0f * std::max(s->max_abs, 1e-30f);
    for (int64_t k = 0; k < K; ++k) {
        const float x = hp[k * pd], y = hp[k * pd + 1], z = (pd == 3) ? hp[k * pd + 2] : 0.0f;
        if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
            return fail(UVC_EINVAL, "pose " + std::to_string(k) + ": a pose coordinate is not finite");
        const float z0 = z + dzmin, z1 = z + dzmax;
        if (std::fabs(x) > lim || std::fabs(y) > lim || std::fabs(z0) > lim || std::fabs(z1) > lim)
            return fail(UVC_EINVAL, "pose " + std::to_string(k) +
                                        ": a source point lies farther than 2 * max_abs_coord from the origin");
    }
    return UVC_OK;
}

static uint64_t spread_bits(uint64_t v, int stride) {
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (b * stride);
    return r;
}

// Positions 0..kb-1 -> pose rows k0..k0+kb-1 (relative to k0) in Morton order
// of the pose coordinates.
static void pose_order(const std::vector<float>& hp, int pd, int64_t k0, int64_t kb, std::vector<int32_t>& order) {
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int64_t k = 0; k < kb; ++k)
        for (int a = 0; a < pd; ++a) {
            const float v = hp[(k0 + k) * pd + a];
            lo[a] = k ? std::min(lo[a], v) : v;
            hi[a] = k ? std::max(hi[a], v) : v;
        }
    const int bits = pd == 2 ? 16 : 10;
    const double cells = (double)(1u << bits);
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)kb);
    for (int64_t k = 0; k < kb; ++k) {
        uint64_t code = 0;
        for (int a = 0; a < pd; ++a) {
            const double ext = (double)hi[a] - (double)lo[a];
            double q = ext > 0 ? ((double)hp[(k0 + k) * pd + a] - lo[a]) / ext * cells : 0.0;
            q = std::min(std::max(q, 0.0), cells - 1.0);
            code |= spread_bits((uint64_t)q, pd) << (pd - 1 - a);
        }
        key[(size_t)k] = {code, (int32_t)k};
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, int32_t>& a, const std::pair<uint64_t, int32_t>& b) {
                         return a.first < b.first;
                     });
    order.resize((size_t)kb);
    for (int64_t k = 0; k < kb; ++k) order[(size_t)k] = key[(size_t)k].second;
}

static int choose_path(const uvc_scene* s, const uvc_opts* opts) {
    const int p = opts ? opts->path : UVC_PATH_AUTO;
    if (p == UVC_PATH_LBVH || p == UVC_PATH_BRUTE) return p;
    return s->n <= 2048 ? UVC_PATH_BRUTE : UVC_PATH_LBVH;
}

// UVC_PATH_AUTO with a registered tuning table: the table's path, and its
// packet shape, occupancy and LDS tile wherever the caller left them at 0.
// Other options (flags, bands, counters, timing) stay the caller's.
static uvc_opts resolve_auto(const uvc_scene* s, const uvc_lamp* lamp, const uvc_opts* opts) {
    uvc_opts o{};
    o.band_scale = 1.0f;
    if (opts) o = *opts;
    if (o.path != UVC_PATH_AUTO || !s || !lamp) return o;
    uvc_opts t{};
    if (!tune_lookup(nullptr, s->n, lamp->n_src, t)) return o;
    o.path = t.path;
    if (o.packet_poses <= 0) o.packet_poses = t.packet_poses;
    if (o.waves <= 0) o.waves = t.waves;
    if (o.tile_tris <= 0) o.tile_tris = t.tile_tris;
    return o;
}

// Launch the irradiance kernel for P.K poses into P.E / P.vis.
// counter_ext: NULL (a stream-ordered allocation holds the persistent
// loop's 8 work counters for this launch) or 8 caller-provided counters.
static uvc_status launch_irr_impl(const IrrParams& P0, int path, hipStream_t st,
                                  unsigned long long* counter_ext = nullptr) {
    if (P0.K == 0 || P0.N == 0) return UVC_OK;
    IrrParams P = P0;
    const int64_t per = (path == UVC_PATH_BRUTE) ? 64 : ((int64_t)1 << (6 - P.tk_log2));
    P.ntiles = (P.ntargets + per - 1) / per;
    P.nquads = (P.ntiles + 3) / 4;
    P.kgroups = (path == UVC_PATH_BRUTE) ? P.K : ((P.K + (1 << P.tk_log2) - 1) >> P.tk_log2);
    if (P.ntargets == 0) return UVC_OK;
    const uint64_t blocks = (uint64_t)P.nquads * (uint64_t)P.kgroups;
    if (blocks > 0x7fffffffull) return fail(UVC_EUNSUPPORTED, "launch too large; split the poses");
    const bool stats = P.stats != nullptr;
    if (path == UVC_PATH_BRUTE) {
        const size_t shm = (size_t)P.tile_tris * 48;  // 3 float4 per staged triangle
        const bool lv = lamp_variant(P.lamp);
        if (stats && lv)
            hipLaunchKernelGGL((k_irr_brute<true, true>), dim3((unsigned)blocks), dim3(256), shm, st, P);
        else if (stats)
            hipLaunchKernelGGL((k_irr_brute<true, false>), dim3((unsigned)blocks), dim3(256), shm, st, P);
        else if (lv)
            hipLaunchKernelGGL((k_irr_brute<false, true>), dim3((unsigned)blocks), dim3(256), shm, st, P);
        else
            hipLaunchKernelGGL((k_irr_brute<false, false>), dim3((unsigned)blocks), dim3(256), shm, st, P);
    } else {
        // persistent launch: as many workgroups as the variant keeps resident
        // (4 waves each, `waves` per SIMD), draining the items per XCD range
        int cus = 256, dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int waves = stats ? 5 : (P.waves == 8 ? 8 : (P.waves == 6 ? 6 : 5));
        const uint64_t grid = std::min<uint64_t>(blocks, (uint64_t)std::max(1, cus) * (uint64_t)waves);
        PersistArgs Q{nullptr, {}};
        for (int x = 0; x <= 8; ++x) Q.range_off[x] = (int64_t)(blocks * (uint64_t)x / 8u);
        if (counter_ext)
            Q.counter = counter_ext;
        else
            UVC_HIP(hipMallocAsync(reinterpret_cast<void**>(&Q.counter), 8 * sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, Q.counter, 0ull, 8);
        const dim3 g((unsigned)grid), b(256);
        if (!lamp_variant(P.lamp)) {
            if (stats)
                hipLaunchKernelGGL((k_irr_lbvh<true, false>), g, b, 0, st, P, Q);
            else if (waves == 8)
                hipLaunchKernelGGL((k_irr_lbvh_w8<false, false>), g, b, 0, st, P, Q);
            else if (waves == 6)
                hipLaunchKernelGGL((k_irr_lbvh_w6<false, false>), g, b, 0, st, P, Q);
            else
                hipLaunchKernelGGL((k_irr_lbvh<false, false>), g, b, 0, st, P, Q);
        } else {
            if (stats)
                hipLaunchKernelGGL((k_irr_lbvh<true, true>), g, b, 0, st, P, Q);
            else if (waves == 8)
                hipLaunchKernelGGL((k_irr_lbvh_w8<false, true>), g, b, 0, st, P, Q);
            else if (waves == 6)
                hipLaunchKernelGGL((k_irr_lbvh_w6<false, true>), g, b, 0, st, P, Q);
            else
                hipLaunchKernelGGL((k_irr_lbvh<false, true>), g, b, 0, st, P, Q);
        }
        const hipError_t le = hipGetLastError();
        const hipError_t fe = counter_ext ? hipSuccess : hipFreeAsync(Q.counter, st);
        if (le != hipSuccess) return fail(UVC_EDEVICE, std::string("irradiance launch: ") + hipGetErrorString(le));
        if (fe != hipSuccess) return fail(UVC_EDEVICE, std::string("counter release: ") + hipGetErrorString(fe));
        return UVC_OK;
    }
    UVC_HIP(hipGetLastError());
    return UVC_OK;
}

// Launch with optional HIP-event timing of the kernel on the caller's stream.
static uvc_status launch_irr(const IrrParams& P, int path, hipStream_t st, float* kernel_ms,
                             unsigned long long* counter_ext = nullptr) {
    if (!kernel_ms) return launch_irr_impl(P, path, st, counter_ext);
    hipEvent_t e0, e1;
    UVC_HIP(hipEventCreate(&e0));
    UVC_HIP(hipEventCreate(&e1));
    uvc_status r = UVC_OK;
    hipError_t he = hipEventRecord(e0, st);
    if (he == hipSuccess) r = launch_irr_impl(P, path, st, counter_ext);
    if (he == hipSuccess && r == UVC_OK) he = hipEventRecord(e1, st);
    if (he == hipSuccess && r == UVC_OK) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess && r == UVC_OK) he = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != UVC_OK) return r;
    if (he != hipSuccess) return fail(UVC_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(he));
    *kernel_ms += ms;
    return UVC_OK;
}

}  // namespace uvc

using namespace uvc;

struct uvc_csr_job {
    int device = 0;
    int64_t K = 0, N = 0, nnz = 0;
    int64_t* counts = nullptr;  // K row counts (device)
    struct Chunk {
        int32_t* col;
        float* val;
        int64_t nnz;
    };
    std::vector<Chunk> chunks;
};

// Device copy of a pose order (stream-ordered allocation, freed after use).
static uvc_status upload_order(const std::vector<float>& hp, int pd, int64_t k0, int64_t kb, hipStream_t st,
                               int32_t** out) {
    std::vector<int32_t> ord;
    pose_order(hp, pd, k0, kb, ord);
    UVC_HIP(hipMallocAsync(reinterpret_cast<void**>(out), (size_t)std::max<int64_t>(kb, 1) * 4, st));
    hipError_t e = hipMemcpyAsync(*out, ord.data(), (size_t)kb * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // ord is released on return
    if (e != hipSuccess) {
        (void)hipFreeAsync(*out, st);
        *out = nullptr;
        return fail(UVC_EDEVICE, std::string("pose order upload: ") + hipGetErrorString(e));
    }
    return UVC_OK;
}

extern "C" uvc_status uvc_compute_irradiance_dense(const uvc_scene* scene, const float* poses_dev, int64_t K,
                                                   int32_t pose_dim, const uvc_lamp* lamp, const uvc_opts* opts_in,
                                                   float* E_dev, uint32_t* vis_dev, void* hip_stream) {
    const uvc_opts opts_r = resolve_auto(scene, lamp, opts_in);
    const uvc_opts* opts = &opts_r;
    IrrParams P;
    UVC_TRY(make_params(scene, poses_dev, K, pose_dim, lamp, opts, P));
    if (K == 0 || scene->n == 0) return UVC_OK;
    if (!E_dev) return fail(UVC_EINVAL, "E is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<float> hp;
    UVC_TRY(fetch_poses(scene, poses_dev, K, pose_dim, P.lamp, st, hp));
    const int path = choose_path(scene, opts);
    int32_t* dorder = nullptr;
    if (path == UVC_PATH_LBVH) UVC_TRY(upload_order(hp, pose_dim, 0, K, st, &dorder));
    P.pose_order = dorder;
    P.E = E_dev;
    P.vis = vis_dev;
    if (opts && opts->kernel_ms) *opts->kernel_ms = 0.f;
    const uvc_status r = launch_irr(P, path, st, opts ? opts->kernel_ms : nullptr);
    if (dorder) (void)hipFreeAsync(dorder, st);
    return r;
}

// ------------------------------------------------ dense, without allocation
// The dense call allocates two small stream-ordered buffers per call (the
// persistent loop's work counters and the pose visiting order).  For callers
// that cannot allocate, the variant below takes both from one file-scope
// device array instead.  Each device holds its own copy of the array at its
// own address, looked up once per device with hipGetSymbolAddress; host code
// uses only that address.  Layout: 8 work counters at byte 0, the pose
// check word at byte 64, the pose order (int32) from byte 256.
namespace uvc {
constexpr int64_t NOALLOC_MAX_POSES = (int64_t)1 << 20;
constexpr size_t SCR_CHECK = 64, SCR_ORDER = 256;
constexpr size_t SCRATCH_BYTES = SCR_ORDER + (size_t)NOALLOC_MAX_POSES * 4;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up on the
// first call on each device, with that device current).
static uvc_status scratch_address(void** out) {
    int dev = 0;
    UVC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(UVC_EUNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(UVC_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return UVC_OK;
}

// The host-side pose check of the dense call, on the device: *bad receives
// the smallest (k << 1) | c over the offending poses, c = 0 for a
// non-finite coordinate, 1 for a source point farther than lim from the
// origin (left at ~0 when every pose passes).
__global__ void k_check_poses(const float* __restrict__ poses, int64_t K, int pd, float dzmin, float dzmax, float lim,
                              unsigned long long* __restrict__ bad) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= K) return;
    const float x = poses[k * pd], y = poses[k * pd + 1], z = (pd == 3) ? poses[k * pd + 2] : 0.0f;
    unsigned long long code = ~0ull;
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        code = (unsigned long long)k << 1;
    } else {
        const float z0 = z + dzmin, z1 = z + dzmax;
        if (fabsf(x) > lim || fabsf(y) > lim || fabsf(z0) > lim || fabsf(z1) > lim)
            code = ((unsigned long long)k << 1) | 1ull;
    }
    if (code != ~0ull) atomicMin(bad, code);
}

__global__ void k_iota_i32(int32_t* __restrict__ p, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) p[q] = (int32_t)q;
}
}  // namespace uvc

extern "C" uvc_status uvc_compute_irradiance_dense_noalloc(const uvc_scene* scene, const float* poses_dev, int64_t K,
                                                           int32_t pose_dim, const uvc_lamp* lamp,
                                                           const uvc_opts* opts, float* E_dev, uint32_t* vis_dev,
                                                           void* hip_stream) {
    IrrParams P;
    UVC_TRY(make_params(scene, poses_dev, K, pose_dim, lamp, opts, P));
    if (opts && opts->kernel_ms)
        return fail(UVC_EINVAL, "kernel_ms is not available without allocation (timing creates HIP events)");
    if (K > NOALLOC_MAX_POSES)
        return fail(UVC_EINVAL, "K = " + std::to_string(K) + " exceeds the no-allocation limit of " +
                                    std::to_string(NOALLOC_MAX_POSES) + " poses");
    if (K == 0 || scene->n == 0) return UVC_OK;
    if (!E_dev) return fail(UVC_EINVAL, "E is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    void* base = nullptr;
    UVC_TRY(scratch_address(&base));
    unsigned long long* counters = reinterpret_cast<unsigned long long*>(base);
    unsigned long long* checkw = reinterpret_cast<unsigned long long*>((char*)base + SCR_CHECK);
    int32_t* order = reinterpret_cast<int32_t*>((char*)base + SCR_ORDER);
    float dzmin = P.lamp.dz[0], dzmax = P.lamp.dz[0];
    for (int j = 1; j < P.lamp.S; ++j) {
        dzmin = std::min(dzmin, P.lamp.dz[j]);
        dzmax = std::max(dzmax, P.lamp.dz[j]);
    }
    const float lim = 2.0f * std::max(scene->max_abs, 1e-30f);
    const unsigned gk = (unsigned)((K + 255) / 256);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, checkw, ~0ull, 1);
    hipLaunchKernelGGL(k_check_poses, dim3(gk), dim3(256), 0, st, poses_dev, K, pose_dim, dzmin, dzmax, lim, checkw);
    UVC_HIP(hipGetLastError());
    unsigned long long bad = 0;
    UVC_HIP(hipMemcpyAsync(&bad, checkw, 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    if (bad != ~0ull) {
        const std::string k = std::to_string(bad >> 1);
        if ((bad & 1ull) == 0) return fail(UVC_EINVAL, "pose " + k + ": a pose coordinate is not finite");
        return fail(UVC_EINVAL, "pose " + k + ": a source point lies farther than 2 * max_abs_coord from the origin");
    }
    const int path = choose_path(scene, opts);
    if (path == UVC_PATH_LBVH) {
        // poses are visited in the caller's order (the dense call sorts them
        // into a compact 2D order first); every entry is computed on its own,
        // so the order changes no bit of the result
        hipLaunchKernelGGL(k_iota_i32, dim3(gk), dim3(256), 0, st, order, K);
        UVC_HIP(hipGetLastError());
        P.pose_order = order;
    }
    P.E = E_dev;
    P.vis = vis_dev;
    return launch_irr(P, path, st, nullptr, counters);
}

static void free_job(uvc_csr_job* j) {
    if (!j) return;
    if (j->counts) (void)hipFree(j->counts);
    for (auto& c : j->chunks) {
        if (c.col) (void)hipFree(c.col);
        if (c.val) (void)hipFree(c.val);
    }
    delete j;
}

extern "C" uvc_status uvc_compute_irradiance_csr_begin(const uvc_scene* scene, const float* poses_dev, int64_t K,
                                                       int32_t pose_dim, const uvc_lamp* lamp, const uvc_opts* opts_in,
                                                       void* hip_stream, uvc_csr_job** job, int64_t* nnz) {
    const uvc_opts opts_r = resolve_auto(scene, lamp, opts_in);
    const uvc_opts* opts = &opts_r;
    if (!job || !nnz) return fail(UVC_EINVAL, "job / nnz output is NULL");
    *job = nullptr;
    *nnz = 0;
    IrrParams P;
    UVC_TRY(make_params(scene, poses_dev, K, pose_dim, lamp, opts, P));
    hipStream_t st = (hipStream_t)hip_stream;
    uvc_csr_job* J = new uvc_csr_job();
    (void)hipGetDevice(&J->device);
    J->K = K;
    J->N = scene->n;
    if (K == 0 || scene->n == 0) {
        uvc_status r = dalloc_n(&J->counts, (size_t)std::max<int64_t>(K, 1), "row counts");
        if (r != UVC_OK) {
            free_job(J);
            return r;
        }
        if (K > 0 && hipMemsetAsync(J->counts, 0, (size_t)K * 8, st) != hipSuccess) {
            free_job(J);
            return fail(UVC_EDEVICE, "hipMemsetAsync failed");
        }
        *job = J;
        return UVC_OK;
    }
    std::vector<float> hp;
    uvc_status r = fetch_poses(scene, poses_dev, K, pose_dim, P.lamp, st, hp);
    if (r != UVC_OK) {
        free_job(J);
        return r;
    }
    const int64_t N = scene->n;
    const int64_t budget = (int64_t)1 << 28;  // dense scratch entries per batch
    const int64_t Kb = std::max<int64_t>(1, std::min<int64_t>(K, budget / N));
    float* scratch = nullptr;
    int64_t* offs = nullptr;
    if ((r = dalloc_n(&J->counts, (size_t)K, "row counts")) != UVC_OK ||
        (r = dalloc_n(&scratch, (size_t)Kb * N, "dense batch scratch")) != UVC_OK ||
        (r = dalloc_n(&offs, (size_t)Kb + 1, "batch offsets")) != UVC_OK) {
        if (scratch) (void)hipFree(scratch);
        if (offs) (void)hipFree(offs);
        free_job(J);
        return r;
    }
    const int path = choose_path(scene, opts);
    if (opts && opts->kernel_ms) *opts->kernel_ms = 0.f;
    hipError_t he = hipSuccess;
    for (int64_t k0 = 0; k0 < K && r == UVC_OK; k0 += Kb) {
        const int64_t kb = std::min(Kb, K - k0);
        IrrParams Q = P;
        Q.poses = poses_dev + k0 * pose_dim;
        Q.K = kb;
        Q.E = scratch;
        Q.vis = nullptr;
        int32_t* dorder = nullptr;
        if (path == UVC_PATH_LBVH && (r = upload_order(hp, pose_dim, k0, kb, st, &dorder)) != UVC_OK) break;
        Q.pose_order = dorder;
        r = launch_irr(Q, path, st, opts ? opts->kernel_ms : nullptr);
        if (dorder) (void)hipFreeAsync(dorder, st);
        if (r != UVC_OK) break;
        const unsigned rb = (unsigned)((kb * 64 + 255) / 256);
        hipLaunchKernelGGL(k_row_count, dim3(rb), dim3(256), 0, st, scratch, kb, N, J->counts + k0);
        hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, J->counts + k0, offs, kb, (int64_t)0);
        int64_t bnnz = 0;
        he = hipMemcpyAsync(&bnnz, offs + kb, 8, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) {
            r = fail(UVC_EDEVICE, std::string("CSR batch: ") + hipGetErrorString(he));
            break;
        }
        uvc_csr_job::Chunk c{nullptr, nullptr, bnnz};
        if ((r = dalloc_n(&c.col, (size_t)std::max<int64_t>(bnnz, 1), "CSR columns")) != UVC_OK) break;
        if ((r = dalloc_n(&c.val, (size_t)std::max<int64_t>(bnnz, 1), "CSR values")) != UVC_OK) {
            (void)hipFree(c.col);
            break;
        }
        J->chunks.push_back(c);
        hipLaunchKernelGGL(k_row_gather, dim3(rb), dim3(256), 0, st, scratch, kb, N, offs, c.col, c.val);
        he = hipGetLastError();
        if (he != hipSuccess) {
            r = fail(UVC_EDEVICE, std::string("CSR gather: ") + hipGetErrorString(he));
            break;
        }
        J->nnz += bnnz;
    }
    if (r == UVC_OK) {
        he = hipStreamSynchronize(st);
        if (he != hipSuccess) r = fail(UVC_EDEVICE, std::string("CSR begin: ") + hipGetErrorString(he));
    }
    (void)hipFree(scratch);
    (void)hipFree(offs);
    if (r != UVC_OK) {
        free_job(J);
        return r;
    }
    *nnz = J->nnz;
    *job = J;
    return UVC_OK;
}

extern "C" uvc_status uvc_compute_irradiance_csr_finish(uvc_csr_job* J, int64_t* row_ptr, int32_t* col, float* val,
                                                        void* hip_stream) {
    if (!J) return fail(UVC_EINVAL, "job is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    if (!row_ptr || (J->nnz > 0 && (!col || !val))) {
        free_job(J);
        return fail(UVC_EINVAL, "NULL CSR output buffer");
    }
    uvc_status r = UVC_OK;
    if (J->K == 0) {
        if (hipMemsetAsync(row_ptr, 0, 8, st) != hipSuccess) r = fail(UVC_EDEVICE, "hipMemsetAsync failed");
    } else {
        hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, J->counts, row_ptr, J->K, (int64_t)0);
        int64_t at = 0;
        for (auto& c : J->chunks) {
            if (c.nnz > 0) {
                if (hipMemcpyAsync(col + at, c.col, (size_t)c.nnz * 4, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                    hipMemcpyAsync(val + at, c.val, (size_t)c.nnz * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) {
                    r = fail(UVC_EDEVICE, "CSR copy failed");
                    break;
                }
            }
            at += c.nnz;
        }
    }
    if (r == UVC_OK && hipStreamSynchronize(st) != hipSuccess) r = fail(UVC_EDEVICE, "CSR finish sync failed");
    free_job(J);
    return r;
}

extern "C" void uvc_csr_job_destroy(uvc_csr_job* J) {
    if (!J) return;
    (void)hipDeviceSynchronize();
    free_job(J);
}

// ------------------------------------------------------------- batched host
struct uvc_batch {
    int device = 0;
    int32_t n_rooms = 0;
    std::vector<IrrParams> rooms;     // host copies (per-room launches)
    IrrParams* d_rooms = nullptr;
    int64_t* d_item_off = nullptr;
    int32_t* d_room_of = nullptr;
    int32_t* d_orders = nullptr;      // all rooms' pose orders, concatenated
    unsigned long long* d_counter = nullptr;
    int32_t n_queue = 0;
    int64_t total = 0;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;  // library-owned: the legacy stream cannot be captured
};

static void free_batch(uvc_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    void* ptrs[] = {b->d_rooms, b->d_item_off, b->d_room_of, b->d_orders, b->d_counter};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete b;
}

extern "C" uvc_status uvc_batch_create(const uvc_scene* const* scenes, int32_t n_rooms, const float* const* poses_dev,
                                       const int64_t* K, int32_t pose_dim, const uvc_lamp* lamp, const uvc_opts* opts,
                                       const char* tune_table_json, float* const* E_dev, void* hip_stream,
                                       uvc_batch** out) {
    if (!out) return fail(UVC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_rooms < 0 || (n_rooms > 0 && (!scenes || !poses_dev || !K || !E_dev)))
        return fail(UVC_EINVAL, "invalid batch arrays");
    hipStream_t st = (hipStream_t)hip_stream;
    uvc_batch* b = new uvc_batch();
    (void)hipGetDevice(&b->device);
    b->n_rooms = n_rooms;
    std::vector<std::vector<int32_t>> orders((size_t)n_rooms);
    int64_t order_total = 0;
    for (int32_t r = 0; r < n_rooms; ++r) {
        // per room: the tuning table's packet shape and occupancy for its
        // size class (hierarchy path; the caller's options otherwise)
        uvc_opts ro{};
        ro.band_scale = 1.0f;
        if (opts) ro = *opts;
        uvc_opts t{};
        if (scenes && scenes[r] && lamp &&
            (tune_table_json || ro.path == UVC_PATH_AUTO) &&
            tune_lookup(tune_table_json, scenes[r]->n, lamp->n_src, t) && t.path == UVC_PATH_LBVH) {
            ro.packet_poses = t.packet_poses;
            ro.waves = t.waves;
        }
        ro.path = UVC_PATH_LBVH;
        IrrParams P;
        uvc_status st_ = make_params(scenes[r], poses_dev[r], K[r], pose_dim, lamp, &ro, P);
        if (st_ == UVC_OK && lamp_variant(P.lamp))
            st_ = fail(UVC_EUNSUPPORTED, "the many-room batch takes uniform lamps only");
        if (st_ == UVC_OK && K[r] > 0 && scenes[r]->n > 0 && !E_dev[r]) st_ = fail(UVC_EINVAL, "E is NULL");
        std::vector<float> hp;
        if (st_ == UVC_OK) st_ = fetch_poses(scenes[r], poses_dev[r], K[r], pose_dim, P.lamp, st, hp);
        if (st_ != UVC_OK) {
            free_batch(b);
            return fail(st_, "room " + std::to_string(r) + ": " + uvc_last_error());
        }
        pose_order(hp, pose_dim, 0, K[r], orders[(size_t)r]);
        P.E = E_dev[r];
        P.vis = nullptr;
        P.stats = nullptr;
        const int64_t per = (int64_t)1 << (6 - P.tk_log2);
        P.ntiles = (P.ntargets + per - 1) / per;
        P.nquads = (P.ntiles + 3) / 4;
        P.kgroups = (P.K + (1 << P.tk_log2) - 1) >> P.tk_log2;
        b->rooms.push_back(P);
        order_total += K[r];
    }
    uvc_status r = UVC_OK;
    if ((r = dalloc_n(&b->d_orders, (size_t)std::max<int64_t>(order_total, 1), "batch pose orders")) != UVC_OK ||
        (r = dalloc_n(&b->d_rooms, (size_t)std::max<int32_t>(n_rooms, 1), "batch room table")) != UVC_OK ||
        (r = dalloc_n(&b->d_item_off, (size_t)n_rooms + 1, "batch queue")) != UVC_OK ||
        (r = dalloc_n(&b->d_room_of, (size_t)std::max<int32_t>(n_rooms, 1), "batch queue")) != UVC_OK ||
        (r = dalloc_n(&b->d_counter, 8, "batch counters")) != UVC_OK) {
        free_batch(b);
        return r;
    }
    // pose orders into one arena
    std::vector<int32_t> all((size_t)std::max<int64_t>(order_total, 1));
    int64_t at = 0;
    for (int32_t q = 0; q < n_rooms; ++q) {
        std::copy(orders[(size_t)q].begin(), orders[(size_t)q].end(), all.begin() + at);
        b->rooms[(size_t)q].pose_order = b->d_orders + at;
        at += K[q];
    }
    // queue: rooms with work, by estimated cost per item (depth ~ log2 N) descending
    std::vector<int32_t> qorder;
    for (int32_t q = 0; q < n_rooms; ++q)
        if (b->rooms[(size_t)q].K > 0 && b->rooms[(size_t)q].N > 0) qorder.push_back(q);
    std::stable_sort(qorder.begin(), qorder.end(), [&](int32_t a, int32_t c) {
        return b->rooms[(size_t)a].N > b->rooms[(size_t)c].N;
    });
    std::vector<int64_t> off(qorder.size() + 1, 0);
    for (size_t q = 0; q < qorder.size(); ++q) {
        const IrrParams& P = b->rooms[(size_t)qorder[q]];
        off[q + 1] = off[q] + P.nquads * P.kgroups;
    }
    b->n_queue = (int32_t)qorder.size();
    b->total = off.back();
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->grid = std::max(1, cus * 6);  // 6 workgroups of 4 waves per CU: 6 waves per SIMD
    hipError_t e = hipMemcpyAsync(b->d_orders, all.data(), all.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && n_rooms > 0)
        e = hipMemcpyAsync(b->d_rooms, b->rooms.data(), b->rooms.size() * sizeof(IrrParams), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_item_off, off.data(), off.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !qorder.empty())
        e = hipMemcpyAsync(b->d_room_of, qorder.data(), qorder.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_batch(b);
        return fail(UVC_EDEVICE, std::string("batch upload: ") + hipGetErrorString(e));
    }
    *out = b;
    return UVC_OK;
}

static uvc_status batch_enqueue(uvc_batch* b, hipStream_t st) {
    BatchArgs A{b->d_rooms, b->rooms.empty() ? LampArgs{} : b->rooms[0].lamp, b->d_item_off, b->d_room_of, b->n_queue,
                b->total, {b->d_counter, {}}};
    for (int x = 0; x <= 8; ++x) A.q.range_off[x] = b->total * x / 8;
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, b->d_counter, 0ull, 8);
    hipLaunchKernelGGL(k_irr_batched, dim3((unsigned)b->grid), dim3(256), 0, st, A);
    UVC_HIP(hipGetLastError());
    return UVC_OK;
}

extern "C" uvc_status uvc_batch_run(uvc_batch* b, int32_t mode, float* kernel_ms, void* hip_stream) {
    if (!b) return fail(UVC_EINVAL, "batch is NULL");
    if (mode < 0 || mode > 2) return fail(UVC_EINVAL, "mode must be 0, 1 or 2");
    hipStream_t st = (hipStream_t)hip_stream;
    if (b->total == 0) return UVC_OK;
    if (mode == UVC_BATCH_GRAPH && !b->exec) {
        // capture once on a library stream; the executable graph is then
        // launched on whatever stream the caller passes
        if (!b->capture_stream) UVC_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = b->capture_stream;
        UVC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const uvc_status r = batch_enqueue(b, cs);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (r != UVC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(UVC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        b->graph = g;
        UVC_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kernel_ms) {
        UVC_HIP(hipEventCreate(&e0));
        UVC_HIP(hipEventCreate(&e1));
        UVC_HIP(hipEventRecord(e0, st));
    }
    uvc_status r = UVC_OK;
    if (mode == UVC_BATCH_GRAPH) {
        const hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
    } else if (mode == UVC_BATCH_PERSISTENT) {
        r = batch_enqueue(b, st);
    } else {
        for (const IrrParams& P : b->rooms) {
            if (P.K == 0 || P.N == 0) continue;
            if ((r = launch_irr_impl(P, UVC_PATH_LBVH, st)) != UVC_OK) break;
        }
    }
    if (kernel_ms) {
        float ms = 0.f;
        hipError_t e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (r == UVC_OK && e != hipSuccess) r = fail(UVC_EDEVICE, std::string("batch timing: ") + hipGetErrorString(e));
        *kernel_ms = ms;
    }
    return r;
}

extern "C" void uvc_batch_destroy(uvc_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    free_batch(b);
}

extern "C" uvc_status uvc_compute_irradiance_targets(const uvc_scene* scene, const float* poses_dev, int64_t K,
                                                     int32_t pose_dim, const uvc_lamp* lamp, const uvc_opts* opts_in,
                                                     const int32_t* targets_dev, int64_t n_targets, float* E_dev,
                                                     uint32_t* vis_dev, void* hip_stream) {
    const uvc_opts opts_r = resolve_auto(scene, lamp, opts_in);
    const uvc_opts* opts = &opts_r;
    IrrParams P;
    UVC_TRY(make_params(scene, poses_dev, K, pose_dim, lamp, opts, P));
    if (n_targets < 0) return fail(UVC_EINVAL, "n_targets < 0");
    if (K == 0 || scene->n == 0 || n_targets == 0) return UVC_OK;
    if (!E_dev || !targets_dev) return fail(UVC_EINVAL, "E or targets is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<float> hp;
    UVC_TRY(fetch_poses(scene, poses_dev, K, pose_dim, P.lamp, st, hp));
    // targets are input element indices: check the range and map them to leaf slots
    std::vector<int32_t> ht((size_t)n_targets), perm((size_t)scene->n), slot((size_t)scene->n);
    UVC_HIP(hipMemcpyAsync(ht.data(), targets_dev, (size_t)n_targets * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(perm.data(), scene->perm, (size_t)scene->n * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    for (int64_t s2 = 0; s2 < scene->n; ++s2) slot[(size_t)perm[(size_t)s2]] = (int32_t)s2;
    for (int64_t j = 0; j < n_targets; ++j) {
        if (ht[(size_t)j] < 0 || ht[(size_t)j] >= scene->n)
            return fail(UVC_EINVAL, "target " + std::to_string(j) + " is not an element index");
        ht[(size_t)j] = slot[(size_t)ht[(size_t)j]];
    }
    int32_t* dslots = nullptr;
    UVC_HIP(hipMallocAsync(reinterpret_cast<void**>(&dslots), (size_t)n_targets * 4, st));
    hipError_t he = hipMemcpyAsync(dslots, ht.data(), (size_t)n_targets * 4, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
        (void)hipFreeAsync(dslots, st);
        return fail(UVC_EDEVICE, std::string("targets upload: ") + hipGetErrorString(he));
    }
    const int path = choose_path(scene, opts);
    int32_t* dorder = nullptr;
    uvc_status r = UVC_OK;
    if (path == UVC_PATH_LBVH) r = upload_order(hp, pose_dim, 0, K, st, &dorder);
    if (r == UVC_OK) {
        P.pose_order = dorder;
        P.targets = dslots;
        P.ntargets = n_targets;
        P.ld = n_targets;
        P.E = E_dev;
        P.vis = vis_dev;
        if (opts && opts->kernel_ms) *opts->kernel_ms = 0.f;
        r = launch_irr(P, path, st, opts ? opts->kernel_ms : nullptr);
    }
    if (dorder) (void)hipFreeAsync(dorder, st);
    (void)hipFreeAsync(dslots, st);
    return r;
}
