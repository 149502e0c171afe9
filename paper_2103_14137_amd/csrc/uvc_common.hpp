// Internal declarations of the HIP irradiance library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/uvc.h"

namespace uvc {

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);
uvc_status fail(uvc_status s, const std::string& msg);

#define UVC_HIP(call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::uvc::fail(UVC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define UVC_TRY(expr)                        \
    do {                                     \
        uvc_status s_ = (expr);              \
        if (s_ != UVC_OK) return s_;         \
    } while (0)

// Allocation helper that reports UVC_ENOMEM with the size.
uvc_status dalloc(void** p, size_t bytes, const char* what);

template <class T>
uvc_status dalloc_n(T** p, size_t n, const char* what) {
    return dalloc(reinterpret_cast<void**>(p), n * sizeof(T), what);
}

// --------------------------------------------------------- layout constants
// Triangle record, 80 bytes, in leaf-slot order: v0.xyz v1.xyz v2.xyz in the
// input vertex order, the FP32 edge vectors e01 = v1-v0, e12 = v2-v1,
// e20 = v0-v2, L = the largest |component| of the three edges, and the input
// triangle index (int bits).
constexpr int TRI_WORDS = 20;
constexpr int TRI_E01 = 9, TRI_E12 = 12, TRI_E20 = 15, TRI_L = 18, TRI_ID = 19;
// Element record, 32 bytes, in leaf-slot order: centroid xyz, unit normal
// xyz, input triangle index (int bits), near-list cut radius rho_t.
constexpr int ELEM_WORDS = 8;
// Near lists: element slot s owns near[near_off[s] .. near_off[s+1]), the
// slots of every triangle other than s whose padded box meets the ball of
// radius rho_n = NEAR_SCALE * L_s around the centroid (L_s = the element's
// largest |edge component|), except triangles whose FP64 plane side at the
// centroid is exactly zero (the predicate can never report those).  The
// traversal may then stop each segment rho_t = rho_n (1 - 2^-10) short of its
// target: every point it skips lies inside the ball.
// (Measured on the ward: 0.25 costs 0.07 near-list tests per segment and
// is 3 % faster than 1.0, which costs 1.25; 2.0 is 28 % slower.)
constexpr float NEAR_SCALE = 0.25f;
// Hierarchy node, 64 bytes: left box lo xyz hi xyz, right box lo xyz hi xyz,
// left ref, right ref (>= 0 internal, < 0 leaf slot ~ref), hint axis/order,
// hint split coordinate as an order key (float_key).
constexpr int NODE_WORDS = 16;

// Signed integer that orders like the float (non-NaN; -0 sorts below +0), so
// that a coordinate comparison can run on the scalar unit.
__host__ __device__ inline int32_t float_key(float f) {
    int32_t b;
    __builtin_memcpy(&b, &f, 4);
    return b ^ ((b >> 31) & 0x7fffffff);
}

// Decision bands of the FP32 fast path (multiplied by opts.band_scale).
// Front-facing: |<d, n>| > TAU_F * |d|_1.
// Edge orientations U, V, W (computed as D . ((vi - O) x (vj - vi))):
//   |U| > TAU_E * |D|_1 * G * (L + 2^-28 G) with G the largest |coordinate| of
//   v0-O, v1-O, v2-O and L that of the three edge vectors.
// Plane sides: |s| > TAU_P * |x|_inf * |e1|_inf * |e2|_inf with x = O-v0 or
//   T-v0 and e1, e2 the triangle's edge vectors from v0.
constexpr float TAU_F = 1.0f / 524288.0f;   // 2^-19
constexpr float TAU_E = 1.0f / 65536.0f;    // 2^-16
constexpr float TAU_P = 1.0f / 8192.0f;     // 2^-13

// Box padding relative to the scene's largest |coordinate|.
constexpr float PAD_REL = 1.0f / 262144.0f; // 2^-18

// A lamp as the kernels read it (a kernel argument).
struct LampArgs {
    int32_t S;
    float dz[32];
    float pw[32];      // P_j / (4 pi)
    // emission pattern (read by the lamp-variant kernels only)
    int32_t nprof;     // 0: uniform; else the table's node count (2..33)
    float ph;          // (nprof - 1) / 2
    float prof[33];
    uint32_t up, down; // hemisphere masks
};

// Launch options from a tuning table (json text, or NULL: the table
// registered with uvc_set_tune_table) for an n-triangle scene and n_src
// sources; false when the table has no entry for that size class.
bool tune_lookup(const char* json, int64_t n, int n_src, uvc_opts& o);

// Validates a lamp of the C ABI and fills its kernel form.
uvc_status lamp_args(const uvc_lamp* lamp, LampArgs& L);

// Emission weight of the lamp's table (L.nprof >= 2) at cos(theta): linear
// interpolation between equally spaced nodes over [-1, 1].  The table is
// uniform across the wave; the two bracketing entries are picked with a
// select chain, not an indexed load.
__device__ __forceinline__ float table_weight(const LampArgs& L, float ct) {
#pragma clang fp contract(off)
    const int last = L.nprof - 1;
    const float u = fminf(fmaxf((ct + 1.0f) * L.ph, 0.0f), (float)last);
    const int q = min((int)u, last - 1);
    const float f = u - (float)q;
    float a = L.prof[0], b = L.prof[1];
    for (int qq = 1; qq < last; ++qq) {
        const bool here = q == qq;
        a = here ? L.prof[qq] : a;
        b = here ? L.prof[qq + 1] : b;
    }
    return a + f * (b - a);
}

}  // namespace uvc

struct uvc_scene {
    int device = 0;
    int64_t n = 0;              // triangles = elements
    int32_t depth = 0;          // hierarchy depth (root = 1)
    float max_abs = 0.f;        // largest |vertex coordinate|
    float pad = 0.f;            // absolute box padding
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float* tri = nullptr;       // n x TRI_WORDS
    float* elem = nullptr;      // n x ELEM_WORDS (slot order)
    float* elem_c = nullptr;    // n x 3 (input order)
    float* elem_n = nullptr;    // n x 3 (input order)
    float* elem_a = nullptr;    // n (input order)
    int32_t* perm = nullptr;    // slot -> input index
    uint32_t* codes = nullptr;  // sorted Morton codes
    float* nodes = nullptr;     // (n-1) x NODE_WORDS
    int32_t* near_off = nullptr;  // n + 1
    int32_t* near = nullptr;      // near_off[n] slots
    int64_t n_near = 0;
};
