// Area-integrated irradiance (Sec. IV-C, the visibility-cube procedure): the
// paper's entry is the mean irradiance over the visible part of a triangle,
// found by emitting each source's power through the pixels of a cube map,
// crediting every pixel to the triangle it sees first, and dividing each
// triangle's collected power by its area.  Here each pixel is one
// closest-hit ray through the pixel centre, traced through the scene
// hierarchy.
//
// Work decomposition: one wavefront = an 8 x 8 tile of pixels of one cube
// face of one source of one pose (coherent directions from one origin).
// Collection: the pixel powers go into a per-(pose, triangle) fixed-point
// accumulator (units of 2^-40 W, unsigned 64-bit) with integer atomics,
// which are associative, so the result does not depend on the order in
// which waves finish; lanes of a wave that hit the same triangle are summed
// in the wave first, so each (wave, triangle) pair costs one atomic.
#include "uvc_common.hpp"
#include "closest_hit.hpp"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace uvc {
namespace {

constexpr double FIX_ONE = 1099511627776.0;  // 2^40 units per watt
constexpr int AREA_MAX_RES = 1024;

struct AreaParams {
    const float* tri;
    const float* elem;
    const float* nodes;
    int64_t N;
    const float* poses;   // pose rows of this launch
    int pd;
    int R, T;             // pixels per face edge, 8 x 8 tiles per face edge
    float L;              // length of the traced direction vectors
    const float* dom;     // R x R pixel solid angles (the same on every face)
    unsigned long long* acc;  // launch poses x N, input element order
    int64_t items;        // poses x S x 6 x T x T tiles
    LampArgs lamp;
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_area_cube(AreaParams A) {
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * 4 + w;
    if (item >= A.items) return;  // uniform per wave
    const int64_t TT = (int64_t)A.T * A.T;
    const int64_t tile = item % TT;
    int64_t rest = item / TT;
    const int f = (int)(rest % 6);
    rest /= 6;
    const int j = (int)(rest % A.lamp.S);
    const int64_t kk = rest / A.lamp.S;
    const int a = (int)(tile / A.T) * 8 + (lane >> 3), b = (int)(tile % A.T) * 8 + (lane & 7);
    bool valid = a < A.R && b < A.R;
    // pixel centre direction on face f (axis f / 2, outward sign by parity)
    const float invR = 1.0f / (float)A.R;
    const float uc = (float)(2 * a + 1) * invR - 1.0f, vc = (float)(2 * b + 1) * invR - 1.0f;
    const int ax = f >> 1;
    const float sg = (f & 1) ? -1.0f : 1.0f;
    const float d0 = ax == 0 ? sg : (ax == 1 ? vc : uc);
    const float d1 = ax == 1 ? sg : (ax == 2 ? vc : uc);
    const float d2 = ax == 2 ? sg : (ax == 0 ? vc : uc);
    if ((A.lamp.up >> j) & 1u) valid = valid && d2 > 0.0f;
    if ((A.lamp.down >> j) & 1u) valid = valid && d2 < 0.0f;
    const float* pp = A.poses + kk * A.pd;
    const float ox = pp[0], oy = pp[1], oz = (A.pd == 3 ? pp[2] : 0.0f) + A.lamp.dz[j];
    CRay r;
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.dx = d0 * A.L; r.dy = d1 * A.L; r.dz = d2 * A.L;
    auto ginv = [](float d) { return 1.0f / ((fabsf(d) < 1e-30f) ? copysignf(1e-30f, d) : d); };
    r.ix = ginv(r.dx); r.iy = ginv(r.dy); r.iz = ginv(r.dz);
    r.nx = -ox * r.ix; r.ny = -oy * r.iy; r.nz = -oz * r.iz;
    r.tbest = valid ? 1.0f : -1.0f;  // an invalid lane enters no box
    r.best = -1;
    closest_hit_walk<true>(r, A.tri, A.nodes, A.N, lane);
    int key = -1;
    unsigned long long q = 0;
    if (valid && r.best >= 0) {
        const float* e = A.elem + (int64_t)r.best * ELEM_WORDS;
        const float dn = d0 * e[3] + d1 * e[4] + d2 * e[5];
        if (dn < 0.0f) {  // the ray reaches the triangle's front side
            float wgt = 1.0f;
            if (A.lamp.nprof > 0) wgt = table_weight(A.lamp, d2 / sqrtf(d0 * d0 + d1 * d1 + d2 * d2));
            const double pw = (double)A.lamp.pw[j] * (double)wgt * (double)A.dom[a * A.R + b];
            q = (unsigned long long)llrint(pw * FIX_ONE);
            key = __float_as_int(e[6]);
        }
    }
    // sum the lanes that hit the same triangle, one atomic per triangle
    unsigned long long todo = __ballot(key >= 0);
    unsigned long long* row = A.acc + kk * A.N;
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int k0 = __builtin_amdgcn_readlane(key, leader);
        const bool mine = key == k0;
        const unsigned long long s = wave_sum_u64(mine ? q : 0ull);
        if (lane == leader) atomicAdd(row + k0, s);
        todo &= ~__ballot(mine);
    }
}

__global__ void k_fill_acc(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0ull;
}

// E[k, i] = collected power / area (FP64, rounded once); power[k] = sum over
// the row (integer sum, exact).  One workgroup per pose row.
__global__ __launch_bounds__(256) void k_area_finish(const unsigned long long* __restrict__ acc, int64_t N,
                                                     const float* __restrict__ area, float* __restrict__ E,
                                                     double* __restrict__ power) {
    __shared__ unsigned long long red[256];
    const int64_t k = blockIdx.x;
    const unsigned long long* row = acc + k * N;
    unsigned long long s = 0;
    for (int64_t i = threadIdx.x; i < N; i += 256) {
        const unsigned long long v = row[i];
        s += v;
        E[k * N + i] = (float)(((double)v / FIX_ONE) / (double)area[i]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && power) power[k] = (double)red[0] / FIX_ONE;
}

__global__ void k_fill_zero_f64(double* __restrict__ p, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0.0;
}

}  // namespace
}  // namespace uvc

using namespace uvc;

extern "C" uvc_status uvc_compute_irradiance_area(const uvc_scene* scene, const float* poses_dev, int64_t K,
                                                  int32_t pose_dim, const uvc_lamp* lamp, int32_t face_res,
                                                  float* E_dev, double* power_dev, void* hip_stream) {
    if (!scene) return fail(UVC_EINVAL, "scene is NULL");
    if (K < 0 || (pose_dim != 2 && pose_dim != 3)) return fail(UVC_EINVAL, "invalid K or pose_dim");
    LampArgs L;
    UVC_TRY(lamp_args(lamp, L));
    double ptot = 0.0;
    for (int j = 0; j < L.S; ++j) ptot += (double)lamp->power_w[j];
    if (ptot > 4194304.0) return fail(UVC_EINVAL, "total lamp power above 2^22 W (fixed-point collection range)");
    const int R = face_res == 0 ? 512 : face_res;
    if (R < 1 || R > AREA_MAX_RES) return fail(UVC_EINVAL, "face_res must lie in [1, 1024] (0: 512)");
    if (K == 0) return UVC_OK;
    if (!poses_dev) return fail(UVC_EINVAL, "poses is NULL");
    if (scene->n > 0 && !E_dev) return fail(UVC_EINVAL, "E is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<float> hp((size_t)K * pose_dim);
    UVC_HIP(hipMemcpyAsync(hp.data(), poses_dev, hp.size() * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    float reach = std::max(scene->max_abs, 1e-30f);
    float dzmax = 0.f;
    for (int j = 0; j < L.S; ++j) dzmax = std::max(dzmax, std::fabs(L.dz[j]));
    for (float v : hp) {
        if (!std::isfinite(v)) return fail(UVC_EINVAL, "pose coordinate is not finite");
        reach = std::max(reach, std::fabs(v) + dzmax);
    }
    const int64_t N = scene->n;
    if (N == 0) {
        if (power_dev)
            hipLaunchKernelGGL(k_fill_zero_f64, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, power_dev, K);
        UVC_HIP(hipGetLastError());
        return UVC_OK;
    }
    // pixel solid angles: the exact solid angle of each pixel's square on
    // the unit-distance face plane (FP64, rounded once)
    std::vector<float> hdom((size_t)R * R);
    auto corner = [](double x, double y) { return std::atan2(x * y, std::sqrt(1.0 + x * x + y * y)); };
    for (int a = 0; a < R; ++a) {
        const double u0 = -1.0 + 2.0 * a / R, u1 = -1.0 + 2.0 * (a + 1) / R;
        for (int b = 0; b < R; ++b) {
            const double v0 = -1.0 + 2.0 * b / R, v1 = -1.0 + 2.0 * (b + 1) / R;
            hdom[(size_t)a * R + b] = (float)(corner(u1, v1) - corner(u0, v1) - corner(u1, v0) + corner(u0, v0));
        }
    }
    float* dom = nullptr;
    unsigned long long* acc = nullptr;
    UVC_TRY(dalloc_n(&dom, hdom.size(), "cube pixel solid angles"));
    const int T = (R + 7) / 8;
    const int64_t per_pose = (int64_t)L.S * 6 * T * T;
    const int64_t kc = std::max<int64_t>(1, std::min<int64_t>({K, ((int64_t)1 << 27) / N,
                                                               ((int64_t)1 << 32) / per_pose}));
    uvc_status r = UVC_OK;
    hipError_t e = hipMemcpyAsync(dom, hdom.data(), hdom.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("solid angle upload: ") + hipGetErrorString(e));
    if (r == UVC_OK) r = dalloc_n(&acc, (size_t)kc * N, "area accumulator");
    AreaParams A{};
    A.tri = scene->tri;
    A.elem = scene->elem;
    A.nodes = scene->nodes;
    A.N = N;
    A.pd = pose_dim;
    A.R = R;
    A.T = T;
    A.L = 4.0f * reach + 1.0f;
    A.dom = dom;
    A.acc = acc;
    A.lamp = L;
    for (int64_t k0 = 0; r == UVC_OK && k0 < K; k0 += kc) {
        const int64_t kb = std::min(kc, K - k0);
        A.poses = poses_dev + k0 * pose_dim;
        A.items = kb * per_pose;
        hipLaunchKernelGGL(k_fill_acc, dim3(1024), dim3(256), 0, st, acc, kb * N);
        hipLaunchKernelGGL(k_area_cube, dim3((unsigned)((A.items + 3) / 4)), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_area_finish, dim3((unsigned)kb), dim3(256), 0, st, (const unsigned long long*)acc, N,
                           (const float*)scene->elem_a, E_dev + k0 * N, power_dev ? power_dev + k0 : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("area launch: ") + hipGetErrorString(e));
    }
    e = hipStreamSynchronize(st);
    if (r == UVC_OK && e != hipSuccess) r = fail(UVC_EDEVICE, std::string("area irradiance: ") + hipGetErrorString(e));
    (void)hipFree(acc);
    (void)hipFree(dom);
    return r;
}
