// Learned pose ranker: cheap per-pose visibility features and a small MLP
// that scores poses (forward, backward and Adam on the GPU).  The ranked
// plan that uses the scores (keep the top-scoring poses, assemble E on them
// only, solve the dosage LP, price the pruned poses with its duals) lives
// with the column generation in the ranked-plan source.
//
// Features of pose k: 16 x 16 closest-hit rays from the point (x, y, z + h)
// over an equal-area direction set (16 azimuths x 16 bands uniform in the
// vertical direction cosine, cell centres).  Each hit adds the area its ray
// subtends, dOmega r^2 / max(|cos|, 0.05), to one of 8 distance bins
// ([0, .5, 1, 1.5, 2, 3, 4, 6, inf) m) x 8 |cos| bins; the 64 features are
// log1p of the bin sums.
//
// MLP: 64 -> 128 -> 128 -> 1, ReLU, FP32 parameters laid out as
// W1[128][64], b1[128], W2[128][128], b2[128], W3[128], b3 (24,961 floats);
// binary cross-entropy on the logit; Adam.
#include "uvc_common.hpp"
#include "closest_hit.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace uvc {

constexpr int FEAT = 64;
constexpr int H1 = 128, H2 = 128;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + H1 * FEAT, OFF_W2 = OFF_B1 + H1, OFF_B2 = OFF_W2 + H2 * H1,
                  OFF_W3 = OFF_B2 + H2, OFF_B3 = OFF_W3 + H2, N_PARAMS = OFF_B3 + 1;

// ------------------------------------------------------------- features
__global__ __launch_bounds__(256) void k_rank_features(const float* __restrict__ tri, const float* __restrict__ elem,
                                                       const float* __restrict__ nodes, int64_t N,
                                                       const float* __restrict__ poses, int64_t K, int pd, float h,
                                                       float L, float* __restrict__ feat) {
    __shared__ int sbin[256];
    __shared__ float sw[256];
    const int64_t k = blockIdx.x;
    const int j = threadIdx.x, lane = j & 63;
    const float* pp = poses + k * pd;
    const float ox = pp[0], oy = pp[1], oz = (pd == 3 ? pp[2] : 0.f) + h;
    const int a = j & 15, b = j >> 4;
    const float phi = 6.283185307179586f * ((float)a + 0.5f) / 16.0f;
    const float cz = -1.0f + 2.0f * ((float)b + 0.5f) / 16.0f;
    const float rxy = sqrtf(fmaxf(0.f, 1.0f - cz * cz));
    const float ux = rxy * cosf(phi), uy = rxy * sinf(phi), uz = cz;
    CRay r;
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.dx = ux * L; r.dy = uy * L; r.dz = uz * L;
    auto ginv = [](float d) { return 1.0f / ((fabsf(d) < 1e-30f) ? copysignf(1e-30f, d) : d); };
    r.ix = ginv(r.dx); r.iy = ginv(r.dy); r.iz = ginv(r.dz);
    r.nx = -ox * r.ix; r.ny = -oy * r.iy; r.nz = -oz * r.iz;
    r.tbest = 1.0f;
    r.best = -1;
    closest_hit_walk<false>(r, tri, nodes, N, lane);
    int bin = -1;
    float wgt = 0.f;
    if (r.best >= 0) {
        const float* e = elem + (int64_t)r.best * ELEM_WORDS;
        const float c0 = fabsf(ux * e[3] + uy * e[4] + uz * e[5]);
        const float c = (c0 == c0) ? fminf(c0, 1.0f) : 0.0f;
        const float dist = r.tbest * L;
        const float edges[7] = {0.5f, 1.0f, 1.5f, 2.0f, 3.0f, 4.0f, 6.0f};
        int db = 0;
        for (int q = 0; q < 7; ++q) db += dist >= edges[q] ? 1 : 0;
        const int cb = min(7, (int)(c * 8.0f));
        bin = db * 8 + cb;
        wgt = (4.0f * 3.14159265358979f / 256.0f) * dist * dist / fmaxf(c, 0.05f);
    }
    sbin[j] = bin;
    sw[j] = wgt;
    __syncthreads();
    if (j < FEAT) {
        float acc = 0.f;
        for (int q = 0; q < 256; ++q)
            if (sbin[q] == j) acc += sw[q];
        feat[k * FEAT + j] = log1pf(acc);
    }
}

// ------------------------------------------------------------------- MLP
__device__ __forceinline__ float bf16r(float x) {
    // round to the nearest bfloat16 (ties to even), kept in an FP32 register
    const unsigned u = __float_as_uint(x);
    const unsigned r = u + 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(r & 0xffff0000u);
}

// Forward pass for 16 samples per block of 128 threads; optionally stores
// the pre-activations (for the backward pass).
constexpr int MB = 16;

__global__ __launch_bounds__(128) void k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X,
                                                 const int32_t* __restrict__ idx, int64_t B, int bf16,
                                                 float* __restrict__ score, float* __restrict__ z1,
                                                 float* __restrict__ z2) {
    __shared__ float xs[MB][FEAT];
    __shared__ float h1[MB][H1];
    __shared__ float h2[MB][H2];
    const int o = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * MB;
    for (int q = o; q < MB * FEAT; q += 128) {
        const int s = q / FEAT, i = q % FEAT;
        const int64_t row = (s0 + s < B) ? (idx ? (int64_t)idx[s0 + s] : s0 + s) : -1;
        const float v = row >= 0 ? X[row * FEAT + i] : 0.f;
        xs[s][i] = bf16 ? bf16r(v) : v;
    }
    __syncthreads();
    for (int s = 0; s < MB; ++s) {
        float a = P[OFF_B1 + o];
        for (int i = 0; i < FEAT; ++i) {
            const float w = P[OFF_W1 + o * FEAT + i];
            a = fmaf(bf16 ? bf16r(w) : w, xs[s][i], a);
        }
        if (z1 && s0 + s < B) z1[(s0 + s) * H1 + o] = a;
        const float r = fmaxf(a, 0.f);
        h1[s][o] = bf16 ? bf16r(r) : r;
    }
    __syncthreads();
    for (int s = 0; s < MB; ++s) {
        float a = P[OFF_B2 + o];
        for (int i = 0; i < H1; ++i) {
            const float w = P[OFF_W2 + o * H1 + i];
            a = fmaf(bf16 ? bf16r(w) : w, h1[s][i], a);
        }
        if (z2 && s0 + s < B) z2[(s0 + s) * H2 + o] = a;
        const float r = fmaxf(a, 0.f);
        h2[s][o] = bf16 ? bf16r(r) : r;
    }
    __syncthreads();
    if (o < MB && s0 + o < B) {
        float a = P[OFF_B3];
        for (int i = 0; i < H2; ++i) {
            const float w = P[OFF_W3 + i];
            a = fmaf(bf16 ? bf16r(w) : w, h2[o][i], a);
        }
        score[s0 + o] = a;
    }
}

// Per-sample backward: dscore = (sigmoid(s) - y) / B, then deltas of the two
// hidden layers; also the per-sample loss.
__global__ __launch_bounds__(128) void k_mlp_delta(const float* __restrict__ P, const float* __restrict__ score,
                                                   const float* __restrict__ y, const int32_t* __restrict__ idx,
                                                   const float* __restrict__ z1,
                                                   const float* __restrict__ z2, int64_t B, float* __restrict__ ds,
                                                   float* __restrict__ d2, float* __restrict__ d1,
                                                   float* __restrict__ loss) {
    __shared__ float sd2[H2];
    const int64_t s = blockIdx.x;
    const int o = threadIdx.x;
    const float sc = score[s], yy = y[idx ? (int64_t)idx[s] : s];
    const float p = 1.0f / (1.0f + expf(-sc));
    const float g = (p - yy) / (float)B;
    if (o == 0) {
        ds[s] = g;
        loss[s] = fmaxf(sc, 0.f) - sc * yy + log1pf(expf(-fabsf(sc)));
    }
    const float dz2 = (z2[s * H2 + o] > 0.f) ? g * P[OFF_W3 + o] : 0.f;
    d2[s * H2 + o] = dz2;
    sd2[o] = dz2;
    __syncthreads();
    float a = 0.f;
    for (int q = 0; q < H2; ++q) a = fmaf(P[OFF_W2 + q * H1 + o], sd2[q], a);
    d1[s * H1 + o] = (z1[s * H1 + o] > 0.f) ? a : 0.f;
}

// Gradient of every parameter: one thread per parameter, fixed-order sum
// over the batch.
__global__ void k_mlp_grad(const float* __restrict__ X, const int32_t* __restrict__ idx, const float* __restrict__ z1,
                           const float* __restrict__ z2,
                           const float* __restrict__ ds, const float* __restrict__ d2, const float* __restrict__ d1,
                           const float* __restrict__ loss, int64_t B, float* __restrict__ G,
                           float* __restrict__ loss_sum) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= N_PARAMS) return;
    float acc = 0.f;
    if (q < OFF_B1) {
        const int o = (int)(q / FEAT), i = (int)(q % FEAT);
        for (int64_t s = 0; s < B; ++s) acc = fmaf(d1[s * H1 + o], X[(idx ? (int64_t)idx[s] : s) * FEAT + i], acc);
    } else if (q < OFF_W2) {
        const int o = (int)(q - OFF_B1);
        for (int64_t s = 0; s < B; ++s) acc += d1[s * H1 + o];
    } else if (q < OFF_B2) {
        const int o = (int)((q - OFF_W2) / H1), i = (int)((q - OFF_W2) % H1);
        for (int64_t s = 0; s < B; ++s) acc = fmaf(d2[s * H2 + o], fmaxf(z1[s * H1 + i], 0.f), acc);
    } else if (q < OFF_W3) {
        const int o = (int)(q - OFF_B2);
        for (int64_t s = 0; s < B; ++s) acc += d2[s * H2 + o];
    } else if (q < OFF_B3) {
        const int i = (int)(q - OFF_W3);
        for (int64_t s = 0; s < B; ++s) acc = fmaf(ds[s], fmaxf(z2[s * H2 + i], 0.f), acc);
    } else {
        for (int64_t s = 0; s < B; ++s) acc += ds[s];
        float l = 0.f;
        for (int64_t s = 0; s < B; ++s) l += loss[s];
        *loss_sum = l / (float)B;
    }
    G[q] = acc;
}

// 1 - beta comes from the host (rounded once from FP64): forming it in FP32
// from a rounded beta would be off by up to 1e-5 relative for beta2 = 0.999.
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ G, int64_t n, float lr, float b1, float b2, float ob1, float ob2,
                       float eps, float c1, float c2) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float g = G[q];
    const float mm = b1 * m[q] + ob1 * g;
    const float vv = b2 * v[q] + ob2 * g * g;
    m[q] = mm;
    v[q] = vv;
    P[q] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Non-learned baseline score: the total visible area seen by the feature
// rays, sum_b expm1(feature_b), summed in bin order.
__global__ void k_area_score(const float* __restrict__ feat, int64_t K, float* __restrict__ score) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= K) return;
    float a = 0.f;
    for (int b = 0; b < FEAT; ++b) a += expm1f(feat[k * FEAT + b]);
    score[k] = a;
}

}  // namespace uvc

using namespace uvc;

extern "C" int64_t uvc_ranker_param_count(void) { return N_PARAMS; }

extern "C" uvc_status uvc_ranker_features(const uvc_scene* scene, const float* poses_dev, int64_t K,
                                          int32_t pose_dim, float src_height, float* feat_dev, void* hip_stream) {
    if (!scene) return fail(UVC_EINVAL, "scene is NULL");
    if (K < 0 || (pose_dim != 2 && pose_dim != 3)) return fail(UVC_EINVAL, "invalid K or pose_dim");
    if (!std::isfinite(src_height)) return fail(UVC_EINVAL, "feature source height is not finite");
    if (K == 0) return UVC_OK;
    if (!poses_dev || !feat_dev) return fail(UVC_EINVAL, "NULL poses or features");
    if (K > (int64_t)INT32_MAX) return fail(UVC_EINVAL, "K too large");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<float> hp((size_t)K * pose_dim);
    UVC_HIP(hipMemcpyAsync(hp.data(), poses_dev, hp.size() * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    for (float v : hp)
        if (!std::isfinite(v)) return fail(UVC_EINVAL, "pose coordinate is not finite");
    if (scene->n == 0) {
        UVC_HIP(hipMemsetAsync(feat_dev, 0, (size_t)K * FEAT * 4, st));
        return UVC_OK;
    }
    float reach = std::max(scene->max_abs, 1e-30f);
    for (float v : hp) reach = std::max(reach, std::fabs(v) + std::fabs(src_height));
    const float L = 4.0f * reach + 1.0f;
    hipLaunchKernelGGL(k_rank_features, dim3((unsigned)K), dim3(256), 0, st, scene->tri, scene->elem, scene->nodes,
                       scene->n, poses_dev, K, pose_dim, src_height, L, feat_dev);
    UVC_HIP(hipGetLastError());
    return UVC_OK;
}

extern "C" uvc_status uvc_ranker_forward(const float* params_dev, const float* feat_dev, int64_t B, int32_t bf16,
                                         float* score_dev, void* hip_stream) {
    if (B < 0) return fail(UVC_EINVAL, "B < 0");
    if (B == 0) return UVC_OK;
    if (!params_dev || !feat_dev || !score_dev) return fail(UVC_EINVAL, "NULL ranker buffer");
    if (B > (int64_t)INT32_MAX * MB) return fail(UVC_EINVAL, "B too large");
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((B + MB - 1) / MB)), dim3(128), 0, (hipStream_t)hip_stream,
                       params_dev, feat_dev, (const int32_t*)nullptr, B, bf16 ? 1 : 0, score_dev, (float*)nullptr,
                       (float*)nullptr);
    UVC_HIP(hipGetLastError());
    return UVC_OK;
}

extern "C" uvc_status uvc_ranker_area_score(const float* feat_dev, int64_t K, float* score_dev, void* hip_stream) {
    if (K < 0) return fail(UVC_EINVAL, "K < 0");
    if (K == 0) return UVC_OK;
    if (!feat_dev || !score_dev) return fail(UVC_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(k_area_score, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, feat_dev,
                       K, score_dev);
    UVC_HIP(hipGetLastError());
    return UVC_OK;
}

extern "C" uvc_status uvc_ranker_train_step(float* params_dev, float* adam_m, float* adam_v, const float* feat_dev,
                                            const float* label_dev, const int32_t* idx_dev, int64_t B, float lr,
                                            int64_t step, float* grad_out_dev, float* loss_out, void* hip_stream) {
    if (B <= 0 || step < 1) return fail(UVC_EINVAL, "B must be positive and step >= 1");
    if (B > (1 << 24)) return fail(UVC_EINVAL, "batch too large");
    if (!params_dev || !adam_m || !adam_v || !feat_dev || !label_dev) return fail(UVC_EINVAL, "NULL ranker buffer");
    if (!std::isfinite(lr) || lr < 0.f) return fail(UVC_EINVAL, "learning rate must be finite and >= 0");
    hipStream_t st = (hipStream_t)hip_stream;
    float* buf = nullptr;
    const size_t nb = (size_t)B * (2 * H1 + 2 * H2 + 3) + (size_t)N_PARAMS + 1;
    UVC_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), nb * 4, st));
    float *score = buf, *z1 = score + B, *z2 = z1 + B * H1, *ds = z2 + B * H2, *d2 = ds + B, *d1 = d2 + B * H2,
          *loss = d1 + B * H1, *G = loss + B, *lsum = G + N_PARAMS;
    float* Gp = grad_out_dev ? grad_out_dev : G;
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((B + MB - 1) / MB)), dim3(128), 0, st, params_dev, feat_dev, idx_dev,
                       B, 0, score, z1, z2);
    hipLaunchKernelGGL(k_mlp_delta, dim3((unsigned)B), dim3(128), 0, st, params_dev, score, label_dev, idx_dev, z1, z2,
                       B, ds, d2, d1, loss);
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((N_PARAMS + 255) / 256)), dim3(256), 0, st, feat_dev, idx_dev, z1,
                       z2, ds, d2, d1, loss, B, Gp, lsum);
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)step)), c2 = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((N_PARAMS + 255) / 256)), dim3(256), 0, st, params_dev, adam_m, adam_v,
                       Gp, N_PARAMS, lr, b1, b2, (float)(1.0 - 0.9), (float)(1.0 - 0.999), 1e-8f, c1, c2);
    hipError_t e = hipGetLastError();
    float l = 0.f;
    if (e == hipSuccess) e = hipMemcpyAsync(&l, lsum, 4, hipMemcpyDeviceToHost, st);
    (void)hipFreeAsync(buf, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(UVC_EDEVICE, std::string("ranker train step: ") + hipGetErrorString(e));
    if (loss_out) *loss_out = l;
    return UVC_OK;
}
