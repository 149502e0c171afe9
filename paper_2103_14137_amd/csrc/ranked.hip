// Ranked plan: prune the candidate poses with a score, assemble E on the
// kept poses only and solve the relaxed dosage LP (Sec. IV-D) on that
// restricted matrix, then price the pruned poses with the LP's duals
// (column generation): a pose whose reduced cost 1 + y_b - sum_i E[k,i] y_i
// is negative would lower the objective, so the most negative ones join the
// restricted set and the LP is solved again.  When no pruned pose prices
// out, the restricted plan is optimal for the LP over all candidates.  The
// full candidate set remains the fallback.
#include "uvc_common.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace uvc {
namespace {

__global__ void k_gather_rows(const float* __restrict__ src, const int32_t* __restrict__ rows, int64_t n, int dim,
                              float* __restrict__ dst) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n * dim) return;
    dst[q] = src[(int64_t)rows[q / dim] * dim + q % dim];
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) p[q] = v;
}

__global__ void k_scatter_f64(const double* __restrict__ src, const int32_t* __restrict__ rows, int64_t n,
                              double* __restrict__ dst) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) dst[rows[q]] = src[q];
}

// colmax[j] = max_k E[k * n + j]: one thread per column, rows read in order
// (a row of n consecutive floats is read by consecutive threads).
__global__ void k_colmax(const float* __restrict__ E, int64_t K, int64_t n, float* __restrict__ out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    float m = 0.f;
    for (int64_t k = 0; k < K; ++k) m = fmaxf(m, E[k * n + j]);
    out[j] = m;
}

// Pricing: r[k] -= sum_j Ec[k,j] y[j] over one block of c element columns
// (FP64, fixed order: per thread a strided partial, then a tree).
__global__ __launch_bounds__(256) void k_price(const float* __restrict__ Ec, int64_t c, const double* __restrict__ y,
                                               double* __restrict__ r) {
    __shared__ double red[256];
    const int64_t k = blockIdx.x;
    double a = 0.0;
    for (int64_t j = threadIdx.x; j < c; j += 256) a += (double)Ec[k * c + j] * y[j];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) r[k] -= red[0];
}

// Largest entry of each pose row over the priced columns (to learn which
// elements no candidate sees at all): colmax over rows for c columns.
__global__ void k_colmax_any(const float* __restrict__ Ec, int64_t K, int64_t c, float* __restrict__ out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= c) return;
    float m = 0.f;
    for (int64_t k = 0; k < K; ++k) m = fmaxf(m, Ec[k * c + j]);
    out[j] = m;
}

// Per-block partial sums of E^2 (FP64) for the Frobenius norm.
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ E, int64_t n, double* __restrict__ part) {
    __shared__ double red[256];
    double a = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
        const double v = E[q];
        a += v * v;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Per column i: a = sum_k E[k,i] t_k (FP64, ascending k), visible = some
// E[k,i] > 0, shortfall = max(0, mu - a) over visible columns.  Per block:
// the shortfall sum, the count of shortfalls above short_tol, and the sum of
// E^2 (FP64) of the block's columns, reduced in a fixed tree order.
constexpr int EV_TB = 256;
__global__ __launch_bounds__(EV_TB) void k_plan_eval(const float* __restrict__ E, int64_t K, int64_t N,
                                                     const double* __restrict__ t, double mu, double short_tol,
                                                     double* __restrict__ part_short, double* __restrict__ part_e2,
                                                     int64_t* __restrict__ part_n, int64_t* __restrict__ part_vis) {
    __shared__ double s_short[EV_TB], s_e2[EV_TB];
    __shared__ int64_t s_n[EV_TB], s_v[EV_TB];
    const int64_t i = blockIdx.x * (int64_t)EV_TB + threadIdx.x;
    double sh = 0.0, e2 = 0.0;
    int64_t ns = 0, nv = 0;
    if (i < N) {
        double a = 0.0;
        bool vis = false;
        for (int64_t k = 0; k < K; ++k) {
            const double e = (double)E[k * N + i];
            a += e * t[k];
            e2 += e * e;
            vis = vis || e > 0.0;
        }
        if (vis) {
            nv = 1;
            sh = a < mu ? mu - a : 0.0;
            ns = sh > short_tol ? 1 : 0;
        }
    }
    s_short[threadIdx.x] = sh;
    s_e2[threadIdx.x] = e2;
    s_n[threadIdx.x] = ns;
    s_v[threadIdx.x] = nv;
    __syncthreads();
    for (int w = EV_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_short[threadIdx.x] += s_short[threadIdx.x + w];
            s_e2[threadIdx.x] += s_e2[threadIdx.x + w];
            s_n[threadIdx.x] += s_n[threadIdx.x + w];
            s_v[threadIdx.x] += s_v[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_short[blockIdx.x] = s_short[0];
        part_e2[blockIdx.x] = s_e2[0];
        part_n[blockIdx.x] = s_n[0];
        part_vis[blockIdx.x] = s_v[0];
    }
}

unsigned grid_of(int64_t n, int tb) { return (unsigned)((n + tb - 1) / tb); }

struct Dev {
    void* p = nullptr;
    Dev() = default;
    Dev(const Dev&) = delete;
    Dev& operator=(const Dev&) = delete;
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    ~Dev() { reset(); }
};

template <class T>
uvc_status alloc(Dev& d, int64_t n, const char* what) {
    return dalloc(&d.p, (size_t)std::max<int64_t>(n, 1) * sizeof(T), what);
}

struct Events {
    hipEvent_t e[8] = {};
    ~Events() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

float ms_between(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

}  // namespace
}  // namespace uvc

using namespace uvc;

extern "C" uvc_status uvc_plan_ranked(const uvc_scene* scene, const float* poses_dev, int64_t K, int32_t pose_dim,
                                      const uvc_lamp* lamp, const uvc_opts* opts, int32_t score_mode,
                                      const float* params_dev, int32_t bf16, float keep_frac, float feature_height,
                                      double penalty, double mu_min, double t_max, double tol, int32_t max_iter,
                                      int32_t max_rounds, double* t_out_dev, double* sigma_out_dev,
                                      int32_t* kept_host, uvc_plan_info* info, void* hip_stream) {
    if (!scene || !poses_dev || !lamp || !t_out_dev || !sigma_out_dev || !info)
        return fail(UVC_EINVAL, "NULL scene, poses, lamp, outputs or info");
    if (K < 1 || (pose_dim != 2 && pose_dim != 3)) return fail(UVC_EINVAL, "K must be >= 1 and pose_dim 2 or 3");
    if (K > (int64_t)INT32_MAX) return fail(UVC_EINVAL, "K too large");
    if (score_mode != UVC_RANK_MLP && score_mode != UVC_RANK_AREA && score_mode != UVC_RANK_NONE)
        return fail(UVC_EINVAL, "unknown score_mode");
    if (score_mode == UVC_RANK_MLP && !params_dev) return fail(UVC_EINVAL, "MLP scoring needs params_dev");
    if (!(keep_frac > 0.f && keep_frac <= 1.f)) return fail(UVC_EINVAL, "keep_frac must lie in (0, 1]");
    if (max_rounds < 0 || max_rounds > 1000) return fail(UVC_EINVAL, "max_rounds must lie in [0, 1000]");
    if (!std::isfinite(penalty)) return fail(UVC_EINVAL, "penalty must be finite");
    const int64_t N = scene->n;
    if (N < 1) return fail(UVC_EINVAL, "empty scene");
    hipStream_t st = (hipStream_t)hip_stream;
    uvc_opts o{};
    if (opts) o = *opts;
    o.stats_dev = nullptr;
    o.kernel_ms = nullptr;
    *info = uvc_plan_info{};
    info->min_reduced_cost = std::nan("");
    Events ev;
    for (auto& x : ev.e) UVC_HIP(hipEventCreate(&x));
    UVC_HIP(hipEventRecord(ev.e[0], st));
    uvc_lp_info li{};
    Dev pen;  // the LP penalty, one value per element
    UVC_TRY(alloc<double>(pen, N, "penalty"));
    auto set_penalty = [&](double p) -> uvc_status {
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_of(N, 256)), dim3(256), 0, st, (double*)pen.p, p, N);
        UVC_HIP(hipGetLastError());
        return UVC_OK;
    };

    // p <= 0: the LP's own default over the full matrix
    auto full_plan = [&](hipEvent_t before, hipEvent_t after, double p) -> uvc_status {
        Dev E;
        UVC_TRY(alloc<float>(E, K * N, "E (full candidate set)"));
        UVC_TRY(uvc_compute_irradiance_dense(scene, poses_dev, K, pose_dim, lamp, &o, (float*)E.p, nullptr, st));
        if (p > 0.0) UVC_TRY(set_penalty(p));
        UVC_HIP(hipEventRecord(before, st));
        const uvc_status s =
            uvc_solve_dosage_lp((const float*)E.p, nullptr, nullptr, K, N, p > 0.0 ? (const double*)pen.p : nullptr, mu_min,
                                t_max, tol, max_iter, t_out_dev, sigma_out_dev, nullptr, &li, st);
        UVC_HIP(hipEventRecord(after, st));
        if (s != UVC_OK && s != UVC_ENOTCONV) return s;
        info->n_kept = K;
        info->objective = li.objective;
        info->penalty = li.penalty;
        info->lp_iterations += li.iterations;
        info->lp_converged = s == UVC_OK ? 1 : 0;
        if (kept_host)
            for (int64_t k = 0; k < K; ++k) kept_host[k] = (int32_t)k;
        return UVC_OK;
    };

    if (score_mode == UVC_RANK_NONE) {
        UVC_TRY(full_plan(ev.e[1], ev.e[2], penalty));
        UVC_HIP(hipEventSynchronize(ev.e[2]));
        info->ms_E = ms_between(ev.e[0], ev.e[1]);
        info->ms_lp = ms_between(ev.e[1], ev.e[2]);
        info->ms_total = ms_between(ev.e[0], ev.e[2]);
        return UVC_OK;
    }

    // 1. features and scores
    Dev feat, score;
    UVC_TRY(alloc<float>(feat, K * 64, "ranker features"));
    UVC_TRY(alloc<float>(score, K, "ranker scores"));
    UVC_TRY(uvc_ranker_features(scene, poses_dev, K, pose_dim, feature_height, (float*)feat.p, st));
    UVC_HIP(hipEventRecord(ev.e[1], st));
    if (score_mode == UVC_RANK_MLP)
        UVC_TRY(uvc_ranker_forward(params_dev, (const float*)feat.p, K, bf16, (float*)score.p, st));
    else
        UVC_TRY(uvc_ranker_area_score((const float*)feat.p, K, (float*)score.p, st));
    std::vector<float> hs((size_t)K);
    UVC_HIP(hipMemcpyAsync(hs.data(), score.p, (size_t)K * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    // 2. keep the ceil(keep_frac K) best scores (ties: lower index first)
    const int64_t keep0 = std::min<int64_t>(K, std::max<int64_t>(1, (int64_t)std::ceil((double)keep_frac * (double)K)));
    std::vector<int32_t> order((size_t)K);
    std::iota(order.begin(), order.end(), 0);
    auto better = [&](int32_t a, int32_t b) {
        const float sa = hs[(size_t)a], sb = hs[(size_t)b];
        const bool na = sa != sa, nb = sb != sb;  // NaN scores rank last
        if (na != nb) return nb;
        if (!na && sa != sb) return sa > sb;
        return a < b;
    };
    std::partial_sort(order.begin(), order.begin() + keep0, order.end(), better);
    std::vector<int32_t> kept(order.begin(), order.begin() + keep0);
    std::sort(kept.begin(), kept.end());
    UVC_HIP(hipEventRecord(ev.e[2], st));

    // 3. the LP penalty.  The default, 1.001 ||E||_F, is taken over the whole
    // candidate set, so that the restricted LPs, the pricing and the
    // fallback all solve the LP over all K poses with the same p.  The norm
    // streams E through a bounded buffer, pose rows in blocks (E itself is
    // not kept).
    double p_lp = penalty;
    if (!(p_lp > 0.0)) {
        const int64_t kc = std::max<int64_t>(1, std::min<int64_t>(K, ((int64_t)1 << 26) / N));
        Dev Eb, part;
        const int nb = 1024;
        UVC_TRY(alloc<float>(Eb, kc * N, "E block (penalty)"));
        UVC_TRY(alloc<double>(part, nb, "norm partials"));
        std::vector<double> h(nb);
        double e2 = 0.0;
        for (int64_t k0 = 0; k0 < K; k0 += kc) {
            const int64_t kb = std::min(kc, K - k0);
            UVC_TRY(uvc_compute_irradiance_dense(scene, poses_dev + k0 * pose_dim, kb, pose_dim, lamp, &o,
                                                 (float*)Eb.p, nullptr, st));
            hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(256), 0, st, (const float*)Eb.p, kb * N, (double*)part.p);
            UVC_HIP(hipGetLastError());
            UVC_HIP(hipMemcpyAsync(h.data(), part.p, nb * 8, hipMemcpyDeviceToHost, st));
            UVC_HIP(hipStreamSynchronize(st));
            for (double v : h) e2 += v;
        }
        p_lp = 1.001 * std::sqrt(e2);
    }
    UVC_HIP(hipEventRecord(ev.e[3], st));

    // 4. restricted LP, then pricing rounds
    const int64_t add_cap = std::max<int64_t>(16, keep0);
    const double rc_tol = 1e-6;
    // every restricted LP is solved to tol: a looser tolerance for the rounds
    // that add poses (1e-4, then the accepted set solved again to tol) took
    // 1.4x as long over 59 held-out rooms, the repeated final solve costing
    // more than the iterations it saved
    std::vector<uint8_t> in_set((size_t)K, 0), dark((size_t)N, 0);  // dark: no candidate sees it
    std::vector<uint8_t> dropped_once((size_t)K, 0);
    for (int32_t k : kept) in_set[(size_t)k] = 1;
    Dev tred, dkept;
    std::vector<hipEvent_t> marks;  // per round: E start, LP start, pricing start, pricing end
    std::vector<float> seen_kept;   // last round: per element, max of E over the kept poses
    bool fallback = false, optimal = false;
    for (int round = 0; !fallback && !optimal; ++round) {
        const int64_t keep = (int64_t)kept.size();
        hipEvent_t mk[4];
        for (auto& x : mk) {
            UVC_HIP(hipEventCreate(&x));
            marks.push_back(x);
        }
        UVC_HIP(hipEventRecord(mk[0], st));
        Dev red_poses, Ered, yd;
        tred.reset();
        dkept.reset();
        UVC_TRY(alloc<int32_t>(dkept, keep, "kept pose list"));
        UVC_TRY(alloc<float>(red_poses, keep * pose_dim, "kept poses"));
        UVC_TRY(alloc<float>(Ered, keep * N, "E (kept poses)"));
        UVC_TRY(alloc<double>(tred, keep, "restricted dwell times"));
        UVC_TRY(alloc<double>(yd, N + 1, "LP duals"));
        UVC_HIP(hipMemcpyAsync(dkept.p, kept.data(), (size_t)keep * 4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_gather_rows, dim3(grid_of(keep * pose_dim, 256)), dim3(256), 0, st, poses_dev,
                           (const int32_t*)dkept.p, keep, pose_dim, (float*)red_poses.p);
        UVC_HIP(hipGetLastError());
        UVC_TRY(uvc_compute_irradiance_dense(scene, (const float*)red_poses.p, keep, pose_dim, lamp, &o,
                                             (float*)Ered.p, nullptr, st));
        if (round == 0) UVC_TRY(set_penalty(p_lp));
        UVC_HIP(hipEventRecord(mk[1], st));
        const uvc_status lps = uvc_solve_dosage_lp((const float*)Ered.p, nullptr, nullptr, keep, N, (const double*)pen.p, mu_min, t_max,
                                                   tol, max_iter, (double*)tred.p,
                                                   sigma_out_dev, (double*)yd.p, &li, st);
        if (lps != UVC_OK && lps != UVC_ENOTCONV) return lps;
        UVC_HIP(hipEventRecord(mk[2], st));
        info->n_kept = keep;
        info->objective = li.objective;
        info->lp_iterations += li.iterations;
        info->lp_converged = lps == UVC_OK ? 1 : 0;
        info->rounds = round + 1;
        // an LP stopped at its iteration limit is used as it is when its
        // relative residuals and gap are within 1e-6 (a few LPs stall near
        // 1e-7, and so does the full LP of the same room); otherwise the
        // plan falls back to the full candidate set
        const bool near = lps == UVC_ENOTCONV &&
                          std::max(li.primal_residual, std::max(li.dual_residual, li.gap)) <= 1e-6;
        if (lps != UVC_OK && !near) {
            fallback = true;
            UVC_HIP(hipEventRecord(mk[3], st));
            break;
        }
        if (keep == K) {
            optimal = true;
            UVC_HIP(hipEventRecord(mk[3], st));
            break;
        }
        {
            Dev cmk;
            UVC_TRY(alloc<float>(cmk, N, "kept column maxima"));
            hipLaunchKernelGGL(k_colmax_any, dim3(grid_of(N, 256)), dim3(256), 0, st, (const float*)Ered.p, keep, N,
                               (float*)cmk.p);
            UVC_HIP(hipGetLastError());
            seen_kept.resize((size_t)N);
            UVC_HIP(hipMemcpyAsync(seen_kept.data(), cmk.p, (size_t)N * 4, hipMemcpyDeviceToHost, st));
        }
        // price every pruned pose against the elements with a nonzero dual
        std::vector<double> hy((size_t)N + 1);
        UVC_HIP(hipMemcpyAsync(hy.data(), yd.p, ((size_t)N + 1) * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        const double yb = hy[(size_t)N];
        double ymax = 0.0;
        for (int64_t i = 0; i < N; ++i) ymax = std::max(ymax, hy[(size_t)i]);
        std::vector<int32_t> pe;
        std::vector<double> py;
        for (int64_t i = 0; i < N; ++i)
            if (!dark[(size_t)i] && hy[(size_t)i] > 1e-9 * ymax) {
                pe.push_back((int32_t)i);
                py.push_back(hy[(size_t)i]);
            }
        std::vector<double> rc((size_t)K, 1.0 + yb);
        if (!pe.empty()) {
            const int64_t np = (int64_t)pe.size();
            const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(np, ((int64_t)1 << 26) / K));
            Dev dpe, dpy, Ec, rdev, cm;
            UVC_TRY(alloc<int32_t>(dpe, np, "priced elements"));
            UVC_TRY(alloc<double>(dpy, np, "priced duals"));
            UVC_TRY(alloc<float>(Ec, K * chunk, "pricing block"));
            UVC_TRY(alloc<double>(rdev, K, "reduced costs"));
            UVC_TRY(alloc<float>(cm, chunk, "pricing column maxima"));
            UVC_HIP(hipMemcpyAsync(dpe.p, pe.data(), (size_t)np * 4, hipMemcpyHostToDevice, st));
            UVC_HIP(hipMemcpyAsync(dpy.p, py.data(), (size_t)np * 8, hipMemcpyHostToDevice, st));
            UVC_HIP(hipMemcpyAsync(rdev.p, rc.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
            std::vector<float> hm((size_t)chunk);
            for (int64_t c0 = 0; c0 < np; c0 += chunk) {
                const int64_t c = std::min(chunk, np - c0);
                UVC_TRY(uvc_compute_irradiance_targets(scene, poses_dev, K, pose_dim, lamp, &o,
                                                       (const int32_t*)dpe.p + c0, c, (float*)Ec.p, nullptr, st));
                hipLaunchKernelGGL(k_price, dim3((unsigned)K), dim3(256), 0, st, (const float*)Ec.p, c,
                                   (const double*)dpy.p + c0, (double*)rdev.p);
                hipLaunchKernelGGL(k_colmax_any, dim3(grid_of(c, 256)), dim3(256), 0, st, (const float*)Ec.p, K, c,
                                   (float*)cm.p);
                UVC_HIP(hipGetLastError());
                UVC_HIP(hipMemcpyAsync(hm.data(), cm.p, (size_t)c * 4, hipMemcpyDeviceToHost, st));
                UVC_HIP(hipStreamSynchronize(st));
                for (int64_t j = 0; j < c; ++j)
                    if (hm[(size_t)j] == 0.f) dark[(size_t)pe[(size_t)(c0 + j)]] = 1;
                info->n_priced += c;
            }
            UVC_HIP(hipMemcpyAsync(rc.data(), rdev.p, (size_t)K * 8, hipMemcpyDeviceToHost, st));
            UVC_HIP(hipStreamSynchronize(st));
        }
        UVC_HIP(hipEventRecord(mk[3], st));
        std::vector<int32_t> cand;
        double rmin = 0.0;
        for (int64_t k = 0; k < K; ++k)
            if (!in_set[(size_t)k]) {
                rmin = std::min(rmin, rc[(size_t)k]);
                if (rc[(size_t)k] < -rc_tol) cand.push_back((int32_t)k);
            }
        info->min_reduced_cost = rmin;
        if (cand.empty()) {
            optimal = true;
        } else if (info->rounds_added >= max_rounds) {
            fallback = true;
        } else {
            // kept poses without dwell whose reduced cost is clearly positive
            // leave the set (each pose at most once): the restricted LPs stay
            // near the support; a pose that prices negative later rejoins
            {
                std::vector<double> ht((size_t)keep);
                UVC_HIP(hipMemcpyAsync(ht.data(), tred.p, (size_t)keep * 8, hipMemcpyDeviceToHost, st));
                UVC_HIP(hipStreamSynchronize(st));
                double tmx = 0.0;
                for (double v : ht) tmx = std::max(tmx, v);
                const double margin = 1e-2 * (1.0 + std::fabs(yb));
                std::vector<int32_t> stay;
                stay.reserve(kept.size());
                for (int64_t q = 0; q < keep; ++q) {
                    const int32_t k = kept[(size_t)q];
                    if (!dropped_once[(size_t)k] && ht[(size_t)q] <= 1e-9 * tmx && rc[(size_t)k] > margin) {
                        in_set[(size_t)k] = 0;
                        dropped_once[(size_t)k] = 1;
                        info->n_dropped += 1;
                    } else {
                        stay.push_back(k);
                    }
                }
                kept.swap(stay);
            }
            const int64_t na = std::min<int64_t>((int64_t)cand.size(), add_cap);
            std::partial_sort(cand.begin(), cand.begin() + na, cand.end(), [&](int32_t a, int32_t b) {
                return rc[(size_t)a] != rc[(size_t)b] ? rc[(size_t)a] < rc[(size_t)b] : a < b;
            });
            for (int64_t q = 0; q < na; ++q) {
                kept.push_back(cand[(size_t)q]);
                in_set[(size_t)cand[(size_t)q]] = 1;
            }
            info->n_added += na;
            info->rounds_added += 1;
            std::sort(kept.begin(), kept.end());
        }
    }
    UVC_HIP(hipEventRecord(ev.e[5], st));
    if (fallback) {
        info->fell_back = 1;
        // the full candidate set with the caller's penalty (<= 0: the LP's own
        // default over the full matrix, the same p as p_lp up to the order of
        // the norm's sum), so that the fallback is exactly the full plan
        UVC_TRY(full_plan(ev.e[6], ev.e[7], penalty));
    } else {
        const int64_t keep = (int64_t)kept.size();
        // elements the kept poses leave unseen sit out of the restricted LP
        // at sigma_i = mu_min; those some candidate sees (priced, not dark)
        // belong to the full LP's objective with their p mu_min
        if (keep < K && !seen_kept.empty()) {
            int64_t unseen = 0;
            for (int64_t i = 0; i < N; ++i) unseen += (seen_kept[(size_t)i] == 0.f && !dark[(size_t)i]) ? 1 : 0;
            info->objective += (double)unseen * p_lp * mu_min;
        }
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_of(K, 256)), dim3(256), 0, st, t_out_dev, 0.0, K);
        hipLaunchKernelGGL(k_scatter_f64, dim3(grid_of(keep, 256)), dim3(256), 0, st, (const double*)tred.p,
                           (const int32_t*)dkept.p, keep, t_out_dev);
        UVC_HIP(hipGetLastError());
        UVC_HIP(hipEventRecord(ev.e[6], st));
        UVC_HIP(hipEventRecord(ev.e[7], st));
        if (kept_host) std::copy(kept.begin(), kept.end(), kept_host);
    }
    if (!fallback) info->penalty = p_lp;
    UVC_HIP(hipEventSynchronize(ev.e[7]));
    info->ms_features = ms_between(ev.e[0], ev.e[1]);
    info->ms_score = ms_between(ev.e[1], ev.e[2]);
    info->ms_E = ms_between(ev.e[2], ev.e[3]);  // the default penalty's norm pass
    for (size_t r = 0; r + 3 < marks.size(); r += 4) {
        info->ms_E += ms_between(marks[r], marks[r + 1]);
        info->ms_lp += ms_between(marks[r + 1], marks[r + 2]);
        info->ms_price += ms_between(marks[r + 2], marks[r + 3]);
    }
    for (auto x : marks) (void)hipEventDestroy(x);
    info->ms_fallback = ms_between(ev.e[5], ev.e[7]);
    info->ms_total = ms_between(ev.e[0], ev.e[7]);
    return UVC_OK;
}

extern "C" uvc_status uvc_plan_evaluate(const float* E_dev, int64_t K, int64_t N, const double* t_dev,
                                        double mu_min, double penalty, double* objective, double* shortfall,
                                        int64_t* n_short, int64_t* n_visible, void* hip_stream) {
    if (!E_dev || !t_dev || !objective) return fail(UVC_EINVAL, "NULL E, t or objective");
    if (K < 1 || N < 1) return fail(UVC_EINVAL, "empty matrix");
    if (!(mu_min > 0.0) || !std::isfinite(mu_min) || !std::isfinite(penalty))
        return fail(UVC_EINVAL, "mu_min must be positive and the penalty finite");
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t nb = (N + EV_TB - 1) / EV_TB;
    if (nb > (int64_t)INT32_MAX) return fail(UVC_EINVAL, "N too large");
    Dev ps, pe, pn, pv;
    UVC_TRY(alloc<double>(ps, nb, "evaluation partials"));
    UVC_TRY(alloc<double>(pe, nb, "evaluation partials"));
    UVC_TRY(alloc<int64_t>(pn, nb, "evaluation partials"));
    UVC_TRY(alloc<int64_t>(pv, nb, "evaluation partials"));
    hipLaunchKernelGGL(k_plan_eval, dim3((unsigned)nb), dim3(EV_TB), 0, st, E_dev, K, N, t_dev, mu_min,
                       1e-6 * mu_min, (double*)ps.p, (double*)pe.p, (int64_t*)pn.p, (int64_t*)pv.p);
    UVC_HIP(hipGetLastError());
    std::vector<double> hs((size_t)nb), he((size_t)nb), ht((size_t)K);
    std::vector<int64_t> hn((size_t)nb), hv((size_t)nb);
    UVC_HIP(hipMemcpyAsync(hs.data(), ps.p, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(he.data(), pe.p, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(hn.data(), pn.p, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(hv.data(), pv.p, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(ht.data(), t_dev, (size_t)K * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    double sh = 0.0, e2 = 0.0, tsum = 0.0;
    int64_t ns = 0, nv = 0;
    for (int64_t b = 0; b < nb; ++b) {
        sh += hs[(size_t)b];
        e2 += he[(size_t)b];
        ns += hn[(size_t)b];
        nv += hv[(size_t)b];
    }
    for (double v : ht) tsum += v;
    const double p = penalty > 0.0 ? penalty : 1.001 * std::sqrt(e2);
    *objective = tsum + p * sh;
    if (shortfall) *shortfall = sh;
    if (n_short) *n_short = ns;
    if (n_visible) *n_visible = nv;
    return UVC_OK;
}
