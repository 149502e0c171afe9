// Route stage (Sec. IV-D, second stage; roadmap distances Sec. IV-B): the
// lamp visits the poses the dosage LP gives a dwell time along a closed
// tour; plan time = sum of dwell times + tour length / v_max.
//
// Distances are grid geodesics through free space: 8-connected cells, step
// costs cell and cell * sqrt(2) in FP64, diagonal steps only between two
// free orthogonal neighbours.  One workgroup per stop relaxes its distance
// field in place until no cell changes; every value ever written is the
// FP64 sum of the steps of some path (accumulated from the stop), and a
// relaxation only lowers a value, so the field converges to the smallest
// such sum for every cell whatever the order of the updates: the value a
// label-setting Dijkstra computes.  The m x m matrix is symmetrised as
// min(d(a, b), d(b, a)).
//
// Tour: nearest neighbour from the first stop, then best-improvement 2-opt
// and, when 2-opt finds nothing, best-improvement Or-opt (segments of 1-3
// stops moved elsewhere, same orientation), until no move improves by more
// than 1e-12 of the tour length.  One workgroup holds the tour in LDS and
// evaluates every move of a pass in parallel; the best move is the one with
// the smallest FP64 delta, ties broken by the lowest move index, so the
// tour does not depend on the reduction order.
#include "uvc_common.hpp"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace uvc {
namespace {

constexpr int RT_TB = 1024;
constexpr int ROUTE_MAX_STOPS = 4096;
constexpr double SQRT2 = 1.4142135623730951;  // nearest double to sqrt(2)

// dist[s][cell] for stop s = blockIdx.x; src[s] = its cell.
__global__ __launch_bounds__(RT_TB) void k_geodesic(const uint8_t* __restrict__ free, int H, int W, double w_o,
                                                     const int64_t* __restrict__ src, double* __restrict__ dist) {
    const int64_t n = (int64_t)H * W;
    double* d = dist + (int64_t)blockIdx.x * n;
    for (int64_t c = threadIdx.x; c < n; c += RT_TB) d[c] = INFINITY;
    __syncthreads();
    if (threadIdx.x == 0) d[src[blockIdx.x]] = 0.0;
    __syncthreads();
    const double w_d = w_o * SQRT2;
    // at most n sweeps: every sweep fixes at least one more cell of every
    // shortest-path tree; in practice a few hundred
    for (int64_t sweep = 0; sweep <= n; ++sweep) {
        int changed = 0;
        for (int64_t c = threadIdx.x; c < n; c += RT_TB) {
            if (!free[c]) continue;
            const int r = (int)(c / W), q = (int)(c % W);
            double best = d[c];
            const bool up = r > 0 && free[c - W], dn = r + 1 < H && free[c + W];
            const bool lf = q > 0 && free[c - 1], rt = q + 1 < W && free[c + 1];
            if (up) best = fmin(best, d[c - W] + w_o);
            if (dn) best = fmin(best, d[c + W] + w_o);
            if (lf) best = fmin(best, d[c - 1] + w_o);
            if (rt) best = fmin(best, d[c + 1] + w_o);
            if (up && lf && free[c - W - 1]) best = fmin(best, d[c - W - 1] + w_d);
            if (up && rt && free[c - W + 1]) best = fmin(best, d[c - W + 1] + w_d);
            if (dn && lf && free[c + W - 1]) best = fmin(best, d[c + W - 1] + w_d);
            if (dn && rt && free[c + W + 1]) best = fmin(best, d[c + W + 1] + w_d);
            if (best < d[c]) {
                d[c] = best;
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
}

// D[a][b] = min(dist_a(cell_b), dist_b(cell_a)); bad = 1 if some pair has
// no free path.
__global__ void k_geo_matrix(const double* __restrict__ dist, int64_t n, const int64_t* __restrict__ src, int m,
                             double* __restrict__ D, int* __restrict__ bad) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= (int64_t)m * m) return;
    const int a = (int)(q / m), b = (int)(q % m);
    const double v = fmin(dist[(int64_t)a * n + src[b]], dist[(int64_t)b * n + src[a]]);
    D[q] = v;
    if (!(v < INFINITY)) *bad = 1;
}

// bad = 1 if some distance is negative or not finite.
__global__ void k_check_dist(const double* __restrict__ D, int64_t n, int* __restrict__ bad) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n && !(D[q] >= 0.0 && D[q] < INFINITY)) *bad = 1;
}

__device__ __forceinline__ bool better(double d, int q, double d2, int q2) { return d < d2 || (d == d2 && q < q2); }

// Smallest (delta, index) over the workgroup (a total order: the result
// does not depend on how the pairs are combined).
__device__ void block_argmin(double& d, int& q, double* sd, int* sq) {
    sd[threadIdx.x] = d;
    sq[threadIdx.x] = q;
    __syncthreads();
    for (int w = RT_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && better(sd[threadIdx.x + w], sq[threadIdx.x + w], sd[threadIdx.x], sq[threadIdx.x])) {
            sd[threadIdx.x] = sd[threadIdx.x + w];
            sq[threadIdx.x] = sq[threadIdx.x + w];
        }
        __syncthreads();
    }
    d = sd[0];
    q = sq[0];
    __syncthreads();
}

__global__ __launch_bounds__(RT_TB) void k_tour(const double* __restrict__ D, int m, int max_moves,
                                                int32_t* __restrict__ tour_out, double* __restrict__ length_out,
                                                int* __restrict__ moves_out) {
    __shared__ int t[ROUTE_MAX_STOPS], tmp[ROUTE_MAX_STOPS];
    __shared__ unsigned char used[ROUTE_MAX_STOPS];
    __shared__ double sd[RT_TB];
    __shared__ int sq[RT_TB];
    __shared__ double s_len;
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += RT_TB) used[i] = 0;
    __syncthreads();
    // nearest neighbour from stop 0 (ties: the lowest index)
    if (tid == 0) {
        t[0] = 0;
        used[0] = 1;
    }
    __syncthreads();
    for (int k = 1; k < m; ++k) {
        const int cur = t[k - 1];
        double bd = INFINITY;
        int bq = 0x7fffffff;
        for (int c = tid; c < m; c += RT_TB)
            if (!used[c] && better(D[(int64_t)cur * m + c], c, bd, bq)) {
                bd = D[(int64_t)cur * m + c];
                bq = c;
            }
        block_argmin(bd, bq, sd, sq);
        if (tid == 0) {
            t[k] = bq;
            used[bq] = 1;
        }
        __syncthreads();
    }
    auto tour_length = [&]() -> double {  // in tour order, one thread
        if (tid == 0) {
            double L = 0.0;
            for (int k = 0; k < m; ++k) L = L + D[(int64_t)t[k] * m + t[(k + 1) % m]];
            s_len = L;
        }
        __syncthreads();
        const double L = s_len;
        __syncthreads();
        return L;
    };
    int moves = 0;
    while (m >= 4 && moves < max_moves) {
        const double eps = 1e-12 * tour_length();
        // 2-opt: q = i m + j
        double bd = INFINITY;
        int bq = 0x7fffffff;
        for (int q = tid; q < m * m; q += RT_TB) {
            const int i = q / m, j = q % m;
            if (i > m - 3 || j < i + 2 || (i == 0 && j == m - 1)) continue;
            const int a = t[i], b = t[i + 1], c = t[j], e = t[(j + 1) % m];
            const double delta = (D[(int64_t)a * m + c] + D[(int64_t)b * m + e]) -
                                 (D[(int64_t)a * m + b] + D[(int64_t)c * m + e]);
            if (better(delta, q, bd, bq)) {
                bd = delta;
                bq = q;
            }
        }
        block_argmin(bd, bq, sd, sq);
        if (bd < -eps) {
            const int i = bq / m, j = bq % m;
            for (int k = tid; k < (j - i) / 2; k += RT_TB) {
                const int x = t[i + 1 + k];
                t[i + 1 + k] = t[j - k];
                t[j - k] = x;
            }
            __syncthreads();
            ++moves;
            continue;
        }
        // Or-opt: q = ((s - 1) m + i) m + p
        bd = INFINITY;
        bq = 0x7fffffff;
        for (int q = tid; q < 3 * m * m; q += RT_TB) {
            const int s = q / (m * m) + 1, i = (q / m) % m, p = q % m;
            if (i < 1 || i > m - s || (p >= i - 1 && p <= i + s - 1)) continue;
            const int f = t[i], l = t[i + s - 1], prev = t[i - 1], nxt = t[(i + s) % m];
            const int u = t[p], v = t[(p + 1) % m];
            const double add = (D[(int64_t)prev * m + nxt] + D[(int64_t)u * m + f]) + D[(int64_t)l * m + v];
            const double rem = (D[(int64_t)prev * m + f] + D[(int64_t)l * m + nxt]) + D[(int64_t)u * m + v];
            const double delta = add - rem;
            if (better(delta, q, bd, bq)) {
                bd = delta;
                bq = q;
            }
        }
        block_argmin(bd, bq, sd, sq);
        if (!(bd < -eps)) break;
        {
            const int s = bq / (m * m) + 1, i = (bq / m) % m, p = bq % m;
            if (tid == 0) {
                // remove the segment, then insert it after the stop that was
                // at position p
                int seg[3];
                for (int k = 0; k < s; ++k) seg[k] = t[i + k];
                int n = 0, at = -1;
                for (int k = 0; k < m; ++k) {
                    if (k >= i && k < i + s) continue;
                    tmp[n] = t[k];
                    if (k == p) at = n;
                    ++n;
                }
                int w = 0;
                for (int k = 0; k <= at; ++k) t[w++] = tmp[k];
                for (int k = 0; k < s; ++k) t[w++] = seg[k];
                for (int k = at + 1; k < n; ++k) t[w++] = tmp[k];
            }
            __syncthreads();
        }
        ++moves;
    }
    const double L = tour_length();
    for (int k = tid; k < m; k += RT_TB) tour_out[k] = t[k];
    if (tid == 0) {
        *length_out = L;
        *moves_out = moves;
    }
}

}  // namespace
}  // namespace uvc

using namespace uvc;

// Stop cells and the device arrays of one geodesic computation.
static uvc_status stop_cells(const float* stops_dev, int32_t m, const uint8_t* free_dev, int32_t H, int32_t W,
                             float x0, float y0, float cell, hipStream_t st, std::vector<int64_t>& src) {
    std::vector<float> hs((size_t)m * 2);
    std::vector<uint8_t> hf((size_t)H * W);
    UVC_HIP(hipMemcpyAsync(hs.data(), stops_dev, hs.size() * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(hf.data(), free_dev, hf.size(), hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    src.resize((size_t)m);
    for (int32_t a = 0; a < m; ++a) {
        const double x = hs[(size_t)a * 2], y = hs[(size_t)a * 2 + 1];
        if (!std::isfinite(x) || !std::isfinite(y)) return fail(UVC_EINVAL, "stop " + std::to_string(a) + " is not finite");
        const double c = std::floor((x - (double)x0) / (double)cell), r = std::floor((y - (double)y0) / (double)cell);
        if (!(c >= 0 && c < W && r >= 0 && r < H) || !hf[(size_t)r * W + (size_t)c])
            return fail(UVC_EINVAL, "stop " + std::to_string(a) + " lies outside the grid or in a blocked cell");
        src[(size_t)a] = (int64_t)r * W + (int64_t)c;
    }
    return UVC_OK;
}

extern "C" uvc_status uvc_route_geodesics(const uint8_t* free_dev, int32_t H, int32_t W, float x0, float y0,
                                          float cell, const float* stops_dev, int32_t m, double* dist_dev,
                                          void* hip_stream) {
    if (H < 1 || W < 1 || !free_dev) return fail(UVC_EINVAL, "empty or NULL free-space grid");
    if (!(cell > 0.f) || !std::isfinite(cell) || !std::isfinite(x0) || !std::isfinite(y0))
        return fail(UVC_EINVAL, "grid cell must be positive and the origin finite");
    if (m < 0 || m > ROUTE_MAX_STOPS) return fail(UVC_EINVAL, "m must lie in [0, 4096]");
    if (m == 0) return UVC_OK;
    if (!stops_dev || !dist_dev) return fail(UVC_EINVAL, "NULL stops or distance output");
    const int64_t n = (int64_t)H * W;
    if ((double)n * (double)m > (double)((int64_t)1 << 31)) return fail(UVC_EINVAL, "grid cells x stops above 2^31");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<int64_t> src;
    UVC_TRY(stop_cells(stops_dev, m, free_dev, H, W, x0, y0, cell, st, src));
    int64_t* dsrc = nullptr;
    double* field = nullptr;
    int* bad = nullptr;
    UVC_TRY(dalloc_n(&dsrc, (size_t)m, "stop cells"));
    uvc_status r = dalloc_n(&field, (size_t)n * m, "distance fields");
    if (r == UVC_OK) r = dalloc_n(&bad, 1, "route flag");
    int hb = 0;
    if (r == UVC_OK) {
        hipError_t e = hipMemcpyAsync(dsrc, src.data(), (size_t)m * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(bad, &hb, 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_geodesic, dim3((unsigned)m), dim3(RT_TB), 0, st, free_dev, H, W,
                               (double)cell, (const int64_t*)dsrc, field);
            const int64_t mm = (int64_t)m * m;
            hipLaunchKernelGGL(k_geo_matrix, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, st,
                               (const double*)field, n, (const int64_t*)dsrc, m, dist_dev, bad);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("geodesics: ") + hipGetErrorString(e));
    }
    (void)hipFree(dsrc);
    (void)hipFree(field);
    (void)hipFree(bad);
    if (r == UVC_OK && hb) r = fail(UVC_EINVAL, "two stops are not connected through free space");
    return r;
}

extern "C" uvc_status uvc_route_tour(const double* dist_dev, int32_t m, int32_t max_moves, int32_t* tour_host,
                                     double* length, int32_t* moves, void* hip_stream) {
    if (m < 0 || m > ROUTE_MAX_STOPS) return fail(UVC_EINVAL, "m must lie in [0, 4096]");
    if (length) *length = 0.0;
    if (moves) *moves = 0;
    if (m == 0) return UVC_OK;
    if (!dist_dev || !tour_host) return fail(UVC_EINVAL, "NULL distances or tour output");
    hipStream_t st = (hipStream_t)hip_stream;
    int32_t* dt = nullptr;
    double* dl = nullptr;
    int* dm = nullptr;
    UVC_TRY(dalloc_n(&dt, (size_t)m, "tour"));
    uvc_status r = dalloc_n(&dl, 1, "tour length");
    if (r == UVC_OK) r = dalloc_n(&dm, 1, "tour moves");
    double hl = 0.0;
    int hm = 0;
    if (r == UVC_OK) {
        // the distances must be finite and nonnegative (the flag reuses dm)
        const int64_t mm = (int64_t)m * m;
        hipError_t e = hipMemcpyAsync(dm, &hm, 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_check_dist, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, st, dist_dev, mm, dm);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&hm, dm, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("tour check: ") + hipGetErrorString(e));
        else if (hm) r = fail(UVC_EINVAL, "distances must be finite and nonnegative");
        hm = 0;
    }
    if (r == UVC_OK) {
        const int cap = max_moves > 0 ? max_moves : 100 * m;
        hipLaunchKernelGGL(k_tour, dim3(1), dim3(RT_TB), 0, st, dist_dev, m, cap, dt, dl, dm);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(tour_host, dt, (size_t)m * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hl, dl, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hm, dm, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("tour: ") + hipGetErrorString(e));
    }
    (void)hipFree(dt);
    (void)hipFree(dl);
    (void)hipFree(dm);
    if (r == UVC_OK) {
        if (length) *length = hl;
        if (moves) *moves = hm;
    }
    return r;
}

extern "C" uvc_status uvc_plan_route(const float* poses_dev, int64_t K, int32_t pose_dim, const double* t_dev,
                                     double rel_threshold, const uint8_t* free_dev, int32_t H, int32_t W, float x0,
                                     float y0, float cell, double v_max, int32_t* stops_host, int32_t* m_out,
                                     double* length, double* plan_time, void* hip_stream) {
    if (K < 0 || (pose_dim != 2 && pose_dim != 3)) return fail(UVC_EINVAL, "invalid K or pose_dim");
    if (!(v_max > 0.0) || !std::isfinite(v_max)) return fail(UVC_EINVAL, "v_max must be positive");
    if (!(rel_threshold >= 0.0) || !(rel_threshold < 1.0)) return fail(UVC_EINVAL, "rel_threshold must lie in [0, 1)");
    if (!stops_host || !m_out || !length || !plan_time) return fail(UVC_EINVAL, "NULL output");
    *m_out = 0;
    *length = 0.0;
    *plan_time = 0.0;
    if (K == 0) return UVC_OK;
    if (!poses_dev || !t_dev) return fail(UVC_EINVAL, "NULL poses or dwell times");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<double> ht((size_t)K);
    std::vector<float> hp((size_t)K * pose_dim);
    UVC_HIP(hipMemcpyAsync(ht.data(), t_dev, (size_t)K * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(hp.data(), poses_dev, hp.size() * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    double tsum = 0.0;
    for (int64_t k = 0; k < K; ++k) {
        if (!std::isfinite(ht[(size_t)k]) || ht[(size_t)k] < 0.0)
            return fail(UVC_EINVAL, "dwell time " + std::to_string(k) + " is negative or not finite");
        tsum += ht[(size_t)k];
    }
    // the stops: poses whose dwell time is above rel_threshold of the total
    std::vector<int32_t> sel;
    std::vector<float> xy;
    for (int64_t k = 0; k < K; ++k)
        if (ht[(size_t)k] > rel_threshold * tsum) {
            sel.push_back((int32_t)k);
            xy.push_back(hp[(size_t)k * pose_dim]);
            xy.push_back(hp[(size_t)k * pose_dim + 1]);
        }
    const int32_t m = (int32_t)sel.size();
    if (m > ROUTE_MAX_STOPS) return fail(UVC_EUNSUPPORTED, "more than 4096 stops");
    *plan_time = tsum;
    if (m == 0) return UVC_OK;
    float* dxy = nullptr;
    double* D = nullptr;
    UVC_TRY(dalloc_n(&dxy, xy.size(), "stops"));
    uvc_status r = dalloc_n(&D, (size_t)m * m, "stop distances");
    std::vector<int32_t> tour((size_t)m);
    double L = 0.0;
    if (r == UVC_OK) {
        hipError_t e = hipMemcpyAsync(dxy, xy.data(), xy.size() * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = fail(UVC_EDEVICE, std::string("stop upload: ") + hipGetErrorString(e));
    }
    if (r == UVC_OK) r = uvc_route_geodesics(free_dev, H, W, x0, y0, cell, dxy, m, D, hip_stream);
    if (r == UVC_OK) r = uvc_route_tour(D, m, 0, tour.data(), &L, nullptr, hip_stream);
    (void)hipFree(dxy);
    (void)hipFree(D);
    if (r != UVC_OK) return r;
    for (int32_t q = 0; q < m; ++q) stops_host[q] = sel[(size_t)tour[(size_t)q]];
    *m_out = m;
    *length = L;
    *plan_time = tsum + L / v_max;
    return UVC_OK;
}
