// Relaxed dosage LP (Sec. IV-D, "simple LP") on the GPU:
//
//   minimise   sum_k t_k + sum_i p_i sigma_i
//   subject to sum_k E[k,i] t_k + sigma_i >= mu_min   (every visible element i)
//              sum_k t_k <= T_max,  t >= 0,  sigma >= 0
//
// Elements no pose sees (all E[k,i] = 0) are dropped: sigma_i = mu_min is
// fixed and their constant p_i mu_min is left out of the objective.
//
// Solver: Mehrotra predictor-corrector interior point method on
//   min c.x  s.t.  G x - s = h,  x >= 0, s >= 0
// with x = (t, sigma), G = [[E^T, I], [-1^T, 0]], h = (mu_min, -T_max),
// c = (1, p).  With D = s^-1 y (rows) and Theta = x^-1 z (columns), the
// Newton system reduces, after eliminating the sigma block (diagonal), to the
// K x K SPD system
//   M dt = r,   M = E diag(d~) E^T + d_b 1 1^T + diag(Theta_t),
//   d~ = D_c Theta_s / (D_c + Theta_s),
// formed on the GPU by an FP64 SYRK over the FP32 matrix and factored by a
// blocked FP64 Cholesky; the two solves per iteration (predictor, corrector)
// reuse the factor.  The O(K + N) vector algebra runs on the host in FP64.
// Every device reduction sums in a fixed order: results are deterministic.
#include "uvc_common.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace uvc {

constexpr int LP_TB = 256;

// ---------------------------------------------------------------- kernels
// colmax[i] = max_k |E[k,i]| ; also per-row-chunk partial sums of E^2 for ||E||_F
__global__ void k_lp_colstats(const float* __restrict__ E, int64_t K, int64_t N, int64_t rows_per,
                              float* __restrict__ colmax_part, double* __restrict__ sq_part) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    const int64_t k0 = blockIdx.y * rows_per, k1 = std::min<int64_t>(K, k0 + rows_per);
    float mx = 0.f;
    double sq = 0.0;
    if (i < N)
        for (int64_t k = k0; k < k1; ++k) {
            const float v = E[k * N + i];
            mx = fmaxf(mx, fabsf(v));
            sq += (double)v * (double)v;
        }
    if (i < N) {
        colmax_part[blockIdx.y * N + i] = mx;
        sq_part[blockIdx.y * N + i] = sq;
    }
}

// rowmax[k] = max_i |E[k,i]| * w[i] (w = current column... row scale of the
// coverage rows) for visible i; one block per row.
__global__ void k_lp_rowmax(const float* __restrict__ E, int64_t N, const double* __restrict__ w,
                            const unsigned char* __restrict__ vis, double* __restrict__ out) {
    __shared__ double red[LP_TB];
    const int64_t k = blockIdx.x;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += LP_TB)
        if (vis[i]) mx = fmax(mx, fabs((double)E[k * N + i]) * w[i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = LP_TB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

// colmax over rows k of |E[k,i]| * w[k]; partial over row chunks.
__global__ void k_lp_colmax_w(const float* __restrict__ E, int64_t K, int64_t N, int64_t rows_per,
                              const double* __restrict__ w, double* __restrict__ part) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    const int64_t k0 = blockIdx.y * rows_per, k1 = std::min<int64_t>(K, k0 + rows_per);
    double mx = 0.0;
    if (i < N)
        for (int64_t k = k0; k < k1; ++k) mx = fmax(mx, fabs((double)E[k * N + i]) * w[k]);
    if (i < N) part[blockIdx.y * N + i] = mx;
}

// part[chunk][i] = sum_{k in chunk} E[k,i] * u[k]   (E^T u, column sums)
__global__ void k_lp_Etu(const float* __restrict__ E, int64_t K, int64_t N, int64_t rows_per,
                         const double* __restrict__ u, double* __restrict__ part) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    const int64_t k0 = blockIdx.y * rows_per, k1 = std::min<int64_t>(K, k0 + rows_per);
    double acc = 0.0;
    if (i < N)
        for (int64_t k = k0; k < k1; ++k) acc += (double)E[k * N + i] * u[k];
    if (i < N) part[blockIdx.y * N + i] = acc;
}

// out[k] = sum_i E[k,i] * v[i]  (E v, row dot products; one block per row,
// fixed-order tree reduction)
__global__ void k_lp_Ev(const float* __restrict__ E, int64_t N, const double* __restrict__ v,
                        double* __restrict__ out) {
    __shared__ double red[LP_TB];
    const int64_t k = blockIdx.x;
    double acc = 0.0;
    const float* row = E + k * N;
    for (int64_t i = threadIdx.x; i < N; i += LP_TB) acc += (double)row[i] * v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = LP_TB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

// out[i] = sum over chunks of part[chunk][i] (fixed order)
__global__ void k_lp_sum_parts(const double* __restrict__ part, int64_t chunks, int64_t N, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    double a = 0.0;
    for (int64_t c = 0; c < chunks; ++c) a += part[c * N + i];
    out[i] = a;
}

__global__ void k_lp_max_parts(const float* __restrict__ part, int64_t chunks, int64_t N, float* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    float a = 0.f;
    for (int64_t c = 0; c < chunks; ++c) a = fmaxf(a, part[c * N + i]);
    out[i] = a;
}

__global__ void k_lp_max_parts_d(const double* __restrict__ part, int64_t chunks, int64_t N,
                                 double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    double a = 0.0;
    for (int64_t c = 0; c < chunks; ++c) a = fmax(a, part[c * N + i]);
    out[i] = a;
}

// Fixed-order block sums of up to 4 vectors of length n (each block writes
// its partial sums; a second pass sums the partials).
__global__ void k_lp_dots(const double* __restrict__ a0, const double* __restrict__ b0, const double* __restrict__ a1,
                          const double* __restrict__ b1, int64_t n, int mode, double* __restrict__ part) {
    __shared__ double red[2][LP_TB];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * LP_TB) {
        if (mode == 0) {  // sum a0*b0, sum a1*b1
            s0 += a0[i] * b0[i];
            if (a1) s1 += a1[i] * b1[i];
        } else if (mode == 2) {  // max a0 (a0 >= 0)
            s0 = fmax(s0, a0[i]);
        } else {          // sum (a0 - b0)^2, sum (a1 - b1)^2
            const double d0 = a0[i] - b0[i];
            s0 += d0 * d0;
            if (a1) {
                const double d1 = a1[i] - b1[i];
                s1 += d1 * d1;
            }
        }
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int s = LP_TB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            if (mode == 2) {
                red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            } else {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ void k_lp_sum_pairs(const double* __restrict__ part, int nb, double* __restrict__ out, int mode) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (mode == 2) {
                s0 = fmax(s0, part[2 * b]);
            } else {
                s0 += part[2 * b];
                s1 += part[2 * b + 1];
            }
        }
        out[0] = s0;
        out[1] = s1;
    }
}


// ------------------------------------------------------- dense FP64 algebra
constexpr int SY_T = 64;   // output tile
constexpr int SY_KC = 16;  // inner chunk

// M[a][b] = sum_i E[a,i] d[i] E[b,i] for the lower tiles (tile row >= tile
// col) of the K x K row-major M.  256 threads, 4 x 4 outputs each.
__global__ __launch_bounds__(256) void k_syrk(const float* __restrict__ E, int64_t K, int64_t N,
                                              const double* __restrict__ d, double* __restrict__ M) {
    __shared__ double As[SY_KC][SY_T + 1];
    __shared__ double Bs[SY_KC][SY_T + 1];
    // lower-triangular tile index -> (tr, tc)
    const int64_t t = blockIdx.x;
    int64_t tr = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((tr + 1) * (tr + 2) / 2 <= t) ++tr;
    while (tr * (tr + 1) / 2 > t) --tr;
    const int64_t tc = t - tr * (tr + 1) / 2;
    const int64_t a0 = tr * SY_T, b0 = tc * SY_T;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4] = {};
    for (int64_t i0 = 0; i0 < N; i0 += SY_KC) {
        for (int q = threadIdx.x; q < SY_T * SY_KC; q += 256) {
            const int r = q / SY_KC, kk = q % SY_KC;
            const int64_t i = i0 + kk;
            const int64_t a = a0 + r, b = b0 + r;
            const double di = (i < N) ? d[i] : 0.0;
            As[kk][r] = (a < K && i < N) ? (double)E[a * N + i] * di : 0.0;
            Bs[kk][r] = (b < K && i < N) ? (double)E[b * N + i] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SY_KC; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = As[kk][ty * 4 + u];
                bv[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            const int64_t a = a0 + ty * 4 + u, b = b0 + tx * 4 + v;
            if (a < K && b < K && b <= a) M[a * K + b] = acc[u][v];
        }
}

// M += db (every lower entry) ; diag += theta_t + reg
__global__ void k_mat_finish(double* __restrict__ M, int64_t K, double db, const double* __restrict__ th,
                             double reg) {
    const int64_t a = blockIdx.y;
    const int64_t b = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (a >= K || b > a) return;
    double v = M[a * K + b] + db;
    if (a == b) v += th[a] + reg;
    M[a * K + b] = v;
}

__global__ void k_get_diag(const double* __restrict__ M, int64_t K, double* __restrict__ out) {
    const int64_t a = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (a < K) out[a] = M[a * K + a];
}

constexpr int CH_B = 32;

// Cholesky of the diagonal block at j0 (size nb <= CH_B), in place (lower).
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ M, int64_t K, int64_t j0, int nb,
                                                   int* __restrict__ fail) {
    __shared__ double A[CH_B][CH_B + 1];
    for (int q = threadIdx.x; q < nb * nb; q += 256) {
        const int r = q / nb, c = q % nb;
        A[r][c] = (c <= r) ? M[(j0 + r) * K + j0 + c] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (threadIdx.x == 0) {
            const double v = A[j][j];
            if (!(v > 0.0)) *fail = 1;
            A[j][j] = sqrt(fmax(v, 1e-300));
        }
        __syncthreads();
        for (int r = j + 1 + threadIdx.x; r < nb; r += 256) A[r][j] /= A[j][j];
        __syncthreads();
        for (int q = threadIdx.x; q < nb * nb; q += 256) {
            const int r = q / nb, c = q % nb;
            if (r > j && c > j && c <= r) A[r][c] -= A[r][j] * A[c][j];
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < nb * nb; q += 256) {
        const int r = q / nb, c = q % nb;
        if (c <= r) M[(j0 + r) * K + j0 + c] = A[r][c];
    }
}

// Rows r >= j0 + nb: L[r, j0:j0+nb] = M[r, j0:j0+nb] L_jj^-T (one row per thread).
__global__ __launch_bounds__(256) void k_chol_trsm(double* __restrict__ M, int64_t K, int64_t j0, int nb) {
    __shared__ double L[CH_B][CH_B + 1];
    for (int q = threadIdx.x; q < nb * nb; q += 256) {
        const int r = q / nb, c = q % nb;
        L[r][c] = (c <= r) ? M[(j0 + r) * K + j0 + c] : 0.0;
    }
    __syncthreads();
    const int64_t r = j0 + nb + blockIdx.x * (int64_t)256 + threadIdx.x;
    if (r >= K) return;
    double x[CH_B];
    for (int c = 0; c < nb; ++c) {
        double v = M[r * K + j0 + c];
        for (int q = 0; q < c; ++q) v -= x[q] * L[c][q];
        x[c] = v / L[c][c];
    }
    for (int c = 0; c < nb; ++c) M[r * K + j0 + c] = x[c];
}

// Trailing update of the lower part: M[a][b] -= sum_q L[a][j0+q] L[b][j0+q]
// for a >= b >= j0 + nb, tiles of 64 x 64.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ M, int64_t K, int64_t j0, int nb) {
    __shared__ double As[CH_B][SY_T + 1];
    __shared__ double Bs[CH_B][SY_T + 1];
    const int64_t t = blockIdx.x;
    int64_t tr = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((tr + 1) * (tr + 2) / 2 <= t) ++tr;
    while (tr * (tr + 1) / 2 > t) --tr;
    const int64_t tc = t - tr * (tr + 1) / 2;
    const int64_t base = j0 + nb;
    const int64_t a0 = base + tr * SY_T, b0 = base + tc * SY_T;
    for (int q = threadIdx.x; q < SY_T * nb; q += 256) {
        const int r = q / nb, kk = q % nb;
        const int64_t a = a0 + r, b = b0 + r;
        As[kk][r] = (a < K) ? M[a * K + j0 + kk] : 0.0;
        Bs[kk][r] = (b < K) ? M[b * K + j0 + kk] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4] = {};
    for (int kk = 0; kk < nb; ++kk)
        for (int u = 0; u < 4; ++u)
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(As[kk][ty * 4 + u], Bs[kk][tx * 4 + v], acc[u][v]);
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            const int64_t a = a0 + ty * 4 + u, b = b0 + tx * 4 + v;
            if (a < K && b <= a) M[a * K + b] -= acc[u][v];
        }
}

// Solve L L^T x = r in place (one workgroup of 1024 threads): forward then
// backward substitution, blocks of 64 unknowns solved by one thread each
// step while the other threads update the remaining right-hand side.
__global__ __launch_bounds__(1024) void k_chol_solve(const double* __restrict__ L, int64_t K, double* __restrict__ x) {
    __shared__ double zb[64];
    // forward: L z = r
    for (int64_t j0 = 0; j0 < K; j0 += 64) {
        const int nb = (int)((K - j0) < 64 ? (K - j0) : 64);
        if (threadIdx.x == 0) {
            for (int c = 0; c < nb; ++c) {
                double v = x[j0 + c];
                for (int q = 0; q < c; ++q) v -= L[(j0 + c) * K + j0 + q] * zb[q];
                zb[c] = v / L[(j0 + c) * K + j0 + c];
                x[j0 + c] = zb[c];
            }
        }
        __syncthreads();
        for (int64_t r = j0 + nb + threadIdx.x; r < K; r += 1024) {
            double v = 0.0;
            for (int q = 0; q < nb; ++q) v += L[r * K + j0 + q] * zb[q];
            x[r] -= v;
        }
        __syncthreads();
    }
    // backward: L^T x = z
    for (int64_t j1 = K; j1 > 0; j1 -= 64) {
        const int64_t j0 = j1 >= 64 ? j1 - 64 : 0;
        const int nb = (int)(j1 - j0);
        if (threadIdx.x == 0) {
            for (int c = nb - 1; c >= 0; --c) {
                double v = x[j0 + c];
                for (int q = c + 1; q < nb; ++q) v -= L[(j0 + q) * K + j0 + c] * zb[q];
                zb[c] = v / L[(j0 + c) * K + j0 + c];
                x[j0 + c] = zb[c];
            }
        }
        __syncthreads();
        // rows above the block: x[r] -= sum_q L[j0+q][r] zb[q]
        for (int64_t r = threadIdx.x; r < j0; r += 1024) {
            double v = 0.0;
            for (int q = 0; q < nb; ++q) v += L[(j0 + q) * K + r] * zb[q];
            x[r] -= v;
        }
        __syncthreads();
    }
}

static inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + LP_TB - 1) / LP_TB); }

// ------------------------------------------------------------------ host
struct LpDev {
    hipStream_t st;
    int64_t K, N, chunks, rows_per;
    const float* E;
    double *vecK = nullptr, *vecN = nullptr, *outN = nullptr, *outK = nullptr, *part = nullptr, *M = nullptr;
    int* fail = nullptr;
    std::vector<void*> owned;
    template <class T>
    uvc_status alloc(T** p, size_t count, const char* what) {
        UVC_TRY(dalloc_n(p, std::max<size_t>(count, 1), what));
        owned.push_back(*p);
        return UVC_OK;
    }
    ~LpDev() {
        for (void* p : owned) (void)hipFree(p);
    }
    // out[i] = sum_k E[k,i] u[k]
    uvc_status Etu(const std::vector<double>& u, std::vector<double>& out) {
        UVC_HIP(hipMemcpyAsync(vecK, u.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_lp_Etu, dim3(nblk(N), (unsigned)chunks), dim3(LP_TB), 0, st, E, K, N, rows_per, vecK,
                           part);
        hipLaunchKernelGGL(k_lp_sum_parts, dim3(nblk(N)), dim3(LP_TB), 0, st, part, chunks, N, outN);
        out.resize((size_t)N);
        UVC_HIP(hipMemcpyAsync(out.data(), outN, (size_t)N * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        return UVC_OK;
    }
    // out[k] = sum_i E[k,i] v[i]
    uvc_status Ev(const std::vector<double>& v, std::vector<double>& out) {
        UVC_HIP(hipMemcpyAsync(vecN, v.data(), (size_t)N * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_lp_Ev, dim3((unsigned)K), dim3(LP_TB), 0, st, E, N, vecN, outK);
        out.resize((size_t)K);
        UVC_HIP(hipMemcpyAsync(out.data(), outK, (size_t)K * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        return UVC_OK;
    }
    // M = E diag(d) E^T + db + diag(th) + reg, then Cholesky in place
    uvc_status factor(const std::vector<double>& d, double db, const std::vector<double>& th, bool& ok) {
        UVC_HIP(hipMemcpyAsync(vecN, d.data(), (size_t)N * 8, hipMemcpyHostToDevice, st));
        UVC_HIP(hipMemcpyAsync(vecK, th.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
        const int64_t T = (K + SY_T - 1) / SY_T;
        hipLaunchKernelGGL(k_syrk, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, st, E, K, N, vecN, M);
        // regularisation relative to the largest diagonal entry
        double dmax = 0.0;
        for (double v : th) dmax = std::max(dmax, v);
        hipLaunchKernelGGL(k_mat_finish, dim3(nblk(K), (unsigned)K), dim3(LP_TB), 0, st, M, K, db, vecK, 0.0);
        // diagonal maximum of M for the regulariser
        std::vector<double> diag((size_t)K);
        hipLaunchKernelGGL(k_get_diag, dim3(nblk(K)), dim3(LP_TB), 0, st, M, K, outK);
        UVC_HIP(hipMemcpyAsync(diag.data(), outK, (size_t)K * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        for (double v : diag) dmax = std::max(dmax, v);
        std::vector<double> regv((size_t)K, 1e-13 * dmax);
        UVC_HIP(hipMemcpyAsync(vecK, regv.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_mat_finish, dim3(nblk(K), (unsigned)K), dim3(LP_TB), 0, st, M, K, 0.0, vecK, 0.0);
        UVC_HIP(hipMemsetAsync(fail, 0, 4, st));
        for (int64_t j0 = 0; j0 < K; j0 += CH_B) {
            const int nb = (int)std::min<int64_t>(CH_B, K - j0);
            hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, M, K, j0, nb, fail);
            const int64_t rest = K - j0 - nb;
            if (rest > 0) {
                hipLaunchKernelGGL(k_chol_trsm, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, st, M, K, j0, nb);
                const int64_t T2 = (rest + SY_T - 1) / SY_T;
                hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T2 * (T2 + 1) / 2)), dim3(256), 0, st, M, K, j0,
                                   nb);
            }
        }
        UVC_HIP(hipGetLastError());
        int f = 0;
        UVC_HIP(hipMemcpyAsync(&f, fail, 4, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        ok = (f == 0);
        return UVC_OK;
    }
    uvc_status solve(std::vector<double>& r) {
        UVC_HIP(hipMemcpyAsync(vecK, r.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(1024), 0, st, M, K, vecK);
        UVC_HIP(hipMemcpyAsync(r.data(), vecK, (size_t)K * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        return UVC_OK;
    }
};

static double norm2(const std::vector<double>& v) {
    double s = 0.0;
    for (double x : v) s += x * x;
    return std::sqrt(s);
}

static uvc_status solve_ipm(const float* E, int64_t K, int64_t N, const double* pen_dev, double mu, double tmax,
                            double tol, int32_t max_iter, double* t_out, double* s_out, uvc_lp_info* info,
                            hipStream_t st) {
    if ((double)K * (double)K * 8.0 > 64e9) return fail(UVC_EUNSUPPORTED, "K too large for the dense normal matrix");
    LpDev D;
    D.st = st;
    D.K = K;
    D.N = N;
    D.E = E;
    D.rows_per = std::max<int64_t>(64, (K + 15) / 16);
    D.chunks = (K + D.rows_per - 1) / D.rows_per;
    float *cmax_part = nullptr, *cmax = nullptr;
    double *sq_part = nullptr, *sq = nullptr;
    UVC_TRY(D.alloc(&cmax_part, (size_t)D.chunks * N, "lp colmax"));
    UVC_TRY(D.alloc(&cmax, N, "lp colmax"));
    UVC_TRY(D.alloc(&sq_part, (size_t)D.chunks * N, "lp norm"));
    UVC_TRY(D.alloc(&sq, N, "lp norm"));
    UVC_TRY(D.alloc(&D.vecK, K, "lp vec"));
    UVC_TRY(D.alloc(&D.vecN, N, "lp vec"));
    UVC_TRY(D.alloc(&D.outN, N, "lp vec"));
    UVC_TRY(D.alloc(&D.outK, K, "lp vec"));
    UVC_TRY(D.alloc(&D.part, (size_t)D.chunks * N, "lp partial sums"));
    UVC_TRY(D.alloc(&D.M, (size_t)K * K, "lp normal matrix"));
    UVC_TRY(D.alloc(&D.fail, 1, "lp flag"));

    hipLaunchKernelGGL(k_lp_colstats, dim3(nblk(N), (unsigned)D.chunks), dim3(LP_TB), 0, st, E, K, N, D.rows_per,
                       cmax_part, sq_part);
    hipLaunchKernelGGL(k_lp_max_parts, dim3(nblk(N)), dim3(LP_TB), 0, st, cmax_part, D.chunks, N, cmax);
    hipLaunchKernelGGL(k_lp_sum_parts, dim3(nblk(N)), dim3(LP_TB), 0, st, sq_part, D.chunks, N, sq);
    std::vector<float> hcmax((size_t)N);
    std::vector<double> hsq((size_t)N);
    UVC_HIP(hipMemcpyAsync(hcmax.data(), cmax, (size_t)N * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(hsq.data(), sq, (size_t)N * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    std::vector<unsigned char> vis((size_t)N);
    double fro2 = 0.0;
    int64_t nvis = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (!std::isfinite(hcmax[(size_t)i])) return fail(UVC_EINVAL, "E has a non-finite entry");
        vis[(size_t)i] = hcmax[(size_t)i] > 0.f;
        nvis += vis[(size_t)i];
        fro2 += hsq[(size_t)i];
    }
    std::vector<double> pen((size_t)N, 1.001 * std::sqrt(fro2));
    if (pen_dev) {
        UVC_HIP(hipMemcpyAsync(pen.data(), pen_dev, (size_t)N * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
    }
    std::vector<double> t((size_t)K, 0.0), sg((size_t)N, mu);
    double obj = 0.0, pres = 0.0, dres = 0.0, rgap = 0.0;
    int32_t it = 0;
    bool converged = nvis == 0;
    if (nvis > 0) {
        // variables over all N columns; invisible elements are held out (their
        // sigma is fixed at mu, their rows and columns carry no weight)
        const int64_t n = K + N, m = N + 1;
        std::vector<double> c((size_t)n, 0.0), h((size_t)m, 0.0);
        for (int64_t k = 0; k < K; ++k) c[(size_t)k] = 1.0;
        for (int64_t i = 0; i < N; ++i) {
            c[(size_t)(K + i)] = vis[(size_t)i] ? pen[(size_t)i] : 0.0;
            h[(size_t)i] = vis[(size_t)i] ? mu : 0.0;
        }
        h[(size_t)N] = -tmax;
        double cmaxv = 0.0;
        for (double v : c) cmaxv = std::max(cmaxv, std::fabs(v));
        const double sc0 = std::max(1.0, std::max(mu, std::sqrt(cmaxv)));
        std::vector<double> x((size_t)n, sc0), z((size_t)n, sc0), s((size_t)m, sc0), y((size_t)m, 1.0);
        for (int64_t i = 0; i < N; ++i)
            if (!vis[(size_t)i]) {
                x[(size_t)(K + i)] = 0.0;
                z[(size_t)(K + i)] = 0.0;
                s[(size_t)i] = 0.0;
                y[(size_t)i] = 0.0;
            }
        const double hn = norm2(h), cn = norm2(c);
        std::vector<double> Etmp, Evt;
        // G x = (E^T t + sigma, -sum t)
        auto Gx = [&](const std::vector<double>& xx, std::vector<double>& out) -> uvc_status {
            std::vector<double> tt(xx.begin(), xx.begin() + K);
            UVC_TRY(D.Etu(tt, Etmp));
            out.assign((size_t)m, 0.0);
            double st_ = 0.0;
            for (int64_t k = 0; k < K; ++k) st_ += tt[(size_t)k];
            for (int64_t i = 0; i < N; ++i) out[(size_t)i] = vis[(size_t)i] ? Etmp[(size_t)i] + xx[(size_t)(K + i)] : 0.0;
            out[(size_t)N] = -st_;
            return UVC_OK;
        };
        // G^T y = (E y_c - y_b, y_c)
        auto GTy = [&](const std::vector<double>& yy, std::vector<double>& out) -> uvc_status {
            std::vector<double> yc((size_t)N);
            for (int64_t i = 0; i < N; ++i) yc[(size_t)i] = vis[(size_t)i] ? yy[(size_t)i] : 0.0;
            UVC_TRY(D.Ev(yc, Evt));
            out.assign((size_t)n, 0.0);
            for (int64_t k = 0; k < K; ++k) out[(size_t)k] = Evt[(size_t)k] - yy[(size_t)N];
            for (int64_t i = 0; i < N; ++i) out[(size_t)(K + i)] = yc[(size_t)i];
            return UVC_OK;
        };
        std::vector<double> gx, gty, rp((size_t)m), rd((size_t)n);
        for (it = 0; it < max_iter; ++it) {
            UVC_TRY(Gx(x, gx));
            UVC_TRY(GTy(y, gty));
            double gap = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                rd[(size_t)j] = (j >= K && !vis[(size_t)(j - K)]) ? 0.0 : c[(size_t)j] - gty[(size_t)j] - z[(size_t)j];
                gap += x[(size_t)j] * z[(size_t)j];
            }
            for (int64_t i = 0; i < m; ++i) {
                rp[(size_t)i] = (i < N && !vis[(size_t)i]) ? 0.0 : h[(size_t)i] - gx[(size_t)i] + s[(size_t)i];
                gap += s[(size_t)i] * y[(size_t)i];
            }
            const double muc = gap / (double)(nvis * 2 + K + 1);
            double po = 0.0, dob = 0.0;
            for (int64_t j = 0; j < n; ++j) po += c[(size_t)j] * x[(size_t)j];
            for (int64_t i = 0; i < m; ++i) dob += h[(size_t)i] * y[(size_t)i];
            pres = norm2(rp) / (1.0 + hn);
            dres = norm2(rd) / (1.0 + cn);
            rgap = std::fabs(po - dob) / (1.0 + std::fabs(po) + std::fabs(dob));
            obj = po;
            if (std::max(pres, std::max(dres, rgap)) <= tol) {
                converged = true;
                break;
            }
            // normal matrix
            std::vector<double> Dr((size_t)m, 0.0), Th((size_t)n, 0.0), dt_((size_t)N, 0.0), tht((size_t)K);
            for (int64_t i = 0; i < m; ++i)
                if (!(i < N && !vis[(size_t)i])) Dr[(size_t)i] = y[(size_t)i] / s[(size_t)i];
            for (int64_t j = 0; j < n; ++j)
                if (!(j >= K && !vis[(size_t)(j - K)])) Th[(size_t)j] = z[(size_t)j] / x[(size_t)j];
            for (int64_t i = 0; i < N; ++i)
                if (vis[(size_t)i]) {
                    const double a = Dr[(size_t)i], b = Th[(size_t)(K + i)];
                    dt_[(size_t)i] = a * b / (a + b);
                }
            for (int64_t k = 0; k < K; ++k) tht[(size_t)k] = Th[(size_t)k];
            bool ok = true;
            UVC_TRY(D.factor(dt_, Dr[(size_t)N], tht, ok));
            if (!ok) break;
            // solve for a direction given complementarity right-hand sides
            auto direction = [&](const std::vector<double>& rxz, const std::vector<double>& rsy, std::vector<double>& dx,
                                 std::vector<double>& dy, std::vector<double>& dz,
                                 std::vector<double>& ds) -> uvc_status {
                std::vector<double> rpp((size_t)m), wv((size_t)m), rhs;
                for (int64_t i = 0; i < m; ++i) {
                    const bool live = !(i < N && !vis[(size_t)i]);
                    rpp[(size_t)i] = live ? rp[(size_t)i] + rsy[(size_t)i] / y[(size_t)i] : 0.0;
                    wv[(size_t)i] = Dr[(size_t)i] * rpp[(size_t)i];
                }
                UVC_TRY(GTy(wv, rhs));
                for (int64_t j = 0; j < n; ++j) {
                    const bool live = !(j >= K && !vis[(size_t)(j - K)]);
                    rhs[(size_t)j] = live ? rhs[(size_t)j] - rd[(size_t)j] + rxz[(size_t)j] / x[(size_t)j] : 0.0;
                }
                // eliminate sigma: rt2 = rt - E (Dc/(Dc+Ts) * rs)
                std::vector<double> q((size_t)N, 0.0), eq;
                for (int64_t i = 0; i < N; ++i)
                    if (vis[(size_t)i]) {
                        const double a = Dr[(size_t)i], b = Th[(size_t)(K + i)];
                        q[(size_t)i] = a / (a + b) * rhs[(size_t)(K + i)];
                    }
                UVC_TRY(D.Ev(q, eq));
                std::vector<double> dtv((size_t)K);
                for (int64_t k = 0; k < K; ++k) dtv[(size_t)k] = rhs[(size_t)k] - eq[(size_t)k];
                UVC_TRY(D.solve(dtv));
                std::vector<double> etd;
                UVC_TRY(D.Etu(dtv, etd));
                dx.assign((size_t)n, 0.0);
                for (int64_t k = 0; k < K; ++k) dx[(size_t)k] = dtv[(size_t)k];
                for (int64_t i = 0; i < N; ++i)
                    if (vis[(size_t)i]) {
                        const double a = Dr[(size_t)i], b = Th[(size_t)(K + i)];
                        dx[(size_t)(K + i)] = (rhs[(size_t)(K + i)] - a * etd[(size_t)i]) / (a + b);
                    }
                // G dx without another E^T pass: (E^T dt + dsigma, -sum dt)
                std::vector<double> gdx((size_t)m, 0.0);
                double sdt = 0.0;
                for (int64_t k = 0; k < K; ++k) sdt += dtv[(size_t)k];
                for (int64_t i = 0; i < N; ++i)
                    if (vis[(size_t)i]) gdx[(size_t)i] = etd[(size_t)i] + dx[(size_t)(K + i)];
                gdx[(size_t)N] = -sdt;
                dy.assign((size_t)m, 0.0);
                ds.assign((size_t)m, 0.0);
                for (int64_t i = 0; i < m; ++i)
                    if (!(i < N && !vis[(size_t)i])) {
                        dy[(size_t)i] = Dr[(size_t)i] * (rpp[(size_t)i] - gdx[(size_t)i]);
                        ds[(size_t)i] = (rsy[(size_t)i] - s[(size_t)i] * dy[(size_t)i]) / y[(size_t)i];
                    }
                // dz from dual feasibility (G^T dy + dz = rd), which keeps the
                // dual residual from drifting when the normal matrix is
                // ill-conditioned near the optimum
                std::vector<double> gtdy;
                UVC_TRY(GTy(dy, gtdy));
                dz.assign((size_t)n, 0.0);
                for (int64_t j = 0; j < n; ++j)
                    if (!(j >= K && !vis[(size_t)(j - K)])) dz[(size_t)j] = rd[(size_t)j] - gtdy[(size_t)j];
                return UVC_OK;
            };
            auto maxstep = [](const std::vector<double>& v, const std::vector<double>& dv) {
                double a = 1.0;
                for (size_t j = 0; j < v.size(); ++j)
                    if (dv[j] < 0.0 && v[j] > 0.0) a = std::min(a, -v[j] / dv[j]);
                return a;
            };
            std::vector<double> rxz((size_t)n), rsy((size_t)m), dx, dy, dz, ds;
            for (int64_t j = 0; j < n; ++j) rxz[(size_t)j] = -x[(size_t)j] * z[(size_t)j];
            for (int64_t i = 0; i < m; ++i) rsy[(size_t)i] = -s[(size_t)i] * y[(size_t)i];
            UVC_TRY(direction(rxz, rsy, dx, dy, dz, ds));
            double ap = std::min(maxstep(x, dx), maxstep(s, ds)), ad = std::min(maxstep(z, dz), maxstep(y, dy));
            double gaff = 0.0;
            for (int64_t j = 0; j < n; ++j) gaff += (x[(size_t)j] + ap * dx[(size_t)j]) * (z[(size_t)j] + ad * dz[(size_t)j]);
            for (int64_t i = 0; i < m; ++i) gaff += (s[(size_t)i] + ap * ds[(size_t)i]) * (y[(size_t)i] + ad * dy[(size_t)i]);
            const double sig = std::pow(gaff / std::max(gap, 1e-300), 3.0);
            for (int64_t j = 0; j < n; ++j) {
                const bool live = !(j >= K && !vis[(size_t)(j - K)]);
                rxz[(size_t)j] = live ? sig * muc - x[(size_t)j] * z[(size_t)j] - dx[(size_t)j] * dz[(size_t)j] : 0.0;
            }
            for (int64_t i = 0; i < m; ++i) {
                const bool live = !(i < N && !vis[(size_t)i]);
                rsy[(size_t)i] = live ? sig * muc - s[(size_t)i] * y[(size_t)i] - ds[(size_t)i] * dy[(size_t)i] : 0.0;
            }
            UVC_TRY(direction(rxz, rsy, dx, dy, dz, ds));
            ap = 0.99 * std::min(maxstep(x, dx), maxstep(s, ds));
            ad = 0.99 * std::min(maxstep(z, dz), maxstep(y, dy));
            for (int64_t j = 0; j < n; ++j) {
                x[(size_t)j] += ap * dx[(size_t)j];
                z[(size_t)j] += ad * dz[(size_t)j];
            }
            for (int64_t i = 0; i < m; ++i) {
                s[(size_t)i] += ap * ds[(size_t)i];
                y[(size_t)i] += ad * dy[(size_t)i];
            }
        }
        obj = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            t[(size_t)k] = std::max(0.0, x[(size_t)k]);
            obj += t[(size_t)k];
        }
        for (int64_t i = 0; i < N; ++i)
            if (vis[(size_t)i]) {
                sg[(size_t)i] = std::max(0.0, x[(size_t)(K + i)]);
                obj += pen[(size_t)i] * sg[(size_t)i];
            }
    }
    if (t_out) UVC_HIP(hipMemcpyAsync(t_out, t.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
    if (s_out) UVC_HIP(hipMemcpyAsync(s_out, sg.data(), (size_t)N * 8, hipMemcpyHostToDevice, st));
    UVC_HIP(hipStreamSynchronize(st));
    if (info) {
        info->objective = obj;
        info->primal_residual = pres;
        info->dual_residual = dres;
        info->gap = rgap;
        info->iterations = it;
        info->n_visible = nvis;
        info->penalty = pen.empty() ? 0.0 : pen[0];
    }
    if (!converged)
        return fail(UVC_ENOTCONV, "LP did not reach tol; residuals " + std::to_string(pres) + " " +
                                      std::to_string(dres) + " " + std::to_string(rgap));
    return UVC_OK;
}

}  // namespace uvc

using namespace uvc;

extern "C" uvc_status uvc_solve_dosage_lp(const float* E_dev, int64_t K, int64_t N, const double* penalty_dev,
                                          double mu_min, double t_max, double tol, int32_t max_iter,
                                          double* t_out_dev, double* sigma_out_dev, uvc_lp_info* info,
                                          void* hip_stream) {
    if (info) *info = uvc_lp_info{};
    if (K < 0 || N < 0) return fail(UVC_EINVAL, "negative LP size");
    if (!(mu_min > 0) || !(t_max > 0) || !(tol > 0) || max_iter <= 0)
        return fail(UVC_EINVAL, "mu_min, t_max, tol and max_iter must be positive");
    if (K == 0 || N == 0) return fail(UVC_EINVAL, "empty LP");
    if (!E_dev) return fail(UVC_EINVAL, "E is NULL");
    try {
        return solve_ipm(E_dev, K, N, penalty_dev, mu_min, t_max, tol, max_iter, t_out_dev, sigma_out_dev, info,
                         (hipStream_t)hip_stream);
    } catch (const std::exception& e) {
        return fail(UVC_ENOMEM, std::string("host exception: ") + e.what());
    }
}
