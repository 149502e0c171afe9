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
// reuse the factor.  The iterate and all O(K + N) vector algebra stay on the
// device in FP64; per iteration the host reads back a few reduced scalars
// (residual norms, step lengths, the affine complementarity gap).
// Every device reduction sums in a fixed order: results are deterministic.
#include "uvc_common.hpp"

#include <chrono>
#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <cfloat>
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
            // NaN and Inf both record Inf (fmaxf would drop a NaN), which the
            // host reports as a non-finite entry
            mx = (fabsf(v) <= FLT_MAX) ? fmaxf(mx, fabsf(v)) : INFINITY;
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
// Both products below take the occupancy map of E (64 rows x 256 columns
// per block, see k_occ; occ = nullptr: none) and skip the all-zero blocks.
// A skipped term is E[k,i] * x = +-0 added to a sum that starts at +0 and
// never is -0, so the results are the same bits as without the map.
constexpr int OCC_R = 64, OCC_C = 256;
static_assert(OCC_C == LP_TB, "a workgroup of k_lp_Etu covers one occupancy block of columns");

__global__ void k_lp_Etu(const float* __restrict__ E, int64_t K, int64_t N, int64_t rows_per,
                         const double* __restrict__ u, double* __restrict__ part,
                         const unsigned char* __restrict__ occ, int64_t nc) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    const int64_t k0 = blockIdx.y * rows_per, k1 = std::min<int64_t>(K, k0 + rows_per);
    double acc = 0.0;
    if (i < N)
        for (int64_t k = k0; k < k1;) {
            const int64_t t = k / OCC_R, kend = std::min<int64_t>(k1, (t + 1) * OCC_R);
            if (occ && !occ[t * nc + blockIdx.x]) {
                k = kend;
                continue;
            }
            for (; k < kend; ++k) acc += (double)E[k * N + i] * u[k];
        }
    if (i < N) part[blockIdx.y * N + i] = acc;
}

// out[k] = sum_i E[k,i] * v[i]  (E v, row dot products; one block per row,
// fixed-order tree reduction)
__global__ void k_lp_Ev(const float* __restrict__ E, int64_t N, const double* __restrict__ v,
                        double* __restrict__ out, double scale, const unsigned char* __restrict__ occ, int64_t nc) {
    __shared__ double red[LP_TB];
    const int64_t k = blockIdx.x;
    double acc = 0.0;
    const float* row = E + k * N;
    const unsigned char* orow = occ ? occ + (k / OCC_R) * nc : nullptr;
    // 64 blocks' flags per ballot (one per lane, the same in every wave),
    // then the set blocks in ascending order: no load waits on a flag
    const int lane = threadIdx.x & 63;
    const int64_t nb = (N + OCC_C - 1) / OCC_C;
    for (int64_t jb = 0; jb < nb; jb += 64) {
        unsigned long long m = __ballot(jb + lane < nb && (!orow || orow[jb + lane]));
        while (m) {
            const int b = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int64_t i = (jb + b) * OCC_C + threadIdx.x;
            if (i < N) acc += (double)row[i] * v[i];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = LP_TB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0] * scale;
}

// out[i] = scale * sum over chunks of part[chunk][i] (fixed order)
__global__ void k_lp_sum_parts(const double* __restrict__ part, int64_t chunks, int64_t N, double* __restrict__ out,
                               double scale) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    double a = 0.0;
    for (int64_t c = 0; c < chunks; ++c) a += part[c * N + i];
    out[i] = a * scale;
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
constexpr int SY_KC = 32;  // inner chunk (columns of E per LDS stage)
constexpr int SY_OC = 256; // occupancy block: 64 rows x 256 columns of E
static_assert(SY_T == OCC_R && SY_OC == OCC_C, "one occupancy map serves the products and the normal matrix");

// occ[r * nc + c] = 1 iff E has a nonzero in rows [64 r, 64 r + 64) and
// columns [256 c, 256 c + 256); one workgroup per block, thread q on column q.
__global__ __launch_bounds__(256) void k_occ(const float* __restrict__ E, int64_t K, int64_t N, int64_t nc,
                                             unsigned char* __restrict__ occ) {
    const int64_t c = blockIdx.x, r = blockIdx.y;
    const int64_t i = c * SY_OC + threadIdx.x;
    int nz = 0;
    if (i < N)
        for (int64_t a = r * SY_T; a < std::min<int64_t>(K, r * SY_T + SY_T); ++a) nz |= E[a * N + i] != 0.0f;
    nz = __syncthreads_or(nz);
    if (threadIdx.x == 0) occ[r * nc + c] = nz ? 1 : 0;
}

// M[a][b] = sum_i E[a,i] d[i] E[b,i] for the lower tiles (tile row >= tile
// col) of the K x K row-major M, on the FP64 matrix cores.  A workgroup of
// four waves owns a 64 x 64 tile; wave w computes the 32 x 32 block
// (rows 32 (w / 2), cols 32 (w % 2)) as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64.  Per chunk of SY_KC columns of E, the two 64-row
// panels are staged in LDS in FP64 (the row panel scaled by d).  Operand
// layout of the instruction: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k; result D[i][j] in lane j + 16 (i % 4), element i / 4.
// With splits > 1, workgroup (tile, s) covers columns [s N / splits,
// (s + 1) N / splits) and writes the partial product to M + s K^2.
// With occ (k_occ's map, nc blocks per row tile), a 256-column block where
// either tile's rows of E are all zero is skipped: its products are exact
// zeros (E >= 0, d >= 0), so M is the same bit for bit, and a sparse E (poses
// that see only their own rooms) costs only the blocks both tiles touch.
typedef double dbl4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_syrk(const float* __restrict__ E, int64_t K, int64_t N,
                                              const double* __restrict__ d, double* __restrict__ M, int splits,
                                              const unsigned char* __restrict__ occ, int64_t nc) {
    __shared__ double As[SY_KC][SY_T + 1];
    __shared__ double Bs[SY_KC][SY_T + 1];
    // lower-triangular tile index -> (tr, tc)
    const int64_t t = blockIdx.x;
    int64_t tr = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((tr + 1) * (tr + 2) / 2 <= t) ++tr;
    while (tr * (tr + 1) / 2 > t) --tr;
    const int64_t tc = t - tr * (tr + 1) / 2;
    const int64_t a0 = tr * SY_T, b0 = tc * SY_T;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    dbl4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const int64_t per = ((N + splits - 1) / splits + SY_KC - 1) / SY_KC * SY_KC;
    const int64_t ib = (int64_t)blockIdx.y * per, ie = std::min<int64_t>(N, ib + per);
    double* Mo = M + (int64_t)blockIdx.y * K * K;
    // staging: thread q loads column kk = q % SY_KC of rows q / SY_KC + (256 / SY_KC) u
    constexpr int SU = SY_T * SY_KC / 256;
    const int sr = threadIdx.x / SY_KC, skk = threadIdx.x % SY_KC;
    // the next chunk's loads are issued before the current chunk's matrix
    // operations, so that their latency is covered
    float ea[SU], eb[SU];
    double di = 0.0;
    // out-of-range rows and columns load a clamped in-range address and are
    // zeroed by a select (no branches around the loads)
    auto fetch = [&](int64_t i0) {
        const int64_t i = i0 + skk;
        const bool iok = i < ie;
        const int64_t ic = iok ? i : ie - 1;
        di = d[ic];
        di = iok ? di : 0.0;
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int64_t a = a0 + sr + (256 / SY_KC) * u, b = b0 + sr + (256 / SY_KC) * u;
            const float va = E[(a < K ? a : K - 1) * N + ic], vb = E[(b < K ? b : K - 1) * N + ic];
            ea[u] = a < K ? va : 0.0f;
            eb[u] = (iok && b < K) ? vb : 0.0f;
        }
    };
    // first column >= i of a block both tiles touch (ie if none); the chunks
    // of SY_KC columns stay aligned, since ib and SY_OC are multiples of SY_KC
    auto next_active = [&](int64_t i) -> int64_t {
        if (occ)
            while (i < ie && !(occ[tr * nc + i / SY_OC] && occ[tc * nc + i / SY_OC])) i = (i / SY_OC + 1) * SY_OC;
        return std::min(i, ie);
    };
    int64_t i0 = next_active(ib);
    if (i0 < ie) fetch(i0);
    while (i0 < ie) {
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            As[skk][sr + (256 / SY_KC) * u] = (double)ea[u] * di;
            Bs[skk][sr + (256 / SY_KC) * u] = (double)eb[u];
        }
        __syncthreads();
        // the map is consulted only where a new 256-column block starts
        const int64_t i1 = ((i0 + SY_KC) % SY_OC) ? std::min(i0 + SY_KC, ie) : next_active(i0 + SY_KC);
        if (i1 < ie) fetch(i1);
#pragma unroll
        for (int ks = 0; ks < SY_KC / 4; ++ks) {
            const int kk = 4 * ks + lk;
            const double fa0 = As[kk][wr + li], fa1 = As[kk][wr + 16 + li];
            const double fb0 = Bs[kk][wc + li], fb1 = Bs[kk][wc + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa0, fb0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa0, fb1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa1, fb0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa1, fb1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
        i0 = i1;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t a = a0 + wr + 16 * m + 4 * e + lk, b = b0 + wc + 16 * n + li;
                if (a < K && b < K && b <= a) Mo[a * K + b] = acc[m][n][e];
            }
}

// M = ms M + db (every lower entry) ; diag += theta_t + reg
__global__ void k_mat_finish(double* __restrict__ M, int64_t K, double ms, double db, const double* __restrict__ th,
                             double reg) {
    const int64_t a = blockIdx.y;
    const int64_t b = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (a >= K || b > a) return;
    double v = ms * M[a * K + b] + db;
    if (a == b) v += th[a] + reg;
    M[a * K + b] = v;
}

__global__ void k_get_diag(const double* __restrict__ M, int64_t K, double* __restrict__ out) {
    const int64_t a = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (a < K) out[a] = M[a * K + a];
}

constexpr int CH_B = 32;
constexpr int LP_CENTRALITY = 2;  // centrality correctors tried per iteration

// Cholesky of the diagonal block at j0 (size nb <= CH_B), in place (lower).
// Right-looking on the unscaled block: step j subtracts
// A[r][j] A[c][j] / A[j][j] from every entry below and right of the pivot
// (one barrier per step); afterwards column j is scaled by 1 / sqrt(A[j][j]),
// which gives L with L[j][j] = sqrt(A[j][j]).
__device__ __forceinline__ void chol_diag_block(double* __restrict__ M, int64_t K, int64_t j0, int nb,
                                                int* __restrict__ fail, double (*A)[CH_B + 1]) {
    for (int q = threadIdx.x; q < nb * nb; q += 256) {
        const int r = q / nb, c = q % nb;
        A[r][c] = (c <= r) ? M[(j0 + r) * K + j0 + c] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const double piv = A[j][j];
        if (!(piv > 0.0)) {
            if (threadIdx.x == 0) *fail = 1;
        }
        const double inv = 1.0 / fmax(piv, 1e-300);
        const int w = nb - 1 - j;  // trailing block size
        for (int q = threadIdx.x; q < w * w; q += 256) {
            const int r = j + 1 + q / w, c = j + 1 + q % w;
            if (c <= r) A[r][c] -= A[r][j] * A[c][j] * inv;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < nb * nb; q += 256) {
        const int r = q / nb, c = q % nb;
        if (c <= r) M[(j0 + r) * K + j0 + c] = A[r][c] / sqrt(fmax(A[c][c], 1e-300));
    }
}

__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ M, int64_t K, int64_t j0, int nb,
                                                   int* __restrict__ fail) {
    __shared__ double A[CH_B][CH_B + 1];
    chol_diag_block(M, K, j0, nb, fail, A);
}

// Rows r >= j0 + nb: L[r, j0:j0+nb] = M[r, j0:j0+nb] L_jj^-T (one row per
// thread).  The diagonal block sits in LDS; each thread keeps its row's
// unknowns in its own LDS column (conflict-free), so nothing spills.
__global__ __launch_bounds__(256) void k_chol_trsm(double* __restrict__ M, int64_t K, int64_t j0, int nb) {
    __shared__ double L[CH_B][CH_B + 1];
    __shared__ double inv[CH_B];
    __shared__ double X[CH_B][256];
    for (int q = threadIdx.x; q < nb * nb; q += 256) {
        const int r = q / nb, c = q % nb;
        L[r][c] = (c <= r) ? M[(j0 + r) * K + j0 + c] : 0.0;
    }
    __syncthreads();
    if ((int)threadIdx.x < nb) inv[threadIdx.x] = 1.0 / L[threadIdx.x][threadIdx.x];
    __syncthreads();
    const int64_t r = j0 + nb + blockIdx.x * (int64_t)256 + threadIdx.x;
    if (r >= K) return;
    const int t = threadIdx.x;
    for (int c = 0; c < nb; ++c) X[c][t] = M[r * K + j0 + c];
    for (int c = 0; c < nb; ++c) {
        double v = X[c][t];
        for (int q = 0; q < c; ++q) v -= X[q][t] * L[c][q];
        X[c][t] = v * inv[c];
    }
    for (int c = 0; c < nb; ++c) M[r * K + j0 + c] = X[c][t];
}

// Trailing update of the lower part: M[a][b] -= sum_q L[a][j0+q] L[b][j0+q]
// for a >= b >= j0 + nb, tiles of 64 x 64.  The workgroup of the first tile,
// which holds the whole next diagonal block (size next_nb <= CH_B), then
// factors that block, so the next panel needs no separate launch for it.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ M, int64_t K, int64_t j0, int nb,
                                                     int next_nb, int* __restrict__ fail) {
    __shared__ double As[CH_B][SY_T + 1];
    __shared__ double Bs[CH_B][SY_T + 1];
    __shared__ double Ad[CH_B][CH_B + 1];
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
    if (t == 0 && next_nb > 0) {
        __syncthreads();
        chol_diag_block(M, K, base, next_nb, fail, Ad);
    }
}

// Lane c's value of v for the whole wave (c uniform): two v_readlane.
__device__ __forceinline__ double lane_bcast(double v, int c) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, c);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), c);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Blocked triangular solves spread over the chip, one launch per 64-row
// block.  Forward (L z = r): launch j0 applies the solved block jp = j0 - 64
// to every row below it (workgroup 0 to the rows of block j0, the others to
// the rows from j0 + 64 on, 64 rows each) and workgroup 0 then solves the
// diagonal block j0 (one wave, lane r holding unknown r).  Backward (L^T x
// = z): launch j0 applies the solved block jq = j0 + 64 to every unknown
// before it (workgroup 0 to those of block j0, the others to 256 unknowns
// each below j0) and workgroup 0 then solves the transposed block j0.  Only
// workgroup 0 writes the unknowns of block j0, and the next launch reads
// them, so no launch depends on another workgroup of itself.
constexpr int TS_B = 64;      // block size
constexpr int TS_ROWS = 64;   // rows per workgroup in the forward update
constexpr int TS_COLS = 256;  // unknowns per workgroup in the backward update

// x[r] -= sum_c L[r][jp + c] z[c] for rows r in [r0, r1): 16 lanes per row
// (4 columns each), 16 rows per pass of 256 threads, the loads of four passes
// issued together.
__device__ __forceinline__ void ts_fwd_rows(const double* __restrict__ L, int64_t K, double* __restrict__ x,
                                            int64_t jp, int nbp, const double* zb, int64_t r0, int64_t r1) {
    const int tid = threadIdx.x, rg = tid >> 4, l16 = tid & 15;
    const int c0 = l16 < nbp ? l16 : 0, c1 = l16 + 16 < nbp ? l16 + 16 : 0;
    const int c2 = l16 + 32 < nbp ? l16 + 32 : 0, c3 = l16 + 48 < nbp ? l16 + 48 : 0;
    const double z0 = l16 < nbp ? zb[l16] : 0.0, z1 = l16 + 16 < nbp ? zb[l16 + 16] : 0.0;
    const double z2 = l16 + 32 < nbp ? zb[l16 + 32] : 0.0, z3 = l16 + 48 < nbp ? zb[l16 + 48] : 0.0;
    for (int64_t rb = r0 + rg; rb < r1; rb += 64) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t r = rb + 16 * u;
            v[u] = 0.0;
            if (r < r1) {
                const double* row = L + r * K + jp;
                v[u] = row[c0] * z0 + row[c1] * z1 + row[c2] * z2 + row[c3] * z3;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            for (int o = 8; o > 0; o >>= 1) v[u] += __shfl_xor(v[u], o, 16);
            const int64_t r = rb + 16 * u;
            if (l16 == 0 && r < r1) x[r] -= v[u];
        }
    }
}

// x[c] -= sum_q L[jq + q][c] z[q] for unknowns c in [c0, c1): thread per
// unknown (coalesced across threads), 32 loads issued together.
__device__ __forceinline__ void ts_bwd_cols(const double* __restrict__ L, int64_t K, double* __restrict__ x,
                                            int64_t jq, int nbq, const double* zb, int64_t c0, int64_t c1) {
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int q = 0;
        for (; q + 32 <= nbq; q += 32) {
            double l[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) l[u] = L[(jq + q + u) * K + c];
#pragma unroll
            for (int u = 0; u < 32; ++u) a[u & 7] += l[u] * zb[q + u];
        }
        for (; q < nbq; ++q) a[0] += L[(jq + q) * K + c] * zb[q];
        x[c] -= ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
}

// Diagonal block at j0 (size nb), in place on x[j0 .. j0 + nb): forward
// (lower) or backward (transposed).  All threads stage; wave 0 solves.
__device__ __forceinline__ void ts_diag(const double* __restrict__ L, int64_t K, double* __restrict__ x, int64_t j0,
                                        int nb, bool transposed, double (*Lb)[TS_B + 1], double* zb, double* rd) {
    const int tid = threadIdx.x;
    for (int q = tid; q < TS_B * TS_B; q += blockDim.x) {
        const int r = q / TS_B, c = q % TS_B;
        Lb[r][c] = (r < nb && c <= r) ? L[(j0 + r) * K + j0 + c] : 0.0;
    }
    if (tid < nb) {
        zb[tid] = x[j0 + tid];
        rd[tid] = 1.0 / L[(j0 + tid) * K + j0 + tid];
    }
    __syncthreads();
    if (tid < 64) {
        double v = tid < nb ? zb[tid] : 0.0;
        if (!transposed) {
            for (int c = 0; c < nb; ++c) {
                const double zc = lane_bcast(v, c) * rd[c];
                if (tid == c)
                    v = zc;
                else if (tid > c && tid < nb)
                    v -= Lb[tid][c] * zc;
            }
        } else {
            for (int c = nb - 1; c >= 0; --c) {
                const double zc = lane_bcast(v, c) * rd[c];
                if (tid == c)
                    v = zc;
                else if (tid < c)
                    v -= Lb[c][tid] * zc;
            }
        }
        if (tid < nb) x[j0 + tid] = v;
    }
}

__global__ __launch_bounds__(256) void k_ts_fwd(const double* __restrict__ L, int64_t K, double* __restrict__ x,
                                                int64_t j0) {
    __shared__ double Lb[TS_B][TS_B + 1];
    __shared__ double zb[TS_B], rd[TS_B];
    const int nb = (int)std::min<int64_t>(TS_B, K - j0);
    const int64_t jp = j0 - TS_B;
    if (jp >= 0) {
        if (threadIdx.x < TS_B) zb[threadIdx.x] = x[jp + threadIdx.x];
        __syncthreads();
        if (blockIdx.x == 0) {
            ts_fwd_rows(L, K, x, jp, TS_B, zb, j0, j0 + nb);
        } else {
            const int64_t r0 = j0 + TS_B + (int64_t)(blockIdx.x - 1) * TS_ROWS;
            ts_fwd_rows(L, K, x, jp, TS_B, zb, r0, std::min<int64_t>(K, r0 + TS_ROWS));
        }
        __syncthreads();
    }
    if (blockIdx.x == 0) ts_diag(L, K, x, j0, nb, false, Lb, zb, rd);
}

__global__ __launch_bounds__(256) void k_ts_bwd(const double* __restrict__ L, int64_t K, double* __restrict__ x,
                                                int64_t j0) {
    __shared__ double Lb[TS_B][TS_B + 1];
    __shared__ double zb[TS_B], rd[TS_B];
    const int nb = (int)std::min<int64_t>(TS_B, K - j0);
    const int64_t jq = j0 + TS_B;
    if (jq < K) {
        const int nbq = (int)std::min<int64_t>(TS_B, K - jq);
        if (threadIdx.x < nbq) zb[threadIdx.x] = x[jq + threadIdx.x];
        __syncthreads();
        if (blockIdx.x == 0) {
            ts_bwd_cols(L, K, x, jq, nbq, zb, j0, j0 + nb);
        } else {
            const int64_t c0 = (int64_t)(blockIdx.x - 1) * TS_COLS;
            ts_bwd_cols(L, K, x, jq, nbq, zb, c0, std::min<int64_t>(j0, c0 + TS_COLS));
        }
        __syncthreads();
    }
    if (blockIdx.x == 0) ts_diag(L, K, x, j0, nb, true, Lb, zb, rd);
}

static inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + LP_TB - 1) / LP_TB); }

// L L^T x = r in place (L in the lower part of M): one launch per block and sweep.
static void tri_solve(const double* M, int64_t K, double* x, hipStream_t st) {
    for (int64_t j0 = 0; j0 < K; j0 += TS_B) {
        const int64_t below = std::max<int64_t>(0, K - (j0 + TS_B));
        const unsigned g = 1u + (unsigned)((below + TS_ROWS - 1) / TS_ROWS);
        hipLaunchKernelGGL(k_ts_fwd, dim3(j0 == 0 ? 1u : g), dim3(256), 0, st, M, K, x, j0);
    }
    const int64_t last = ((K - 1) / TS_B) * TS_B;
    for (int64_t j0 = last; j0 >= 0; j0 -= TS_B) {
        const unsigned g = 1u + (unsigned)((j0 + TS_COLS - 1) / TS_COLS);
        hipLaunchKernelGGL(k_ts_bwd, dim3(j0 == last ? 1u : g), dim3(256), 0, st, M, K, x, j0);
    }
}

// -------------------------------------------------- interior point kernels
// Iterate (device, FP64): x = (t[K], sigma[N]), z = (zt[K], zs[N]),
// s = (sc[N], s_b), y = (yc[N], y_b).  Hidden (invisible) elements keep
// every entry at zero.  The budget-row scalars s_b, y_b live on the host;
// the direction's budget components dy_b, ds_b are formed on the device
// (k_ipm_bscal) so that no direction needs a host round trip.
struct IpmPtr {
    // K
    double *xt, *zt, *rdt, *tht, *mvK, *mvK2;
    double *dt[2], *dzt[2];
    // N
    double *xs, *zs, *yc, *sc, *pen, *rpc, *rds, *drc, *ths, *dtil, *rhs, *rpp, *mvN, *u;
    double *dsig[2], *dzs[2], *dyc[2], *dsc[2];
    const unsigned char* vis;
    double* S;  // device scalars, see S_* below
};
enum { S_SUMDT0 = 0, S_DYB0 = 1, S_DSB0 = 2, S_SUMDT1 = 3, S_DYB1 = 4, S_DSB1 = 5, S_REG = 6, S_RED = 8 };
constexpr int IPM_SUMS = 8;

// Residuals: rpc = mu - (E^T t + sigma) + sc, rds = p - yc - zs (visible i);
// rdt = 1 - (E yc - y_b) - zt.
__global__ void k_ipm_resid_N(IpmPtr P, int64_t N, double mu) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    if (P.vis[i]) {
        P.rpc[i] = mu - (P.mvN[i] + P.xs[i]) + P.sc[i];
        P.rds[i] = P.pen[i] - P.yc[i] - P.zs[i];
    } else {
        P.rpc[i] = 0.0;
        P.rds[i] = 0.0;
    }
}
__global__ void k_ipm_resid_K(IpmPtr P, int64_t K, double yb) {
    const int64_t k = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (k < K) P.rdt[k] = 1.0 - (P.mvK[k] - yb) - P.zt[k];
}

// Scalings: drc = yc / sc, ths = zs / sigma, dtil = drc ths / (drc + ths),
// tht = zt / t.
__global__ void k_ipm_scale(IpmPtr P, int64_t K, int64_t N) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i < N) {
        if (P.vis[i]) {
            const double a = P.yc[i] / P.sc[i], b = P.zs[i] / P.xs[i];
            P.drc[i] = a;
            P.ths[i] = b;
            P.dtil[i] = a * b / (a + b);
        } else {
            P.drc[i] = 0.0;
            P.ths[i] = 0.0;
            P.dtil[i] = 0.0;
        }
    }
    if (i < K) P.tht[i] = P.zt[i] / P.xt[i];
}

// Right-hand side of one Newton solve.  Complementarity part: predictor
// (mode 0) -x z; corrector (mode 1) sigmu - x z - dx dz with the predictor
// in slot cd; centrality corrector (mode 2, Gondzio 1996) the move of the
// trial product v = (x + atp dx)(z + atd dz) of the direction in slot cd
// into [0.1, 10] sigmu (no move below -10 sigmu).  The residuals enter
// with weight res (1, or 0 for a centrality corrector).
struct RhsArgs {
    int mode;
    int cd;
    double sigmu;
    double atp, atd;
    double res;
};
__device__ __forceinline__ double centrality(double v, double tgt) {
    const double r = fmin(fmax(v, 0.1 * tgt), 10.0 * tgt) - v;
    return fmax(r, -10.0 * tgt);
}
__device__ __forceinline__ double comp_rhs(double x, double z, double dx, double dz, const RhsArgs& A) {
    if (A.mode == 0) return -x * z;
    if (A.mode == 1) return A.sigmu - x * z - dx * dz;
    return centrality((x + A.atp * dx) * (z + A.atd * dz), A.sigmu);
}
__device__ __forceinline__ double rsy_of(const IpmPtr& P, int64_t i, const RhsArgs& A) {
    return comp_rhs(P.sc[i], P.yc[i], P.dsc[A.cd][i], P.dyc[A.cd][i], A);
}
__device__ __forceinline__ double rxzs_of(const IpmPtr& P, int64_t i, const RhsArgs& A) {
    return comp_rhs(P.xs[i], P.zs[i], P.dsig[A.cd][i], P.dzs[A.cd][i], A);
}

// Direction, part a (elements): rpp = rpc + rsy / yc, wv = drc rpp,
// rhs = wv - rds + rxz / sigma, q = drc / (drc + ths) rhs, u = wv - q.
__global__ void k_dir_a(IpmPtr P, int64_t N, RhsArgs A) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    if (!P.vis[i]) {
        P.rpp[i] = 0.0;
        P.rhs[i] = 0.0;
        P.u[i] = 0.0;
        return;
    }
    const double rpp = A.res * P.rpc[i] + rsy_of(P, i, A) / P.yc[i];
    const double wv = P.drc[i] * rpp;
    const double rhs = wv - A.res * P.rds[i] + rxzs_of(P, i, A) / P.xs[i];
    const double q = P.drc[i] / (P.drc[i] + P.ths[i]) * rhs;
    P.rpp[i] = rpp;
    P.rhs[i] = rhs;
    P.u[i] = wv - q;
}

// Part b (poses): dt = E u - wv_b - rdt + rxz_t / t  (then solved with M).
__global__ void k_dir_b(IpmPtr P, int64_t K, RhsArgs A, double wvb, int d) {
    const int64_t k = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (k >= K) return;
    const double rxz = comp_rhs(P.xt[k], P.zt[k], P.dt[A.cd][k], P.dzt[A.cd][k], A);
    P.dt[d][k] = P.mvK[k] - wvb - A.res * P.rdt[k] + rxz / P.xt[k];
}

// Budget-row components: gdx_b = -sum dt, dy_b = D_b (rpp_b - gdx_b),
// ds_b = (rsy_b - s_b dy_b) / y_b.  One workgroup; fixed-order sum.
__global__ __launch_bounds__(LP_TB) void k_ipm_bscal(IpmPtr P, int64_t K, int d, double Db, double rppb,
                                                     double rsyb, double sb, double yb) {
    __shared__ double red[LP_TB];
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < K; k += LP_TB) a += P.dt[d][k];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = LP_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sdt = red[0];
        const double dyb = Db * (rppb + sdt);
        const double dsb = (rsyb - sb * dyb) / yb;
        P.S[3 * d + 0] = sdt;
        P.S[3 * d + 1] = dyb;
        P.S[3 * d + 2] = dsb;
    }
}

// Part c (elements), with etd = E^T dt in mvN: dsigma, dy_c, ds_c, dz_s.
__global__ void k_dir_c(IpmPtr P, int64_t N, RhsArgs A, int d) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N) return;
    if (!P.vis[i]) {
        P.dsig[d][i] = 0.0;
        P.dyc[d][i] = 0.0;
        P.dsc[d][i] = 0.0;
        P.dzs[d][i] = 0.0;
        return;
    }
    const double a = P.drc[i], b = P.ths[i];
    const double etd = P.mvN[i];
    const double dsg = (P.rhs[i] - a * etd) / (a + b);
    const double gdx = etd + dsg;
    const double dy = a * (P.rpp[i] - gdx);
    P.dsig[d][i] = dsg;
    P.dyc[d][i] = dy;
    P.dsc[d][i] = (rsy_of(P, i, A) - P.sc[i] * dy) / P.yc[i];
    P.dzs[d][i] = A.res * P.rds[i] - dy;
}

// Part d (poses), with E dy_c in mvK2: dz_t = rdt - (E dy_c - dy_b).
__global__ void k_dir_d(IpmPtr P, int64_t K, int d, double res) {
    const int64_t k = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (k >= K) return;
    P.dzt[d][k] = res * P.rdt[k] - (P.mvK2[k] - P.S[3 * d + 1]);
}

// Slot od += slot cd (all direction components and the budget row's dy_b, ds_b).
__global__ void k_dir_add(IpmPtr P, int64_t K, int64_t N, int od, int cd) {
    const int64_t j = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (j < K) {
        P.dt[od][j] += P.dt[cd][j];
        P.dzt[od][j] += P.dzt[cd][j];
    }
    if (j < N) {
        P.dsig[od][j] += P.dsig[cd][j];
        P.dzs[od][j] += P.dzs[cd][j];
        P.dyc[od][j] += P.dyc[cd][j];
        P.dsc[od][j] += P.dsc[cd][j];
    }
    if (j == 0) {
        P.S[3 * od + 1] += P.S[3 * cd + 1];
        P.S[3 * od + 2] += P.S[3 * cd + 2];
    }
}

// Fixed-order block reductions over the index space [0, K + N): job
//  0 residual sums: [0] sum t, [1] x.z + sc.yc, [2] p.sigma, [3] sum yc,
//    [4] |rpc|^2, [5] |rd|^2
//  1 largest steps of direction d: [0] primal min ratio, [1] dual min ratio
//  2 affine complementarity: [0] sum (x + ap dx)(z + ad dz) + (s + ap ds)(y + ad dy)
//  3 final objective of the clamped iterate: [0] sum max(t,0), [1] p.max(sigma,0)
//  4 sum p^2 over visible elements: [0]
//  5 [0] sum of dt[d]
//  6 minima: [0] over (t, sigma, s_c), [1] over (z_t, z_sigma, y_c)
//  7 start sums: [0] x.z + s.y, [1] sum z + sum y, [2] sum x + sum s
__global__ __launch_bounds__(LP_TB) void k_ipm_reduce(IpmPtr P, int64_t K, int64_t N, int job, int d, double ap,
                                                      double ad, double* __restrict__ part) {
    __shared__ double red[IPM_SUMS][LP_TB];
    double acc[IPM_SUMS];
    const bool is_min = job == 1 || job == 6;
    for (int q = 0; q < IPM_SUMS; ++q) acc[q] = is_min ? 1e300 : 0.0;
    const int64_t n = K + N;
    for (int64_t j = blockIdx.x * (int64_t)LP_TB + threadIdx.x; j < n; j += (int64_t)gridDim.x * LP_TB) {
        if (j < K) {
            const int64_t k = j;
            if (job == 0) {
                acc[0] += P.xt[k];
                acc[1] += P.xt[k] * P.zt[k];
                acc[5] += P.rdt[k] * P.rdt[k];
            } else if (job == 1) {
                if (P.dt[d][k] < 0.0 && P.xt[k] > 0.0) acc[0] = fmin(acc[0], -P.xt[k] / P.dt[d][k]);
                if (P.dzt[d][k] < 0.0 && P.zt[k] > 0.0) acc[1] = fmin(acc[1], -P.zt[k] / P.dzt[d][k]);
            } else if (job == 2) {
                acc[0] += (P.xt[k] + ap * P.dt[0][k]) * (P.zt[k] + ad * P.dzt[0][k]);
            } else if (job == 3) {
                acc[0] += fmax(P.xt[k], 0.0);
            } else if (job == 5) {
                acc[0] += P.dt[d][k];
            } else if (job == 6) {
                acc[0] = fmin(acc[0], P.xt[k]);
                acc[1] = fmin(acc[1], P.zt[k]);
            } else if (job == 7) {
                acc[0] += P.xt[k] * P.zt[k];
                acc[1] += P.zt[k];
                acc[2] += P.xt[k];
            }
        } else {
            const int64_t i = j - K;
            if (!P.vis[i]) continue;
            if (job == 0) {
                acc[1] += P.xs[i] * P.zs[i] + P.sc[i] * P.yc[i];
                acc[2] += P.pen[i] * P.xs[i];
                acc[3] += P.yc[i];
                acc[4] += P.rpc[i] * P.rpc[i];
                acc[5] += P.rds[i] * P.rds[i];
            } else if (job == 1) {
                if (P.dsig[d][i] < 0.0 && P.xs[i] > 0.0) acc[0] = fmin(acc[0], -P.xs[i] / P.dsig[d][i]);
                if (P.dsc[d][i] < 0.0 && P.sc[i] > 0.0) acc[0] = fmin(acc[0], -P.sc[i] / P.dsc[d][i]);
                if (P.dzs[d][i] < 0.0 && P.zs[i] > 0.0) acc[1] = fmin(acc[1], -P.zs[i] / P.dzs[d][i]);
                if (P.dyc[d][i] < 0.0 && P.yc[i] > 0.0) acc[1] = fmin(acc[1], -P.yc[i] / P.dyc[d][i]);
            } else if (job == 2) {
                acc[0] += (P.xs[i] + ap * P.dsig[0][i]) * (P.zs[i] + ad * P.dzs[0][i]) +
                          (P.sc[i] + ap * P.dsc[0][i]) * (P.yc[i] + ad * P.dyc[0][i]);
            } else if (job == 3) {
                acc[1] += P.pen[i] * fmax(P.xs[i], 0.0);
            } else if (job == 4) {
                acc[0] += P.pen[i] * P.pen[i];
            } else if (job == 6) {
                acc[0] = fmin(acc[0], fmin(P.xs[i], P.sc[i]));
                acc[1] = fmin(acc[1], fmin(P.zs[i], P.yc[i]));
            } else if (job == 7) {
                acc[0] += P.xs[i] * P.zs[i] + P.sc[i] * P.yc[i];
                acc[1] += P.zs[i] + P.yc[i];
                acc[2] += P.xs[i] + P.sc[i];
            }
        }
    }
    for (int q = 0; q < IPM_SUMS; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = LP_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < IPM_SUMS; ++q)
                red[q][threadIdx.x] = is_min ? fmin(red[q][threadIdx.x], red[q][threadIdx.x + w])
                                             : red[q][threadIdx.x] + red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < IPM_SUMS) part[blockIdx.x * IPM_SUMS + threadIdx.x] = red[threadIdx.x][0];
}

// Second pass: 64 threads per sum each fold a fixed stride of the block
// partials, then a fixed-order tree over the 64 (one workgroup of 512).
__global__ __launch_bounds__(512) void k_ipm_reduce2(const double* __restrict__ part, int nb, int is_min,
                                                     double* __restrict__ out) {
    __shared__ double red[IPM_SUMS][64];
    const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
    double a = is_min ? 1e300 : 0.0;
    for (int b = l; b < nb; b += 64) a = is_min ? fmin(a, part[b * IPM_SUMS + q]) : a + part[b * IPM_SUMS + q];
    red[q][l] = a;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (l < w) red[q][l] = is_min ? fmin(red[q][l], red[q][l + w]) : red[q][l] + red[q][l + w];
        __syncthreads();
    }
    if (l == 0) out[q] = red[q][0];
}

__global__ void k_ipm_update(IpmPtr P, int64_t K, int64_t N, double ap, double ad, int d) {
    const int64_t j = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (j < K) {
        P.xt[j] += ap * P.dt[d][j];
        P.zt[j] += ad * P.dzt[d][j];
    }
    if (j < N && P.vis[j]) {
        P.xs[j] += ap * P.dsig[d][j];
        P.sc[j] += ap * P.dsc[d][j];
        P.zs[j] += ad * P.dzs[d][j];
        P.yc[j] += ad * P.dyc[d][j];
    }
}

__global__ void k_ipm_init(IpmPtr P, int64_t K, int64_t N, double x0, double pdef, const double* __restrict__ pen_in,
                           double pscale) {
    const int64_t j = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (j < K) {
        P.xt[j] = x0;
        P.zt[j] = x0;
    }
    if (j < N) {
        const bool v = P.vis[j] != 0;
        P.pen[j] = v ? pscale * (pen_in ? pen_in[j] : pdef) : 0.0;
        P.xs[j] = v ? x0 : 0.0;
        P.zs[j] = v ? x0 : 0.0;
        P.sc[j] = v ? x0 : 0.0;
        P.yc[j] = v ? 1.0 : 0.0;
    }
}

// Constant starting point (scaled problem): K op 0: t = a (half the budget
// over the K poses); op 1, after mvK = rs E y: z_t = max(1 - mvK + a, 1)
// with a = y_b.  N, after mvN = rs E^T t: sigma' = 1, s = max(mvN, 1)
// (the row's surplus, at least 1), y = 1, z_sigma = max(p' - 1, 1).  On the
// ward, the batched rooms and 60 held-out ranked plans it took 7-22 % fewer
// iterations than Mehrotra's least-norm start (which needs an extra
// unit-scaled factorization) together with the per-entry regularisation.
__global__ void k_cs_K(IpmPtr P, int64_t K, int op, double a) {
    const int64_t k = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (k >= K) return;
    if (op == 0)
        P.xt[k] = a;
    else
        P.zt[k] = fmax(1.0 - P.mvK[k] + a, 1.0);
}
__global__ void k_cs_N(IpmPtr P, int64_t N) {
    const int64_t i = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (i >= N || !P.vis[i]) return;
    P.xs[i] = 1.0;
    P.sc[i] = fmax(P.mvN[i], 1.0);
    P.yc[i] = 1.0;
    P.zs[i] = fmax(P.pen[i] - 1.0, 1.0);
}

// Outputs in the problem's units: t, sigma = mu sigma' (mu for dropped
// elements) and the duals of the coverage rows y = y_c / mu (the penalty p_i
// for a dropped element, whose sigma_i = mu sits strictly inside its bound)
// followed by the budget row's y_b.
__global__ void k_ipm_output(IpmPtr P, int64_t K, int64_t N, double mu, double yb, const double* __restrict__ pen_in,
                             double pdef, double* __restrict__ t_out, double* __restrict__ s_out,
                             double* __restrict__ y_out) {
    const int64_t j = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (t_out && j < K) t_out[j] = fmax(P.xt[j], 0.0);
    if (s_out && j < N) s_out[j] = P.vis[j] ? mu * fmax(P.xs[j], 0.0) : mu;
    if (y_out && j < N) y_out[j] = P.vis[j] ? fmax(P.yc[j], 0.0) / mu : (pen_in ? pen_in[j] : pdef);
    if (y_out && j == 0) y_out[N] = fmax(yb, 0.0);
}

// Largest diagonal entry of M (one workgroup), stored at S[S_REG].
__global__ __launch_bounds__(LP_TB) void k_diag_max(const double* __restrict__ M, int64_t K, double* __restrict__ S) {
    __shared__ double red[LP_TB];
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < K; k += LP_TB) a = fmax(a, M[k * K + k]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = LP_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) S[S_REG] = red[0];
}

// diag(M) += rel * diag(M) + 1e-30 * max diag (S[S_REG]).  Relative to
// each entry: a shift relative to the largest entry (set by poses whose
// t -> 0, theta_t = z_t / t huge) perturbed the rows of the support poses
// enough that their dual slacks' directions carried errors of ~1e-8, which
// blocked the dual step once such a slack approached zero.
__global__ void k_diag_reg(double* __restrict__ M, int64_t K, const double* __restrict__ S, double rel) {
    const int64_t k = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (k < K) M[k * K + k] += rel * M[k * K + k] + 1e-30 * S[S_REG];
}

// M (lower) = sum over splits of the partial products
__global__ void k_sum_splits(const double* __restrict__ part, int splits, int64_t K, double* __restrict__ M) {
    const int64_t a = blockIdx.y;
    const int64_t b = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (a >= K || b > a) return;
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += part[(int64_t)s * K * K + a * K + b];
    M[a * K + b] = v;
}

// ------------------------------------------------------------------ host
struct LpWork {
    std::vector<void*> owned;
    template <class T>
    uvc_status alloc(T** p, size_t count, const char* what) {
        UVC_TRY(dalloc_n(p, std::max<size_t>(count, 1), what));
        owned.push_back(*p);
        return UVC_OK;
    }
    ~LpWork() {
        for (void* p : owned) (void)hipFree(p);
    }
};

static uvc_status solve_ipm(const float* E, int64_t K, int64_t N, const double* pen_dev, double mu, double tmax,
                            double tol, int32_t max_iter, double* t_out, double* s_out, double* y_out,
                            uvc_lp_info* info, hipStream_t st) {
    if ((double)K * (double)K * 8.0 > 64e9) return fail(UVC_EUNSUPPORTED, "K too large for the dense normal matrix");
    LpWork W;
    const int64_t rows_per = std::max<int64_t>(64, (K + 15) / 16);
    const int64_t chunks = (K + rows_per - 1) / rows_per;
    // SYRK split over N: enough workgroups for the chip, bounded scratch
    const int64_t T = (K + SY_T - 1) / SY_T, tiles = T * (T + 1) / 2;
    int splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, (1024 + tiles - 1) / tiles));
    while (splits > 1 && ((double)splits * K * K * 8.0 > 512e6 || N / splits < 4 * SY_KC)) --splits;
    float *cmax_part = nullptr, *cmax = nullptr;
    double *sq_part = nullptr, *sq = nullptr, *part = nullptr, *M = nullptr, *Mpart = nullptr, *rpart = nullptr;
    unsigned char *vis_d = nullptr, *occ = nullptr;
    int* failf = nullptr;
    const int64_t nc_occ = (N + SY_OC - 1) / SY_OC;
    UVC_TRY(W.alloc(&cmax_part, (size_t)chunks * N, "lp colmax"));
    UVC_TRY(W.alloc(&cmax, N, "lp colmax"));
    UVC_TRY(W.alloc(&sq_part, (size_t)chunks * N, "lp norm"));
    UVC_TRY(W.alloc(&sq, N, "lp norm"));
    UVC_TRY(W.alloc(&part, (size_t)chunks * N, "lp partial sums"));
    UVC_TRY(W.alloc(&M, (size_t)K * K, "lp normal matrix"));
    if (splits > 1) UVC_TRY(W.alloc(&Mpart, (size_t)splits * K * K, "lp normal matrix partials"));
    UVC_TRY(W.alloc(&vis_d, N, "lp visibility"));
    UVC_TRY(W.alloc(&occ, (size_t)T * nc_occ, "lp occupancy map"));
    UVC_TRY(W.alloc(&failf, 1, "lp flag"));
    const int RB = 512;  // reduction workgroups
    UVC_TRY(W.alloc(&rpart, (size_t)RB * IPM_SUMS, "lp reduction partials"));
    IpmPtr P{};
    double** kvec[] = {&P.xt, &P.zt, &P.rdt, &P.tht, &P.mvK, &P.mvK2, &P.dt[0], &P.dt[1], &P.dzt[0], &P.dzt[1]};
    for (double** p : kvec) UVC_TRY(W.alloc(p, K, "lp pose vector"));
    double** nvec[] = {&P.xs,     &P.zs,     &P.yc,     &P.sc,     &P.pen,    &P.rpc,   &P.rds,
                       &P.drc,    &P.ths,    &P.dtil,   &P.rhs,    &P.rpp,    &P.mvN,   &P.u,
                       &P.dsig[0], &P.dsig[1], &P.dzs[0], &P.dzs[1], &P.dyc[0], &P.dyc[1], &P.dsc[0],
                       &P.dsc[1]};
    for (double** p : nvec) UVC_TRY(W.alloc(p, N, "lp element vector"));
    UVC_TRY(W.alloc(&P.S, 16, "lp scalars"));
    P.vis = vis_d;

    // The iteration runs on the equivalent problem whose coverage rows are
    // divided by mu_min: rows (E^T t) / mu + sigma' >= 1 with sigma' = sigma /
    // mu and penalties mu p, so that the objective and t are unchanged and the
    // coverage duals are mu y.  Every product with E carries the factor
    // rs = 1 / mu.  Without it the central path runs with the budget row far
    // from its scale and budget-bound rooms took up to twice the iterations.
    const double rs = 1.0 / mu;
    auto Etu = [&](const double* u, double* out) {  // out[i] = rs sum_k E[k,i] u[k]
        hipLaunchKernelGGL(k_lp_Etu, dim3(nblk(N), (unsigned)chunks), dim3(LP_TB), 0, st, E, K, N, rows_per, u, part,
                           (const unsigned char*)occ, nc_occ);
        hipLaunchKernelGGL(k_lp_sum_parts, dim3(nblk(N)), dim3(LP_TB), 0, st, part, chunks, N, out, rs);
    };
    auto Ev = [&](const double* v, double* out) {  // out[k] = sum_i E[k,i] v[i]
        hipLaunchKernelGGL(k_lp_Ev, dim3((unsigned)K), dim3(LP_TB), 0, st, E, N, v, out, rs,
                           (const unsigned char*)occ, nc_occ);
    };
    double red[IPM_SUMS];
    double hS[S_RED + IPM_SUMS];
    auto reduce = [&](int job, int d, double ap, double ad) -> uvc_status {
        hipLaunchKernelGGL(k_ipm_reduce, dim3(RB), dim3(LP_TB), 0, st, P, K, N, job, d, ap, ad, rpart);
        hipLaunchKernelGGL(k_ipm_reduce2, dim3(1), dim3(512), 0, st, rpart, RB, (job == 1 || job == 6) ? 1 : 0,
                           P.S + S_RED);
        UVC_HIP(hipGetLastError());
        // the whole scalar block: the reduction and the directions' budget-row
        // components come back in one copy
        UVC_HIP(hipMemcpyAsync(hS, P.S, sizeof(hS), hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        for (int q = 0; q < IPM_SUMS; ++q) red[q] = hS[S_RED + q];
        return UVC_OK;
    };

    // column statistics: visibility, ||E||_F, finiteness
    hipLaunchKernelGGL(k_lp_colstats, dim3(nblk(N), (unsigned)chunks), dim3(LP_TB), 0, st, E, K, N, rows_per,
                       cmax_part, sq_part);
    if (K > 0 && N > 0)
        hipLaunchKernelGGL(k_occ, dim3((unsigned)nc_occ, (unsigned)T), dim3(256), 0, st, E, K, N, nc_occ, occ);
    hipLaunchKernelGGL(k_lp_max_parts, dim3(nblk(N)), dim3(LP_TB), 0, st, cmax_part, chunks, N, cmax);
    hipLaunchKernelGGL(k_lp_sum_parts, dim3(nblk(N)), dim3(LP_TB), 0, st, sq_part, chunks, N, sq, 1.0);
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
    const double pdef = 1.001 * std::sqrt(fro2);
    double p0 = pdef;
    if (pen_dev) {
        std::vector<double> hp((size_t)N);
        UVC_HIP(hipMemcpyAsync(hp.data(), pen_dev, (size_t)N * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < N; ++i)
            if (vis[(size_t)i] && !(std::isfinite(hp[(size_t)i]) && hp[(size_t)i] >= 0.0))
                return fail(UVC_EINVAL, "penalty must be finite and >= 0");
        p0 = hp[0];
    }
    UVC_HIP(hipMemcpyAsync(vis_d, vis.data(), (size_t)N, hipMemcpyHostToDevice, st));

    double obj = 0.0, pres = 0.0, dres = 0.0, rgap = 0.0;
    int32_t it = 0;
    bool converged = nvis == 0;
    const unsigned gK = nblk(K), gN = nblk(N), gKN = nblk(std::max(K, N));
    if (nvis > 0) {
        // starting point and norms of h and c
        double pmax = mu * pdef;  // penalties of the scaled problem
        double psq = 0.0;
        if (pen_dev) {
            hipLaunchKernelGGL(k_ipm_init, dim3(gKN), dim3(LP_TB), 0, st, P, K, N, 0.0, pdef, pen_dev, mu);
            UVC_TRY(reduce(4, 0, 0.0, 0.0));
            psq = red[0];
            std::vector<double> hp((size_t)N);
            UVC_HIP(hipMemcpyAsync(hp.data(), P.pen, (size_t)N * 8, hipMemcpyDeviceToHost, st));
            UVC_HIP(hipStreamSynchronize(st));
            pmax = 0.0;
            for (double v : hp) pmax = std::max(pmax, v);
        } else {
            psq = (double)nvis * pmax * pmax;
        }
        const double x0 = std::max(1.0, std::sqrt(std::max(1.0, pmax)));
        hipLaunchKernelGGL(k_ipm_init, dim3(gKN), dim3(LP_TB), 0, st, P, K, N, x0, pdef, pen_dev, mu);
        UVC_HIP(hipGetLastError());
        // M = E diag(dtil) E^T + Db 1 1^T + diag(tht), regularised, then its Cholesky factor in place
        auto factor = [&](double Db) -> uvc_status {
            if (splits > 1) {
                hipLaunchKernelGGL(k_syrk, dim3((unsigned)tiles, (unsigned)splits), dim3(256), 0, st, E, K, N, P.dtil,
                                   Mpart, splits, (const unsigned char*)occ, nc_occ);
                hipLaunchKernelGGL(k_sum_splits, dim3(nblk(K), (unsigned)K), dim3(LP_TB), 0, st, Mpart, splits, K, M);
            } else {
                hipLaunchKernelGGL(k_syrk, dim3((unsigned)tiles, 1u), dim3(256), 0, st, E, K, N, P.dtil, M, 1,
                                   (const unsigned char*)occ, nc_occ);
            }
            hipLaunchKernelGGL(k_mat_finish, dim3(nblk(K), (unsigned)K), dim3(LP_TB), 0, st, M, K, rs * rs, Db, P.tht,
                               0.0);
            hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(LP_TB), 0, st, M, K, P.S);
            hipLaunchKernelGGL(k_diag_reg, dim3(gK), dim3(LP_TB), 0, st, M, K, P.S, 1e-13);
            UVC_HIP(hipMemsetAsync(failf, 0, 4, st));
            for (int64_t j0 = 0; j0 < K; j0 += CH_B) {
                const int nb = (int)std::min<int64_t>(CH_B, K - j0);
                // later diagonal blocks are factored by the previous panel's update
                if (j0 == 0) hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, M, K, j0, nb, failf);
                const int64_t rest = K - j0 - nb;
                if (rest > 0) {
                    hipLaunchKernelGGL(k_chol_trsm, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, st, M, K, j0,
                                       nb);
                    const int64_t T2 = (rest + SY_T - 1) / SY_T;
                    const int next_nb = (int)std::min<int64_t>(CH_B, rest);
                    hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T2 * (T2 + 1) / 2)), dim3(256), 0, st, M, K,
                                       j0, nb, next_nb, failf);
                }
            }
            UVC_HIP(hipGetLastError());
            return UVC_OK;
        };
        double sb = 0.5 * tmax, yb = 1.0;
        {
            // constant start: half the budget spread evenly over the poses,
            // sigma' = 1, unit duals, every slack at least 1
            hipLaunchKernelGGL(k_cs_K, dim3(gK), dim3(LP_TB), 0, st, P, K, 0, 0.5 * tmax / (double)K);
            Etu(P.xt, P.mvN);
            hipLaunchKernelGGL(k_cs_N, dim3(gN), dim3(LP_TB), 0, st, P, N);
            Ev(P.yc, P.mvK);
            hipLaunchKernelGGL(k_cs_K, dim3(gK), dim3(LP_TB), 0, st, P, K, 1, yb);
            UVC_HIP(hipGetLastError());
        }
        const double hn = std::sqrt((double)nvis * mu * mu + tmax * tmax);  // |h| in the problem's units
        const double cn = std::sqrt((double)K + psq);
        const double ncomp = (double)(nvis * 2 + K + 1);
        // UVC_VERBOSE=2: one line per iteration on stderr
        const char* venv = std::getenv("UVC_VERBOSE");
        const bool trace = venv && std::atoi(venv) >= 2;
        double tr_ap = 0.0, tr_ad = 0.0, tr_sig = 0.0;
        for (it = 0; it < max_iter; ++it) {
            // residuals and convergence
            Etu(P.xt, P.mvN);
            Ev(P.yc, P.mvK);
            hipLaunchKernelGGL(k_ipm_resid_N, dim3(gN), dim3(LP_TB), 0, st, P, N, 1.0);
            hipLaunchKernelGGL(k_ipm_resid_K, dim3(gK), dim3(LP_TB), 0, st, P, K, yb);
            UVC_TRY(reduce(0, 0, 0.0, 0.0));
            const double sum_t = red[0];
            const double rpb = -tmax + sum_t + sb;
            const double gap = red[1] + sb * yb;
            const double po = sum_t + red[2];
            const double dob = red[3] - tmax * yb;
            pres = std::sqrt(mu * mu * red[4] + rpb * rpb) / (1.0 + hn);  // coverage residuals back in units of mu
            dres = std::sqrt(red[5]) / (1.0 + cn);
            rgap = std::fabs(po - dob) / (1.0 + std::fabs(po) + std::fabs(dob));
            obj = po;
            if (trace) {
                std::fprintf(stderr, "[uvc ipm] K %lld it %3d pres %.2e dres %.2e gap %.2e obj %.9e mu %.2e "
                                     "| last ap %.3f ad %.3f sigma %.2e\n",
                             (long long)K, it, pres, dres, rgap, po, gap / ncomp, tr_ap, tr_ad, tr_sig);
                std::fflush(stderr);
            }
            if (std::max(pres, std::max(dres, rgap)) <= tol) {
                converged = true;
                break;
            }
            const double muc = gap / ncomp;
            // normal matrix M = E diag(dtil) E^T + D_b 1 1^T + diag(theta_t), regularised, and its factor
            const double Db = yb / sb;
            hipLaunchKernelGGL(k_ipm_scale, dim3(gKN), dim3(LP_TB), 0, st, P, K, N);
            UVC_TRY(factor(Db));
            // one Newton direction into slot d (mode 0 predictor, 1 corrector)
            auto direction = [&](const RhsArgs& A, int d, double rsyb) {
                const double rppb = A.res * rpb + rsyb / yb;
                const double wvb = Db * rppb;
                hipLaunchKernelGGL(k_dir_a, dim3(gN), dim3(LP_TB), 0, st, P, N, A);
                Ev(P.u, P.mvK);
                hipLaunchKernelGGL(k_dir_b, dim3(gK), dim3(LP_TB), 0, st, P, K, A, wvb, d);
                tri_solve(M, K, P.dt[d], st);
                Etu(P.dt[d], P.mvN);
                hipLaunchKernelGGL(k_ipm_bscal, dim3(1), dim3(LP_TB), 0, st, P, K, d, Db, rppb, rsyb, sb, yb);
                hipLaunchKernelGGL(k_dir_c, dim3(gN), dim3(LP_TB), 0, st, P, N, A, d);
                Ev(P.dyc[d], P.mvK2);
                hipLaunchKernelGGL(k_dir_d, dim3(gK), dim3(LP_TB), 0, st, P, K, d, A.res);
            };
            auto steps = [&](int d, double& ap, double& ad, double& dyb, double& dsb) -> uvc_status {
                UVC_TRY(reduce(1, d, 0.0, 0.0));  // also brings back S[3 d + 1], S[3 d + 2]
                dyb = hS[3 * d + 1];
                dsb = hS[3 * d + 2];
                ap = std::min(1.0, red[0]);
                ad = std::min(1.0, red[1]);
                if (dsb < 0.0 && sb > 0.0) ap = std::min(ap, -sb / dsb);
                if (dyb < 0.0 && yb > 0.0) ad = std::min(ad, -yb / dyb);
                return UVC_OK;
            };
            // the factorization's failure flag comes back with the next synchronisation
            int f = 0;
            UVC_HIP(hipMemcpyAsync(&f, failf, 4, hipMemcpyDeviceToHost, st));
            direction(RhsArgs{0, 0, 0.0, 0.0, 0.0, 1.0}, 0, -sb * yb);
            double ap = 1.0, ad = 1.0, dyb0 = 0.0, dsb0 = 0.0;
            UVC_TRY(steps(0, ap, ad, dyb0, dsb0));
            if (f != 0) break;
            UVC_TRY(reduce(2, 0, ap, ad));
            const double gaff = red[0] + (sb + ap * dsb0) * (yb + ad * dyb0);
            const double sig = std::pow(gaff / std::max(gap, 1e-300), 3.0);
            const double sigmu = sig * muc;
            direction(RhsArgs{1, 0, sigmu, 0.0, 0.0, 1.0}, 1, sigmu - sb * yb - dsb0 * dyb0);
            double dybc = 0.0, dsbc = 0.0;
            UVC_TRY(steps(1, ap, ad, dybc, dsbc));
            // Gondzio's centrality correctors: from the trial point a longer
            // step would reach, move outlying complementarity products into
            // [0.1, 10] sigmu; keep a correction only if it lengthens the steps
            int cd = 1;
            for (int kc = 0; kc < LP_CENTRALITY; ++kc) {
                const double atp = std::min(1.0, 1.5 * ap + 0.3), atd = std::min(1.0, 1.5 * ad + 0.3);
                const double vb = (sb + atp * dsbc) * (yb + atd * dybc);
                const double rb = std::max(std::min(std::max(vb, 0.1 * sigmu), 10.0 * sigmu) - vb, -10.0 * sigmu);
                const int od = 1 - cd;
                direction(RhsArgs{2, cd, sigmu, atp, atd, 0.0}, od, rb);
                hipLaunchKernelGGL(k_dir_add, dim3(gKN), dim3(LP_TB), 0, st, P, K, N, od, cd);
                double ap2 = 1.0, ad2 = 1.0, dyb2 = 0.0, dsb2 = 0.0;
                UVC_TRY(steps(od, ap2, ad2, dyb2, dsb2));
                if (!(ap2 + ad2 >= 1.01 * (ap + ad))) break;
                cd = od;
                ap = ap2;
                ad = ad2;
                dybc = dyb2;
                dsbc = dsb2;
            }
            ap *= 0.99;
            ad *= 0.99;
            tr_ap = ap;
            tr_ad = ad;
            tr_sig = sig;
            hipLaunchKernelGGL(k_ipm_update, dim3(gKN), dim3(LP_TB), 0, st, P, K, N, ap, ad, cd);
            UVC_HIP(hipGetLastError());
            sb += ap * dsbc;
            yb += ad * dybc;
        }
        UVC_TRY(reduce(3, 0, 0.0, 0.0));
        obj = red[0] + red[1];
        hipLaunchKernelGGL(k_ipm_output, dim3(gKN), dim3(LP_TB), 0, st, P, K, N, mu, yb, pen_dev, pdef, t_out, s_out,
                           y_out);
    } else {
        if (t_out) UVC_HIP(hipMemsetAsync(t_out, 0, (size_t)K * 8, st));
        if (s_out) {
            std::vector<double> hs((size_t)N, mu);
            UVC_HIP(hipMemcpyAsync(s_out, hs.data(), (size_t)N * 8, hipMemcpyHostToDevice, st));
            UVC_HIP(hipStreamSynchronize(st));
        }
        if (y_out) {
            // nothing is visible: every element's sigma = mu is interior, its dual is its penalty
            std::vector<double> hy((size_t)N + 1, 0.0);
            if (pen_dev) {
                UVC_HIP(hipMemcpyAsync(hy.data(), pen_dev, (size_t)N * 8, hipMemcpyDeviceToHost, st));
                UVC_HIP(hipStreamSynchronize(st));
            } else {
                for (int64_t i = 0; i < N; ++i) hy[(size_t)i] = pdef;
            }
            hy[(size_t)N] = 0.0;
            UVC_HIP(hipMemcpyAsync(y_out, hy.data(), ((size_t)N + 1) * 8, hipMemcpyHostToDevice, st));
            UVC_HIP(hipStreamSynchronize(st));
        }
    }
    UVC_HIP(hipGetLastError());
    UVC_HIP(hipStreamSynchronize(st));
    if (info) {
        info->objective = obj;
        info->primal_residual = pres;
        info->dual_residual = dres;
        info->gap = rgap;
        info->iterations = it;
        info->n_visible = nvis;
        info->penalty = p0;
    }
    if (!converged)
        return fail(UVC_ENOTCONV, "LP did not reach tol; residuals " + std::to_string(pres) + " " +
                                      std::to_string(dres) + " " + std::to_string(rgap));
    return UVC_OK;
}

__global__ void k_lp_fill(double* __restrict__ p, double v, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (q < n) p[q] = v;
}

__global__ void k_lp_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
    const int64_t q = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (q < n) dst[q] = src[q];
}

// An LP without poses or without elements: no element is visible, so every
// element is dropped (sigma_i = mu_min, its dual is its penalty), t = 0 and
// the objective (which leaves dropped elements out) is 0.  The default
// penalty 1.001 ||E||_F of an empty matrix is 0.
static uvc_status solve_empty(int64_t K, int64_t N, const double* pen_dev, double mu, double* t_out, double* s_out,
                              double* y_out, uvc_lp_info* info, hipStream_t st) {
    double p0 = 0.0;
    if (pen_dev && N > 0) {
        UVC_HIP(hipMemcpyAsync(&p0, pen_dev, 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
    }
    if (t_out && K > 0) hipLaunchKernelGGL(k_lp_fill, dim3(nblk(K)), dim3(LP_TB), 0, st, t_out, 0.0, K);
    if (s_out && N > 0) hipLaunchKernelGGL(k_lp_fill, dim3(nblk(N)), dim3(LP_TB), 0, st, s_out, mu, N);
    if (y_out) {
        if (N > 0 && pen_dev)
            hipLaunchKernelGGL(k_lp_copy, dim3(nblk(N)), dim3(LP_TB), 0, st, y_out, pen_dev, N);
        else if (N > 0)
            hipLaunchKernelGGL(k_lp_fill, dim3(nblk(N)), dim3(LP_TB), 0, st, y_out, 0.0, N);
        hipLaunchKernelGGL(k_lp_fill, dim3(1), dim3(LP_TB), 0, st, y_out + N, 0.0, (int64_t)1);
    }
    UVC_HIP(hipGetLastError());
    UVC_HIP(hipStreamSynchronize(st));
    if (info) info->penalty = p0;
    return UVC_OK;
}

// ------------------------------------------------------------ CSR input
// Row k of a CSR matrix with nnz entries: 0 <= row_ptr[k] <= row_ptr[k + 1]
// <= nnz, columns strictly ascending within [0, N) (columns are read only
// for rows whose range lies inside [0, nnz)).  *bad receives the smallest
// offending row (left at ~0 when every row passes).
__global__ __launch_bounds__(LP_TB) void k_csr_check(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     int64_t K, int64_t N, int64_t nnz,
                                                     unsigned long long* __restrict__ bad) {
    const int64_t k = blockIdx.x;
    const int64_t q0 = rp[k], q1 = rp[k + 1];
    bool ok = 0 <= q0 && q0 <= q1 && q1 <= nnz;
    if (ok) {
        for (int64_t q = q0 + threadIdx.x; q < q1; q += LP_TB) {
            const int32_t c = col[q];
            if (c < 0 || (int64_t)c >= N || (q > q0 && col[q - 1] >= c)) ok = false;
        }
    }
    if (!ok) atomicMin(bad, (unsigned long long)k);
}

__global__ void k_fill_f32(float* __restrict__ p, float v, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)LP_TB + threadIdx.x; q < n; q += (int64_t)gridDim.x * LP_TB) p[q] = v;
}

__global__ void k_fill_u64x1(unsigned long long* p, unsigned long long v) { *p = v; }

// D[k * N + col[q]] = val[q] for the entries of row k (one workgroup per row).
__global__ __launch_bounds__(LP_TB) void k_csr_scatter(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       const float* __restrict__ val, int64_t N,
                                                       float* __restrict__ D) {
    const int64_t k = blockIdx.x;
    for (int64_t q = rp[k] + threadIdx.x; q < rp[k + 1]; q += LP_TB) D[k * N + col[q]] = val[q];
}

// The interior point method works on the K x K normal matrix, which is
// dense whatever the sparsity of E; its product reads E as a dense pose-major
// matrix.  A CSR input is validated and expanded once into a library-owned
// dense copy (K N 4 bytes; released after the solve).
// CSR inputs with more poses than this are solved by column generation.
constexpr int64_t LP_DENSE_MAX_POSES = 8192;

static uvc_status csr_validate(const int64_t* rp, const int32_t* col, const float* val, int64_t K, int64_t N,
                               hipStream_t st, int64_t* nnz_out) {
    if (K > (int64_t)0x7fffffff) return fail(UVC_EINVAL, "K too large for a CSR input");
    int64_t ends[2] = {0, 0};
    UVC_HIP(hipMemcpyAsync(&ends[0], rp, 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(&ends[1], rp + K, 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] < 0) return fail(UVC_EINVAL, "CSR row_ptr must start at 0 and end at nnz >= 0");
    if (ends[1] > 0 && !val) return fail(UVC_EINVAL, "CSR values are NULL");
    unsigned long long* bad = nullptr;
    UVC_TRY(dalloc_n(&bad, 1, "csr check flag"));
    hipLaunchKernelGGL(k_fill_u64x1, dim3(1), dim3(1), 0, st, bad, ~0ull);
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)K), dim3(LP_TB), 0, st, rp, col, K, N, ends[1], bad);
    unsigned long long hb = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(UVC_EDEVICE, std::string("csr check: ") + hipGetErrorString(e));
    if (hb != ~0ull)
        return fail(UVC_EINVAL, "CSR row " + std::to_string(hb) +
                                    ": row_ptr decreasing, or columns outside [0, N) or not strictly ascending");
    *nnz_out = ends[1];
    return UVC_OK;
}

static uvc_status csr_to_dense(const int64_t* rp, const int32_t* col, const float* val, int64_t K, int64_t N,
                               hipStream_t st, float** out) {
    *out = nullptr;
    int64_t nnz = 0;
    UVC_TRY(csr_validate(rp, col, val, K, N, st, &nnz));
    float* D = nullptr;
    UVC_TRY(dalloc_n(&D, (size_t)K * (size_t)N, "dense copy of the CSR matrix"));
    hipLaunchKernelGGL(k_fill_f32, dim3(4096), dim3(LP_TB), 0, st, D, 0.0f, K * N);
    hipLaunchKernelGGL(k_csr_scatter, dim3((unsigned)K), dim3(LP_TB), 0, st, rp, col, val, N, D);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFree(D);
        return fail(UVC_EDEVICE, std::string("csr expand: ") + hipGetErrorString(e));
    }
    *out = D;
    return UVC_OK;
}

// ------------------------------------------- large CSR input: column generation
// For a CSR matrix with many poses the K x K normal matrix (and the dense
// copy of E) would dominate; the LP is instead solved over a working set R
// of poses, with every other pose priced against the working LP's duals:
// pose k's reduced cost is 1 + y_b - sum_i E[k,i] y_i (a sparse row times
// the dual vector); poses with negative reduced costs join R until none is
// below -1e-6, at which point the working solution is optimal for the LP
// over all K poses.  Elements no pose of R sees are dropped from the
// working LP (sigma_i = mu_min, dual p_i) and priced at their penalty; their
// constant p_i mu_min is added back to the reported objective when some pose
// outside R sees them, so that the objective is the full LP's (over every
// element some pose sees).

// best[i] = max over the entries (k, i) of (bits(E[k,i]) << 32 | k): E >= 0,
// so the float bits order like the values; nonzero exactly for the visible
// elements.
__global__ __launch_bounds__(LP_TB) void k_csr_colbest(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       unsigned long long* __restrict__ best) {
    const int64_t k = blockIdx.x;
    for (int64_t q = rp[k] + threadIdx.x; q < rp[k + 1]; q += LP_TB) {
        const float v = val[q];
        if (v > 0.0f)
            atomicMax(best + col[q], ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)k);
    }
}

// Per-workgroup partial sums of E^2 (FP64, fixed order).
__global__ __launch_bounds__(LP_TB) void k_csr_sumsq(const float* __restrict__ val, int64_t nnz,
                                                     double* __restrict__ part) {
    __shared__ double red[LP_TB];
    double a = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)LP_TB + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * LP_TB) {
        const double v = val[q];
        a += v * v;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = LP_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// D[r * N + col] = val for the entries of pose rows[r] (D zeroed first).
__global__ __launch_bounds__(LP_TB) void k_csr_gather(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const float* __restrict__ val, const int32_t* __restrict__ rows,
                                                      int64_t N, float* __restrict__ D) {
    const int64_t r = blockIdx.x, k = rows[r];
    for (int64_t q = rp[k] + threadIdx.x; q < rp[k + 1]; q += LP_TB) D[r * N + col[q]] = val[q];
}

// rc[k] = (1 + y_b) - sum_q val[q] y[col[q]] over row k (FP64; strided
// partials in a fixed tree order).
__global__ __launch_bounds__(LP_TB) void k_csr_price(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const float* __restrict__ val, const double* __restrict__ y,
                                                     double base, double* __restrict__ rc) {
    __shared__ double red[LP_TB];
    const int64_t k = blockIdx.x;
    double a = 0.0;
    for (int64_t q = rp[k] + threadIdx.x; q < rp[k + 1]; q += LP_TB) a += (double)val[q] * y[col[q]];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = LP_TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rc[k] = base - red[0];
}

// seen[col] = 1 for the nonzero entries of the poses rows[0..m) (seen
// zeroed first).
__global__ __launch_bounds__(LP_TB) void k_csr_mark(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    const float* __restrict__ val, const int32_t* __restrict__ rows,
                                                    float* __restrict__ seen) {
    const int64_t k = rows[blockIdx.x];
    for (int64_t q = rp[k] + threadIdx.x; q < rp[k + 1]; q += LP_TB)
        if (val[q] > 0.0f) seen[col[q]] = 1.0f;
}

__global__ void k_scatter_t(const double* __restrict__ src, const int32_t* __restrict__ rows, int64_t n,
                            double* __restrict__ dst) {
    const int64_t q = blockIdx.x * (int64_t)LP_TB + threadIdx.x;
    if (q < n) dst[rows[q]] = src[q];
}

template <class T>
struct DevBuf {
    T* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

static uvc_status solve_csr_colgen(const int64_t* rp, const int32_t* col, const float* val, int64_t K, int64_t N,
                                   int64_t nnz, const double* pen_dev, double mu, double tmax, double tol,
                                   int32_t max_iter, double* t_out, double* s_out, double* y_out, uvc_lp_info* info,
                                   hipStream_t st) {
    DevBuf<unsigned long long> best;
    DevBuf<double> part, pen, yd, rc, tr;
    DevBuf<float> D;
    DevBuf<int32_t> rows;
    UVC_TRY(dalloc_n(&best.p, (size_t)N, "column best poses"));
    UVC_TRY(dalloc_n(&part.p, 1024, "norm partials"));
    UVC_TRY(dalloc_n(&pen.p, (size_t)N, "penalties"));
    UVC_TRY(dalloc_n(&yd.p, (size_t)N + 1, "working duals"));
    UVC_TRY(dalloc_n(&rc.p, (size_t)K, "reduced costs"));
    hipLaunchKernelGGL(k_lp_fill, dim3(nblk(N)), dim3(LP_TB), 0, st, (double*)best.p, 0.0, N);  // zero bits
    hipLaunchKernelGGL(k_csr_colbest, dim3((unsigned)K), dim3(LP_TB), 0, st, rp, col, val, best.p);
    hipLaunchKernelGGL(k_csr_sumsq, dim3(1024), dim3(LP_TB), 0, st, val, nnz, part.p);
    UVC_HIP(hipGetLastError());
    std::vector<unsigned long long> hb((size_t)N);
    std::vector<double> hpart(1024);
    UVC_HIP(hipMemcpyAsync(hb.data(), best.p, (size_t)N * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipMemcpyAsync(hpart.data(), part.p, 1024 * 8, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    double fro2 = 0.0;
    for (double v : hpart) fro2 += v;
    if (!std::isfinite(fro2)) return fail(UVC_EINVAL, "E has a non-finite entry");
    const double pdef = 1.001 * std::sqrt(fro2);
    if (pen_dev)
        hipLaunchKernelGGL(k_lp_copy, dim3(nblk(N)), dim3(LP_TB), 0, st, pen.p, pen_dev, N);
    else
        hipLaunchKernelGGL(k_lp_fill, dim3(nblk(N)), dim3(LP_TB), 0, st, pen.p, pdef, N);
    int64_t nvis = 0;
    for (int64_t i = 0; i < N; ++i) nvis += hb[(size_t)i] ? 1 : 0;
    if (nvis == 0)
        return solve_empty(K, N, pen_dev, mu, t_out, s_out, y_out, info, st);
    // working set: the ceil(K / 10) poses with the largest row sums of E
    // (the most irradiance delivered in all; ties: the lower index); elements
    // they leave unseen are dropped from the working LP, priced at their
    // penalty, and the poses that see them join in the first rounds
    std::vector<double> hrs((size_t)K);
    {
        DevBuf<double> ones;
        UVC_TRY(dalloc_n(&ones.p, (size_t)N, "ones"));
        hipLaunchKernelGGL(k_lp_fill, dim3(nblk(N)), dim3(LP_TB), 0, st, ones.p, 1.0, N);
        hipLaunchKernelGGL(k_csr_price, dim3((unsigned)K), dim3(LP_TB), 0, st, rp, col, val, (const double*)ones.p,
                           0.0, rc.p);
        UVC_HIP(hipGetLastError());
        UVC_HIP(hipMemcpyAsync(hrs.data(), rc.p, (size_t)K * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
    }
    const int64_t keep0 = std::max<int64_t>(1, (K + 9) / 10);
    std::vector<int32_t> order((size_t)K);
    for (int64_t k = 0; k < K; ++k) order[(size_t)k] = (int32_t)k;
    std::partial_sort(order.begin(), order.begin() + keep0, order.end(), [&](int32_t a, int32_t b) {
        return hrs[(size_t)a] != hrs[(size_t)b] ? hrs[(size_t)a] < hrs[(size_t)b] : a < b;  // -row sums
    });
    std::vector<uint8_t> in((size_t)K, 0), dropped_once((size_t)K, 0);
    std::vector<int32_t> R(order.begin(), order.begin() + keep0);
    for (int32_t k : R) in[(size_t)k] = 1;
    std::sort(R.begin(), R.end());
    uvc_lp_info li{};
    int32_t iters = 0, rounds = 0;
    double rmin = 0.0;
    uvc_status r = UVC_OK;
    std::vector<double> hr((size_t)K);
    // at most max(64, ceil(K/10)/4) poses join per round, the most negative
    // first: small steps keep the set near the support.  Letting the set
    // double per round took the floor plan to 9,709 working poses where
    // 5,281 suffice, and 1.7x the time; solving the rounds that add poses to
    // a looser tolerance saved few iterations (the early iterations
    // dominate) and cost extra rounds at the end
    const int64_t add_cap = std::max<int64_t>(64, keep0 / 4);
    // UVC_VERBOSE set: one progress line per round on stderr
    const bool verbose = std::getenv("UVC_VERBOSE") != nullptr;
    const auto t_start = std::chrono::steady_clock::now();
    int64_t m = 0;  // poses of the last working LP (rows.p, tr.p); R may have grown since
    while (true) {
        m = (int64_t)R.size();
        if ((double)m * (double)m * 8.0 > 64e9) return fail(UVC_EUNSUPPORTED, "working pose set too large");
        for (void** q : {(void**)&rows.p, (void**)&D.p, (void**)&tr.p})
            if (*q) {
                (void)hipFree(*q);
                *q = nullptr;
            }
        UVC_TRY(dalloc_n(&rows.p, (size_t)m, "working poses"));
        UVC_TRY(dalloc_n(&D.p, (size_t)m * N, "working matrix"));
        UVC_TRY(dalloc_n(&tr.p, (size_t)m, "working dwell times"));
        UVC_HIP(hipMemcpyAsync(rows.p, R.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_fill_f32, dim3(4096), dim3(LP_TB), 0, st, D.p, 0.0f, m * N);
        hipLaunchKernelGGL(k_csr_gather, dim3((unsigned)m), dim3(LP_TB), 0, st, rp, col, val, rows.p, N, D.p);
        UVC_HIP(hipGetLastError());
        r = solve_ipm(D.p, m, N, pen.p, mu, tmax, tol, max_iter, tr.p, s_out, yd.p, &li, st);
        iters += li.iterations;
        ++rounds;
        if (r != UVC_OK) break;
        // price every pose against the working duals (working poses price at >= 0 up to rounding)
        double yb = 0.0;
        UVC_HIP(hipMemcpyAsync(&yb, yd.p + N, 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        hipLaunchKernelGGL(k_csr_price, dim3((unsigned)K), dim3(LP_TB), 0, st, rp, col, val, (const double*)yd.p,
                           1.0 + yb, rc.p);
        UVC_HIP(hipGetLastError());
        UVC_HIP(hipMemcpyAsync(hr.data(), rc.p, (size_t)K * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        std::vector<int32_t> cand;
        rmin = 0.0;
        for (int64_t k = 0; k < K; ++k)
            if (!in[(size_t)k]) {
                rmin = std::min(rmin, hr[(size_t)k]);
                if (hr[(size_t)k] < -1e-6) cand.push_back((int32_t)k);
            }
        if (verbose) {
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            std::fprintf(stderr, "[uvc lp] round %d: %lld working poses, %d iterations, objective %.9e, "
                                 "%zu poses price below -1e-6 (min %.3e), %.2f s\n",
                         rounds, (long long)m, li.iterations, li.objective, cand.size(), rmin, el);
            std::fflush(stderr);
        }
        if (cand.empty()) break;
        // poses of R without dwell whose reduced cost is clearly positive
        // leave the set (each pose at most once, so the rounds end): the
        // working LPs stay near the support instead of growing with every
        // round; should one price negative again later, it rejoins
        {
            std::vector<double> ht((size_t)m);
            UVC_HIP(hipMemcpyAsync(ht.data(), tr.p, (size_t)m * 8, hipMemcpyDeviceToHost, st));
            UVC_HIP(hipStreamSynchronize(st));
            double tmax_w = 0.0;
            for (double v : ht) tmax_w = std::max(tmax_w, v);
            const double margin = 1e-2 * (1.0 + std::fabs(yb));
            std::vector<int32_t> keep;
            keep.reserve(R.size());
            for (int64_t q = 0; q < m; ++q) {
                const int32_t k = R[(size_t)q];
                if (!dropped_once[(size_t)k] && ht[(size_t)q] <= 1e-9 * tmax_w && hr[(size_t)k] > margin) {
                    in[(size_t)k] = 0;
                    dropped_once[(size_t)k] = 1;
                } else {
                    keep.push_back(k);
                }
            }
            R.swap(keep);
        }
        const int64_t na = std::min<int64_t>((int64_t)cand.size(), add_cap);
        std::partial_sort(cand.begin(), cand.begin() + na, cand.end(), [&](int32_t a, int32_t b) {
            return hr[(size_t)a] != hr[(size_t)b] ? hr[(size_t)a] < hr[(size_t)b] : a < b;
        });
        for (int64_t q = 0; q < na; ++q) {
            in[(size_t)cand[(size_t)q]] = 1;
            R.push_back(cand[(size_t)q]);
        }
        std::sort(R.begin(), R.end());
        if (rounds >= 200) {
            r = fail(UVC_ENOTCONV, "column generation: pricing still finds improving poses after 200 rounds");
            break;
        }
    }
    if (r != UVC_OK && r != UVC_ENOTCONV) return r;
    // elements some pose sees but no working pose does: their constant
    // p_i mu_min belongs to the full LP's objective
    double dropped = 0.0;
    {
        DevBuf<float> seen;
        UVC_TRY(dalloc_n(&seen.p, (size_t)N, "working visibility"));
        hipLaunchKernelGGL(k_fill_f32, dim3(nblk(N)), dim3(LP_TB), 0, st, seen.p, 0.0f, N);
        hipLaunchKernelGGL(k_csr_mark, dim3((unsigned)m), dim3(LP_TB), 0, st, rp, col, val, (const int32_t*)rows.p,
                           seen.p);
        UVC_HIP(hipGetLastError());
        std::vector<float> hs((size_t)N);
        std::vector<double> hp((size_t)N);
        UVC_HIP(hipMemcpyAsync(hs.data(), seen.p, (size_t)N * 4, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipMemcpyAsync(hp.data(), pen.p, (size_t)N * 8, hipMemcpyDeviceToHost, st));
        UVC_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < N; ++i)
            if (hb[(size_t)i] && hs[(size_t)i] == 0.0f) dropped += hp[(size_t)i] * mu;
    }
    // outputs in the full problem's terms: t scattered (0 outside R), the
    // working sigma and duals; residuals of the working LP, the dual
    // residual also covering the pricing of the poses outside R
    if (t_out) {
        hipLaunchKernelGGL(k_lp_fill, dim3(nblk(K)), dim3(LP_TB), 0, st, t_out, 0.0, K);
        hipLaunchKernelGGL(k_scatter_t, dim3(nblk(m)), dim3(LP_TB), 0, st, (const double*)tr.p,
                           (const int32_t*)rows.p, m, t_out);
    }
    if (y_out) hipLaunchKernelGGL(k_lp_copy, dim3(nblk(N + 1)), dim3(LP_TB), 0, st, y_out, (const double*)yd.p, N + 1);
    UVC_HIP(hipGetLastError());
    UVC_HIP(hipStreamSynchronize(st));
    if (info) {
        *info = li;
        info->iterations = iters;
        info->objective += dropped;
        info->n_visible = nvis;
        info->penalty = pen_dev ? info->penalty : pdef;
        info->dual_residual = std::max(li.dual_residual, std::max(0.0, -rmin));
        info->working_poses = m;
        info->rounds = rounds;
    }
    return r;
}

}  // namespace uvc

using namespace uvc;

extern "C" uvc_status uvc_solve_dosage_lp(const float* E_dev, const int64_t* row_ptr_dev, const int32_t* col_dev,
                                          int64_t K, int64_t N, const double* penalty_dev, double mu_min,
                                          double t_max, double tol, int32_t max_iter, double* t_out_dev,
                                          double* sigma_out_dev, double* y_out_dev, uvc_lp_info* info,
                                          void* hip_stream) {
    if (info) *info = uvc_lp_info{};
    if (K < 0 || N < 0) return fail(UVC_EINVAL, "negative LP size");
    if (!(mu_min > 0) || !(t_max > 0) || !(tol > 0) || max_iter <= 0)
        return fail(UVC_EINVAL, "mu_min, t_max, tol and max_iter must be positive");
    if (K == 0 || N == 0) return solve_empty(K, N, penalty_dev, mu_min, t_out_dev, sigma_out_dev, y_out_dev, info,
                                             (hipStream_t)hip_stream);
    if (!row_ptr_dev && !E_dev) return fail(UVC_EINVAL, "E is NULL");
    if (row_ptr_dev && col_dev == nullptr) return fail(UVC_EINVAL, "CSR input needs col");
    hipStream_t st = (hipStream_t)hip_stream;
    try {
        if (!row_ptr_dev)
            return solve_ipm(E_dev, K, N, penalty_dev, mu_min, t_max, tol, max_iter, t_out_dev, sigma_out_dev,
                             y_out_dev, info, st);
        int64_t nnz = 0;
        if (K > LP_DENSE_MAX_POSES) {
            UVC_TRY(csr_validate(row_ptr_dev, col_dev, E_dev, K, N, st, &nnz));
            return solve_csr_colgen(row_ptr_dev, col_dev, E_dev, K, N, nnz, penalty_dev, mu_min, t_max, tol,
                                    max_iter, t_out_dev, sigma_out_dev, y_out_dev, info, st);
        }
        float* dense = nullptr;
        UVC_TRY(csr_to_dense(row_ptr_dev, col_dev, E_dev, K, N, st, &dense));
        const uvc_status r = solve_ipm(dense, K, N, penalty_dev, mu_min, t_max, tol, max_iter, t_out_dev,
                                       sigma_out_dev, y_out_dev, info, st);
        (void)hipFree(dense);
        return r;
    } catch (const std::exception& e) {
        return fail(UVC_ENOMEM, std::string("host exception: ") + e.what());
    }
}
