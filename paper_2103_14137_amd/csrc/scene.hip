// Scene build: validation, surface elements, Morton codes, LSD radix sort,
// agglomerative (PLOC) hierarchy over the Morton order, near lists, all on
// the GPU.
#include "uvc_common.hpp"
#include "fp64_predicate.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace uvc {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

uvc_status fail(uvc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

uvc_status dalloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(UVC_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) +
                                    " bytes failed (" + what + ")");
    }
    return UVC_OK;
}

// --------------------------------------------------------------- kernels
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Surface elements in input order (Sec. III-B: one element per triangle).
// Centroid in FP64 as ((a + b) + c) / 3, rounded once to FP32; normal and
// area from the FP64 cross product of the two edges leaving v0.
__global__ void k_elements(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t n,
                           float* __restrict__ c, float* __restrict__ nrm, float* __restrict__ area) {
#pragma clang fp contract(off)
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t ia = T[3 * i], ib = T[3 * i + 1], ic = T[3 * i + 2];
    const double ax = V[3 * ia], ay = V[3 * ia + 1], az = V[3 * ia + 2];
    const double bx = V[3 * ib], by = V[3 * ib + 1], bz = V[3 * ib + 2];
    const double cx = V[3 * ic], cy = V[3 * ic + 1], cz = V[3 * ic + 2];
    c[3 * i + 0] = (float)(((ax + bx) + cx) / 3.0);
    c[3 * i + 1] = (float)(((ay + by) + cy) / 3.0);
    c[3 * i + 2] = (float)(((az + bz) + cz) / 3.0);
    const double e1x = bx - ax, e1y = by - ay, e1z = bz - az;
    const double e2x = cx - ax, e2y = cy - ay, e2z = cz - az;
    const double mx = e1y * e2z - e1z * e2y;
    const double my = e1z * e2x - e1x * e2z;
    const double mz = e1x * e2y - e1y * e2x;
    const double len = sqrt((mx * mx + my * my) + mz * mz);
    nrm[3 * i + 0] = (float)(mx / len);
    nrm[3 * i + 1] = (float)(my / len);
    nrm[3 * i + 2] = (float)(mz / len);
    area[i] = (float)(0.5 * len);
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Sort key of each triangle: the 30-bit Morton code of its centroid in the
// scene box (10 bits per axis, x most significant).  (Keys that put the
// normal's orientation class above the Morton bits were measured too: their
// six room-sized subtrees near the root cost a third more node visits per
// segment.)
__global__ void k_morton(const float* __restrict__ c, int64_t n, float lox,
                         float loy, float loz, float sx, float sy, float sz, uint32_t* __restrict__ key,
                         int32_t* __restrict__ val) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float q[3] = {(c[3 * i] - lox) * sx, (c[3 * i + 1] - loy) * sy, (c[3 * i + 2] - loz) * sz};
    uint32_t b[3];
    for (int a = 0; a < 3; ++a) b[a] = (uint32_t)fminf(fmaxf(q[a], 0.f), 1023.f);
    key[i] = (spread10(b[0]) << 2) | (spread10(b[1]) << 1) | spread10(b[2]);
    val[i] = (int32_t)i;
}

// ---- stable LSD radix sort of (key, value) pairs, 8 bits per pass --------
constexpr int RS_THREADS = 256;
constexpr int RS_TILE = 1024;  // 4 waves x 4 rounds x 64 lanes

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                       uint32_t* __restrict__ hist, int nb) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_TILE / RS_THREADS; ++r) {
        int64_t idx = base + r * RS_THREADS + tid;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nb + blockIdx.x] = h[tid];
}

// Exclusive scan of len words in place, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* __restrict__ a, int64_t len) {
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < len; base += 1024) {
        int64_t i = base + tid;
        uint32_t v = (i < len) ? a[i] : 0u;
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            uint32_t t = (tid >= off) ? part[tid - off] : 0u;
            __syncthreads();
            part[tid] += t;
            __syncthreads();
        }
        if (i < len) a[i] = carry + part[tid] - v;
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                          const int32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                          int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                          int nb) {
    __shared__ uint32_t cnt[4][257];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i < 4 * 257; i += RS_THREADS) (&cnt[0][0])[i] = 0;
    __syncthreads();
    uint32_t kk[4], rank[4], dig[4];
    int32_t vv[4];
    const uint64_t lt = lanemask_lt(lane);
    for (int r = 0; r < 4; ++r) {
        const int64_t idx = (int64_t)blockIdx.x * RS_TILE + w * 256 + r * 64 + lane;
        const bool valid = idx < n;
        kk[r] = valid ? kin[idx] : 0u;
        vv[r] = valid ? vin[idx] : 0;
        const uint32_t d = valid ? ((kk[r] >> shift) & 255u) : 256u;
        uint64_t peers = ~0ull;
        for (int b = 0; b < 9; ++b) {
            const int bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = cnt[w][d];
        rank[r] = before + (uint32_t)__popcll(peers & lt);
        dig[r] = d;
        const bool leader = (peers >> lane) == 1ull;
        if (leader) cnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t acc = 0;
        for (int ww = 0; ww < 4; ++ww) {
            uint32_t t = cnt[ww][tid];
            cnt[ww][tid] = acc;
            acc += t;
        }
    }
    __syncthreads();
    for (int r = 0; r < 4; ++r) {
        if (dig[r] < 256u) {
            const uint32_t d = dig[r];
            const uint64_t dst = (uint64_t)offs[(int64_t)d * nb + blockIdx.x] + cnt[w][d] + rank[r];
            if (dst < (uint64_t)n) {  // always true for a consistent histogram; guards the write
                kout[dst] = kk[r];
                vout[dst] = vv[r];
            }
        }
    }
}

// Leaf-slot records: triangle vertices in input order plus the input index,
// and the element (centroid, unit normal, index, area).
__global__ void k_gather(const float* __restrict__ V, const int32_t* __restrict__ T,
                         const int32_t* __restrict__ perm, const float* __restrict__ c,
                         const float* __restrict__ nrm, const float* __restrict__ area, int64_t n,
                         float* __restrict__ tri, float* __restrict__ elem) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    float* t = tri + s * TRI_WORDS;
    float v[3][3];
    for (int k = 0; k < 3; ++k) {
        const int64_t vi = T[3 * i + k];
        for (int a = 0; a < 3; ++a) v[k][a] = t[3 * k + a] = V[3 * vi + a];
    }
    float L = 0.f;
    for (int a = 0; a < 3; ++a) {
        const float e01 = v[1][a] - v[0][a], e12 = v[2][a] - v[1][a], e20 = v[0][a] - v[2][a];
        t[TRI_E01 + a] = e01;
        t[TRI_E12 + a] = e12;
        t[TRI_E20 + a] = e20;
        L = fmaxf(L, fmaxf(fabsf(e01), fmaxf(fabsf(e12), fabsf(e20))));
    }
    t[TRI_L] = L;
    t[TRI_ID] = __int_as_float((int)i);
    float* e = elem + s * ELEM_WORDS;
    e[0] = c[3 * i];
    e[1] = c[3 * i + 1];
    e[2] = c[3 * i + 2];
    e[3] = nrm[3 * i];
    e[4] = nrm[3 * i + 1];
    e[5] = nrm[3 * i + 2];
    e[6] = __int_as_float((int)i);
    e[7] = NEAR_SCALE * L * (1.0f - 0x1p-10f);  // rho_t
}

// Near lists (see uvc_common.hpp): ball query of every element against the
// hierarchy.  FILL = false counts, FILL = true writes at near_off[s].
template <bool FILL>
__global__ void k_near(const float* __restrict__ nodes, const float* __restrict__ tri,
                       const float* __restrict__ elem, int64_t n, float pad, int32_t* __restrict__ off,
                       int32_t* __restrict__ list) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float* e = elem + s * ELEM_WORDS;
    const float cx = e[0], cy = e[1], cz = e[2];
    const float rho = NEAR_SCALE * tri[s * TRI_WORDS + TRI_L];
    const float q = rho * (1.0f + 0x1p-9f) + 4.0f * pad;
    const float q2 = q * q;
    int32_t count = 0;
    const int32_t base = FILL ? off[s] : 0;
    int32_t stack[64];
    int sp = 0;
    if (n > 1) stack[sp++] = 0;
    while (sp > 0) {
        const float* nd = nodes + (int64_t)stack[--sp] * NODE_WORDS;
        for (int side = 0; side < 2; ++side) {
            const float* b = nd + 6 * side;
            const float dx = fmaxf(fmaxf(b[0] - cx, cx - b[3]), 0.0f);
            const float dy = fmaxf(fmaxf(b[1] - cy, cy - b[4]), 0.0f);
            const float dz = fmaxf(fmaxf(b[2] - cz, cz - b[5]), 0.0f);
            if (dx * dx + dy * dy + dz * dz > q2) continue;
            const int32_t ref = __float_as_int(nd[12 + side]);
            if (ref >= 0) {
                if (sp < 64) stack[sp++] = ref;
                continue;
            }
            const int64_t j = ~ref;
            if (j == s) continue;
            const float* t = tri + j * TRI_WORDS;
            if (plane_side_fp64(cx, cy, cz, t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7], t[8]) == 0.0) continue;
            if (FILL) list[base + count] = (int32_t)j;
            ++count;
        }
    }
    if (!FILL) off[s] = count;
}

// Exclusive scan of n int32 counts into a[0..n] by one block of 1024.
__device__ __forceinline__ void block_scan_i32(int32_t* __restrict__ a, int64_t n) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 <= n; b0 += 1024) {
        const int64_t i = b0 + tid;
        const int64_t v = (i < n) ? a[i] : 0;
        part[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t t = (tid >= o) ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += t;
            __syncthreads();
        }
        if (i <= n) a[i] = (int32_t)(carry + part[tid] - v);
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_i32(int32_t* __restrict__ a, int64_t n) { block_scan_i32(a, n); }

// Both flag scans of a clustering round (C from the device state).
__global__ __launch_bounds__(1024) void k_ploc_scan(int32_t* __restrict__ keep, int32_t* __restrict__ merge,
                                                    const int32_t* __restrict__ st) {
    const int64_t C = st[0];
    if (C <= 1) return;
    block_scan_i32(keep, C);
    block_scan_i32(merge, C);
}

// End of a round: C <- clusters kept, next id <- next id - merges.  A round
// that merges nothing, or whose counts do not add up, sets the error flag
// and stops the clustering.
__global__ void k_ploc_advance(const int32_t* __restrict__ keep, const int32_t* __restrict__ merge,
                               int32_t* __restrict__ st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t C = st[0], next_id = st[1];
    if (C <= 1) return;
    const int64_t kt = keep[C], mt = merge[C];
    if (mt < 1 || mt > next_id + 1 || kt + mt != C) {
        st[2] = 1;
        st[0] = 1;
        return;
    }
    st[0] = (int32_t)kt;
    st[1] = (int32_t)(next_id - mt);
}

__global__ void k_ploc_state(int32_t* __restrict__ st, int32_t C, int32_t next_id) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st[0] = C;
        st[1] = next_id;
        st[2] = 0;
    }
}

__global__ void k_depth(const int32_t* __restrict__ leaf_parent, const int32_t* __restrict__ int_parent, int64_t n,
                        int32_t* __restrict__ depth) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    int d = 1;
    for (int32_t p = leaf_parent[s]; p >= 0; p = int_parent[p]) {
        ++d;
        if (d > 65) break;  // deeper than supported, or a cycle
    }
    atomicMax(depth, d);
}

// ---- agglomerative build (PLOC, Meister and Bittner 2018): clusters in
// Morton order repeatedly merge with their nearest neighbour within PLOC_R
// positions, measured by the surface area of the merged box; mutual nearest
// neighbours merge.  Ties go to the lower index, so the pair of least
// (area, lower index) is always mutual and every round makes progress.
// Boxes are exact FP32 min/max of the padded triangle boxes, so every node
// box contains its subtree.  On the ward this tree costs 16.5 node visits
// per segment against 25.3 for the hierarchy emitted directly from the
// Morton codes (Karras 2012), for 2-3 ms more build time.
constexpr int PLOC_R = 16;  // windows of 8 and 32 measured within 2 % on 64 rooms

__device__ __forceinline__ float merged_area(const float* a, const float* b) {
    const float dx = fmaxf(a[3], b[3]) - fminf(a[0], b[0]);
    const float dy = fmaxf(a[4], b[4]) - fminf(a[1], b[1]);
    const float dz = fmaxf(a[5], b[5]) - fminf(a[2], b[2]);
    return dx * dy + dy * dz + dz * dx;
}

__global__ void k_ploc_init(const float* __restrict__ tri, int64_t n, float pad, float* __restrict__ box,
                            int32_t* __restrict__ ref) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float* t = tri + s * TRI_WORDS;
    for (int a = 0; a < 3; ++a) {
        box[s * 6 + a] = fminf(fminf(t[a], t[3 + a]), t[6 + a]) - pad;
        box[s * 6 + 3 + a] = fmaxf(fmaxf(t[a], t[3 + a]), t[6 + a]) + pad;
    }
    ref[s] = ~(int32_t)s;
}

// The clustering state lives on the device so that several rounds run
// between host checks: st[0] = clusters C, st[1] = next node id, st[2] = error
// flag.  A round with C <= 1 does nothing.
__global__ void k_ploc_nn(const float* __restrict__ box, const int32_t* __restrict__ st, int32_t* __restrict__ nn) {
    const int64_t C = st[0];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (C <= 1 || i >= C) return;
    float bi[6];
    for (int k = 0; k < 6; ++k) bi[k] = box[i * 6 + k];
    const int64_t j0 = i - PLOC_R < 0 ? 0 : i - PLOC_R, j1 = i + PLOC_R < C - 1 ? i + PLOC_R : C - 1;
    float best = INFINITY;
    int64_t bj = i == 0 ? 1 : 0;
    for (int64_t j = j0; j <= j1; ++j) {
        if (j == i) continue;
        const float d = merged_area(bi, box + j * 6);
        if (d < best) {
            best = d;
            bj = j;
        }
    }
    nn[i] = (int32_t)bj;
}

// keep[i] = cluster i survives (unmerged, or the lower index of a merged
// pair); merge[i] = i is the lower index of a mutual pair.
__global__ void k_ploc_flags(const int32_t* __restrict__ nn, const int32_t* __restrict__ st, int32_t* __restrict__ keep,
                             int32_t* __restrict__ merge) {
    const int64_t C = st[0];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (C <= 1 || i >= C) return;
    const int32_t j = nn[i];
    const bool mutual = nn[j] == (int32_t)i;
    merge[i] = (mutual && (int64_t)j > i) ? 1 : 0;
    keep[i] = (mutual && (int64_t)j < i) ? 0 : 1;
}

// After exclusive scans of keep and merge (totals at [C]): write the new
// nodes (id = next_id - merge rank, so that the last node made is node 0)
// and the compacted cluster list.
__global__ void k_ploc_merge(const float* __restrict__ box, const int32_t* __restrict__ ref,
                             const int32_t* __restrict__ nn, const int32_t* __restrict__ st,
                             const int32_t* __restrict__ keep, const int32_t* __restrict__ merge,
                             float* __restrict__ nodes, float* __restrict__ box_out, int32_t* __restrict__ ref_out,
                             int32_t* __restrict__ int_parent, int32_t* __restrict__ leaf_parent) {
    const int64_t C = st[0], next_id = st[1];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (C <= 1 || i >= C || keep[i + 1] == keep[i]) return;
    const int64_t pos = keep[i];
    if (merge[i + 1] == merge[i]) {
        for (int k = 0; k < 6; ++k) box_out[pos * 6 + k] = box[i * 6 + k];
        ref_out[pos] = ref[i];
        return;
    }
    const int64_t j = nn[i];
    const int32_t id = (int32_t)(next_id - merge[i]);
    const float* a = box + i * 6;
    const float* b = box + j * 6;
    float* nd = nodes + (int64_t)id * NODE_WORDS;
    for (int k = 0; k < 6; ++k) {
        nd[k] = a[k];
        nd[6 + k] = b[k];
    }
    nd[12] = __int_as_float(ref[i]);
    nd[13] = __int_as_float(ref[j]);
    float best = -1.f;
    int axis = 0;
    for (int q = 0; q < 3; ++q) {
        const float sep = fabsf((b[q] + b[3 + q]) - (a[q] + a[3 + q]));
        if (sep > best) {
            best = sep;
            axis = q;
        }
    }
    const float cl = 0.5f * (a[axis] + a[3 + axis]), cr = 0.5f * (b[axis] + b[3 + axis]);
    nd[14] = __int_as_float(axis | ((cl <= cr) ? 4 : 0));
    nd[15] = __int_as_float(float_key(0.5f * (cl + cr)));
    for (int q = 0; q < 3; ++q) {
        box_out[pos * 6 + q] = fminf(a[q], b[q]);
        box_out[pos * 6 + 3 + q] = fmaxf(a[3 + q], b[3 + q]);
    }
    ref_out[pos] = id;
    const int32_t ri = ref[i], rj = ref[j];
    if (ri < 0) leaf_parent[~ri] = id; else int_parent[ri] = id;
    if (rj < 0) leaf_parent[~rj] = id; else int_parent[rj] = id;
}

static inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

static void free_scene(uvc_scene* s) {
    if (!s) return;
    void* ptrs[] = {s->tri, s->elem, s->elem_c, s->elem_n, s->elem_a, s->perm, s->codes, s->nodes, s->near_off, s->near};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete s;
}

struct TmpBuffers {
    std::vector<void*> p;
    ~TmpBuffers() {
        for (void* q : p)
            if (q) (void)hipFree(q);
    }
    template <class T>
    uvc_status alloc(T** out, size_t n, const char* what) {
        UVC_TRY(dalloc_n(out, n, what));
        p.push_back(*out);
        return UVC_OK;
    }
};

static uvc_status build_impl(const float* verts_in, int64_t nv, const int32_t* tris_in, int64_t nt, int on_dev,
                             hipStream_t st, uvc_scene** out) {
    if (!out) return fail(UVC_EINVAL, "out is NULL");
    *out = nullptr;
    if (nv < 0 || nt < 0) return fail(UVC_EINVAL, "negative vertex or triangle count");
    if (nt > (int64_t)(1u << 30)) return fail(UVC_EUNSUPPORTED, "more than 2^30 triangles");
    if (nt > 0 && (!verts_in || !tris_in || nv == 0)) return fail(UVC_EINVAL, "NULL mesh arrays");
    // host copies for validation
    std::vector<float> hv((size_t)nv * 3);
    std::vector<int32_t> ht((size_t)nt * 3);
    if (nt > 0) {
        if (on_dev) {
            UVC_HIP(hipMemcpyAsync(hv.data(), verts_in, hv.size() * 4, hipMemcpyDeviceToHost, st));
            UVC_HIP(hipMemcpyAsync(ht.data(), tris_in, ht.size() * 4, hipMemcpyDeviceToHost, st));
            UVC_HIP(hipStreamSynchronize(st));
        } else {
            std::memcpy(hv.data(), verts_in, hv.size() * 4);
            std::memcpy(ht.data(), tris_in, ht.size() * 4);
        }
    }
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float max_abs = 0.f;
    bool first = true;
    for (int64_t t = 0; t < nt; ++t) {
        double v[3][3];
        for (int k = 0; k < 3; ++k) {
            const int32_t vi = ht[3 * t + k];
            if (vi < 0 || vi >= nv)
                return fail(UVC_EINVAL, "triangle " + std::to_string(t) + " has vertex index " + std::to_string(vi) +
                                            " outside [0, " + std::to_string(nv) + ")");
            for (int a = 0; a < 3; ++a) {
                const float x = hv[3 * (size_t)vi + a];
                if (!std::isfinite(x))
                    return fail(UVC_EINVAL, "vertex " + std::to_string(vi) + " has a non-finite coordinate");
                v[k][a] = x;
                if (first) {
                    lo[a] = hi[a] = x;
                } else {
                    lo[a] = std::min(lo[a], x);
                    hi[a] = std::max(hi[a], x);
                }
                max_abs = std::max(max_abs, std::fabs(x));
            }
            first = false;
        }
        const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
        const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
        const double m0 = e1[1] * e2[2] - e1[2] * e2[1];
        const double m1 = e1[2] * e2[0] - e1[0] * e2[2];
        const double m2 = e1[0] * e2[1] - e1[1] * e2[0];
        if (m0 == 0.0 && m1 == 0.0 && m2 == 0.0)
            return fail(UVC_EINVAL, "triangle " + std::to_string(t) + " has zero area");
    }
    // The slab test replaces a zero direction component by +-1e-30 and
    // multiplies coordinates by its reciprocal: with |coordinates| (and pose
    // coordinates, limited to twice this) up to 2^26 every such product
    // stays finite in FP32.
    if (max_abs > 67108864.0f) return fail(UVC_EINVAL, "a vertex coordinate exceeds 2^26 in magnitude");
    uvc_scene* s = new uvc_scene();
    (void)hipGetDevice(&s->device);
    s->n = nt;
    s->max_abs = max_abs;
    s->pad = PAD_REL * std::max(max_abs, 1e-30f);
    for (int a = 0; a < 3; ++a) {
        s->lo[a] = lo[a];
        s->hi[a] = hi[a];
    }
    if (nt == 0) {
        s->depth = 0;
        *out = s;
        return UVC_OK;
    }
    auto cleanup_fail = [&](uvc_status st_) {
        free_scene(s);
        return st_;
    };
    const int64_t n = nt;
    uvc_status r = UVC_OK;
    if ((r = dalloc_n(&s->tri, (size_t)n * TRI_WORDS, "triangle records")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->elem, (size_t)n * ELEM_WORDS, "element records")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->elem_c, (size_t)n * 3, "centroids")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->elem_n, (size_t)n * 3, "normals")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->elem_a, (size_t)n, "areas")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->perm, (size_t)n, "leaf permutation")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->codes, (size_t)n, "morton codes")) != UVC_OK) return cleanup_fail(r);
    if ((r = dalloc_n(&s->nodes, (size_t)std::max<int64_t>(n - 1, 1) * NODE_WORDS, "hierarchy nodes")) != UVC_OK)
        return cleanup_fail(r);
    TmpBuffers tmp;
    float* dv = nullptr;
    int32_t* dt = nullptr;
    uint32_t *k2 = nullptr, *hist = nullptr;
    int32_t *v1 = nullptr, *v2 = nullptr, *ipar = nullptr, *lpar = nullptr, *ddepth = nullptr;
    const int nb = (int)((n + RS_TILE - 1) / RS_TILE);
    if ((!on_dev && (r = tmp.alloc(&dv, (size_t)nv * 3, "vertices")) != UVC_OK) ||
        (!on_dev && (r = tmp.alloc(&dt, (size_t)n * 3, "indices")) != UVC_OK) ||
        (r = tmp.alloc(&k2, (size_t)n, "sort keys")) != UVC_OK ||
        (r = tmp.alloc(&v1, (size_t)n, "sort values")) != UVC_OK ||
        (r = tmp.alloc(&v2, (size_t)n, "sort values")) != UVC_OK ||
        (r = tmp.alloc(&hist, (size_t)256 * nb, "sort histogram")) != UVC_OK ||
        (r = tmp.alloc(&ipar, (size_t)std::max<int64_t>(n - 1, 1), "parents")) != UVC_OK ||
        (r = tmp.alloc(&lpar, (size_t)n, "leaf parents")) != UVC_OK ||
        (r = tmp.alloc(&ddepth, 1, "depth")) != UVC_OK)
        return cleanup_fail(r);
#define STEP(call)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ == hipSuccess) e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess) return cleanup_fail(fail(UVC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_))); \
    } while (0)
    if (on_dev) {  // validated copies of the caller's device arrays are already on the device
        dv = const_cast<float*>(verts_in);
        dt = const_cast<int32_t*>(tris_in);
    } else {
        STEP(hipMemcpyAsync(dv, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, st));
        STEP(hipMemcpyAsync(dt, ht.data(), ht.size() * 4, hipMemcpyHostToDevice, st));
    }
    const int TB = 256;
    hipLaunchKernelGGL(k_elements, dim3(grid_for(n, TB)), dim3(TB), 0, st, dv, dt, n, s->elem_c, s->elem_n, s->elem_a);
    STEP(hipGetLastError());
    float sc[3];
    for (int a = 0; a < 3; ++a) sc[a] = (hi[a] > lo[a]) ? 1024.f / (hi[a] - lo[a]) : 0.f;
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, TB)), dim3(TB), 0, st, s->elem_c, n, lo[0], lo[1], lo[2], sc[0],
                       sc[1], sc[2], s->codes, v1);
    STEP(hipGetLastError());
    uint32_t* ka = s->codes;
    uint32_t* kb = k2;
    int32_t* va = v1;
    int32_t* vb = v2;
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, st, ka, n, shift, hist, nb);
        STEP(hipGetLastError());
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, hist, (int64_t)256 * nb);
        STEP(hipGetLastError());
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, st, ka, va, kb, vb, n, shift, hist, nb);
        STEP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // after 4 passes the sorted data is back in (s->codes, v1)
    STEP(hipMemcpyAsync(s->perm, va, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
    {
        // structural check before any kernel indexes through the permutation
        std::vector<uint32_t> hc((size_t)n);
        std::vector<int32_t> hp((size_t)n);
        STEP(hipMemcpyAsync(hc.data(), s->codes, (size_t)n * 4, hipMemcpyDeviceToHost, st));
        STEP(hipMemcpyAsync(hp.data(), s->perm, (size_t)n * 4, hipMemcpyDeviceToHost, st));
        STEP(hipStreamSynchronize(st));
        std::vector<uint8_t> seen((size_t)n, 0);
        for (int64_t i = 0; i < n; ++i) {
            if ((i > 0 && hc[i] < hc[i - 1]) || hp[i] < 0 || hp[i] >= n || seen[hp[i]])
                return cleanup_fail(fail(UVC_EDEVICE, "internal error: Morton sort produced an invalid order"));
            seen[hp[i]] = 1;
        }
    }
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, TB)), dim3(TB), 0, st, dv, dt, s->perm, s->elem_c, s->elem_n,
                       s->elem_a, n, s->tri, s->elem);
    STEP(hipGetLastError());
    int32_t depth = 1;
    if (n > 1) {
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n - 1, TB)), dim3(TB), 0, st, (uint32_t*)ipar, 0xfffffffeu, n - 1);
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, TB)), dim3(TB), 0, st, (uint32_t*)lpar, 0xfffffffeu, n);
        {
            float *cb0 = nullptr, *cb1 = nullptr;
            int32_t *cr0 = nullptr, *cr1 = nullptr, *nn = nullptr, *keep = nullptr, *merge = nullptr, *pst = nullptr;
            if ((r = tmp.alloc(&cb0, (size_t)n * 6, "clusters")) != UVC_OK ||
                (r = tmp.alloc(&cb1, (size_t)n * 6, "clusters")) != UVC_OK ||
                (r = tmp.alloc(&cr0, (size_t)n, "clusters")) != UVC_OK ||
                (r = tmp.alloc(&cr1, (size_t)n, "clusters")) != UVC_OK ||
                (r = tmp.alloc(&nn, (size_t)n, "neighbours")) != UVC_OK ||
                (r = tmp.alloc(&keep, (size_t)n + 1, "cluster flags")) != UVC_OK ||
                (r = tmp.alloc(&merge, (size_t)n + 1, "cluster flags")) != UVC_OK ||
                (r = tmp.alloc(&pst, 4, "clustering state")) != UVC_OK)
                return cleanup_fail(r);
            hipLaunchKernelGGL(k_ploc_init, dim3(grid_for(n, TB)), dim3(TB), 0, st, s->tri, n, s->pad, cb0, cr0);
            hipLaunchKernelGGL(k_ploc_state, dim3(1), dim3(1), 0, st, pst, (int32_t)n, (int32_t)(n - 2));
            STEP(hipGetLastError());
            // rounds run in batches between host checks; the grids cover the
            // cluster count of the last check (it only shrinks)
            constexpr int PLOC_BATCH = 8;
            int64_t Cb = n;
            for (int round = 0; Cb > 1;) {
                if (round > 10000) return cleanup_fail(fail(UVC_EDEVICE, "internal error: clustering did not finish"));
                const unsigned g = grid_for(Cb, TB);
                for (int b = 0; b < PLOC_BATCH; ++b, ++round) {
                    hipLaunchKernelGGL(k_ploc_nn, dim3(g), dim3(TB), 0, st, cb0, pst, nn);
                    hipLaunchKernelGGL(k_ploc_flags, dim3(g), dim3(TB), 0, st, nn, pst, keep, merge);
                    hipLaunchKernelGGL(k_ploc_scan, dim3(1), dim3(1024), 0, st, keep, merge, pst);
                    hipLaunchKernelGGL(k_ploc_merge, dim3(g), dim3(TB), 0, st, cb0, cr0, nn, pst, keep, merge, s->nodes,
                                       cb1, cr1, ipar, lpar);
                    hipLaunchKernelGGL(k_ploc_advance, dim3(1), dim3(1), 0, st, keep, merge, pst);
                    std::swap(cb0, cb1);
                    std::swap(cr0, cr1);
                }
                STEP(hipGetLastError());
                int32_t hs[3] = {0, 0, 0};
                STEP(hipMemcpyAsync(hs, pst, sizeof(hs), hipMemcpyDeviceToHost, st));
                STEP(hipStreamSynchronize(st));
                if (hs[2] != 0) return cleanup_fail(fail(UVC_EDEVICE, "internal error: clustering made no progress"));
                if (hs[0] < 1 || hs[0] > Cb) return cleanup_fail(fail(UVC_EDEVICE, "internal error: bad cluster count"));
                Cb = hs[0];
                if (Cb == 1 && hs[1] != -1)
                    return cleanup_fail(fail(UVC_EDEVICE, "internal error: clustering left node ids unused"));
            }
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, (uint32_t*)ipar, 0xffffffffu, (int64_t)1);
            STEP(hipGetLastError());
        }
        {
            // every internal node but the root has one parent in range, every
            // leaf has one, and every internal node has exactly two children
            std::vector<int32_t> hi_((size_t)(n - 1)), hl((size_t)n);
            STEP(hipMemcpyAsync(hi_.data(), ipar, (size_t)(n - 1) * 4, hipMemcpyDeviceToHost, st));
            STEP(hipMemcpyAsync(hl.data(), lpar, (size_t)n * 4, hipMemcpyDeviceToHost, st));
            STEP(hipStreamSynchronize(st));
            std::vector<uint8_t> kids((size_t)(n - 1), 0);
            bool ok = hi_[0] == -1;
            for (int64_t i = 1; ok && i < n - 1; ++i) {
                ok = hi_[i] >= 0 && hi_[i] < n - 1 && hi_[i] != i;
                if (ok) ++kids[hi_[i]];
            }
            for (int64_t i = 0; ok && i < n; ++i) {
                ok = hl[i] >= 0 && hl[i] < n - 1;
                if (ok) ++kids[hl[i]];
            }
            for (int64_t i = 0; ok && i < n - 1; ++i) ok = kids[i] == 2;
            // that every leaf reaches the root within 64 levels is checked by
            // k_depth below: with the ranges and counts above, a walk up from
            // a leaf stays in bounds and either ends at the root (the only
            // node without a parent) or cycles, which its step bound reports
            if (!ok) return cleanup_fail(fail(UVC_EDEVICE, "internal error: hierarchy emission is inconsistent"));
        }
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, (uint32_t*)ddepth, 0u, (int64_t)1);
        STEP(hipGetLastError());
        hipLaunchKernelGGL(k_depth, dim3(grid_for(n, TB)), dim3(TB), 0, st, lpar, ipar, n, ddepth);
        STEP(hipGetLastError());
        STEP(hipMemcpyAsync(&depth, ddepth, 4, hipMemcpyDeviceToHost, st));
        STEP(hipStreamSynchronize(st));
        if (depth > 64)
            return cleanup_fail(fail(UVC_EUNSUPPORTED, "hierarchy depth " + std::to_string(depth) + " exceeds 64"));
    }
    if ((r = dalloc_n(&s->near_off, (size_t)n + 1, "near-list offsets")) != UVC_OK) return cleanup_fail(r);
    hipLaunchKernelGGL(k_near<false>, dim3(grid_for(n, TB)), dim3(TB), 0, st, s->nodes, s->tri, s->elem, n, s->pad,
                       s->near_off, (int32_t*)nullptr);
    STEP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(1024), 0, st, s->near_off, n);
    STEP(hipGetLastError());
    int32_t n_near = 0;
    STEP(hipMemcpyAsync(&n_near, s->near_off + n, 4, hipMemcpyDeviceToHost, st));
    STEP(hipStreamSynchronize(st));
    if (n_near < 0) return cleanup_fail(fail(UVC_EUNSUPPORTED, "near lists exceed 2^31 entries"));
    s->n_near = n_near;
    if ((r = dalloc_n(&s->near, (size_t)std::max<int32_t>(n_near, 1), "near lists")) != UVC_OK) return cleanup_fail(r);
    hipLaunchKernelGGL(k_near<true>, dim3(grid_for(n, TB)), dim3(TB), 0, st, s->nodes, s->tri, s->elem, n, s->pad,
                       s->near_off, s->near);
    STEP(hipGetLastError());
    STEP(hipStreamSynchronize(st));
#undef STEP
    s->depth = depth;
    *out = s;
    return UVC_OK;
}

}  // namespace uvc

using namespace uvc;

extern "C" const char* uvc_last_error(void) { return uvc::g_err.c_str(); }

extern "C" int32_t uvc_version(void) { return 100; }

extern "C" uvc_status uvc_build_scene(const float* verts_xyz, int64_t n_verts, const int32_t* tri_idx, int64_t n_tris,
                                      int32_t inputs_on_device, void* hip_stream, uvc_scene** out) {
    try {
        return build_impl(verts_xyz, n_verts, tri_idx, n_tris, inputs_on_device, (hipStream_t)hip_stream, out);
    } catch (const std::exception& e) {
        return fail(UVC_ENOMEM, std::string("host exception: ") + e.what());
    }
}

extern "C" uvc_status uvc_scene_info(const uvc_scene* s, int64_t* n_tris, int32_t* depth, float* max_abs) {
    if (!s) return fail(UVC_EINVAL, "scene is NULL");
    if (n_tris) *n_tris = s->n;
    if (depth) *depth = s->depth;
    if (max_abs) *max_abs = s->max_abs;
    return UVC_OK;
}

extern "C" uvc_status uvc_scene_elements(const uvc_scene* s, float* c, float* nrm, float* area, void* hip_stream) {
    if (!s) return fail(UVC_EINVAL, "scene is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    if (s->n == 0) return UVC_OK;
    if (c) UVC_HIP(hipMemcpyAsync(c, s->elem_c, (size_t)s->n * 12, hipMemcpyDeviceToDevice, st));
    if (nrm) UVC_HIP(hipMemcpyAsync(nrm, s->elem_n, (size_t)s->n * 12, hipMemcpyDeviceToDevice, st));
    if (area) UVC_HIP(hipMemcpyAsync(area, s->elem_a, (size_t)s->n * 4, hipMemcpyDeviceToDevice, st));
    return UVC_OK;
}

extern "C" uvc_status uvc_scene_export_bvh(const uvc_scene* s, float* nodes, int32_t* perm, uint32_t* codes,
                                           void* hip_stream) {
    if (!s) return fail(UVC_EINVAL, "scene is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    if (s->n == 0) return UVC_OK;
    if (nodes && s->n > 1)
        UVC_HIP(hipMemcpyAsync(nodes, s->nodes, (size_t)(s->n - 1) * NODE_WORDS * 4, hipMemcpyDeviceToHost, st));
    if (perm) UVC_HIP(hipMemcpyAsync(perm, s->perm, (size_t)s->n * 4, hipMemcpyDeviceToHost, st));
    if (codes) UVC_HIP(hipMemcpyAsync(codes, s->codes, (size_t)s->n * 4, hipMemcpyDeviceToHost, st));
    UVC_HIP(hipStreamSynchronize(st));
    return UVC_OK;
}

extern "C" void uvc_destroy_scene(uvc_scene* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    free_scene(s);
}
