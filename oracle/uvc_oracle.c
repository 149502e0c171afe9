/*
 * CPU oracle for the irradiance matrix -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, brute-force FP64 evaluation of what the paper defines:
 *   - one surface element per mesh triangle (Sec. III-B, discrete
 *     formulation), sampled at its centroid;
 *   - the inverse-square, cosine-weighted point-source irradiance of Sec. IV-C
 *     (equation "inverse square law"), counted only when the element faces the
 *     source with a strictly positive cosine and nothing else lies on the
 *     segment between them;
 *   - extended lamps as several point sources whose contributions add
 *     (Sec. IV-C, "Non-Point Light Sources").
 * Every (pose, source, element) segment is tested against every triangle.
 * Only the test suite, the smoke check and the benchmark's CPU baseline may
 * load this library; the product path never does.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no contraction, no reassociation: every FP64 operation below is one IEEE
 * operation in the written order).
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

typedef struct { double x, y, z; } d3;

static d3 ld(const float* p) { d3 r = {(double)p[0], (double)p[1], (double)p[2]}; return r; }
static d3 sub(d3 a, d3 b) { d3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static d3 cross(d3 a, d3 b) {
    d3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static double dot(d3 a, d3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }

/* Surface elements.  Centroid: ((a + b) + c) / 3 in FP64, rounded once to
 * FP32 -- this FP32 point is the element's sampling point, the target of its
 * occlusion segments.  m = (b - a) x (c - a) in FP64; unit normal m / |m|;
 * area |m| / 2. */
void oracle_elements(const float* verts, const int32_t* tris, int64_t n,
                     float* c32, double* n64, double* area64, double* m64)
{
    for (int64_t i = 0; i < n; ++i) {
        d3 a = ld(verts + 3 * (int64_t)tris[3 * i + 0]);
        d3 b = ld(verts + 3 * (int64_t)tris[3 * i + 1]);
        d3 c = ld(verts + 3 * (int64_t)tris[3 * i + 2]);
        c32[3 * i + 0] = (float)(((a.x + b.x) + c.x) / 3.0);
        c32[3 * i + 1] = (float)(((a.y + b.y) + c.y) / 3.0);
        c32[3 * i + 2] = (float)(((a.z + b.z) + c.z) / 3.0);
        d3 m = cross(sub(b, a), sub(c, a));
        double len = sqrt(dot(m, m));
        n64[3 * i + 0] = m.x / len;
        n64[3 * i + 1] = m.y / len;
        n64[3 * i + 2] = m.z / len;
        area64[i] = 0.5 * len;
        m64[3 * i + 0] = m.x;
        m64[3 * i + 1] = m.y;
        m64[3 * i + 2] = m.z;
    }
}

/* Front-facing test: <p - c, m> > 0, strict (the paper requires a strictly
 * positive inner product with the surface normal). */
static int front64(d3 p, d3 c, d3 m) { return dot(sub(p, c), m) > 0.0; }

/* Segment / triangle occlusion predicate.
 * The open segment O->T (0 < t < 1) meets the closed triangle v0 v1 v2 iff
 *  (1) O and T lie strictly on opposite sides of the triangle's plane, and
 *  (2) the line through O and T passes through the closed triangle: the three
 *      edge orientations D . ((vi - O) x (vj - O)) with D = T - O, taken for
 *      the edges (v1,v2), (v2,v0), (v0,v1), are not of mixed strict sign.
 * A degenerate triangle (m = 0) never occludes.  An edge shared by two
 * triangles enters them with opposite vertex order, so its orientation is
 * computed as exact negatives of each other and no segment slips between
 * the two triangles. */
static int hit64(d3 O, d3 T, d3 v0, d3 v1, d3 v2)
{
    d3 m = cross(sub(v1, v0), sub(v2, v0));
    double sO = dot(sub(O, v0), m);
    double sT = dot(sub(T, v0), m);
    if (!((sO > 0.0 && sT < 0.0) || (sO < 0.0 && sT > 0.0))) return 0;
    d3 D = sub(T, O);
    d3 a = sub(v0, O), b = sub(v1, O), c = sub(v2, O);
    double U = dot(D, cross(b, c));
    double V = dot(D, cross(c, a));
    double W = dot(D, cross(a, b));
    int neg = (U < 0.0) || (V < 0.0) || (W < 0.0);
    int pos = (U > 0.0) || (V > 0.0) || (W > 0.0);
    return !(neg && pos);
}

int oracle_hit(const float* O, const float* T, const float* v0, const float* v1, const float* v2)
{
    return hit64(ld(O), ld(T), ld(v0), ld(v1), ld(v2));
}

/* Reciprocal visibility test used by the invariant checks: is any triangle
 * other than `skip` hit by the open segment O->T? */
int oracle_segment_blocked(const float* verts, const int32_t* tris, int64_t n,
                           const float* O, const float* T, int64_t skip)
{
    d3 o = ld(O), t = ld(T);
    for (int64_t m = 0; m < n; ++m) {
        if (m == skip) continue;
        d3 v0 = ld(verts + 3 * (int64_t)tris[3 * m + 0]);
        d3 v1 = ld(verts + 3 * (int64_t)tris[3 * m + 1]);
        d3 v2 = ld(verts + 3 * (int64_t)tris[3 * m + 2]);
        if (hit64(o, t, v0, v1, v2)) return 1;
    }
    return 0;
}

/* Angular emission weight of a source (Sec. IV-C allows point sources with
 * their own emission pattern; the default is uniform, weight 1).  The
 * pattern is a table of n_prof >= 2 values at cos(theta) = -1 + 2 q /
 * (n_prof - 1), q = 0 .. n_prof - 1, interpolated linearly; theta is the
 * angle between the upward vertical through the source and the direction
 * from the source to the element. */
static double emission_weight(double cos_theta, int32_t n_prof, const float* prof)
{
    if (n_prof <= 0) return 1.0;
    double u = (cos_theta + 1.0) * 0.5 * (double)(n_prof - 1);
    if (u < 0.0) u = 0.0;
    if (u > (double)(n_prof - 1)) u = (double)(n_prof - 1);
    int q = (int)floor(u);
    if (q > n_prof - 2) q = n_prof - 2;
    double f = u - (double)q;
    return (double)prof[q] + f * ((double)prof[q + 1] - (double)prof[q]);
}

/* Irradiance entries for a list of (pose, element) pairs.
 *   poses: K x pose_dim floats (x, y) or (x, y, z); source j sits at
 *          (x, y, z + dz[j]) with the height sum taken in FP32 (z = 0 for
 *          pose_dim 2).
 *   E_out[p]   = sum over sources j (ascending) of
 *                P_j * w_j * max(0, <p_j - c, n>) / (4 pi |p_j - c|^3) * V_j
 *   vis_out[p] = bit j set iff V_j = 1: the source emits towards the
 *                element (hemisphere masks below), the element faces it, and
 *                nothing blocks the segment.
 * Emission pattern: w_j = emission_weight(cos theta) with the lamp's table
 * (n_prof = 0: w_j = 1).  A source whose bit is set in up_mask emits only
 * into the open half-space above its own height (element centroid z >
 * source z), one whose bit is set in down_mask only below it.
 * The element's own triangle is excluded from its occlusion test by index. */
int oracle_irradiance_pairs_lamp(const float* verts, const int32_t* tris, int64_t n,
                                 const float* poses, int64_t K, int32_t pose_dim,
                                 int32_t S, const float* dz, const float* power,
                                 int32_t n_prof, const float* prof, uint32_t up_mask, uint32_t down_mask,
                                 const int64_t* pk, const int64_t* pi, int64_t npairs,
                                 double* E_out, uint32_t* vis_out, int32_t nthreads)
{
    if (S < 1 || S > 32 || (pose_dim != 2 && pose_dim != 3)) return -1;
    if (n_prof == 1 || n_prof > 33 || (n_prof > 1 && !prof) || (up_mask & down_mask)) return -1;
    (void)K;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const double four_pi = 4.0 * M_PI;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < npairs; ++q) {
        int64_t k = pk[q], i = pi[q];
        d3 a = ld(verts + 3 * (int64_t)tris[3 * i + 0]);
        d3 b = ld(verts + 3 * (int64_t)tris[3 * i + 1]);
        d3 cc = ld(verts + 3 * (int64_t)tris[3 * i + 2]);
        float cf[3] = {(float)(((a.x + b.x) + cc.x) / 3.0),
                       (float)(((a.y + b.y) + cc.y) / 3.0),
                       (float)(((a.z + b.z) + cc.z) / 3.0)};
        d3 c = ld(cf);
        d3 m = cross(sub(b, a), sub(cc, a));
        double len = sqrt(dot(m, m));
        d3 nrm = {m.x / len, m.y / len, m.z / len};
        const float* pp = poses + pose_dim * k;
        float zb = (pose_dim == 3) ? pp[2] : 0.0f;
        double acc = 0.0;
        uint32_t bits = 0;
        for (int j = 0; j < S; ++j) {
            float pz = zb + dz[j]; /* FP32 sum */
            float pf[3] = {pp[0], pp[1], pz};
            d3 p = ld(pf);
            if (((up_mask >> j) & 1u) && !(c.z > p.z)) continue;
            if (((down_mask >> j) & 1u) && !(c.z < p.z)) continue;
            if (!front64(p, c, m)) continue;
            int blocked = 0;
            for (int64_t mm = 0; mm < n && !blocked; ++mm) {
                if (mm == i) continue;
                d3 v0 = ld(verts + 3 * (int64_t)tris[3 * mm + 0]);
                d3 v1 = ld(verts + 3 * (int64_t)tris[3 * mm + 1]);
                d3 v2 = ld(verts + 3 * (int64_t)tris[3 * mm + 2]);
                blocked = hit64(p, c, v0, v1, v2);
            }
            if (blocked) continue;
            d3 d = sub(p, c);
            double r2 = dot(d, d);
            double r = sqrt(r2);
            double s = dot(d, nrm);
            if (s < 0.0) s = 0.0;
            double w = emission_weight((c.z - p.z) / r, n_prof, prof);
            acc += (double)power[j] * w * s / (four_pi * r2 * r);
            bits |= 1u << j;
        }
        E_out[q] = acc;
        vis_out[q] = bits;
    }
    return 0;
}

/* The uniform lamp (weight 1, no hemisphere masks). */
int oracle_irradiance_pairs(const float* verts, const int32_t* tris, int64_t n,
                            const float* poses, int64_t K, int32_t pose_dim,
                            int32_t S, const float* dz, const float* power,
                            const int64_t* pk, const int64_t* pi, int64_t npairs,
                            double* E_out, uint32_t* vis_out, int32_t nthreads)
{
    return oracle_irradiance_pairs_lamp(verts, tris, n, poses, K, pose_dim, S, dz, power, 0, 0, 0u, 0u, pk, pi,
                                        npairs, E_out, vis_out, nthreads);
}

/* ---------------------------------------------------------------------------
 * Area-integrated irradiance (Sec. IV-C, the visibility-cube procedure).
 * Each source emits through the pixels of a cube around it: face f (axis
 * ax = f / 2, sign +1 for even f, -1 for odd f) holds R x R pixels over
 * (u, v) in [-1, 1]^2; pixel (a, b) spans u in [-1 + 2a/R, -1 + 2(a+1)/R]
 * (likewise v with b) and its centre direction has component ax = sign,
 * component (ax+1) mod 3 = u_c and component (ax+2) mod 3 = v_c.  Its
 * solid angle is the exact solid angle of that square on the plane at unit
 * distance, dOmega = F(u1,v1) - F(u0,v1) - F(u1,v0) + F(u0,v0) with
 * F(x, y) = atan2(x y, sqrt(1 + x^2 + y^2)).  The pixel carries the power
 * e = P_j w_j(cos theta) dOmega / (4 pi) (w_j: the emission table at the
 * centre direction, 1 for uniform emission; a hemisphere mask drops pixels
 * whose centre direction points into the masked half: d_z <= 0 for an
 * upward-only source, d_z >= 0 for a downward-only one).  The ray through
 * the pixel centre meets its closest triangle (smallest plane parameter
 * t > 0 among the closed triangles it passes through; equal t: the lower
 * index); that triangle collects e if the ray reaches its front side
 * (D . m < 0, m its normal; a back side keeps nothing).  The entry is the
 * collected power over the triangle's area, F_i / |s_i|.
 * amb_out counts, per (pose, triangle), pixels whose decision is close to
 * a tie: the ray passes within a relative 1e-5 of the edge of a triangle
 * at least as close as the winner (or of the winner), two hits lie within a
 * relative 1e-5 in t, or the winner is met within 1e-5 of edge-on; such a
 * pixel counts for the winner and for every such near triangle.  (Edge
 * closeness of a ray: the smallest |orientation| D . (p x q) over
 * |D| |p| |q| for the triangle's vertices p, q relative to the origin.)
 * power_out[k] = the power collected over all triangles for pose k. */
static double omega_corner(double x, double y) { return atan2(x * y, sqrt(1.0 + x * x + y * y)); }

int oracle_area_irradiance(const float* verts, const int32_t* tris, int64_t n,
                           const float* poses, int64_t K, int32_t pose_dim,
                           int32_t S, const float* dz, const float* power,
                           int32_t n_prof, const float* prof, uint32_t up_mask, uint32_t down_mask,
                           int32_t R, double* E_out, int32_t* amb_out, double* power_out, int32_t nthreads)
{
    if (S < 1 || S > 32 || (pose_dim != 2 && pose_dim != 3) || R < 1) return -1;
    if (n_prof == 1 || n_prof > 33 || (n_prof > 1 && !prof) || (up_mask & down_mask)) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const double four_pi = 4.0 * M_PI;
    const double rel = 1e-5;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < K; ++k) {
        double* F = E_out + k * n;
        int32_t* amb = amb_out + k * n;
        for (int64_t m = 0; m < n; ++m) { F[m] = 0.0; amb[m] = 0; }
        const float* pp = poses + pose_dim * k;
        float zb = (pose_dim == 3) ? pp[2] : 0.0f;
        double landed = 0.0;
        for (int j = 0; j < S; ++j) {
            float pz = zb + dz[j]; /* FP32 sum */
            float pf[3] = {pp[0], pp[1], pz};
            d3 O = ld(pf);
            for (int f = 0; f < 6; ++f) {
                int ax = f / 2;
                double sgn = (f % 2 == 0) ? 1.0 : -1.0;
                for (int a = 0; a < R; ++a) {
                    double u0 = -1.0 + 2.0 * a / R, u1 = -1.0 + 2.0 * (a + 1) / R, uc = 0.5 * (u0 + u1);
                    for (int b = 0; b < R; ++b) {
                        double v0 = -1.0 + 2.0 * b / R, v1 = -1.0 + 2.0 * (b + 1) / R, vc = 0.5 * (v0 + v1);
                        double dir[3];
                        dir[ax] = sgn;
                        dir[(ax + 1) % 3] = uc;
                        dir[(ax + 2) % 3] = vc;
                        d3 D = {dir[0], dir[1], dir[2]};
                        if (((up_mask >> j) & 1u) && !(D.z > 0.0)) continue;
                        if (((down_mask >> j) & 1u) && !(D.z < 0.0)) continue;
                        double dom = omega_corner(u1, v1) - omega_corner(u0, v1) - omega_corner(u1, v0)
                                     + omega_corner(u0, v0);
                        double dl = sqrt(dot(D, D));
                        double w = emission_weight(D.z / dl, n_prof, prof);
                        double e = (double)power[j] * w * dom / four_pi;
                        /* closest hit by brute force */
                        int64_t best = -1;
                        double tbest = INFINITY, dmbest = 0.0, grbest = 1.0;
                        for (int64_t m = 0; m < n; ++m) {
                            d3 A = ld(verts + 3 * (int64_t)tris[3 * m + 0]);
                            d3 B = ld(verts + 3 * (int64_t)tris[3 * m + 1]);
                            d3 C = ld(verts + 3 * (int64_t)tris[3 * m + 2]);
                            d3 mm = cross(sub(B, A), sub(C, A));
                            double dm = dot(D, mm);
                            if (dm == 0.0) continue;
                            double t = dot(sub(A, O), mm) / dm;
                            if (!(t > 0.0)) continue;
                            d3 a3 = sub(A, O), b3 = sub(B, O), c3 = sub(C, O);
                            double U = dot(D, cross(b3, c3)), V = dot(D, cross(c3, a3)), W = dot(D, cross(a3, b3));
                            int neg = (U < 0.0) || (V < 0.0) || (W < 0.0);
                            int pos = (U > 0.0) || (V > 0.0) || (W > 0.0);
                            if (neg && pos) continue;
                            if (t < tbest || (t == tbest && m < best)) {
                                tbest = t;
                                best = m;
                                dmbest = dm / (dl * sqrt(dot(mm, mm)));
                                double sa = sqrt(dot(a3, a3)), sb = sqrt(dot(b3, b3)), sc = sqrt(dot(c3, c3));
                                double g = fmin(fmin(fabs(U) / (dl * sb * sc), fabs(V) / (dl * sc * sa)),
                                                fabs(W) / (dl * sa * sb));
                                grbest = g;
                            }
                        }
                        if (best < 0) continue;
                        int ambiguous = grbest <= rel || fabs(dmbest) <= rel;
                        /* near triangles: close in t, or grazed at a distance not beyond the winner */
                        for (int64_t m = 0; m < n; ++m) {
                            if (m == best) continue;
                            d3 A = ld(verts + 3 * (int64_t)tris[3 * m + 0]);
                            d3 B = ld(verts + 3 * (int64_t)tris[3 * m + 1]);
                            d3 C = ld(verts + 3 * (int64_t)tris[3 * m + 2]);
                            d3 mm = cross(sub(B, A), sub(C, A));
                            double dm = dot(D, mm);
                            if (dm == 0.0) continue;
                            double t = dot(sub(A, O), mm) / dm;
                            if (!(t > 0.0) || t > tbest * (1.0 + rel)) continue;
                            d3 a3 = sub(A, O), b3 = sub(B, O), c3 = sub(C, O);
                            double U = dot(D, cross(b3, c3)), V = dot(D, cross(c3, a3)), W = dot(D, cross(a3, b3));
                            double sa = sqrt(dot(a3, a3)), sb = sqrt(dot(b3, b3)), sc = sqrt(dot(c3, c3));
                            double u = U / (dl * sb * sc), v = V / (dl * sc * sa), ww = W / (dl * sa * sb);
                            int inside = !(((u < 0) || (v < 0) || (ww < 0)) && ((u > 0) || (v > 0) || (ww > 0)));
                            /* outside (mixed signs): how far the ray is from making all three orientations
                               one sign, either way; inside: a tie in t with the winner */
                            double mn = fmin(fmin(u, v), ww), mx = fmax(fmax(u, v), ww);
                            double miss = fmin(-mn, mx);
                            int near = inside ? (t >= tbest * (1.0 - rel)) : (fabs(miss) <= rel);
                            if (near) {
                                amb[m] += 1;
                                ambiguous = 1;
                            }
                        }
                        if (ambiguous) amb[best] += 1;
                        if (dmbest < 0.0) {
                            F[best] += e;
                            landed += e;
                        }
                    }
                }
            }
        }
        for (int64_t m = 0; m < n; ++m) {
            d3 A = ld(verts + 3 * (int64_t)tris[3 * m + 0]);
            d3 B = ld(verts + 3 * (int64_t)tris[3 * m + 1]);
            d3 C = ld(verts + 3 * (int64_t)tris[3 * m + 2]);
            d3 mm = cross(sub(B, A), sub(C, A));
            F[m] = F[m] / (0.5 * sqrt(dot(mm, mm)));
        }
        if (power_out) power_out[k] = landed;
    }
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
