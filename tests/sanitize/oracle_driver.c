/* Runs the CPU oracle's entry points on a small closed scene (a unit cube
 * inside a box room) so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks every array access and operation they
 * make.  Exit status 0 = every call returned success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_irradiance_pairs_lamp(const float*, const int32_t*, int64_t, const float*, int64_t, int32_t, int32_t,
                                 const float*, const float*, int32_t, const float*, uint32_t, uint32_t,
                                 const int64_t*, const int64_t*, int64_t, double*, uint32_t*, int32_t);
int oracle_area_irradiance(const float*, const int32_t*, int64_t, const float*, int64_t, int32_t, int32_t,
                           const float*, const float*, int32_t, const float*, uint32_t, uint32_t, int32_t, double*,
                           int32_t*, double*, int32_t);
void oracle_elements(const float*, const int32_t*, int64_t, float*, double*, double*, double*);
int oracle_segment_blocked(const float*, const int32_t*, int64_t, const float*, const float*, int64_t);

static void box(float* v, int32_t* t, int vo, float lo, float hi, int inward) {
    for (int q = 0; q < 8; ++q) {
        v[3 * (vo + q) + 0] = (q & 1) ? hi : lo;
        v[3 * (vo + q) + 1] = (q & 2) ? hi : lo;
        v[3 * (vo + q) + 2] = (q & 4) ? hi : lo;
    }
    static const int f[12][3] = {{0, 2, 1}, {1, 2, 3}, {4, 5, 6}, {5, 7, 6}, {0, 1, 4}, {1, 5, 4},
                                 {2, 6, 3}, {3, 6, 7}, {0, 4, 2}, {2, 4, 6}, {1, 3, 5}, {3, 7, 5}};
    for (int q = 0; q < 12; ++q)
        for (int c = 0; c < 3; ++c) t[3 * q + c] = vo + f[q][inward ? 2 - c : c];
}

int main(void) {
    float v[16 * 3];
    int32_t t[24 * 3];
    box(v, t, 0, 0.0f, 4.0f, 1);
    box(v, t + 36, 8, 1.5f, 2.5f, 0);
    const int64_t n = 24;
    float c[24 * 3];
    double nn[24 * 3], area[24], m[24 * 3];
    oracle_elements(v, t, n, c, nn, area, m);
    const float poses[3 * 2] = {0.7f, 0.6f, 3.1f, 0.9f, 0.5f, 3.3f};
    const float dz[2] = {0.5f, 1.2f}, pw[2] = {40.0f, 40.0f}, prof[5] = {0.2f, 0.5f, 1.0f, 0.7f, 0.4f};
    int64_t pk[3 * 24], pi[3 * 24];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 24; ++i) {
            pk[k * 24 + i] = k;
            pi[k * 24 + i] = i;
        }
    double E[3 * 24];
    uint32_t vis[3 * 24];
    int bad = 0;
    bad |= oracle_irradiance_pairs_lamp(v, t, n, poses, 3, 2, 2, dz, pw, 0, NULL, 0u, 0u, pk, pi, 72, E, vis, 2);
    bad |= oracle_irradiance_pairs_lamp(v, t, n, poses, 3, 2, 2, dz, pw, 5, prof, 1u, 2u, pk, pi, 72, E, vis, 2);
    double Ea[3 * 24], landed[3];
    int32_t amb[3 * 24];
    bad |= oracle_area_irradiance(v, t, n, poses, 3, 2, 2, dz, pw, 5, prof, 0u, 0u, 8, Ea, amb, landed, 2);
    const float O[3] = {0.5f, 0.5f, 0.5f}, T[3] = {3.5f, 3.5f, 2.0f};
    (void)oracle_segment_blocked(v, t, n, O, T, -1);
    if (bad) {
        fprintf(stderr, "an oracle call failed\n");
        return 1;
    }
    printf("ok\n");
    return 0;
}
