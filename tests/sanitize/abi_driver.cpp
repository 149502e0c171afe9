// Calls the library's host-side validation and parsing paths (no GPU work:
// every call below is rejected, or handled, before any HIP call) in a build
// whose host code has AddressSanitizer and UndefinedBehaviorSanitizer, so
// that they check the argument checks and the tuning-table parser.  Exit
// status 0 = every call returned the expected status.
#include <cstdio>
#include <cstring>
#include <string>

#include "uvc.h"

static int expect(const char* what, uvc_status got, uvc_status want) {
    if (got == want) return 0;
    std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, uvc_last_error());
    return 1;
}

int main() {
    int bad = 0;
    // tuning tables: well formed, malformed, truncated, empty, cleared
    const char* good = "{\n  \"n10_s1\": {\"path\": 1, \"packet_poses\": 16, \"waves\": 6, \"tile_tris\": 512, "
                       "\"rays_per_s\": 1.0e9},\n  \"n12_s8\": {\"path\": 2, \"packet_poses\": 4, \"waves\": 8, "
                       "\"tile_tris\": 256, \"rays_per_s\": 2.0e9}\n}\n";
    bad |= expect("good table", uvc_set_tune_table(good), UVC_OK);
    bad |= expect("bad packet", uvc_set_tune_table("{\"n3_s1\": {\"path\": 1, \"packet_poses\": 3}}"), UVC_EINVAL);
    bad |= expect("truncated", uvc_set_tune_table("{\"n3_s1\": {\"path\": 1, \"packet_po"), UVC_OK);
    bad |= expect("unterminated key", uvc_set_tune_table("{\"n3_s1"), UVC_OK);
    bad |= expect("empty", uvc_set_tune_table(""), UVC_OK);
    std::string big = "{";
    for (int q = 0; q < 200; ++q)
        big += "\"n" + std::to_string(q) + "_s1\": {\"path\": 1, \"packet_poses\": 8, \"waves\": 5, \"tile_tris\": 64},";
    big += "}";
    bad |= expect("large table", uvc_set_tune_table(big.c_str()), UVC_OK);
    bad |= expect("clear", uvc_set_tune_table(nullptr), UVC_OK);
    // argument checks that return before any device work
    bad |= expect("dense NULL scene", uvc_compute_irradiance_dense(nullptr, nullptr, 1, 2, nullptr, nullptr, nullptr,
                                                                    nullptr, nullptr), UVC_EINVAL);
    uvc_lamp lamp{};
    float dz[33], pw[33], prof[40];
    for (int q = 0; q < 33; ++q) dz[q] = 0.1f * q, pw[q] = 1.0f;
    for (int q = 0; q < 40; ++q) prof[q] = 1.0f;
    lamp.n_src = 33;
    lamp.dz = dz;
    lamp.power_w = pw;
    bad |= expect("area 33 sources", uvc_compute_irradiance_area(nullptr, nullptr, 1, 2, &lamp, 8, nullptr, nullptr,
                                                                  nullptr), UVC_EINVAL);
    bad |= expect("lp negative K", uvc_solve_dosage_lp(nullptr, nullptr, nullptr, -1, 3, nullptr, 280.0, 1.0, 1e-9, 10,
                                                        nullptr, nullptr, nullptr, nullptr, nullptr), UVC_EINVAL);
    bad |= expect("lp bad mu", uvc_solve_dosage_lp(nullptr, nullptr, nullptr, 2, 3, nullptr, -1.0, 1.0, 1e-9, 10,
                                                    nullptr, nullptr, nullptr, nullptr, nullptr), UVC_EINVAL);
    uvc_lp_info info;
    bad |= expect("lp CSR without col", uvc_solve_dosage_lp(nullptr, (const int64_t*)8, nullptr, 2, 3, nullptr, 280.0,
                                                             1.0, 1e-9, 10, nullptr, nullptr, nullptr, &info, nullptr),
                  UVC_EINVAL);
    bad |= expect("geodesics empty grid", uvc_route_geodesics(nullptr, 0, 5, 0.f, 0.f, 1.f, nullptr, 1, nullptr,
                                                               nullptr), UVC_EINVAL);
    bad |= expect("tour too many stops", uvc_route_tour(nullptr, 5000, 0, nullptr, nullptr, nullptr, nullptr),
                  UVC_EINVAL);
    int32_t stops[4], m = 0;
    double L = 0.0, T = 0.0;
    bad |= expect("route bad v_max", uvc_plan_route(nullptr, 1, 2, nullptr, 0.0, nullptr, 1, 1, 0.f, 0.f, 1.f, -1.0,
                                                     stops, &m, &L, &T, nullptr), UVC_EINVAL);
    bad |= expect("batch NULL out", uvc_batch_create(nullptr, 0, nullptr, nullptr, 2, nullptr, nullptr, nullptr,
                                                     nullptr, nullptr, nullptr), UVC_EINVAL);
    lamp.n_src = 2;
    lamp.n_prof = 40;
    lamp.profile = prof;
    bad |= expect("area long table", uvc_compute_irradiance_area(nullptr, nullptr, 1, 2, &lamp, 8, nullptr, nullptr,
                                                                  nullptr), UVC_EINVAL);
    if (std::strlen(uvc_last_error()) == 0) bad = 1;
    if (!bad) std::printf("ok\n");
    return bad;
}
