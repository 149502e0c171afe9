// Autotuner for the irradiance kernels: probes launch variants on a subset
// of the poses, scores them by occlusion rays per second, and keeps the best
// per (mesh-size bucket, source count) in a small JSON table on disk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "uvc_common.hpp"

namespace {

struct Entry {
    int path = UVC_PATH_LBVH, packet_poses = 16, waves = 6, tile_tris = 512;
    double rays_per_s = 0.0;
};

std::string bucket_key(int64_t n, int s) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= std::max<int64_t>(n, 1)) ++b;
    return "n" + std::to_string(b) + "_s" + std::to_string(s);
}

// The table is a flat JSON object written by write_table; read_table parses
// exactly that layout: {"key": {"path": P, "packet_poses": T, "waves": W,
// "tile_tris": L, "rays_per_s": R}, ...}
int read_int(const std::string& body, const char* name, int dflt) {
    const std::string k = std::string("\"") + name + "\":";
    const size_t at = body.find(k);
    if (at == std::string::npos) return dflt;
    return std::atoi(body.c_str() + at + k.size());
}

double read_num(const std::string& body, const char* name) {
    const std::string k = std::string("\"") + name + "\":";
    const size_t at = body.find(k);
    if (at == std::string::npos) return 0.0;
    return std::atof(body.c_str() + at + k.size());
}

std::map<std::string, Entry> parse_table(const std::string& s) {
    std::map<std::string, Entry> t;
    size_t pos = 0;
    while (true) {
        const size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = s.find('"', q0 + 1);
        const size_t b0 = s.find('{', q1);
        const size_t b1 = s.find('}', b0);
        if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
        const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        std::string body = s.substr(b0, b1 - b0 + 1);
        body.erase(std::remove(body.begin(), body.end(), ' '), body.end());
        Entry e;
        e.path = read_int(body, "path", e.path);
        e.packet_poses = read_int(body, "packet_poses", e.packet_poses);
        e.waves = read_int(body, "waves", e.waves);
        e.tile_tris = read_int(body, "tile_tris", e.tile_tris);
        e.rays_per_s = read_num(body, "rays_per_s");
        t[key] = e;
        pos = b1 + 1;
    }
    return t;
}

std::map<std::string, Entry> read_table(const char* path) {
    if (!path) return {};
    std::ifstream f(path);
    if (!f) return {};
    std::stringstream ss;
    ss << f.rdbuf();
    return parse_table(ss.str());
}

// The table registered with uvc_set_tune_table (consulted by UVC_PATH_AUTO
// and by batches created without a table of their own).
std::mutex g_tune_mu;
std::map<std::string, Entry> g_tune;

void fill_opts(const Entry& e, uvc_opts& o) {
    o.path = e.path;
    o.packet_poses = e.packet_poses;
    o.waves = e.waves;
    o.tile_tris = e.tile_tris;
}

bool write_table(const char* path, const std::map<std::string, Entry>& t) {
    if (!path) return true;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : t) {
            const Entry& e = kv.second;
            char buf[256];
            std::snprintf(buf, sizeof(buf),
                          "  \"%s\": {\"path\": %d, \"packet_poses\": %d, \"waves\": %d, \"tile_tris\": %d, "
                          "\"rays_per_s\": %.6e}%s\n",
                          kv.first.c_str(), e.path, e.packet_poses, e.waves, e.tile_tris, e.rays_per_s,
                          ++i < t.size() ? "," : "");
            f << buf;
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" uvc_status uvc_autotune(const uvc_scene* scene, const float* poses_dev, int64_t K, int32_t pose_dim,
                                   const uvc_lamp* lamp, int32_t probe_poses, const char* table_path,
                                   int32_t force, uvc_opts* best, void* hip_stream) {
    if (!scene || !lamp || !best) return uvc::fail(UVC_EINVAL, "NULL scene, lamp or best");
    int64_t n = 0;
    uvc_status st = uvc_scene_info(scene, &n, nullptr, nullptr);
    if (st != UVC_OK) return st;
    const std::string key = bucket_key(n, lamp->n_src);
    auto table = read_table(table_path);
    auto fill = [&](const Entry& e) {
        *best = uvc_opts{};
        best->path = e.path;
        best->packet_poses = e.packet_poses;
        best->waves = e.waves;
        best->tile_tris = e.tile_tris;
        best->band_scale = 1.0f;
    };
    if (!force && table.count(key)) {
        fill(table[key]);
        return UVC_OK;
    }
    if (K <= 0 || n <= 0) {
        fill(Entry{});
        return UVC_OK;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    // the probe must be large enough for the persistent loop to run in its
    // steady state (a few hundred poses leave most workgroups idle at the
    // end and favour small packets): at least 2^25 entries, at most K poses
    const int64_t want = std::max<int64_t>(probe_poses > 0 ? probe_poses : 256, ((int64_t)1 << 25) / std::max<int64_t>(n, 1));
    const int64_t P = std::max<int64_t>(1, std::min<int64_t>(K, want));
    float* E = nullptr;
    unsigned long long* stats = nullptr;
    if (hipMalloc(&E, (size_t)P * n * 4) != hipSuccess || hipMalloc(&stats, 8 * UVC_STAT_N) != hipSuccess) {
        if (E) (void)hipFree(E);
        (void)hipGetLastError();
        return uvc::fail(UVC_ENOMEM, "autotune probe buffers");
    }
    // the default options first (16 poses per packet, 6 waves per SIMD)
    std::vector<Entry> cands;
    {
        Entry e;
        e.path = UVC_PATH_LBVH;
        e.packet_poses = 16;
        e.waves = 6;
        cands.push_back(e);
    }
    for (int tp : {4, 8, 16, 32, 64})
        for (int w : {5, 6, 8}) {
            if (tp == 16 && w == 6) continue;
            Entry e;
            e.path = UVC_PATH_LBVH;
            e.packet_poses = tp;
            e.waves = w;
            cands.push_back(e);
        }
    // brute force costs N segment/triangle tests per segment: only small
    // meshes can win with it
    if (n <= 16384)
        for (int tt : {256, 512, 1024, 2048}) {
            Entry e;
            e.path = UVC_PATH_BRUTE;
            e.tile_tris = tt;
            cands.push_back(e);
        }
    // rays in the probe (identical for every variant)
    uvc_opts o{};
    o.band_scale = 1.0f;
    o.path = UVC_PATH_LBVH;
    o.stats_dev = reinterpret_cast<uint64_t*>(stats);
    (void)hipMemsetAsync(stats, 0, 8 * UVC_STAT_N, s);
    st = uvc_compute_irradiance_dense(scene, poses_dev, P, pose_dim, lamp, &o, E, nullptr, s);
    unsigned long long hs[UVC_STAT_N] = {};
    if (st == UVC_OK && hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, s) == hipSuccess)
        (void)hipStreamSynchronize(s);
    const double rays = (double)hs[UVC_STAT_RAYS];
    // every variant: one warm launch, then the median of three timed ones
    // (a single timing picked shapes whose lead was noise); a variant slower
    // than 1.5x the best so far after its warm launch is not re-timed.  The
    // default options (first candidate) stay unless another variant is more
    // than 2 % faster.
    auto timed = [&](const Entry& c, double bound, double& med) -> uvc_status {
        uvc_opts v{};
        v.band_scale = 1.0f;
        v.path = c.path;
        v.packet_poses = c.packet_poses;
        v.waves = c.waves;
        v.tile_tris = c.tile_tris;
        float ms = 0.f;
        v.kernel_ms = &ms;
        UVC_TRY(uvc_compute_irradiance_dense(scene, poses_dev, P, pose_dim, lamp, &v, E, nullptr, s));  // warm
        med = 1e300;
        if (ms > bound) return UVC_OK;
        float t[3];
        for (float& x : t) {
            UVC_TRY(uvc_compute_irradiance_dense(scene, poses_dev, P, pose_dim, lamp, &v, E, nullptr, s));
            x = ms;
        }
        std::sort(t, t + 3);
        med = t[1];
        return UVC_OK;
    };
    Entry win = cands[0];
    double best_ms = 1e300, win_ms = 1e300;
    for (const Entry& c : cands) {
        if (st != UVC_OK) break;
        double med = 1e300;
        st = timed(c, 1.5 * best_ms, med);
        if (st != UVC_OK) break;
        best_ms = std::min(best_ms, med);
        if (&c == &cands[0] || med < 0.98 * win_ms) {
            win_ms = med;
            win = c;
        }
    }
    best_ms = win_ms;
    (void)hipFree(E);
    (void)hipFree(stats);
    if (st != UVC_OK) return st;
    win.rays_per_s = rays / (best_ms * 1e-3);
    table[key] = win;
    fill(win);
    if (!write_table(table_path, table))
        return uvc::fail(UVC_EINVAL, std::string("cannot write the tuning table ") + table_path);
    return UVC_OK;
}

namespace uvc {
// Launch options of the table entry for this scene size and source count
// (json: a table text, or NULL for the registered table).  Returns false
// (o unchanged) when the table has no entry for the bucket.
bool tune_lookup(const char* json, int64_t n, int n_src, uvc_opts& o) {
    const std::string key = bucket_key(n, n_src);
    if (json) {
        const auto t = parse_table(json);
        const auto it = t.find(key);
        if (it == t.end()) return false;
        fill_opts(it->second, o);
        return true;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    fill_opts(it->second, o);
    return true;
}
}  // namespace uvc

extern "C" uvc_status uvc_set_tune_table(const char* json) {
    std::map<std::string, Entry> t;
    if (json) {
        t = parse_table(json);
        for (const auto& kv : t) {
            const Entry& e = kv.second;
            const bool ok_tp = e.packet_poses >= 1 && e.packet_poses <= 64 && (e.packet_poses & (e.packet_poses - 1)) == 0;
            if ((e.path != UVC_PATH_LBVH && e.path != UVC_PATH_BRUTE) || !ok_tp ||
                (e.waves != 5 && e.waves != 6 && e.waves != 8) || e.tile_tris < 1 || e.tile_tris > 2048)
                return uvc::fail(UVC_EINVAL, "tuning table entry " + kv.first + " has invalid options");
        }
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune = std::move(t);
    return UVC_OK;
}
