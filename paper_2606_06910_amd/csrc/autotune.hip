// autotune.hip -- per-shape choice of the z-march tile height (rows per
// thread) and z-chunk length, timed on the device with HIP events, cached in a
// small JSON file keyed by device, storage, shape bucket and layer width.
#include "fdtd_host.hpp"
#include "fdtd_launch.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

namespace {
struct Plan {
    int ry, zchunk, tk, cols;
    double ms;
};

std::string shape_key(const fdtd_ctx *ctx, const ShotH &s) {
    char buf[256];
    int lmax = 0;
    for (int f = 0; f < 6; ++f) lmax = std::max(lmax, (int)s.c.cpml[f]);
    snprintf(buf, sizeof buf, "gfx950|stor%d|%dx%dx%d|L%d|g%d%d|s%d", ctx->storage, (s.nx + 15) / 16,
             (s.ny + 15) / 16, (s.nz + 15) / 16, lmax, s.gy, s.gz, s.s);
    return buf;
}

// minimal reader for the cache written below:
// {"entries": [{"key": "...", "ry": R, "zchunk": Z, "tk": K, "cols": C, "ms": T}, ...]}
std::map<std::string, Plan> read_cache(const char *path) {
    std::map<std::string, Plan> out;
    if (!path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string t = ss.str();
    size_t pos = 0;
    auto num = [&](const std::string &obj, const char *name, double dflt) {
        std::string pat = std::string("\"") + name + "\":";
        size_t p = obj.find(pat);
        if (p == std::string::npos) return dflt;
        return atof(obj.c_str() + p + pat.size());
    };
    while ((pos = t.find('{', pos + 1)) != std::string::npos) {
        size_t end = t.find('}', pos);
        if (end == std::string::npos) break;
        std::string obj = t.substr(pos, end - pos + 1);
        size_t k = obj.find("\"key\":");
        if (k != std::string::npos) {
            size_t q0 = obj.find('"', k + 6);
            size_t q1 = q0 == std::string::npos ? q0 : obj.find('"', q0 + 1);
            if (q0 != std::string::npos && q1 != std::string::npos) {
                Plan p{(int)num(obj, "ry", 2), (int)num(obj, "zchunk", 64), (int)num(obj, "tk", 1),
                       (int)num(obj, "cols", 1), num(obj, "ms", 0)};
                const bool ok_ry = p.cols == 2 ? (p.ry == 1 || p.ry == 2 || p.ry == 4)
                                               : (p.cols == 1 && (p.ry == 1 || p.ry == 2 || p.ry == 4 || p.ry == 8));
                if (ok_ry && p.zchunk >= 16 && p.zchunk <= 4096)
                    out[obj.substr(q0 + 1, q1 - q0 - 1)] = p;
            }
        }
        pos = end;
    }
    return out;
}

void write_cache(const char *path, const std::map<std::string, Plan> &m) {
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\"entries\": [\n");
    size_t i = 0;
    for (auto &kv : m) {
        fprintf(f, "  {\"key\": \"%s\", \"ry\": %d, \"zchunk\": %d, \"tk\": %d, \"cols\": %d, \"ms\": %.6f}%s\n",
                kv.first.c_str(), kv.second.ry, kv.second.zchunk, kv.second.tk, kv.second.cols, kv.second.ms,
                ++i < m.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}
}  // namespace

extern "C" int fdtd_autotune(fdtd_ctx *ctx, const char *cache_path) {
    if (!ctx) return FDTD_EINVAL;
    int rc = fdtd_ready(ctx);
    if (rc) return rc;
    std::map<std::string, Plan> cache = read_cache(cache_path);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        ctx->err = "hipEventCreate failed";
        return FDTD_EHIP;
    }
    // candidates: the default plan, then tile shapes (x points per lane, rows) x z-chunk
    // lengths (4096: whole columns)
    const int ry_c[7] = {1, 2, 4, 8, 1, 2, 4};
    const int cx_c[7] = {1, 1, 1, 1, 2, 2, 2};
    const int zc_c[4] = {32, 64, 128, 4096};
    for (size_t i = 0; i < ctx->shots.size(); ++i) {
        ShotH &s = ctx->shots[i];
        if (s.variant == FDTD_VARIANT_NAIVE) continue;
        const std::string key = shape_key(ctx, s);
        auto it = cache.find(key);
        if (it != cache.end()) {
            s.ry = it->second.ry;
            s.zchunk = it->second.zchunk;
            s.zcols = it->second.cols;
            continue;
        }
        Plan best{s.ry, s.zchunk, 1, s.zcols, 1e30};
        const int ry0 = s.ry, zc0 = s.zchunk, cx0 = s.zcols;
        for (int c = -1; c < 28; ++c) {
            s.ry = c < 0 ? ry0 : ry_c[c / 4];
            s.zcols = c < 0 ? cx0 : cx_c[c / 4];
            s.zchunk = c < 0 ? zc0 : zc_c[c % 4];
            {
                rc = fdtd_rewrite_work(ctx);
                if (rc) return rc;
                for (int k = 0; k < 2; ++k) fdtd_enqueue_step_shot(ctx, (int)i);
                const int reps = 6;
                (void)hipEventRecord(e0, ctx->stream);
                for (int k = 0; k < reps; ++k) fdtd_enqueue_step_shot(ctx, (int)i);
                (void)hipEventRecord(e1, ctx->stream);
                if (hipEventSynchronize(e1) != hipSuccess) {
                    ctx->err = "autotune: device error while timing";
                    return FDTD_EHIP;
                }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                double per = ms / reps;
                if (per < best.ms) best = Plan{s.ry, s.zchunk, 1, s.zcols, per};
            }
        }
        s.ry = best.ry;
        s.zchunk = best.zchunk;
        s.zcols = best.cols;
        cache[key] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rc = fdtd_rewrite_work(ctx);
    if (rc) return rc;
    fdtd_clear_graphs(ctx);
    write_cache(cache_path, cache);
    return fdtd_zero_state(ctx);
}
