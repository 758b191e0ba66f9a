// Autotuner cache and defaults.
#include "hx_tune.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "hx_runtime.hpp"

namespace hx {

static std::mutex g_tune_mu;
static std::map<std::string, TunedGeom> g_tune;
static bool g_tune_loaded = false;

static int size_class(int64_t n) {
    int c = 0;
    while (n > 1) { n >>= 1; ++c; }
    return c;
}

TuneKey tune_key_1d(int dtype, int64_t n, int steps, bool ghost) {
    char b[128];
    snprintf(b, sizeof b, "stencil1d/%s/n2^%d/s%d%s", dtype ? "f64" : "f32", size_class(n), steps,
             ghost ? "/ghost" : "");
    return TuneKey{b};
}

TuneKey tune_key_2d(int dtype, int64_t ny, int64_t nx, int steps) {
    char b[128];
    snprintf(b, sizeof b, "stencil2d/%s/ny2^%d/nx2^%d/s%d", dtype ? "f64" : "f32", size_class(ny),
             size_class(nx), steps);
    return TuneKey{b};
}

TuneKey tune_key_batched(int dtype, int64_t total, int count, int steps) {
    char b[128];
    snprintf(b, sizeof b, "batched1d/%s/cells2^%d/count2^%d/s%d", dtype ? "f64" : "f32",
             size_class(total), size_class(count), steps);
    return TuneKey{b};
}

// The file is a flat JSON object {"key": [cpl, steps, wpg, rows, grid, mode], ...}
// written and read only by this library.
static void load_file_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("HX_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        std::string key = s.substr(pos + 1, end - pos - 1);
        size_t lb = s.find('[', end), rb = s.find(']', end);
        if (lb == std::string::npos || rb == std::string::npos) break;
        TunedGeom g;
        int v[6] = {0, 0, 0, 0, 0, 0};
        sscanf(s.c_str() + lb + 1, "%d , %d , %d , %d , %d , %d", &v[0], &v[1], &v[2], &v[3],
               &v[4], &v[5]);
        g.cpl = v[0]; g.steps = v[1]; g.wpg = v[2]; g.rows = v[3]; g.grid = v[4]; g.mode = v[5];
        g_tune[key] = g;
        pos = rb + 1;
    }
}

bool tune_lookup(const TuneKey& k, TunedGeom* g) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_file_locked();
    auto it = g_tune.find(k.s);
    if (it == g_tune.end()) return false;
    *g = it->second;
    return true;
}

void tune_store(const TuneKey& k, const TunedGeom& g) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_file_locked();
    g_tune[k.s] = g;
}

Geom1D default_geom_1d(Ctx* c, const TuneKey& k) {
    (void)c;
    TunedGeom t;
    Geom1D g;
    if (tune_lookup(k, &t) && t.cpl) {
        g.cpl = t.cpl;
        g.steps = t.steps;
        g.wpg = t.wpg ? t.wpg : 4;
        g.halo = 0;
        return g;
    }
    // Heuristic: 32 cells per lane, a time block of up to 32 steps.
    g.cpl = 32;
    g.steps = 32;
    g.wpg = 4;
    g.halo = 0;
    return g;
}

}  // namespace hx

using namespace hx;

extern "C" {

hx_status hx_tune_cache_save(const char* path) {
    if (!path) return HX_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_file_locked();
    FILE* f = fopen(path, "w");
    if (!f) return HX_ERR_ARG;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto& kv : g_tune) {
        const TunedGeom& g = kv.second;
        fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d, %d]%s\n", kv.first.c_str(), g.cpl, g.steps,
                g.wpg, g.rows, g.grid, g.mode, (++i < g_tune.size()) ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    return HX_OK;
}

hx_status hx_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = true;
    return HX_OK;
}

}  // extern "C"
