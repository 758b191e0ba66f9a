// Autotuner cache and defaults.
#include "hx_tune.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>
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
    // Heuristic: 32 cells per lane, a time block of up to 50 steps (the
    // fastest measured on MI355X for long runs: 75% of the VALU issue rate).
    g.cpl = 32;
    g.steps = 50;
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

// ------------------------------------------------------------------ search
namespace {

using clk = std::chrono::steady_clock;

// One launch of `a`, in seconds, timed like time_plan: `reps` launches
// chained on one stream after a warm-up, their HIP-event spans in a timing
// context, else their host time over reps.  Negative on any failure.
double time_stencil(hx_ctx ctx, const hx_stencil_args& a, int reps) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    hx_event warm = 0;
    if (hx_launch_stencil(ctx, &a, nullptr, 0, &warm) != HX_OK) return -1;
    if (hx_wait(ctx, warm, -1) != HX_OK) {
        hx_event_release(ctx, warm);
        return -1;
    }
    std::vector<hx_event> evs;
    hx_event prev = warm;
    const auto t0 = clk::now();
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) {
        hx_event ev = 0;
        ok = hx_launch_stencil(ctx, &a, &prev, 1, &ev) == HX_OK;
        if (ok) evs.push_back(prev = ev);
    }
    if (ok) ok = hx_wait(ctx, prev, -1) == HX_OK;
    const double host = std::chrono::duration<double>(clk::now() - t0).count() / reps;
    double gpu = 0.0;
    bool spans = ok && c->timing;
    for (hx_event e : evs) {
        double x = 0, y = 0;
        if (spans && hx_event_span(ctx, e, e, &x, &y) == HX_OK) gpu += (y - x) * 1e-3;
        else spans = false;
    }
    hx_event_release(ctx, warm);
    for (hx_event e : evs) hx_event_release(ctx, e);
    if (!ok || evs.empty()) return -1;
    return spans ? gpu / (double)evs.size() : host;
}

}  // namespace

extern "C" hx_status hx_tune_stencil(hx_ctx ctx, const hx_stencil_args* args, int budget_ms,
                                     hx_stencil_args* best) {
    if (!ctx || !args || !best) return HX_ERR_ARG;
    const bool two_d = args->dims == 2;
    const bool ghost = args->bc_lo == HX_BC_GHOST || args->bc_hi == HX_BC_GHOST;
    std::vector<hx_stencil_args> cands;
    auto add = [&](int cpl, int tb, int wpg, int rows) {
        hx_stencil_args a = *args;
        a.cells_per_lane = cpl;
        a.time_block = ghost ? 0 : tb;
        a.waves_per_group = wpg;
        a.rows_per_block = rows;
        cands.push_back(a);
    };
    const int S = std::max(args->steps, 1);
    if (!two_d) {
        const int tbs[] = {8, 16, 25, 32, 50, 64, 100};
        for (int cpl : {32, 16, 64, 8})
            for (int tb : tbs) {
                const int d = std::min(tb, S);
                if (d > max_time_block_1d(args->dtype, cpl)) continue;
                for (int wpg : {4, 2}) add(cpl, d, wpg, 0);
                if (tb >= S) break;
            }
    } else {
        for (int cpl : {4, 8})
            for (int tb : {16, 12, 10, 8, 6, 4}) {
                const int d = std::min(tb, S);
                if (!stencil2d_supported(args->dtype, cpl, d)) continue;
                for (int rows : {128, 256, 64, 512}) add(cpl, d, 4, rows);
                if (tb >= S) break;
            }
    }
    const auto t_start = clk::now();
    double best_t = 1e30;
    bool found = false;
    for (const hx_stencil_args& a : cands) {
        if (found && std::chrono::duration<double, std::milli>(clk::now() - t_start).count() >
                         budget_ms)
            break;
        const double t = time_stencil(ctx, a, 2);
        if (t > 0 && t < best_t) {
            best_t = t;
            *best = a;
            found = true;
        }
    }
    if (!found) return HX_ERR_ARG;
    TunedGeom g;
    g.cpl = best->cells_per_lane;
    g.steps = best->time_block ? best->time_block : std::min(args->steps, 32);
    g.wpg = best->waves_per_group;
    g.rows = best->rows_per_block;
    const TuneKey k = two_d ? tune_key_2d(args->dtype, args->ny, args->nx, args->steps)
                            : tune_key_1d(args->dtype, args->nx, args->steps, ghost);
    tune_store(k, g);
    return HX_OK;
}

namespace {

// One launch of `plan`, in seconds: `reps` launches chained on one stream
// after a warm-up launch; in a timing context the mean of their HIP-event
// spans (GPU time of each launch), otherwise the host time of the chained
// launches over reps (the launches are queued back to back, so only the
// GPU-side gaps between them add).  Negative on any failure.
double time_plan(hx_ctx ctx, hx_plan plan, int reps) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    hx_event warm = 0;
    if (hx_launch_batched(ctx, plan, nullptr, 0, &warm) != HX_OK) return -1;
    if (hx_wait(ctx, warm, -1) != HX_OK) {
        hx_event_release(ctx, warm);
        return -1;
    }
    std::vector<hx_event> evs;
    hx_event prev = warm;
    const auto t0 = clk::now();
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) {
        hx_event ev = 0;
        ok = hx_launch_batched(ctx, plan, &prev, 1, &ev) == HX_OK;
        if (ok) evs.push_back(prev = ev);
    }
    if (ok) ok = hx_wait(ctx, prev, -1) == HX_OK;
    const double host = std::chrono::duration<double>(clk::now() - t0).count() / reps;
    double gpu = 0.0;
    bool spans = ok && c->timing;
    for (hx_event e : evs) {
        double a = 0, b = 0;
        if (spans && hx_event_span(ctx, e, e, &a, &b) == HX_OK) gpu += (b - a) * 1e-3;
        else spans = false;
    }
    hx_event_release(ctx, warm);
    for (hx_event e : evs) hx_event_release(ctx, e);
    if (!ok || evs.empty()) return -1;
    return spans ? gpu / (double)evs.size() : host;
}

}  // namespace

// The pass depths worth trying for a run of T steps: the divisors of T that a
// fused pass can take (at most 64 steps), from the deepest, down to T/8 steps
// (eight passes), and at least the deepest one.
static std::vector<int> pass_depths(int T) {
    std::vector<int> ds;
    for (int d = std::min(T, 64); d >= 1; --d)
        if (T % d == 0 && (ds.empty() || T / d <= 8)) ds.push_back(d);
    if (ds.empty()) ds.push_back(std::max(T, 0));
    return ds;
}

extern "C" hx_status hx_tune_batched(hx_ctx ctx, const hx_batch_desc* desc, int budget_ms,
                                     hx_batch_desc* best) {
    if (!ctx || !desc || !best || desc->mode != HX_BATCH_PERSISTENT || desc->steps < 0)
        return HX_ERR_ARG;
    const auto t_start = clk::now();
    const int T = desc->steps;
    double best_t = 1e30;
    bool found = false;
    // candidates, the likely fastest first: per pass depth D (deepest first),
    // the propagator form (f32) over its walks, then the direct form over
    // cells per lane, waves per group and the persistent grid; a candidate the
    // plan rejects (depth beyond a geometry's limit, halos too short, ...) is
    // skipped.  The cost of a candidate is T / D times its pass.
    std::vector<hx_batch_desc> cands;
    for (int D : pass_depths(T)) {
        if (desc->dtype == HX_F32)
            // the block walk at one and four waves per group, the interleaved
            // walk, the plan's own choice and spans
            for (int k = 0; k < 6; ++k) {
                static const int kSpan[6] = {-2, -2, -1, 0, 128, 40};
                hx_batch_desc d = *desc;
                d.steps = D;
                d.form = HX_FORM_PROPAGATOR;
                d.span_blocks = kSpan[k];
                d.waves_per_group = k == 1 ? 4 : (k == 0 ? 1 : 0);
                cands.push_back(d);
            }
        for (int cpl : {16, 32, 8, 64})
            for (int wpg : {4, 2, 1})
                for (int grid : {-1, 64, 16}) {
                    if (grid != -1 && wpg != 4) continue;  // the persistent grid at 4 only
                    if (cpl == 64 && (wpg != 4 || grid != -1)) continue;
                    hx_batch_desc d = *desc;
                    d.steps = D;
                    d.form = HX_FORM_DIRECT;
                    d.cells_per_lane = cpl;
                    d.grid_waves_per_cu = grid;
                    d.waves_per_group = wpg;
                    d.span_blocks = 0;
                    cands.push_back(d);
                }
    }
    for (const hx_batch_desc& d : cands) {
        if (found &&
            std::chrono::duration<double, std::milli>(clk::now() - t_start).count() > budget_ms)
            break;
        hx_plan plan = 0;
        if (hx_plan_create_batched(ctx, &d, &plan) != HX_OK) continue;
        const double pass = time_plan(ctx, plan, 3);
        hx_plan_destroy(ctx, plan);
        if (pass <= 0) continue;
        const double t = pass * (d.steps > 0 ? T / d.steps : 1);
        if (t < best_t) {
            best_t = t;
            *best = d;
            found = true;
        }
    }
    if (!found) return HX_ERR_ARG;
    int64_t total = 0;
    for (int i = 0; i < desc->count; ++i) total += desc->segs[i].n;
    TunedGeom g;
    g.cpl = best->cells_per_lane;
    g.steps = best->steps;
    g.wpg = best->waves_per_group;
    g.grid = best->grid_waves_per_cu;
    g.mode = 1 + best->form;
    g.rows = best->form == HX_FORM_PROPAGATOR ? best->span_blocks : 0;
    // under the run's key (its depth is the answer) and the pass's key (a plan
    // made for one pass of that depth finds its geometry)
    tune_store(tune_key_batched(desc->dtype, total, desc->count, T), g);
    if (best->steps != T) tune_store(tune_key_batched(desc->dtype, total, desc->count, best->steps), g);
    return HX_OK;
}
