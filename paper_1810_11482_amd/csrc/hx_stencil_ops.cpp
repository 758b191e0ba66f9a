// hx_launch_stencil: argument validation, launch geometry and the pass
// schedule for the 1D and 2D heat stencils.
#include <algorithm>
#include <string>
#include <vector>

#include "hx_internal.h"
#include "hx_runtime.hpp"
#include "hx_tune.hpp"

namespace hx {

static inline size_t esize(int dtype) { return dtype == HX_F64 ? 8 : 4; }
static inline int vec_cells(int dtype) { return dtype == HX_F64 ? 2 : 4; }
static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

static bool valid_bc(int b) { return b == HX_BC_PERIODIC || b == HX_BC_DIRICHLET0 || b == HX_BC_GHOST; }

// Largest time block a 1D tile of `cpl` cells per lane can take: it must keep
// at least one vector of output cells.
int max_time_block_1d(int dtype, int cpl) {
    const int vn = vec_cells(dtype);
    return (64 * cpl - vn) / 2 / vn * vn;
}

static hx_status launch_1d(Ctx* c, const hx_stencil_args* a, const hx_event* deps, int ndeps,
                           hx_event* out) {
    const int dt = a->dtype;
    const size_t es = esize(dt);
    const int64_t n = a->nx;
    if (n <= 0) return c->fail(HX_ERR_ARG, "nx must be positive");
    if (!valid_bc(a->bc_lo) || !valid_bc(a->bc_hi)) return c->fail(HX_ERR_ARG, "bad boundary");
    if ((a->bc_lo == HX_BC_PERIODIC) != (a->bc_hi == HX_BC_PERIODIC))
        return c->fail(HX_ERR_ARG, "periodic must apply to both ends");
    const bool ghost = a->bc_lo == HX_BC_GHOST || a->bc_hi == HX_BC_GHOST;

    std::vector<Access> acc;
    Access ac{};
    char *pin = nullptr, *pout = nullptr, *ptmp = nullptr, *plo = nullptr, *phi = nullptr;
    const size_t bytes = (size_t)n * es;
    hx_status s = resolve_range(c, a->in, a->in_offset, bytes, &pin, &ac, false);
    if (s) return s;
    acc.push_back(ac);
    s = resolve_range(c, a->out, a->out_offset, bytes, &pout, &ac, true);
    if (s) return s;
    if (ac.buf_slot == acc[0].buf_slot && ac.lo < acc[0].hi && acc[0].lo < ac.hi)
        return c->fail(HX_ERR_ARG, "in and out overlap");
    acc.push_back(ac);

    Geom1D g;
    TuneKey key = tune_key_1d(dt, n, a->steps, ghost);
    Geom1D def = default_geom_1d(c, key);
    g.cpl = a->cells_per_lane ? a->cells_per_lane : def.cpl;
    if (g.cpl != 8 && g.cpl != 16 && g.cpl != 32 && g.cpl != 64)
        return c->fail(HX_ERR_ARG, "cells_per_lane must be 8, 16, 32 or 64");
    g.wpg = a->waves_per_group ? a->waves_per_group : def.wpg;
    if (g.wpg != 1 && g.wpg != 2 && g.wpg != 4)
        return c->fail(HX_ERR_ARG, "waves_per_group must be 1, 2 or 4");
    const int maxd = max_time_block_1d(dt, g.cpl);
    int D = a->time_block ? a->time_block : std::min(def.steps, maxd);
    if (a->steps < 0) return c->fail(HX_ERR_ARG, "negative steps");
    if (ghost) {
        if (a->halo_width <= 0) return c->fail(HX_ERR_ARG, "GHOST needs halo_width > 0");
        if (a->steps > a->halo_width)
            return c->fail(HX_ERR_ARG, "steps exceed halo_width (the halo must cover the light cone)");
        D = a->steps;  // one fused pass
        if (a->time_block && a->time_block < a->steps)
            return c->fail(HX_ERR_ARG, "a GHOST run is one pass: time_block must be >= steps");
        const size_t hb = (size_t)a->halo_width * es;
        if (a->bc_lo == HX_BC_GHOST) {
            s = resolve_range(c, a->halo_lo, a->halo_lo_offset, hb, &plo, &ac, false);
            if (s) return s;
            acc.push_back(ac);
        }
        if (a->bc_hi == HX_BC_GHOST) {
            s = resolve_range(c, a->halo_hi, a->halo_hi_offset, hb, &phi, &ac, false);
            if (s) return s;
            acc.push_back(ac);
        }
    }
    if (D < 1) D = 1;
    if (D > maxd)
        return c->fail(HX_ERR_ARG, "time block " + std::to_string(D) + " exceeds the tile limit " +
                                       std::to_string(maxd) + " for cells_per_lane " +
                                       std::to_string(g.cpl));
    const int passes = a->steps == 0 ? 1 : (a->steps + D - 1) / D;
    if (passes > 1) {
        if (a->tmp == 0)
            return c->fail(HX_ERR_ARG, "a run of more than one pass needs a tmp buffer");
        s = resolve_range(c, a->tmp, a->tmp_offset, bytes, &ptmp, &ac, true);
        if (s) return c->fail(s, "a run of more than one pass needs a valid tmp buffer");
        for (const Access& x : acc)
            if (x.buf_slot == ac.buf_slot && x.lo < ac.hi && ac.lo < x.hi)
                return c->fail(HX_ERR_ARG, "tmp overlaps another operand");
        acc.push_back(ac);
    }

    Seg1D seg{};
    seg.n = n;
    seg.r = a->r;
    seg.bc_lo = a->bc_lo;
    seg.bc_hi = a->bc_hi;
    seg.hw = a->halo_width;
    seg.halo_lo = plo;
    seg.halo_hi = phi;
    const int steps = a->steps;
    const int vn = vec_cells(dt);
    std::string what = "stencil1d n=" + std::to_string(n) + " steps=" + std::to_string(steps);
    return c->submit(
        SC_COMPUTE, deps, ndeps, acc, what,
        [=](hipStream_t st) -> hipError_t {
            // passes ping-pong so that the last one lands in out
            const char* src = pin;
            int left = steps;
            for (int p = 0; p < passes; ++p) {
                const int d = (p == passes - 1) ? left : D;
                char* dst = ((passes - 1 - p) % 2 == 0) ? pout : ptmp;
                Seg1D sg = seg;
                sg.in = src;
                sg.out = dst;
                Geom1D gg = g;
                gg.steps = d;
                gg.halo = std::max(vn, round_up(d, vn));
                hipError_t e = launch_stencil1d(dt, sg, gg, st);
                if (e != hipSuccess) return e;
                src = dst;
                left -= d;
            }
            return hipSuccess;
        },
        out);
}

// Largest fused depth the 2D kernel supports that is <= limit.
static int depth2d_at_most(int dtype, int cpl, int limit) {
    for (int d = limit; d >= 1; --d)
        if (stencil2d_supported(dtype, cpl, d)) return d;
    return 0;
}

static hx_status launch_2d(Ctx* c, const hx_stencil_args* a, const hx_event* deps, int ndeps,
                           hx_event* out) {
    const int dt = a->dtype;
    const size_t es = esize(dt);
    const int vn = vec_cells(dt);
    const int64_t nx = a->nx, ny = a->ny;
    if (nx <= 0 || ny <= 0) return c->fail(HX_ERR_ARG, "nx and ny must be positive");
    if (a->steps < 0) return c->fail(HX_ERR_ARG, "negative steps");
    auto ok = [](int b) { return b == HX_BC_DIRICHLET0 || b == HX_BC_GHOST; };
    if (!ok(a->bc_lo) || !ok(a->bc_hi))
        return c->fail(HX_ERR_ARG, "2D top/bottom must be DIRICHLET0 or GHOST");
    const bool ghost = a->bc_lo == HX_BC_GHOST || a->bc_hi == HX_BC_GHOST;
    std::vector<Access> acc;
    Access ac{};
    char *pin = nullptr, *pout = nullptr, *ptmp = nullptr, *ptop = nullptr, *pbot = nullptr;
    const size_t bytes = (size_t)nx * (size_t)ny * es;
    hx_status s = resolve_range(c, a->in, a->in_offset, bytes, &pin, &ac, false);
    if (s) return s;
    acc.push_back(ac);
    s = resolve_range(c, a->out, a->out_offset, bytes, &pout, &ac, true);
    if (s) return s;
    if (ac.buf_slot == acc[0].buf_slot && ac.lo < acc[0].hi && acc[0].lo < ac.hi)
        return c->fail(HX_ERR_ARG, "in and out overlap");
    acc.push_back(ac);

    TunedGeom tg;
    const bool tuned = tune_lookup(tune_key_2d(dt, ny, nx, a->steps), &tg);
    Geom2D g{};
    g.cpl = a->cells_per_lane ? a->cells_per_lane : (tuned && tg.cpl ? tg.cpl : 4);
    g.wpg = a->waves_per_group ? a->waves_per_group : (tuned && tg.wpg ? tg.wpg : 4);
    g.rows = a->rows_per_block ? a->rows_per_block : (tuned && tg.rows ? tg.rows : 256);
    if (g.wpg != 1 && g.wpg != 2 && g.wpg != 4)
        return c->fail(HX_ERR_ARG, "waves_per_group must be 1, 2 or 4");
    if (g.rows < 1) return c->fail(HX_ERR_ARG, "rows_per_block must be positive");
    if (!stencil2d_supported(dt, g.cpl, 1))
        return c->fail(HX_ERR_ARG, "2D cells_per_lane must be 4 (or 8 for f32)");
    int D = a->time_block ? a->time_block : (tuned && tg.steps ? tg.steps : 8);
    std::vector<int> plan;  // fused depth of each pass
    if (ghost) {
        if (a->halo_width <= 0) return c->fail(HX_ERR_ARG, "GHOST needs halo_width > 0");
        if (a->steps > a->halo_width)
            return c->fail(HX_ERR_ARG, "steps exceed halo_width");
        if (a->steps > 0 && !stencil2d_supported(dt, g.cpl, a->steps))
            return c->fail(HX_ERR_ARG, "a GHOST run is one fused pass: steps must be 1..8, 10, "
                                       "12 or 16 (f32, 4 columns per lane)");
        plan.push_back(a->steps);
        const size_t hb = (size_t)a->halo_width * (size_t)nx * es;
        if (a->bc_lo == HX_BC_GHOST) {
            s = resolve_range(c, a->halo_lo, a->halo_lo_offset, hb, &ptop, &ac, false);
            if (s) return s;
            acc.push_back(ac);
        }
        if (a->bc_hi == HX_BC_GHOST) {
            s = resolve_range(c, a->halo_hi, a->halo_hi_offset, hb, &pbot, &ac, false);
            if (s) return s;
            acc.push_back(ac);
        }
    } else {
        if (D < 1 || !stencil2d_supported(dt, g.cpl, D))
            return c->fail(HX_ERR_ARG, "unsupported 2D time_block");
        int left = a->steps;
        while (left > 0) {
            const int d = depth2d_at_most(dt, g.cpl, std::min(D, left));
            plan.push_back(d);
            left -= d;
        }
        if (plan.empty()) plan.push_back(0);
    }
    const int passes = (int)plan.size();
    if (passes > 1) {
        if (a->tmp == 0)
            return c->fail(HX_ERR_ARG, "a run of more than one pass needs a tmp buffer");
        s = resolve_range(c, a->tmp, a->tmp_offset, bytes, &ptmp, &ac, true);
        if (s) return s;
        for (const Access& x : acc)
            if (x.buf_slot == ac.buf_slot && x.lo < ac.hi && ac.lo < x.hi)
                return c->fail(HX_ERR_ARG, "tmp overlaps another operand");
        acc.push_back(ac);
    }
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const bool aligned = (nx % vn == 0) && al(pin) && al(pout) && (!ptmp || al(ptmp)) &&
                         (!ptop || al(ptop)) && (!pbot || al(pbot));
    Band2D band{};
    band.nx = nx;
    band.ny = ny;
    band.r = a->r;
    band.bc_top = a->bc_lo;
    band.bc_bot = a->bc_hi;
    band.hw = a->halo_width;
    band.halo_top = ptop;
    band.halo_bot = pbot;
    band.aligned = aligned ? 1 : 0;
    std::string what = "stencil2d " + std::to_string(ny) + "x" + std::to_string(nx) +
                       " steps=" + std::to_string(a->steps);
    return c->submit(
        SC_COMPUTE, deps, ndeps, acc, what,
        [=](hipStream_t st) -> hipError_t {
            const char* src = pin;
            for (int p = 0; p < passes; ++p) {
                char* dst = ((passes - 1 - p) % 2 == 0) ? pout : ptmp;
                Band2D bb = band;
                bb.in = src;
                bb.out = dst;
                if (p > 0) { bb.bc_top = HX_BC_DIRICHLET0; bb.bc_bot = HX_BC_DIRICHLET0; }
                if (plan[p] == 0) {
                    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
                    if (e != hipSuccess) return e;
                } else {
                    Geom2D gg = g;
                    gg.steps = plan[p];
                    gg.halo = std::max(vn, round_up(plan[p], vn));
                    hipError_t e = launch_stencil2d(dt, bb, gg, st);
                    if (e != hipSuccess) return e;
                }
                src = dst;
            }
            return hipSuccess;
        },
        out);
}

}  // namespace hx

using namespace hx;

hx_status hx::launch_stencil_locked(Ctx* c, const hx_stencil_args* a, const hx_event* deps,
                                   int ndeps, hx_event* out) {
    if (!a || !out) return c->fail(HX_ERR_ARG, "null argument");
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    if (a->dtype != HX_F32 && a->dtype != HX_F64) return c->fail(HX_ERR_ARG, "bad dtype");
    hipSetDevice(c->device);
    if (a->dims == 1) return launch_1d(c, a, deps, ndeps, out);
    if (a->dims == 2) return launch_2d(c, a, deps, ndeps, out);
    return c->fail(HX_ERR_ARG, "dims must be 1 or 2");
}

extern "C" hx_status hx_launch_stencil(hx_ctx ctx, const hx_stencil_args* a, const hx_event* deps,
                                       int ndeps, hx_event* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    return launch_stencil_locked(c, a, deps, ndeps, out);
}
