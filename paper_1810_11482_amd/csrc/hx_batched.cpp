// Batched 1D plans: many independent (or halo-coupled) segments advanced by
// one fused pass in a single operation.
//
//  PERSISTENT  one launch over a flat tile table (segment, tile) built once
//              at plan creation, largest segments first: either one wave per
//              tile, or a persistent grid of a few waves per CU striding over
//              the table.  Tiles are of equal size, so a static stride
//              balances the grid without atomics.
//  GRAPH       one kernel launch per segment, captured once into a hipGraph
//              and replayed as a single graph launch.
//  PLAIN       the comparator: one launch per segment per time step.
//
// A PERSISTENT plan evaluates its pass in one of two forms: DIRECT (the tile
// kernels, step by step) or PROPAGATOR (one convolution with the D-step
// propagator on the matrix cores, f32; see hx_prop1d.hip).  For the latter
// the plan holds each distinct r's taps and, for contiguous spans, a table of
// per-wave spans; the interleaved walk (segments of one size and one rate)
// needs only the segment table.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "hx_internal.h"
#include "hx_runtime.hpp"
#include "hx_tune.hpp"

using namespace hx;

namespace {

enum { PLAN_BATCHED = 1 };

struct BatchPlan {
    int dtype = 0;
    int steps = 0;
    int mode = 0;
    Geom1D g{};
    std::vector<Seg1D> segs;        // host copy (GRAPH / PLAIN modes)
    std::vector<char*> tmps;        // PLAIN: per-segment ping-pong space
    Seg1D* segs_dev = nullptr;
    uint32_t* tseg_dev = nullptr;
    uint32_t* tidx_dev = nullptr;
    int64_t ntiles = 0;
    int64_t grid_waves = 0;
    int64_t per_seg = 0;  // tiles of every segment when all are equal (table unused)
    bool scaled = true;    // every segment runs the rescaled update
    bool prop = false;     // PROPAGATOR form
    PropSeg* psegs_dev = nullptr;
    PropWave* pwaves_dev = nullptr;
    float* taps_dev = nullptr;
    int64_t pwaves = 0;
    int pskip = 0;         // outer window chunks no segment multiplies
    bool pil = false;      // interleaved walk (segments of one size and one rate)
    bool pbw = false;      // block walk (the same segments), its tap table and
    void* ptab_dev = nullptr;  // waves per workgroup
    int pwpg = 1;
    int64_t pblocks = 0;   // interleaved: 1024-cell blocks in all, and per segment
    int64_t pbps = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Access> acc;
    int device = 0;
};

void destroy_plan(void* p) {
    BatchPlan* b = static_cast<BatchPlan*>(p);
    hipSetDevice(b->device);
    hipDeviceSynchronize();
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->cap) hipStreamDestroy(b->cap);
    if (b->segs_dev) hipFree(b->segs_dev);
    if (b->tseg_dev) hipFree(b->tseg_dev);
    if (b->tidx_dev) hipFree(b->tidx_dev);
    if (b->psegs_dev) hipFree(b->psegs_dev);
    if (b->pwaves_dev) hipFree(b->pwaves_dev);
    if (b->taps_dev) hipFree(b->taps_dev);
    if (b->ptab_dev) hipFree(b->ptab_dev);
    delete b;
}

size_t esz(int dt) { return dt == HX_F64 ? 8 : 4; }
int vecn(int dt) { return dt == HX_F64 ? 2 : 4; }

// The D-step propagator: [1] convolved D times with [r, 1 - 2r, r], in FP64.
std::vector<double> propagator(double r, int D) {
    std::vector<double> p(1, 1.0);
    for (int t = 0; t < D; ++t) {
        std::vector<double> q(p.size() + 2, 0.0);
        for (size_t k = 0; k < p.size(); ++k) {
            q[k] += r * p[k];
            q[k + 1] += (1.0 - 2.0 * r) * p[k];
            q[k + 2] += r * p[k];
        }
        p.swap(q);
    }
    return p;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Why a segment cannot take the propagator form of a D-step pass (nullptr if
// it can).
const char* prop_unfit(const Seg1D& s, int D) {
    int OD, NC;
    if (!prop1d_geometry(D, &OD, &NC)) return "steps must be 1..64";
    if (s.n % 4) return "n must be a multiple of 4";
    if (!aligned16(s.in) || !aligned16(s.out)) return "in and out must be 16-byte aligned";
    if (s.bc_lo == HX_BC_PERIODIC && s.bc_hi == HX_BC_PERIODIC) {
        if (s.n < D) return "a periodic segment needs n >= steps";
        return nullptr;
    }
    if (s.bc_lo != HX_BC_GHOST || s.bc_hi != HX_BC_GHOST)
        return "both ends must be PERIODIC or both GHOST";
    if (s.hw < 4 * ((D + 3) / 4)) return "halo_width must be at least 4 * ceil(steps / 4)";
    const float* lo_end = static_cast<const float*>(s.halo_lo) + s.hw;
    if (!aligned16(lo_end) || !aligned16(s.halo_hi))
        return "the end of halo_lo and the start of halo_hi must be 16-byte aligned";
    return nullptr;
}

// Blocks per wave: the span that fills the device in whole rounds of
// `slots` concurrent waves at the least modelled cost, rounds x (span + a
// start-up of about eight iterations: the taps, the first two blocks).
int choose_span(const std::vector<int64_t>& blocks, int64_t slots) {
    int best = 64;
    double best_cost = 1e300;
    for (int ni = 8; ni <= 256; ++ni) {
        int64_t w = 0;
        for (int64_t b : blocks) w += (b + ni - 1) / ni;
        const double cost = (double)((w + slots - 1) / slots) * (ni + 8);
        if (cost < best_cost) {
            best_cost = cost;
            best = ni;
        }
    }
    return best;
}

}  // namespace

extern "C" hx_status hx_propagator_coefficients(double r, int steps, double* taps) {
    if (!taps || steps < 0 || steps > (1 << 20) || !std::isfinite(r)) return HX_ERR_ARG;
    const std::vector<double> p = propagator(r, steps);
    std::copy(p.begin(), p.end(), taps);
    return HX_OK;
}

extern "C" hx_status hx_plan_create_batched(hx_ctx ctx, const hx_batch_desc* d, hx_plan* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!d || !out) return c->fail(HX_ERR_ARG, "null argument");
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    if (d->dtype != HX_F32 && d->dtype != HX_F64) return c->fail(HX_ERR_ARG, "bad dtype");
    if (d->count < 1 || !d->segs) return c->fail(HX_ERR_ARG, "count >= 1 segments required");
    if (d->steps < 0) return c->fail(HX_ERR_ARG, "negative steps");
    if (d->mode != HX_BATCH_PERSISTENT && d->mode != HX_BATCH_GRAPH && d->mode != HX_BATCH_PLAIN)
        return c->fail(HX_ERR_ARG, "bad mode");
    if (d->form != HX_FORM_DIRECT && d->form != HX_FORM_PROPAGATOR && d->form != HX_FORM_AUTO)
        return c->fail(HX_ERR_ARG, "bad form");
    if (d->form == HX_FORM_PROPAGATOR && (d->mode != HX_BATCH_PERSISTENT || d->dtype != HX_F32))
        return c->fail(HX_ERR_ARG, "the propagator form needs a PERSISTENT f32 batch");
    if (d->span_blocks < -2 || d->span_blocks > kSpanMax)
        return c->fail(HX_ERR_ARG, "span_blocks must be -2 .. " + std::to_string(kSpanMax));
    hipSetDevice(c->device);
    const size_t es = esz(d->dtype);
    const int vn = vecn(d->dtype);

    auto* bp = new BatchPlan();
    bp->device = c->device;
    bp->dtype = d->dtype;
    bp->steps = d->steps;
    bp->mode = d->mode;
    int64_t total = 0;
    for (int i = 0; i < d->count; ++i) total += d->segs[i].n;
    TunedGeom tg;
    const bool tuned = tune_lookup(tune_key_batched(d->dtype, total, d->count, d->steps), &tg);
    bp->g.cpl = d->cells_per_lane ? d->cells_per_lane : (tuned && tg.cpl ? tg.cpl : 16);
    bp->g.wpg = d->waves_per_group ? d->waves_per_group : (tuned && tg.wpg ? tg.wpg : 4);
    if (bp->g.cpl != 8 && bp->g.cpl != 16 && bp->g.cpl != 32 && bp->g.cpl != 64) {
        delete bp;
        return c->fail(HX_ERR_ARG, "cells_per_lane must be 8, 16, 32 or 64");
    }
    if (bp->g.wpg != 1 && bp->g.wpg != 2 && bp->g.wpg != 4) {
        delete bp;
        return c->fail(HX_ERR_ARG, "waves_per_group must be 1, 2 or 4");
    }
    const int fused = (d->mode == HX_BATCH_PLAIN) ? 1 : d->steps;
    bp->g.steps = fused;
    bp->g.halo = std::max(vn, (fused + vn - 1) / vn * vn);

    for (int i = 0; i < d->count; ++i) {
        const hx_segment& s = d->segs[i];
        auto bad = [&](hx_status st, const std::string& m) {
            delete bp;
            return c->fail(st, "segment " + std::to_string(i) + ": " + m);
        };
        if (s.n <= 0) return bad(HX_ERR_ARG, "n must be positive");
        auto okbc = [](int b) { return b >= HX_BC_PERIODIC && b <= HX_BC_GHOST; };
        if (!okbc(s.bc_lo) || !okbc(s.bc_hi)) return bad(HX_ERR_ARG, "bad boundary");
        if ((s.bc_lo == HX_BC_PERIODIC) != (s.bc_hi == HX_BC_PERIODIC))
            return bad(HX_ERR_ARG, "periodic must apply to both ends");
        const bool ghost = s.bc_lo == HX_BC_GHOST || s.bc_hi == HX_BC_GHOST;
        if (ghost && (s.halo_width < d->steps || s.halo_width <= 0))
            return bad(HX_ERR_ARG, "halo_width must cover the steps");
        if (ghost && d->mode == HX_BATCH_PLAIN && d->steps > 1)
            return bad(HX_ERR_ARG, "a halo-coupled segment cannot be run step by step alone");
        Seg1D sg{};
        char *pi = nullptr, *po = nullptr, *pl = nullptr, *ph = nullptr, *pt = nullptr;
        Access a{};
        hx_status st = resolve_range(c, s.in, s.in_offset, (size_t)s.n * es, &pi, &a, false);
        if (st) return bad(st, "in");
        bp->acc.push_back(a);
        Access ao{};
        st = resolve_range(c, s.out, s.out_offset, (size_t)s.n * es, &po, &ao, true);
        if (st) return bad(st, "out");
        if (ao.buf_slot == a.buf_slot && ao.lo < a.hi && a.lo < ao.hi)
            return bad(HX_ERR_ARG, "in and out overlap");
        bp->acc.push_back(ao);
        if (s.bc_lo == HX_BC_GHOST) {
            st = resolve_range(c, s.halo_lo, s.halo_lo_offset, (size_t)s.halo_width * es, &pl, &a,
                               false);
            if (st) return bad(st, "halo_lo");
            bp->acc.push_back(a);
        }
        if (s.bc_hi == HX_BC_GHOST) {
            st = resolve_range(c, s.halo_hi, s.halo_hi_offset, (size_t)s.halo_width * es, &ph, &a,
                               false);
            if (st) return bad(st, "halo_hi");
            bp->acc.push_back(a);
        }
        if (d->mode == HX_BATCH_PLAIN && d->steps > 1) {
            if (s.tmp == 0) return bad(HX_ERR_ARG, "PLAIN with more than one step needs tmp");
            st = resolve_range(c, s.tmp, s.tmp_offset, (size_t)s.n * es, &pt, &a, true);
            if (st) return bad(st, "tmp");
            bp->acc.push_back(a);
        }
        sg.in = pi;
        sg.out = po;
        sg.halo_lo = pl;
        sg.halo_hi = ph;
        sg.n = s.n;
        sg.r = s.r;
        sg.bc_lo = s.bc_lo;
        sg.bc_hi = s.bc_hi;
        sg.hw = s.halo_width;
        sg.shift = tile_shift(pi, (int)es);
        set_rate_1d(sg, d->steps);
        if (sg.period == 0) bp->scaled = false;
        bp->segs.push_back(sg);
        bp->tmps.push_back(pt);
    }

    // form: PROPAGATOR when asked (every segment must qualify) or, for AUTO,
    // when tuned so or untuned and every segment qualifies
    if (d->mode == HX_BATCH_PERSISTENT && d->dtype == HX_F32 && d->form != HX_FORM_DIRECT) {
        const char* why = nullptr;
        int bad_seg = -1;
        for (size_t i = 0; i < bp->segs.size() && !why; ++i) {
            why = prop_unfit(bp->segs[i], d->steps);
            if (why) bad_seg = (int)i;
        }
        if (d->form == HX_FORM_PROPAGATOR && why) {
            delete bp;
            return c->fail(HX_ERR_ARG, "propagator form: segment " + std::to_string(bad_seg) +
                                           ": " + why);
        }
        const bool tuned_direct = tuned && tg.mode == 1 + HX_FORM_DIRECT;
        bp->prop = !why && !(d->form == HX_FORM_AUTO && tuned_direct);
    }
    if (!bp->prop && fused > max_time_block_1d(d->dtype, bp->g.cpl)) {
        delete bp;
        return c->fail(HX_ERR_ARG, "steps exceed the fused-pass limit of the tile geometry");
    }

    if (bp->prop) {
        // taps of each distinct r, then the segments and the per-wave spans
        std::map<double, size_t> tap_at;
        std::map<double, uint32_t> levels_of, levels16_of;
        std::map<double, int32_t> texp_of;
        std::map<double, double> err_of, err16_of;
        std::vector<float> taps;
        const int D = d->steps;
        for (const Seg1D& sg : bp->segs)
            if (!tap_at.count(sg.r)) {
                tap_at[sg.r] = taps.size();
                const std::vector<double> p = propagator(sg.r, D);
                levels_of[sg.r] = prop1d_levels(p.data(), D);
                levels16_of[sg.r] = prop1d_levels16(p.data(), D);
                texp_of[sg.r] = prop1d_tap_exp(p.data(), D);
                err_of[sg.r] = prop1d_err_bound(p.data(), D, levels_of[sg.r], false, 0);
                err16_of[sg.r] =
                    prop1d_err_bound(p.data(), D, levels16_of[sg.r], true, texp_of[sg.r]);
                for (double v : p) taps.push_back((float)v);
            }
        hipDeviceProp_t prop;
        hipGetDeviceProperties(&prop, c->device);
        int OD = 0, NC = 0;
        prop1d_geometry(D, &OD, &NC);
        // outer chunks that every segment skips (level 0 on both sides)
        int skip = NC;
        for (const auto& kv : levels_of) {
            int k = 0;
            while (k < NC / 2 && ((kv.second >> (2 * k)) & 3) == 0 &&
                   ((kv.second >> (2 * (NC - 1 - k))) & 3) == 0)
                ++k;
            skip = std::min(skip, k);
        }
        bp->pskip = std::min(skip, std::min(2, (NC - 1) / 2));
        // the walk: one wave per block or interleaved when asked
        // (span_blocks = -2, -1) or, with no span given or tuned, whenever
        // every segment has the same size and rate; otherwise contiguous spans
        bool il_ok = levels_of.size() == 1;
        for (const Seg1D& sg : bp->segs) il_ok = il_ok && sg.n == bp->segs[0].n;
        const int64_t bps = (bp->segs[0].n + 1023) / 1024;
        il_ok = il_ok && bps * (int64_t)bp->segs.size() < (int64_t(1) << 32);
        if (d->span_blocks < 0 && !il_ok) {
            destroy_plan(bp);
            return c->fail(HX_ERR_ARG, "span_blocks = -1 or -2 (the interleaved or the block "
                                       "walk) needs segments of one size and one rate");
        }
        if (d->span_blocks == -2 && bp->segs.size() > 65535) {
            destroy_plan(bp);
            return c->fail(HX_ERR_ARG, "span_blocks = -2 (the block walk) takes at most 65535 "
                                       "segments");
        }
        const bool tuned_span = d->form == HX_FORM_AUTO && tuned && tg.rows != 0;
        // untuned, equal segments take the block walk (the interleaved walk
        // where there are more segments than a grid dimension holds)
        const bool bw_ok = il_ok && bp->segs.size() <= 65535;
        const bool dflt = d->span_blocks == 0 && (!tuned_span || tg.rows < 0);
        bp->pbw = bw_ok && (d->span_blocks == -2 || (dflt && (!tuned_span || tg.rows == -2)));
        bp->pil = !bp->pbw && il_ok && (d->span_blocks == -1 || dflt);
        if (bp->pil || bp->pbw) {
            // the fp16 walks' levels decide their dropped chunks
            const uint32_t m = levels16_of.begin()->second;
            int k = 0;
            while (k < NC / 2 && ((m >> (2 * k)) & 3) == 0 && ((m >> (2 * (NC - 1 - k))) & 3) == 0)
                ++k;
            bp->pskip = std::min(k, std::min(2, (NC - 1) / 2));
        }
        const int64_t slots =
            (int64_t)prop.multiProcessorCount *
            prop1d_waves_per_cu(D, bp->pskip, bp->pil ? PROP_IL : PROP_SPAN);
        std::vector<int64_t> blocks;
        for (const Seg1D& sg : bp->segs) blocks.push_back((sg.n + 1023) / 1024);
        const int ni = (bp->pil || bp->pbw) ? 0
                       : d->span_blocks > 0 ? d->span_blocks
                       : (tuned_span && tg.rows > 0)
                           ? tg.rows
                           : choose_span(blocks, slots);
        std::vector<PropWave> waves;
        if (bp->pil || bp->pbw) {
            bp->pbps = bps;
            bp->pblocks = bps * (int64_t)bp->segs.size();
            // one round of resident waves, unless a wave would then take more
            // blocks than it can list for stepping
            bp->pwaves = std::max(std::min<int64_t>(bp->pblocks, slots),
                                  (bp->pblocks + kIlMax - 1) / kIlMax);
        }
        for (size_t i = 0; i < bp->segs.size() && !bp->pil && !bp->pbw; ++i)
            for (int64_t b0 = 0; b0 < blocks[i]; b0 += ni) {
                PropWave w{};
                w.seg = (uint32_t)i;
                w.blk0 = (uint32_t)b0;
                w.ni = (uint32_t)std::min<int64_t>(ni, blocks[i] - b0);
                w.interior = (b0 >= 1 && 1024 * (b0 + w.ni + 1) <= bp->segs[i].n) ? 1u : 0u;
                waves.push_back(w);
            }
        if ((int64_t)waves.size() >= (int64_t(1) << 31) || blocks.back() >= (int64_t(1) << 32)) {
            destroy_plan(bp);
            return c->fail(HX_ERR_RANGE, "the batch has too many propagator waves");
        }
        if (!bp->pil && !bp->pbw) bp->pwaves = (int64_t)waves.size();
        std::vector<uint16_t> tab16;
        if (bp->pbw) {
            // waves per workgroup: given, tuned, else one (4 when asked, on
            // consecutive blocks; other counts are rejected)
            bp->pwpg = d->waves_per_group ? d->waves_per_group
                                          : (tuned_span && tg.wpg ? tg.wpg : 1);
            if (bp->pwpg != 1 && bp->pwpg != 4) {
                destroy_plan(bp);
                return c->fail(HX_ERR_ARG, "the block walk takes 1 or 4 waves per group");
            }
            const double r0 = bp->segs[0].r;
            tab16 = prop1d_bw_table(taps.data() + tap_at[r0], D, bp->pskip, texp_of[r0]);
            bp->pwaves = bp->pblocks;
        }
        bool ok = hipMalloc(&bp->taps_dev, 4 * taps.size()) == hipSuccess &&
                  hipMalloc(&bp->psegs_dev, sizeof(PropSeg) * bp->segs.size()) == hipSuccess &&
                  (bp->pil || bp->pbw ||
                   hipMalloc(&bp->pwaves_dev, sizeof(PropWave) * waves.size()) == hipSuccess) &&
                  (!bp->pbw || (!tab16.empty() &&
                                hipMalloc(&bp->ptab_dev, 2 * tab16.size()) == hipSuccess));
        std::vector<PropSeg> ps;
        if (ok) {
            for (const Seg1D& sg : bp->segs) {
                PropSeg q{};
                q.in = static_cast<const float*>(sg.in);
                q.out = static_cast<float*>(sg.out);
                q.n = sg.n;
                q.coef = bp->taps_dev + tap_at[sg.r];
                q.levels = levels_of[sg.r];
                q.levels16 = levels16_of[sg.r];
                q.texp = texp_of[sg.r];
                q.r = (float)sg.r;
                // the accuracy check's threshold for the walk this plan runs
                q.chk = (bp->pil || bp->pbw)
                            ? (float)std::ldexp(err16_of[sg.r], 21 + 15 + q.texp)
                            : (float)std::ldexp(err_of[sg.r], 21);
                if (sg.bc_lo == HX_BC_PERIODIC) {
                    q.lo_base = q.in + sg.n;
                    q.hi_base = q.in;
                    q.lo_av = q.hi_av = sg.n;
                } else {
                    q.lo_base = static_cast<const float*>(sg.halo_lo) + sg.hw;
                    q.hi_base = static_cast<const float*>(sg.halo_hi);
                    q.lo_av = q.hi_av = 4 * (sg.hw / 4);
                }
                ps.push_back(q);
            }
            ok = hipMemcpy(bp->taps_dev, taps.data(), 4 * taps.size(), hipMemcpyHostToDevice) ==
                     hipSuccess &&
                 hipMemcpy(bp->psegs_dev, ps.data(), sizeof(PropSeg) * ps.size(),
                           hipMemcpyHostToDevice) == hipSuccess &&
                 (bp->pil || bp->pbw ||
                  hipMemcpy(bp->pwaves_dev, waves.data(), sizeof(PropWave) * waves.size(),
                            hipMemcpyHostToDevice) == hipSuccess) &&
                 (!bp->pbw || hipMemcpy(bp->ptab_dev, tab16.data(), 2 * tab16.size(),
                                        hipMemcpyHostToDevice) == hipSuccess);
        }
        if (!ok) {
            hipGetLastError();
            destroy_plan(bp);
            return c->fail(HX_ERR_OOM, "could not allocate the propagator tables");
        }
    } else if (d->mode == HX_BATCH_PERSISTENT) {
        // tile table, largest segments first
        std::vector<int> order(d->count);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return bp->segs[a].n > bp->segs[b].n; });
        std::vector<uint32_t> tseg, tidx;
        for (int i : order) {
            const int64_t nt = tiles_1d(bp->segs[i], bp->g);
            for (int64_t t = 0; t < nt; ++t) {
                tseg.push_back((uint32_t)i);
                tidx.push_back((uint32_t)t);
            }
        }
        bp->ntiles = (int64_t)tseg.size();
        if (bp->ntiles >= (int64_t(1) << 31)) {
            destroy_plan(bp);
            return c->fail(HX_ERR_RANGE, "the batch has more than 2^31 tiles");
        }
        const int64_t nt0 = tiles_1d(bp->segs[0], bp->g);
        bool uniform = true;
        for (const Seg1D& sg : bp->segs)
            if (tiles_1d(sg, bp->g) != nt0) uniform = false;
        if (uniform) {
            // equal tile counts: the table is in segment order, so index = seg * nt0 + tile
            for (size_t i = 0; i < tseg.size(); ++i) {
                tseg[i] = (uint32_t)(i / nt0);
                tidx[i] = (uint32_t)(i % nt0);
            }
            bp->per_seg = nt0;
        }
        // Grid: `wpc` > 0 persistent waves per CU striding over the tiles
        // (software-pipelined), otherwise (the default after tuning) one wave
        // per tile, the faster form measured on MI355X for fused passes.
        const int wpc = d->grid_waves_per_cu ? d->grid_waves_per_cu
                                             : (tuned && tg.grid ? tg.grid : 0);
        hipDeviceProp_t prop;
        hipGetDeviceProperties(&prop, c->device);
        // one wave per tile needs 64 * ntiles work-items, under 2^32
        const int64_t flat_max = (int64_t(1) << 32) / 64 - 1;
        if (wpc <= 0)
            bp->grid_waves = std::min<int64_t>(bp->ntiles, flat_max);
        else
            bp->grid_waves = std::min<int64_t>(bp->ntiles, (int64_t)prop.multiProcessorCount * wpc);
        bool ok = hipMalloc(&bp->segs_dev, sizeof(Seg1D) * bp->segs.size()) == hipSuccess &&
                  hipMalloc(&bp->tseg_dev, 4 * tseg.size()) == hipSuccess &&
                  hipMalloc(&bp->tidx_dev, 4 * tidx.size()) == hipSuccess;
        ok = ok &&
             hipMemcpy(bp->segs_dev, bp->segs.data(), sizeof(Seg1D) * bp->segs.size(),
                       hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(bp->tseg_dev, tseg.data(), 4 * tseg.size(), hipMemcpyHostToDevice) ==
                 hipSuccess &&
             hipMemcpy(bp->tidx_dev, tidx.data(), 4 * tidx.size(), hipMemcpyHostToDevice) ==
                 hipSuccess;
        if (!ok) {
            hipGetLastError();
            destroy_plan(bp);
            return c->fail(HX_ERR_OOM, "could not allocate the batch tables");
        }
    } else if (d->mode == HX_BATCH_GRAPH) {
        bool ok = hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            for (const Seg1D& sg : bp->segs)
                if (launch_stencil1d(bp->dtype, sg, bp->g, bp->cap) != hipSuccess) ok = false;
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(bp->cap, &g) != hipSuccess) ok = false;
            bp->graph = g;
        }
        ok = ok && hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            hipGetLastError();
            destroy_plan(bp);
            return c->fail(HX_ERR_HIP, "graph capture of the batch failed");
        }
    }
    *out = c->add_plan(PLAN_BATCHED, bp, destroy_plan);
    return HX_OK;
}

extern "C" hx_status hx_launch_batched(hx_ctx ctx, hx_plan plan, const hx_event* deps, int ndeps,
                                       hx_event* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    Plan* p = c->get_plan(plan, PLAN_BATCHED);
    if (!p) return c->fail(HX_ERR_INVALID, "invalid batched plan");
    c->capture_plan(plan);
    hipSetDevice(c->device);
    BatchPlan* bp = static_cast<BatchPlan*>(p->impl);
    std::string what = "batched1d x" + std::to_string(bp->segs.size());
    return c->submit(
        SC_COMPUTE, deps, ndeps, bp->acc, what,
        [bp](hipStream_t st) -> hipError_t {
            if (bp->prop && bp->pbw)
                return launch_prop1d_bw(bp->psegs_dev, bp->ptab_dev,
                                        (int64_t)bp->segs.size(), bp->pbps, bp->pwpg,
                                        bp->steps, bp->pskip, st);
            if (bp->prop && bp->pil)
                return launch_prop1d_il(bp->psegs_dev, bp->pblocks, bp->pbps, bp->pwaves,
                                        bp->steps, bp->pskip, st);
            if (bp->prop)
                return launch_prop1d(bp->psegs_dev, bp->pwaves_dev, bp->pwaves, bp->steps,
                                     bp->pskip, st);
            if (bp->mode == HX_BATCH_PERSISTENT)
                return launch_stencil1d_batched(bp->dtype, bp->segs_dev, bp->tseg_dev,
                                                bp->tidx_dev, bp->ntiles, bp->g, bp->grid_waves,
                                                bp->per_seg, bp->scaled, st);
            if (bp->mode == HX_BATCH_GRAPH) return hipGraphLaunch(bp->exec, st);
            // PLAIN: step by step, ping-pong so the last step lands in out
            const int S = bp->steps;
            for (size_t i = 0; i < bp->segs.size(); ++i) {
                const Seg1D& s0 = bp->segs[i];
                const void* src = s0.in;
                for (int t = 0; t < std::max(S, 1); ++t) {
                    Seg1D sg = s0;
                    sg.in = src;
                    sg.out = (S <= 1 || (S - 1 - t) % 2 == 0) ? s0.out : bp->tmps[i];
                    Geom1D g = bp->g;
                    g.steps = S == 0 ? 0 : 1;
                    hipError_t e = launch_stencil1d(bp->dtype, sg, g, st);
                    if (e != hipSuccess) return e;
                    src = sg.out;
                }
            }
            return hipSuccess;
        },
        out);
}

extern "C" hx_status hx_plan_destroy(hx_ctx ctx, hx_plan plan) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Plan* p = c->get_plan(plan, -1);
    if (!p) return HX_ERR_INVALID;
    if (hx_status s = c->no_capture("hx_plan_destroy")) return s;
    if (p->graph_refs > 0)
        return c->fail(HX_ERR_ARG, "a captured graph still uses this plan: destroy the graph "
                                   "first");
    for (hipStream_t s : c->streams) hipStreamSynchronize(s);
    if (p->destroy) p->destroy(p->impl);
    p->live = false;
    p->impl = nullptr;
    return HX_OK;
}
