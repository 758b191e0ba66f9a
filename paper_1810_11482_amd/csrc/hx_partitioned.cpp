// Partitioned 1D runs composed as future graphs (the paper's partition
// benchmark, Sec. V-A.2 / Algorithm 1, with the stencil of Sec. V-A.1).
//
// hx_run_partitioned: a device-resident array split over `parts` buffers is
// advanced in passes of `time_block` steps.  Node (p, b) reads partition p's
// state of pass b-1 and time_block halo cells straight from the neighbours'
// buffers, writes the other ping-pong buffer, and depends on nodes
// (p-1, b-1), (p, b-1), (p+1, b-1).  Those three edges carry the halo (read
// after write) and also order the next overwrite of a buffer after every read
// of it (node (p, b+1) writes the buffer nodes (p+-1, b) read, and depends on
// them).  The plain form is the same work issued in Algorithm 1's order with
// one step per launch, every launch chained on one stream.
//
// hx_run_pipeline: host-resident input: Algorithm 1's three loops (every H2D
// copy, then one fused kernel pass per partition, then every D2H copy), with
// each kernel depending on its own and its neighbours' copies (it reads its
// halos from their device buffers), so copies of one partition overlap the
// kernels of others and the two copy directions overlap each other.
#include <algorithm>
#include <string>
#include <vector>

#include "hx_internal.h"
#include "hx_runtime.hpp"

using namespace hx;

namespace {

size_t esz(int dtype) { return dtype == HX_F64 ? 8 : 4; }

// Cells per partition unit: 1 for a 1D run, nx for a row of a 2D band.
int64_t unit(const hx_partitioned_desc* d) { return d->dims == 2 ? d->nx : 1; }

// Kernel arguments of one partition node: sizes[p] cells (1D) or rows (2D).
void node_args(const hx_partitioned_desc* d, int p, hx_stencil_args* a) {
    a->dims = d->dims == 2 ? 2 : 1;
    a->dtype = d->dtype;
    a->nx = d->dims == 2 ? d->nx : d->sizes[p];
    a->ny = d->dims == 2 ? d->sizes[p] : 1;
    a->r = d->r;
    a->cells_per_lane = d->cells_per_lane;
    a->waves_per_group = d->waves_per_group;
    a->rows_per_block = d->rows_per_block;
}

hx_status validate(Ctx* c, const hx_partitioned_desc* d) {
    if (!d) return c->fail(HX_ERR_ARG, "null descriptor");
    if (d->dtype != HX_F32 && d->dtype != HX_F64) return c->fail(HX_ERR_ARG, "bad dtype");
    if (d->parts < 1 || !d->sizes || !d->bufs_a || !d->bufs_b)
        return c->fail(HX_ERR_ARG, "parts, sizes and both buffer arrays are required");
    if (d->steps < 0) return c->fail(HX_ERR_ARG, "negative steps");
    for (int p = 0; p < d->parts; ++p)
        if (d->sizes[p] <= 0) return c->fail(HX_ERR_ARG, "partition sizes must be positive");
    if (d->dims != 0 && d->dims != 1 && d->dims != 2) return c->fail(HX_ERR_ARG, "bad dims");
    if (d->dims == 2 && (d->nx <= 0 || d->periodic))
        return c->fail(HX_ERR_ARG, "2D bands need nx > 0 and periodic = 0");
    return HX_OK;
}

}  // namespace

namespace {

// HX_PART_BATCHED for 2D bands: every pass advances all bands in launches of
// up to kMaxBands bands each (one node per launch), each band reading its halo
// rows from its neighbours' buffers of the previous pass.  A node depends on
// every node of the previous pass.
hx_status run_bands_batched(Ctx* c, const hx_partitioned_desc* d, hx_event gate, hx_event* out,
                            int* final_in_b, hx_event* node_events) {
    const int P = d->parts;
    const int dt = d->dtype == HX_F64 ? 1 : 0;
    const int64_t es = dt ? 8 : 4;
    const int vn = dt ? 2 : 4;
    Geom2D g;
    g.cpl = d->cells_per_lane ? d->cells_per_lane : 4;
    g.rows = d->rows_per_block ? d->rows_per_block : 128;
    g.wpg = d->waves_per_group ? d->waves_per_group : 4;
    if (g.wpg != 1 && g.wpg != 2 && g.wpg != 4)
        return c->fail(HX_ERR_ARG, "waves_per_group must be 1, 2 or 4");
    if (g.rows < 1) return c->fail(HX_ERR_ARG, "rows_per_block must be positive");
    const int D = d->time_block > 0 ? d->time_block : std::min(d->steps, 8);
    int64_t min_rows = d->sizes[0];
    for (int p = 1; p < P; ++p) min_rows = std::min(min_rows, d->sizes[p]);
    if (D > min_rows) return c->fail(HX_ERR_ARG, "time_block exceeds the smallest band");
    // pass depths: D, D, ..., remainder; every depth must have a kernel
    std::vector<int> plan;
    for (int left = d->steps; left > 0; left -= std::min(D, left)) plan.push_back(std::min(D, left));
    for (int depth : plan)
        if (!stencil2d_supported(dt, g.cpl, depth))
            return c->fail(HX_ERR_ARG, "unsupported 2D pass depth " + std::to_string(depth));
    const int groups = (P + kMaxBands - 1) / kMaxBands;
    std::vector<hx_event> prev, cur;
    if (gate) {
        hx_event gcopy = 0;
        hx_status s = when_all_locked(c, &gate, 1, &gcopy);
        if (s) return s;
        prev.push_back(gcopy);
    }
    const bool give = node_events != nullptr;
    int node = 0;
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    // On an error, drop our references (node events handed to the caller
    // stay the caller's); what was already queued still runs.
    bool first_pass = true;
    auto unwind = [&](hx_status st) {
        if (!give || first_pass)
            for (hx_event e : prev) release_locked(c, e);
        if (!give)
            for (hx_event e : cur) release_locked(c, e);
        return st;
    };
    for (size_t b = 0; b < plan.size(); ++b) {
        const int depth = plan[b];
        const bool src_a = (b % 2 == 0);
        Geom2D gg = g;
        gg.steps = depth;
        gg.halo = std::max(vn, (depth + vn - 1) / vn * vn);
        for (int gi = 0; gi < groups; ++gi) {
            const int p0 = gi * kMaxBands, p1 = std::min(P, p0 + kMaxBands);
            std::vector<Band2D> bands;
            std::vector<Access> acc;
            for (int p = p0; p < p1; ++p) {
                const hx_buffer in = src_a ? d->bufs_a[p] : d->bufs_b[p];
                const hx_buffer outb = src_a ? d->bufs_b[p] : d->bufs_a[p];
                const int64_t band_bytes = d->sizes[p] * d->nx * es;
                char *pin = nullptr, *pout = nullptr, *ptop = nullptr, *pbot = nullptr;
                Access a{};
                hx_status s = resolve_range(c, in, 0, (size_t)band_bytes, &pin, &a, false);
                if (s) return unwind(s);
                acc.push_back(a);
                s = resolve_range(c, outb, 0, (size_t)band_bytes, &pout, &a, true);
                if (s) return unwind(s);
                acc.push_back(a);
                Band2D bd{};
                bd.nx = d->nx;
                bd.ny = d->sizes[p];
                bd.r = d->r;
                bd.hw = depth;
                bd.bc_top = p > 0 ? HX_BC_GHOST : HX_BC_DIRICHLET0;
                bd.bc_bot = p < P - 1 ? HX_BC_GHOST : HX_BC_DIRICHLET0;
                const size_t hb = (size_t)depth * d->nx * es;
                if (p > 0) {
                    const hx_buffer hbuf = src_a ? d->bufs_a[p - 1] : d->bufs_b[p - 1];
                    s = resolve_range(c, hbuf, (size_t)(d->sizes[p - 1] - depth) * d->nx * es, hb,
                                      &ptop, &a, false);
                    if (s) return unwind(s);
                    acc.push_back(a);
                }
                if (p < P - 1) {
                    const hx_buffer hbuf = src_a ? d->bufs_a[p + 1] : d->bufs_b[p + 1];
                    s = resolve_range(c, hbuf, 0, hb, &pbot, &a, false);
                    if (s) return unwind(s);
                    acc.push_back(a);
                }
                bd.in = pin;
                bd.out = pout;
                bd.halo_top = ptop;
                bd.halo_bot = pbot;
                bd.aligned = (d->nx % vn == 0) && al(pin) && al(pout) && (!ptop || al(ptop)) &&
                             (!pbot || al(pbot));
                bands.push_back(bd);
            }
            hx_event ev = 0;
            const int dtype = dt;
            hx_status s = c->submit(
                SC_COMPUTE, prev.data(), (int)prev.size(), acc,
                "stencil2d batched pass of " + std::to_string(bands.size()) + " bands",
                [bands, gg, dtype](hipStream_t st) -> hipError_t {
                    return launch_stencil2d_bands(dtype, bands.data(), (int)bands.size(), gg, st);
                },
                &ev);
            if (s) return unwind(s);
            cur.push_back(ev);
            if (give) node_events[node++] = ev;
        }
        // prev holds the gate's copy (pass 0) or our own node events
        if (!give || first_pass)
            for (hx_event e : prev) release_locked(c, e);
        prev.swap(cur);
        cur.clear();
        first_pass = false;
    }
    hx_status s;
    if (plan.empty()) {
        s = prev.empty() ? when_all_locked(c, nullptr, 0, out)
                         : when_all_locked(c, prev.data(), (int)prev.size(), out);
        for (hx_event e : prev) release_locked(c, e);
        if (final_in_b) *final_in_b = 0;
        return s;
    }
    s = when_all_locked(c, prev.data(), (int)prev.size(), out);
    if (!give)
        for (hx_event e : prev) release_locked(c, e);
    if (final_in_b) *final_in_b = (plan.size() % 2 == 1);
    return s;
}

}  // namespace

extern "C" hx_status hx_run_partitioned(hx_ctx ctx, const hx_partitioned_desc* d,
                                        const hx_event* deps, int ndeps, hx_event* out,
                                        int* final_in_b, hx_event* node_events) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = validate(c, d);
    if (s) return s;
    if (d->mode == HX_PART_BATCHED) {
        if (d->dims != 2)
            return c->fail(HX_ERR_ARG, "HX_PART_BATCHED runs 2D bands; 1D batches use "
                                       "hx_plan_create_batched");
        if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
        hx_event gate = 0;
        if (ndeps > 0) {
            s = when_all_locked(c, deps, ndeps, &gate);
            if (s) return s;
        }
        s = run_bands_batched(c, d, gate, out, final_in_b, node_events);
        release_locked(c, gate);
        return s;
    }
    if (d->mode != HX_PART_GRAPH && d->mode != HX_PART_PLAIN)
        return c->fail(HX_ERR_ARG, "bad mode");
    const int P = d->parts;
    const bool plain = d->mode == HX_PART_PLAIN;
    const int defD = d->dims == 2 ? 8 : 32;
    int D = plain ? 1 : (d->time_block > 0 ? d->time_block : std::min(d->steps, defD));
    if (D < 1) D = 1;
    int64_t min_size = d->sizes[0];
    for (int p = 1; p < P; ++p) min_size = std::min(min_size, d->sizes[p]);
    if (D > min_size) return c->fail(HX_ERR_ARG, "time_block exceeds the smallest partition");
    const int passes = d->steps == 0 ? 0 : (d->steps + D - 1) / D;
    const size_t es = esz(d->dtype);

    std::vector<hx_event> prev(P, 0), cur(P, 0);
    hx_event chain = 0;  // plain form: every launch after the previous one
    const bool give = node_events != nullptr;  // node events belong to the caller
    hx_event gate = 0;
    if (ndeps > 0) {
        s = when_all_locked(c, deps, ndeps, &gate);
        if (s) return s;
    }
    auto cleanup = [&](hx_status st) {
        if (!give) {
            for (hx_event e : prev) release_locked(c, e);
            for (hx_event e : cur) release_locked(c, e);
        }
        release_locked(c, gate);
        return st;
    };
    int left = d->steps;
    int node = 0;
    for (int b = 0; b < passes; ++b) {
        const int steps_b = std::min(D, left);
        const bool src_a = (b % 2 == 0);
        for (int p = 0; p < P; ++p) {
            const int lp = (p + P - 1) % P, rp = (p + 1) % P;
            hx_stencil_args a{};
            node_args(d, p, &a);
            a.steps = steps_b;
            a.in = src_a ? d->bufs_a[p] : d->bufs_b[p];
            a.out = src_a ? d->bufs_b[p] : d->bufs_a[p];
            const bool has_lo = d->periodic || p > 0;
            const bool has_hi = d->periodic || p < P - 1;
            a.bc_lo = has_lo ? HX_BC_GHOST : HX_BC_DIRICHLET0;
            a.bc_hi = has_hi ? HX_BC_GHOST : HX_BC_DIRICHLET0;
            a.halo_lo = src_a ? d->bufs_a[lp] : d->bufs_b[lp];
            a.halo_lo_offset = (size_t)(d->sizes[lp] - steps_b) * unit(d) * es;
            a.halo_hi = src_a ? d->bufs_a[rp] : d->bufs_b[rp];
            a.halo_hi_offset = 0;
            a.halo_width = steps_b;
            hx_event dv[4];
            int nd = 0;
            if (plain) {
                dv[nd++] = chain ? chain : gate;
            } else if (b == 0) {
                dv[nd++] = gate;
            } else {
                dv[nd++] = prev[p];
                if (has_lo) dv[nd++] = prev[lp];
                if (has_hi) dv[nd++] = prev[rp];
            }
            hx_event ev = 0;
            s = launch_stencil_locked(c, &a, dv, nd, &ev);
            if (s) return cleanup(s);
            cur[p] = ev;
            if (plain) chain = ev;
            if (give) node_events[node] = ev;
            ++node;
        }
        for (int p = 0; p < P; ++p) {
            if (!give) release_locked(c, prev[p]);
            prev[p] = cur[p];
            cur[p] = 0;
        }
        left -= steps_b;
    }
    if (passes == 0) {
        s = when_all_locked(c, &gate, 1, out);
        release_locked(c, gate);
        if (final_in_b) *final_in_b = 0;
        return s;
    }
    s = when_all_locked(c, prev.data(), P, out);
    if (final_in_b) *final_in_b = (passes % 2 == 1);
    cleanup(HX_OK);
    return s;
}

extern "C" hx_status hx_run_pipeline(hx_ctx ctx, const hx_pipeline_desc* pd, const hx_event* deps,
                                     int ndeps, hx_event* out, hx_event* op_events) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!pd || !out) return c->fail(HX_ERR_ARG, "null argument");
    const hx_partitioned_desc* d = &pd->part;
    hx_status s = validate(c, d);
    if (s) return s;
    if (!pd->host_in || !pd->host_out) return c->fail(HX_ERR_ARG, "host_in and host_out required");
    const int P = d->parts;
    const int T = d->steps;
    const size_t es = esz(d->dtype);
    int64_t total = 0, min_size = d->sizes[0];
    std::vector<int64_t> off(P);
    for (int p = 0; p < P; ++p) {
        off[p] = total;
        total += d->sizes[p] * unit(d);
        min_size = std::min(min_size, d->sizes[p]);
    }
    if (T > min_size) return c->fail(HX_ERR_ARG, "steps exceed the smallest partition");
    hx_event gate = 0;
    if (ndeps > 0) {
        s = when_all_locked(c, deps, ndeps, &gate);
        if (s) return s;
    }
    // Operation events go to the caller when op_events is given (H2D, kernel,
    // D2H, each `parts` long, indexed by partition); otherwise they are ours.
    std::vector<hx_event> keep;
    auto record = [&](int slot, hx_event e) {
        if (op_events) op_events[slot] = e;
        else keep.push_back(e);
    };
    const char* hin = static_cast<const char*>(pd->host_in);
    char* hout = static_cast<char*>(pd->host_out);
    auto unwind = [&](hx_status st) {
        for (hx_event e : keep) release_locked(c, e);
        release_locked(c, gate);
        return st;
    };
    // 1) every copy in (Algorithm 1's first loop)
    std::vector<hx_event> ein(P, 0), ek(P, 0);
    for (int p = 0; p < P; ++p) {
        hx_copy_desc cd{};
        cd.dir = HX_H2D;
        cd.host = const_cast<char*>(hin) + off[p] * es;
        cd.buf = d->bufs_a[p];
        cd.bytes = (size_t)(d->sizes[p] * unit(d)) * es;
        s = copy_async_locked(c, &cd, &gate, gate ? 1 : 0, &ein[p]);
        if (s) return unwind(s);
        record(p, ein[p]);
    }
    // 2) one fused pass per partition; its halos are read from the neighbours'
    //    freshly copied buffers, so it waits for their copies too.  Kernels are
    //    issued in the order they can start: partition 0 of a periodic array
    //    needs the last copy in, so it goes last and blocks no stream meanwhile.
    const bool wrap = d->periodic && P > 1 && T > 0;
    for (int q = 0; q < P; ++q) {
        const int p = wrap ? (q + 1) % P : q;
        const int lp = (p + P - 1) % P, rp = (p + 1) % P;
        const bool has_lo = d->periodic || p > 0;
        const bool has_hi = d->periodic || p < P - 1;
        hx_stencil_args a{};
        node_args(d, p, &a);
        a.steps = T;
        a.in = d->bufs_a[p];
        a.out = d->bufs_b[p];
        const bool halo = T > 0;
        a.bc_lo = (has_lo && halo) ? HX_BC_GHOST : HX_BC_DIRICHLET0;
        a.bc_hi = (has_hi && halo) ? HX_BC_GHOST : HX_BC_DIRICHLET0;
        a.halo_lo = d->bufs_a[lp];
        a.halo_lo_offset = (size_t)(d->sizes[lp] - T) * unit(d) * es;
        a.halo_hi = d->bufs_a[rp];
        a.halo_width = T;
        hx_event dv[3];
        int nd = 0;
        dv[nd++] = ein[p];
        if (halo && has_lo) dv[nd++] = ein[lp];
        if (halo && has_hi && rp != lp) dv[nd++] = ein[rp];
        s = launch_stencil_locked(c, &a, dv, nd, &ek[p]);
        if (s) return unwind(s);
        record(P + p, ek[p]);
    }
    // 3) copies out, in the order the kernels can finish (partition 0 of a
    //    periodic array waits for the last copy in, so it goes last)
    std::vector<hx_event> finals;
    for (int q = 0; q < P; ++q) {
        const int p = wrap ? (q + 1) % P : q;
        hx_copy_desc cd{};
        cd.dir = HX_D2H;
        cd.host = hout + off[p] * es;
        cd.buf = d->bufs_b[p];
        cd.bytes = (size_t)(d->sizes[p] * unit(d)) * es;
        hx_event eo = 0;
        s = copy_async_locked(c, &cd, &ek[p], 1, &eo);
        if (s) return unwind(s);
        finals.push_back(eo);
        record(2 * P + p, eo);
    }
    s = when_all_locked(c, finals.data(), (int)finals.size(), out);
    for (hx_event e : keep) release_locked(c, e);
    release_locked(c, gate);
    return s;
}
