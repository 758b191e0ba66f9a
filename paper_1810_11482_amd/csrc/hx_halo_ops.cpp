// Halo plans: a table of pack/unpack descriptors resolved and uploaded once,
// then run as one kernel per hx_launch_halo.
#include <string>
#include <vector>

#include "hx_internal.h"
#include "hx_runtime.hpp"

using namespace hx;

namespace {

enum { PLAN_HALO = 2 };

struct HaloPlan {
    HaloDev* descs = nullptr;
    int64_t* first = nullptr;
    int nd = 0;
    int64_t total = 0;
    std::vector<Access> acc;
    int device = 0;
};

void destroy_halo(void* p) {
    HaloPlan* h = static_cast<HaloPlan*>(p);
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    if (h->descs) hipFree(h->descs);
    if (h->first) hipFree(h->first);
    delete h;
}

}  // namespace

extern "C" hx_status hx_plan_create_halo(hx_ctx ctx, const hx_halo_desc* d, int n, hx_plan* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out || n < 1 || !d) return c->fail(HX_ERR_ARG, "n >= 1 descriptors required");
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    hipSetDevice(c->device);
    auto* h = new HaloPlan();
    h->device = c->device;
    std::vector<HaloDev> dev(n);
    std::vector<int64_t> first(n);
    for (int i = 0; i < n; ++i) {
        const hx_halo_desc& x = d[i];
        auto bad = [&](hx_status st, const std::string& m) {
            delete h;
            return c->fail(st, "halo descriptor " + std::to_string(i) + ": " + m);
        };
        if (x.rows < 0 || x.row_bytes < 0 || x.row_bytes % 4 != 0)
            return bad(HX_ERR_ARG, "rows >= 0 and row_bytes a non-negative multiple of 4");
        if (x.rows > 1 && (x.src_pitch < x.row_bytes || x.dst_pitch < x.row_bytes))
            return bad(HX_ERR_ARG, "pitches must be at least row_bytes");
        const size_t span_s = x.rows ? (size_t)((x.rows - 1) * x.src_pitch + x.row_bytes) : 0;
        const size_t span_d = x.rows ? (size_t)((x.rows - 1) * x.dst_pitch + x.row_bytes) : 0;
        char *ps = nullptr, *pd = nullptr;
        Access as{}, ad{};
        hx_status st = resolve_range(c, x.src, x.src_offset, span_s, &ps, &as, false);
        if (st) return bad(st, "src");
        st = resolve_range(c, x.dst, x.dst_offset, span_d, &pd, &ad, true);
        if (st) return bad(st, "dst");
        if (as.buf_slot == ad.buf_slot && as.lo < ad.hi && ad.lo < as.hi)
            return bad(HX_ERR_ARG, "source and destination spans overlap");
        h->acc.push_back(as);
        h->acc.push_back(ad);
        dev[i] = HaloDev{ps, pd, x.rows, x.row_bytes, x.src_pitch, x.dst_pitch};
        first[i] = h->total;
        h->total += x.rows;
    }
    h->nd = n;
    bool ok = hipMalloc(&h->descs, sizeof(HaloDev) * n) == hipSuccess &&
              hipMalloc(&h->first, sizeof(int64_t) * n) == hipSuccess &&
              hipMemcpy(h->descs, dev.data(), sizeof(HaloDev) * n, hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(h->first, first.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice) ==
                  hipSuccess;
    if (!ok) {
        hipGetLastError();
        destroy_halo(h);
        return c->fail(HX_ERR_OOM, "could not upload the halo table");
    }
    *out = c->add_plan(PLAN_HALO, h, destroy_halo);
    return HX_OK;
}

extern "C" hx_status hx_launch_halo(hx_ctx ctx, hx_plan plan, const hx_event* deps, int ndeps,
                                    hx_event* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    Plan* p = c->get_plan(plan, PLAN_HALO);
    if (!p) return c->fail(HX_ERR_INVALID, "invalid halo plan");
    c->capture_plan(plan);
    hipSetDevice(c->device);
    HaloPlan* h = static_cast<HaloPlan*>(p->impl);
    return c->submit(SC_COMPUTE, deps, ndeps, h->acc, "halo x" + std::to_string(h->nd),
                     [h](hipStream_t st) {
                         return launch_halo(h->descs, h->first, h->nd, h->total, st);
                     },
                     out);
}
