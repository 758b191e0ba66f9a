// Captured future graphs: the operations a program submits between
// hx_graph_begin and hx_graph_end are recorded, with their dependencies, into
// one HIP graph, which hx_graph_launch then replays as a single operation.
//
// The paper's futures cost host work per operation (Sec. V-A.1 and V-A.2
// measure that overhead against the native API).  A program that submits the
// same dependency graph many times (the partitioned run's nodes every pass, the
// copy-kernel-copy chain of the sequential stencil) pays it once here: the
// runtime's dependency resolution runs while the graph is captured, and each
// replay is one hipGraphLaunch.
//
// Capture is HIP stream capture of compute stream 0: while it is open, every
// operation (copies included) queues on that stream in submission order,
// which respects every dependency since a dependency is always submitted
// before its dependants; the graph is therefore one chain, which replays the
// operations without the concurrency separate streams would give them.  (A
// capture over all of the context's streams, joined by markers, ended in a
// crash inside hx_graph_end for the per-partition graph over four compute
// streams, cause not found; the one-stream form is what is offered.)  While a
// capture is open, the events of captured operations stand
// for graph nodes: they order later captured operations and cannot be waited
// on; once the capture ends they are complete (as recorded), so operations
// submitted afterwards do not wait on them.  Blocking or freeing calls
// (waits on captured events, synchronisation, destroys, host tasks, foreign
// streams) return HX_ERR_ARG during a capture.
#include "hx_internal.h"
#include "hx_runtime.hpp"

namespace hx {
namespace {

enum { PLAN_GRAPH = 4 };

struct GraphPlan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Access> acc;  // every byte range the captured operations touch
    std::vector<hx_plan> plans;  // plans and programs kept alive for the replays
    Ctx* ctx = nullptr;
    size_t nodes = 0;
    int device = 0;
};

void destroy_graph(void* p) {
    GraphPlan* g = static_cast<GraphPlan*>(p);
    for (hx_plan h : g->plans)
        if (Plan* q = g->ctx ? g->ctx->get_plan(h, -1) : nullptr) q->graph_refs--;
    hipSetDevice(g->device);
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

// End the open capture of `c` and settle the captured events (complete, or
// failed with `err` when the capture failed; for the hazard checker they are
// joined: they never run by themselves, only the graph's launches do, which
// carry their byte ranges).  Returns the graph (nullptr on failure).
hipGraph_t finish_capture(Ctx* c, hipError_t* err) {
    hipGraph_t g = nullptr;
    *err = hipStreamEndCapture(c->streams[0], &g);
    if (*err == hipSuccess && !g) *err = hipErrorInvalidValue;
    c->capturing = false;
    std::vector<uint32_t> evs;
    evs.swap(c->cap_events);
    for (uint32_t slot : evs) {
        Event& e = c->events[slot];
        e.status = *err == hipSuccess ? HX_OK : HX_ERR_HIP;
        e.kind = EK_DONE;
        if (c->check) c->mark_joined(e.seq);
        c->resolve_waiters(slot);
        c->unref_event(slot);
    }
    // the streams' tails are captured markers, which nothing may wait on now
    for (uint32_t& t : c->stream_tail) {
        if (t) c->unref_event(t);
        t = 0;
    }
    if (*err != hipSuccess && g) {
        hipGraphDestroy(g);
        g = nullptr;
    }
    return g;
}

}  // namespace
}  // namespace hx

using namespace hx;

extern "C" {

hx_status hx_graph_begin(hx_ctx ctx) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context cannot capture");
    if (c->capturing) return c->fail(HX_ERR_ARG, "a graph is already being captured");
    if (c->external0)
        return c->fail(HX_ERR_UNSUPPORTED, "a context on a caller's stream cannot capture");
    hipSetDevice(c->device);
    // the tails recorded before the capture are outside it: forget them
    for (uint32_t& t : c->stream_tail) {
        if (t) c->unref_event(t);
        t = 0;
    }
    // the graph starts after the work already queued on stream 0 in the
    // sense that a replay is ordered by its own launch; work queued on the
    // other streams is not part of it
    hipError_t err = hipStreamBeginCapture(c->streams[0], hipStreamCaptureModeRelaxed);
    if (err != hipSuccess)
        return c->fail(HX_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(err));
    c->capturing = true;
    c->cap_events.clear();
    c->cap_acc.clear();
    c->cap_plans.clear();
    return HX_OK;
}

hx_status hx_graph_end(hx_ctx ctx, hx_plan* graph) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!c->capturing) return c->fail(HX_ERR_ARG, "no graph is being captured");
    hipSetDevice(c->device);
    std::vector<Access> acc;
    acc.swap(c->cap_acc);
    std::vector<hx_plan> plans;
    plans.swap(c->cap_plans);
    const size_t nops = c->cap_events.size();
    hipError_t err;
    hipGraph_t g = finish_capture(c, &err);
    if (!graph) {
        if (g) hipGraphDestroy(g);
        return c->fail(HX_ERR_ARG, "null output graph");
    }
    if (!g) return c->fail(HX_ERR_HIP, std::string("graph capture failed: ") + hipGetErrorString(err));
    GraphPlan* gp = new GraphPlan;
    gp->graph = g;
    gp->device = c->device;
    gp->nodes = nops;
    gp->ctx = c;
    for (hx_plan h : plans)
        if (Plan* q = c->get_plan(h, -1)) {
            q->graph_refs++;
            gp->plans.push_back(h);
        }
    err = hipGraphInstantiate(&gp->exec, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        destroy_graph(gp);
        return c->fail(HX_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err));
    }
    // one range per buffer and direction is enough for the deferred frees and
    // the hazard checker
    for (const Access& a : acc) {
        bool merged = false;
        for (Access& b : gp->acc)
            if (b.buf_slot == a.buf_slot && b.buf_gen == a.buf_gen && b.write == a.write) {
                b.lo = std::min(b.lo, a.lo);
                b.hi = std::max(b.hi, a.hi);
                merged = true;
                break;
            }
        if (!merged) gp->acc.push_back(a);
    }
    *graph = c->add_plan(PLAN_GRAPH, gp, destroy_graph);
    return HX_OK;
}

hx_status hx_graph_launch(hx_ctx ctx, hx_plan graph, const hx_event* deps, int ndeps,
                          hx_event* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    if (c->capturing) return c->fail(HX_ERR_ARG, "a graph cannot be launched inside a capture");
    Plan* p = c->get_plan(graph, PLAN_GRAPH);
    if (!p) return c->fail(HX_ERR_INVALID, "invalid graph");
    GraphPlan* gp = static_cast<GraphPlan*>(p->impl);
    for (const Access& a : gp->acc) {
        const Buffer* b = a.buf_slot < c->buffers.size() ? &c->buffers[a.buf_slot] : nullptr;
        if (!b || !b->live || (b->gen & 0xFFFFFFu) != a.buf_gen)
            return c->fail(HX_ERR_INVALID, "a buffer the graph uses has been destroyed");
    }
    hipSetDevice(c->device);
    hipGraphExec_t exec = gp->exec;
    return c->submit(SC_COMPUTE, deps, ndeps, gp->acc, "graph x" + std::to_string(gp->nodes),
                     [exec](hipStream_t st) { return hipGraphLaunch(exec, st); }, out);
}

hx_status hx_graph_info(hx_ctx ctx, hx_plan graph, int64_t* operations) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Plan* p = c->get_plan(graph, PLAN_GRAPH);
    if (!p || !operations) return HX_ERR_ARG;
    *operations = (int64_t)static_cast<GraphPlan*>(p->impl)->nodes;
    return HX_OK;
}

}  // extern "C"
