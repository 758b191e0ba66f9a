// Runtime core of hx: context, handle tables, events and dependency resolution,
// buffers, the hazard checker.  Operation front ends (copies, stencils, plans,
// the adjoint schedule) live in separate translation units and submit their
// work through Ctx::submit.
#pragma once

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <thread>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hx.h"

namespace hx {

// Handle encoding: [kind:8][generation:24][slot:32]; slot 0 is never used so no
// valid handle is 0.
enum HandleKind : uint64_t { HK_BUFFER = 1, HK_EVENT = 2, HK_PLAN = 3 };

inline uint64_t make_handle(HandleKind k, uint32_t gen, uint32_t slot) {
    return ((uint64_t)k << 56) | ((uint64_t)(gen & 0xFFFFFFu) << 32) | slot;
}
inline HandleKind handle_kind(uint64_t h) { return (HandleKind)(h >> 56); }
inline uint32_t handle_gen(uint64_t h) { return (uint32_t)((h >> 32) & 0xFFFFFFu); }
inline uint32_t handle_slot(uint64_t h) { return (uint32_t)h; }

// A byte range an operation touches, for the hazard checker.
struct Access {
    uint32_t buf_slot;
    uint32_t buf_gen;
    uint64_t lo, hi;  // [lo, hi)
    bool write;
};

enum StreamClass { SC_COMPUTE = 0, SC_H2D = 1, SC_D2H = 2 };

struct Buffer {
    uint32_t gen = 0;
    bool live = false;
    bool owned = false;
    void* ptr = nullptr;
    size_t bytes = 0;
    std::vector<uint32_t> uses;  // event slots holding an internal reference
};

struct Event;
using EnqueueFn = std::function<hipError_t(hipStream_t)>;

enum EventKind { EK_DONE = 0, EK_GPU, EK_USER, EK_COMPOSITE, EK_DEFERRED, EK_HOST };

struct Event {
    uint32_t gen = 0;
    bool in_use = false;
    bool user_ref = false;
    int internal_refs = 0;
    EventKind kind = EK_DONE;
    hx_status status = HX_OK;    // HX_PENDING until final
    hipEvent_t hev = nullptr;    // EK_GPU (and EK_DEFERRED once enqueued)
    hipEvent_t hev_start = nullptr;  // timing contexts: recorded after the waits
    int stream = -1;             // index into Ctx::streams
    uint64_t seq = 0;
    bool enqueued = false;       // GPU work for this event has been queued
    std::vector<uint32_t> deps;  // internal refs: for composites and deferred ops
    std::vector<uint32_t> waiters;  // deferred events waiting on this one
    // deferred operation (EK_DEFERRED until enqueued)
    StreamClass sclass = SC_COMPUTE;
    EnqueueFn fn;
    // host task (EK_HOST): runs on the context's host worker once every
    // dependency has completed
    hx_host_fn hfn = nullptr;
    void* huser = nullptr;
    bool running = false;
    // queued while the context captured a graph: stands for a node of that
    // graph, never queried (final once the capture ends)
    bool captured = false;
};

struct Plan {
    uint32_t gen = 0;
    bool live = false;
    int type = 0;
    void* impl = nullptr;
    std::function<void(void*)> destroy;
    int graph_refs = 0;  // captured graphs whose nodes use this plan's tables or code
};

struct Ctx {
    int device = -1;
    bool host_only = true;
    bool check = false;
    bool timing = false;
    std::recursive_mutex mu;
    std::condition_variable_any cv;
    std::vector<hipStream_t> streams;  // [0..ncompute) compute, then H2D, D2H
    int ncompute = 0;
    bool external0 = false;
    int h2d = -1, d2h = -1;
    std::vector<uint32_t> stream_tail;  // event slot last recorded on each stream (0 = none)
    int rr = 0;
    std::vector<Event> events;
    std::vector<uint32_t> free_events;
    std::vector<hipEvent_t> hev_pool;
    std::vector<Buffer> buffers;
    std::vector<uint32_t> free_buffers;
    struct Zombie { void* ptr; std::vector<uint32_t> uses; };
    std::vector<Zombie> zombies;
    std::vector<Plan> plans;
    std::vector<void*> host_allocs;
    uint64_t next_seq = 1;
    uint64_t inject_seq = 0;
    // host tasks
    std::thread worker;
    bool worker_stop = false;
    std::vector<uint32_t> host_tasks;  // pending EK_HOST events (internal refs)
    void start_worker();
    void worker_loop();
    std::string last_error;

    // graph capture (hx_graph_begin .. hx_graph_end): every operation queued in
    // between goes to compute stream 0, in submission order, and is recorded
    // there into one HIP graph by stream capture
    bool capturing = false;
    std::vector<uint32_t> cap_events;  // captured operations (internal refs)
    std::vector<Access> cap_acc;       // the byte ranges they touch
    std::vector<hx_plan> cap_plans;    // plans and programs the captured operations use
    // note that a captured operation uses plan `h` (no-op outside a capture)
    void capture_plan(hx_plan h) {
        if (capturing && std::find(cap_plans.begin(), cap_plans.end(), h) == cap_plans.end())
            cap_plans.push_back(h);
    }
    // HX_ERR_ARG with a message when a capture is open (calls that block on
    // or free GPU work are not allowed then)
    hx_status no_capture(const char* what) {
        return capturing ? fail(HX_ERR_ARG, std::string(what) + " is not allowed while a graph "
                                                                "is being captured")
                         : HX_OK;
    }
    bool has_captured_leaf(uint32_t slot);

    // hazard checker
    struct CNode { std::vector<uint64_t> deps; bool joined = false; std::string what; };
    std::unordered_map<uint64_t, CNode> cnodes;   // by seq
    struct Rec { uint64_t lo, hi; bool write; uint64_t seq; };
    std::unordered_map<uint64_t, std::vector<Rec>> recs;  // by buffer (slot<<32|gen)
    int64_t hazard_count = 0;
    std::string hazard_text;
    uint64_t visit_stamp = 0;
    std::unordered_map<uint64_t, uint64_t> visited;

    // ---------------------------------------------------------------- helpers
    hx_status fail(hx_status s, const std::string& msg) {
        last_error = msg;
        return s;
    }
    Buffer* get_buffer(hx_buffer h);
    Event* get_event(hx_event h);
    uint32_t new_event(EventKind k);
    void ref_event(uint32_t slot) { events[slot].internal_refs++; }
    void unref_event(uint32_t slot);
    void maybe_free_event(uint32_t slot);
    hx_status refresh(uint32_t slot);  // query and cache final status
    void complete_deferred(uint32_t slot);
    void resolve_waiters(uint32_t slot);
    void collect_leaves(uint32_t slot, std::vector<uint32_t>& out);
    hipEvent_t take_hev();
    void sweep();

    // submit an operation: validates deps, handles injection, deferral, stream
    // choice and dependency waits; on success *out receives the event handle.
    hx_status submit(StreamClass sc, const hx_event* deps, int ndeps,
                     const std::vector<Access>& acc, const std::string& what, EnqueueFn fn,
                     hx_event* out);
    hx_status enqueue_now(uint32_t slot);
    hx_event handle_of(uint32_t slot) { return make_handle(HK_EVENT, events[slot].gen, slot); }

    // checker
    void check_op(uint64_t seq, const std::vector<uint64_t>& dep_seqs,
                  const std::vector<Access>& acc, const std::string& what);
    bool is_ancestor(uint64_t anc, uint64_t node);
    void mark_joined(uint64_t seq);

    // plans
    hx_plan add_plan(int type, void* impl, std::function<void(void*)> destroy);
    Plan* get_plan(hx_plan h, int type);
};

// hx_launch_stencil with the context lock already held.
hx_status launch_stencil_locked(Ctx* c, const hx_stencil_args* a, const hx_event* deps, int ndeps,
                                hx_event* out);
hx_status copy_async_locked(Ctx* c, const hx_copy_desc* d, const hx_event* deps, int ndeps,
                            hx_event* out);
hx_status when_all_locked(Ctx* c, const hx_event* evs, int n, hx_event* out);
void release_locked(Ctx* c, hx_event ev);

// Resolve (buffer, offset, bytes) to a device pointer after a range check.
hx_status resolve_range(Ctx* c, hx_buffer b, size_t offset, size_t bytes, char** ptr,
                        Access* acc, bool write);

}  // namespace hx
