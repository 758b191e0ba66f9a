// hx runtime core: contexts, handles, events and their dependency resolution,
// buffers, pinned host memory, copies and the hazard checker.
//
// Dependency model (the paper's futures, Sec. III-A, with the native
// synchronisation hidden behind them as in Sec. IV-B): every operation gets an
// event.  An operation whose dependencies are all queued on the GPU is queued at
// once on a stream of its class, after a GPU-side stream-wait on each producer
// recorded on another stream (same-stream producers are ordered by the stream
// itself), so no host round trip sits between dependent operations.  A
// dependency on a host-completed (user) event that is not yet set defers the
// operation: it is kept on the host and queued from hx_user_event_set.  Failures
// travel with the events: an operation with a failed dependency never runs and
// completes with HX_ERR_DEP_FAILED.
#include "hx_internal.h"
#include "hx_runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

namespace hx {

static const char* kStatusNames[] = {"HX_OK", "HX_ERR_INVALID", "HX_ERR_ARG", "HX_ERR_NO_DEVICE",
                                     "HX_ERR_HIP", "HX_ERR_OOM", "HX_ERR_DEP_FAILED",
                                     "HX_ERR_TIMEOUT", "HX_ERR_INJECTED", "HX_ERR_HAZARD",
                                     "HX_ERR_UNSUPPORTED", "HX_ERR_RANGE"};

// ------------------------------------------------------------------ handles
Buffer* Ctx::get_buffer(hx_buffer h) {
    if (handle_kind(h) != HK_BUFFER) return nullptr;
    uint32_t slot = handle_slot(h);
    if (slot == 0 || slot >= buffers.size()) return nullptr;
    Buffer& b = buffers[slot];
    if (!b.live || (b.gen & 0xFFFFFFu) != handle_gen(h)) return nullptr;
    return &b;
}

Event* Ctx::get_event(hx_event h) {
    if (handle_kind(h) != HK_EVENT) return nullptr;
    uint32_t slot = handle_slot(h);
    if (slot == 0 || slot >= events.size()) return nullptr;
    Event& e = events[slot];
    if (!e.in_use || !e.user_ref || (e.gen & 0xFFFFFFu) != handle_gen(h)) return nullptr;
    return &e;
}

hipEvent_t Ctx::take_hev() {
    if (!hev_pool.empty()) {
        hipEvent_t h = hev_pool.back();
        hev_pool.pop_back();
        return h;
    }
    hipEvent_t h = nullptr;
    hipEventCreateWithFlags(&h, timing ? hipEventDefault : hipEventDisableTiming);
    return h;
}

uint32_t Ctx::new_event(EventKind k) {
    uint32_t slot;
    if (!free_events.empty()) {
        slot = free_events.back();
        free_events.pop_back();
    } else {
        slot = (uint32_t)events.size();
        events.emplace_back();
    }
    Event& e = events[slot];
    e.gen = ((e.gen + 1) & 0xFFFFFFu) ? e.gen + 1 : 1;
    e.in_use = true;
    e.user_ref = true;
    e.internal_refs = 0;
    e.kind = k;
    e.status = (k == EK_DONE) ? HX_OK : HX_PENDING;
    e.hev = nullptr;
    e.hev_start = nullptr;
    e.stream = -1;
    e.seq = next_seq++;
    e.enqueued = false;
    e.deps.clear();
    e.waiters.clear();
    e.fn = nullptr;
    e.captured = false;
    return slot;
}

void Ctx::unref_event(uint32_t slot) {
    Event& e = events[slot];
    e.internal_refs--;
    maybe_free_event(slot);
}

void Ctx::maybe_free_event(uint32_t slot) {
    Event& e = events[slot];
    if (!e.in_use || e.user_ref || e.internal_refs > 0) return;
    std::vector<uint32_t> deps;
    deps.swap(e.deps);
    if (e.hev) hev_pool.push_back(e.hev);
    if (e.hev_start) hev_pool.push_back(e.hev_start);
    e.hev = nullptr;
    e.hev_start = nullptr;
    e.in_use = false;
    e.fn = nullptr;
    e.waiters.clear();
    free_events.push_back(slot);
    for (uint32_t d : deps) unref_event(d);
}

static bool leaf_ready(const Event& e) {
    if (e.status != HX_PENDING) return true;
    if (e.kind == EK_GPU) return true;
    return false;  // user event not set, host task not run, or deferred op not yet queued
}

void Ctx::collect_leaves(uint32_t slot, std::vector<uint32_t>& out) {
    Event& e = events[slot];
    if (e.kind == EK_COMPOSITE) {
        for (uint32_t d : e.deps) collect_leaves(d, out);
    } else {
        out.push_back(slot);
    }
}

bool Ctx::has_captured_leaf(uint32_t slot) {
    std::vector<uint32_t> leaves;
    collect_leaves(slot, leaves);
    for (uint32_t l : leaves)
        if (events[l].captured && events[l].status == HX_PENDING) return true;
    return false;
}

hx_status Ctx::refresh(uint32_t slot) {
    Event& e = events[slot];
    if (e.status != HX_PENDING || e.captured) return e.status;
    switch (e.kind) {
    case EK_GPU: {
        hipError_t q = hipEventQuery(e.hev);
        if (q == hipSuccess) {
            e.status = HX_OK;
        } else if (q != hipErrorNotReady) {
            e.status = HX_ERR_HIP;
            last_error = std::string("HIP error on a queued operation: ") + hipGetErrorString(q);
        }
        break;
    }
    case EK_COMPOSITE: {
        bool pending = false;
        hx_status result = HX_OK;
        for (uint32_t d : e.deps) {
            hx_status s = refresh(d);
            if (s == HX_PENDING) pending = true;
            else if (s < 0) result = HX_ERR_DEP_FAILED;
        }
        if (result < 0) e.status = result;
        else if (!pending) e.status = HX_OK;
        if (e.status != HX_PENDING) {
            std::vector<uint32_t> deps;
            deps.swap(e.deps);
            for (uint32_t d : deps) unref_event(d);
        }
        break;
    }
    default:
        break;
    }
    return events[slot].status;
}

void Ctx::resolve_waiters(uint32_t slot) {
    std::vector<uint32_t> ws;
    ws.swap(events[slot].waiters);
    for (uint32_t w : ws) {
        Event& e = events[w];
        if (e.in_use && e.kind == EK_DEFERRED && e.status == HX_PENDING) complete_deferred(w);
        unref_event(w);
    }
    cv.notify_all();
}

// Re-examine a deferred operation: fail it, queue it, or keep waiting.
void Ctx::complete_deferred(uint32_t slot) {
    std::vector<uint32_t> leaves;
    for (uint32_t d : events[slot].deps) collect_leaves(d, leaves);
    for (uint32_t l : leaves) {
        if (refresh(l) < 0) {
            Event& e = events[slot];
            e.status = HX_ERR_DEP_FAILED;
            e.kind = EK_DONE;
            e.fn = nullptr;
            std::vector<uint32_t> deps;
            deps.swap(e.deps);
            for (uint32_t d : deps) unref_event(d);
            resolve_waiters(slot);
            return;
        }
    }
    bool blocked = false;
    for (uint32_t l : leaves) {
        if (!leaf_ready(events[l])) {
            blocked = true;
            auto& ws = events[l].waiters;
            if (std::find(ws.begin(), ws.end(), slot) == ws.end()) {
                ws.push_back(slot);
                ref_event(slot);
            }
        }
    }
    if (!blocked) enqueue_now(slot);
}

hx_status Ctx::enqueue_now(uint32_t slot) {
    std::vector<uint32_t> leaves;
    for (uint32_t d : events[slot].deps) collect_leaves(d, leaves);
    Event& e0 = events[slot];
    int s;
    if (capturing) {
        s = 0;  // a captured graph is recorded on the capture's one stream
    } else if (e0.sclass == SC_H2D) {
        s = h2d;
    } else if (e0.sclass == SC_D2H) {
        s = d2h;
    } else {
        s = -1;
        for (uint32_t l : leaves) {
            const Event& le = events[l];
            if (le.kind == EK_GPU && le.stream >= 0 && le.stream < ncompute &&
                stream_tail[le.stream] == l) {
                s = le.stream;
                break;
            }
        }
        if (s < 0) {
            s = rr;
            rr = (rr + 1) % ncompute;
        }
    }
    hipStream_t st = streams[s];
    for (uint32_t l : leaves) {
        const Event& le = events[l];
        if (le.kind != EK_GPU || le.status == HX_OK) continue;
        if (le.stream == s) continue;  // ordered by the stream itself
        hipStreamWaitEvent(st, le.hev, 0);
    }
    if (timing && !capturing) {
        events[slot].hev_start = take_hev();
        hipEventRecord(events[slot].hev_start, st);
    }
    EnqueueFn fn;
    fn.swap(events[slot].fn);
    hipError_t err = fn ? fn(st) : hipSuccess;
    Event& e = events[slot];
    std::vector<uint32_t> deps;
    deps.swap(e.deps);
    if (err != hipSuccess) {
        e.status = HX_ERR_HIP;
        e.kind = EK_DONE;
        last_error = std::string("launch failed: ") + hipGetErrorString(err);
        for (uint32_t d : deps) unref_event(d);
        resolve_waiters(slot);
        return HX_ERR_HIP;
    }
    e.hev = take_hev();
    hipEventRecord(e.hev, st);
    e.stream = s;
    e.kind = EK_GPU;
    e.enqueued = true;
    if (capturing) {
        e.captured = true;
        cap_events.push_back(slot);
        ref_event(slot);
    }
    if (stream_tail[s]) unref_event(stream_tail[s]);
    stream_tail[s] = slot;
    ref_event(slot);
    for (uint32_t d : deps) unref_event(d);
    resolve_waiters(slot);
    return HX_OK;
}

hx_status Ctx::submit(StreamClass sc, const hx_event* deps, int ndeps,
                      const std::vector<Access>& acc, const std::string& what, EnqueueFn fn,
                      hx_event* out) {
    if (host_only) return fail(HX_ERR_NO_DEVICE, "host-only context cannot run GPU work");
    if (!out) return fail(HX_ERR_ARG, "null output event");
    if (ndeps < 0 || (ndeps > 0 && !deps)) return fail(HX_ERR_ARG, "bad dependency list");
    std::vector<uint32_t> dslots;
    for (int i = 0; i < ndeps; ++i) {
        if (deps[i] == 0) continue;
        if (!get_event(deps[i])) return fail(HX_ERR_INVALID, "invalid dependency event");
        dslots.push_back(handle_slot(deps[i]));
    }
    if (capturing) {
        // inside a graph a dependency is another captured operation, or
        // work that has already completed
        for (uint32_t d : dslots) {
            std::vector<uint32_t> leaves;
            collect_leaves(d, leaves);
            for (uint32_t l : leaves)
                if (!events[l].captured && refresh(l) != HX_OK)
                    return fail(HX_ERR_ARG, "while a graph is being captured, a dependency must "
                                            "be an operation of that graph or complete");
        }
        cap_acc.insert(cap_acc.end(), acc.begin(), acc.end());
    }
    sweep();
    uint32_t slot = new_event(EK_DEFERRED);
    const uint64_t seq = events[slot].seq;
    if (seq == inject_seq) {
        Event& e = events[slot];
        e.kind = EK_DONE;
        e.status = HX_ERR_INJECTED;
        last_error = "injected failure at operation " + std::to_string(seq) + " (" + what + ")";
        if (check) cnodes[seq].what = what;
        *out = handle_of(slot);
        return HX_OK;
    }
    if (check) {
        std::vector<uint64_t> dseq;
        for (uint32_t d : dslots) dseq.push_back(events[d].seq);
        check_op(seq, dseq, acc, what);
    }
    // one reference per buffer (not per access) keeps the buffer's memory alive
    // until this operation completes
    std::vector<uint32_t> bslots;
    for (const Access& a : acc)
        if (std::find(bslots.begin(), bslots.end(), a.buf_slot) == bslots.end())
            bslots.push_back(a.buf_slot);
    for (uint32_t bs : bslots) {
        Buffer& b = buffers[bs];
        if (b.uses.size() >= 32) {
            std::vector<uint32_t> keep;
            for (uint32_t u : b.uses) {
                if (refresh(u) == HX_PENDING) keep.push_back(u);
                else unref_event(u);
            }
            b.uses.swap(keep);
        }
        b.uses.push_back(slot);
        ref_event(slot);
    }
    Event& e = events[slot];
    e.sclass = sc;
    e.fn = std::move(fn);
    for (uint32_t d : dslots) {
        e.deps.push_back(d);
        ref_event(d);
    }
    *out = handle_of(slot);
    complete_deferred(slot);
    return HX_OK;
}

// ------------------------------------------------------------- host tasks
// The worker runs a host task once every leaf of its dependencies is final: it
// blocks on a pending GPU leaf (outside the lock) or sleeps on the condition
// variable for host-completed leaves, then calls the function outside the lock
// and completes the task's event with its return status.
void Ctx::start_worker() {
    if (worker.joinable()) return;
    worker = std::thread([this] { worker_loop(); });
}

void Ctx::worker_loop() {
    std::unique_lock<std::recursive_mutex> lk(mu);
    while (!worker_stop) {
        bool ran = false;
        hipEvent_t block_on = nullptr;
        uint32_t block_slot = 0;
        for (size_t i = 0; i < host_tasks.size() && !ran; ++i) {
            const uint32_t slot = host_tasks[i];
            std::vector<uint32_t> leaves;
            for (uint32_t d : events[slot].deps) collect_leaves(d, leaves);
            bool failed = false, pending = false;
            for (uint32_t l : leaves) {
                hx_status st = refresh(l);
                if (st < 0) failed = true;
                else if (st == HX_PENDING) {
                    pending = true;
                    if (!block_on && events[l].kind == EK_GPU) {
                        block_on = events[l].hev;
                        block_slot = l;
                    }
                }
            }
            if (!failed && pending) continue;
            host_tasks.erase(host_tasks.begin() + i);
            Event& e = events[slot];
            hx_status result = HX_ERR_DEP_FAILED;
            if (!failed) {
                hx_host_fn fn = e.hfn;
                void* user = e.huser;
                e.running = true;
                lk.unlock();
                result = fn ? fn(user) : HX_OK;
                lk.lock();
                if (result > 0) result = HX_OK;
            }
            Event& e2 = events[slot];
            e2.running = false;
            e2.status = result;
            e2.kind = EK_DONE;
            std::vector<uint32_t> deps;
            deps.swap(e2.deps);
            for (uint32_t d : deps) unref_event(d);
            if (check && result == HX_OK) mark_joined(e2.seq);
            resolve_waiters(slot);
            unref_event(slot);
            ran = true;
        }
        if (ran) continue;
        if (block_on && !host_only) {
            ref_event(block_slot);
            lk.unlock();
            hipEventSynchronize(block_on);
            lk.lock();
            refresh(block_slot);
            unref_event(block_slot);
        } else {
            cv.wait_for(lk, std::chrono::milliseconds(host_tasks.empty() ? 50 : 1));
        }
    }
}

void Ctx::sweep() {
    if (zombies.empty() || capturing) return;
    std::vector<Zombie> keep;
    for (Zombie& z : zombies) {
        bool busy = false;
        for (uint32_t u : z.uses)
            if (refresh(u) == HX_PENDING) busy = true;
        if (busy) {
            keep.push_back(std::move(z));
        } else {
            for (uint32_t u : z.uses) unref_event(u);
            hipFree(z.ptr);
        }
    }
    zombies.swap(keep);
}

// ----------------------------------------------------------- hazard checker
bool Ctx::is_ancestor(uint64_t anc, uint64_t node) {
    (void)node;
    auto it = visited.find(anc);
    return it != visited.end() && it->second == visit_stamp;
}

void Ctx::check_op(uint64_t seq, const std::vector<uint64_t>& dep_seqs,
                   const std::vector<Access>& acc, const std::string& what) {
    CNode& node = cnodes[seq];
    node.deps = dep_seqs;
    node.what = what;
    // mark every ancestor of this operation
    ++visit_stamp;
    std::vector<uint64_t> stack(dep_seqs.begin(), dep_seqs.end());
    while (!stack.empty()) {
        uint64_t x = stack.back();
        stack.pop_back();
        auto& v = visited[x];
        if (v == visit_stamp) continue;
        v = visit_stamp;
        auto it = cnodes.find(x);
        if (it != cnodes.end())
            for (uint64_t d : it->second.deps) stack.push_back(d);
    }
    for (const Access& a : acc) {
        uint64_t key = ((uint64_t)a.buf_slot << 32) | a.buf_gen;
        auto& list = recs[key];
        for (const Rec& r : list) {
            if (r.seq == seq) continue;
            if (!(a.lo < r.hi && r.lo < a.hi)) continue;
            if (!a.write && !r.write) continue;
            const CNode& prev = cnodes[r.seq];
            if (prev.joined || is_ancestor(r.seq, seq)) continue;
            ++hazard_count;
            char line[256];
            snprintf(line, sizeof line,
                     "hazard: op %llu (%s) %s bytes [%llu,%llu) of buffer %u unordered with op "
                     "%llu (%s) %s\n",
                     (unsigned long long)seq, what.c_str(), a.write ? "writes" : "reads",
                     (unsigned long long)a.lo, (unsigned long long)a.hi, a.buf_slot,
                     (unsigned long long)r.seq, prev.what.c_str(), r.write ? "write" : "read");
            if (hazard_text.size() < 65536) hazard_text += line;
        }
        list.push_back(Rec{a.lo, a.hi, a.write, seq});
    }
}

void Ctx::mark_joined(uint64_t seq) {
    std::vector<uint64_t> stack{seq};
    while (!stack.empty()) {
        uint64_t x = stack.back();
        stack.pop_back();
        auto it = cnodes.find(x);
        if (it == cnodes.end() || it->second.joined) continue;
        it->second.joined = true;
        for (uint64_t d : it->second.deps) stack.push_back(d);
    }
}

// -------------------------------------------------------------------- plans
hx_plan Ctx::add_plan(int type, void* impl, std::function<void(void*)> destroy) {
    uint32_t slot = 0;
    for (uint32_t i = 1; i < plans.size(); ++i)
        if (!plans[i].live) { slot = i; break; }
    if (slot == 0) {
        if (plans.empty()) plans.emplace_back();
        slot = (uint32_t)plans.size();
        plans.emplace_back();
    }
    Plan& p = plans[slot];
    p.gen = ((p.gen + 1) & 0xFFFFFFu) ? p.gen + 1 : 1;
    p.live = true;
    p.type = type;
    p.impl = impl;
    p.destroy = std::move(destroy);
    return make_handle(HK_PLAN, p.gen, slot);
}

Plan* Ctx::get_plan(hx_plan h, int type) {
    if (handle_kind(h) != HK_PLAN) return nullptr;
    uint32_t slot = handle_slot(h);
    if (slot == 0 || slot >= plans.size()) return nullptr;
    Plan& p = plans[slot];
    if (!p.live || (p.gen & 0xFFFFFFu) != handle_gen(h) || (type >= 0 && p.type != type))
        return nullptr;
    return &p;
}

hx_status resolve_range(Ctx* c, hx_buffer h, size_t offset, size_t bytes, char** ptr,
                        Access* acc, bool write) {
    Buffer* b = c->get_buffer(h);
    if (!b) return c->fail(HX_ERR_INVALID, "invalid buffer handle");
    if (offset > b->bytes || bytes > b->bytes - offset)
        return c->fail(HX_ERR_RANGE, "byte range [" + std::to_string(offset) + ", +" +
                                         std::to_string(bytes) + ") outside a buffer of " +
                                         std::to_string(b->bytes) + " bytes");
    *ptr = static_cast<char*>(b->ptr) + offset;
    if (acc) *acc = Access{handle_slot(h), handle_gen(h), offset, offset + bytes, write};
    return HX_OK;
}

}  // namespace hx

using namespace hx;

#define CTX_OR_FAIL(c)                              \
    if (!(c)) return HX_ERR_INVALID;                \
    std::lock_guard<std::recursive_mutex> lk_((c)->mu)

static inline Ctx* C(hx_ctx c) { return reinterpret_cast<Ctx*>(c); }

extern "C" {

const char* hx_status_string(hx_status s) {
    if (s == HX_PENDING) return "HX_PENDING";
    if (s <= 0 && s >= -11) return kStatusNames[-s];
    return "HX_UNKNOWN_STATUS";
}

hx_status hx_device_count(int* count) {
    if (!count) return HX_ERR_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
    *count = n;
    return HX_OK;
}

hx_status hx_device_info(int dev, hx_device_info_t* info) {
    if (!info) return HX_ERR_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return HX_ERR_NO_DEVICE;
    if (dev < 0 || dev >= n) return HX_ERR_ARG;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return HX_ERR_HIP;
    memset(info, 0, sizeof *info);
    snprintf(info->name, sizeof info->name, "%s", p.name);
    snprintf(info->arch, sizeof info->arch, "%s", p.gcnArchName);
    info->compute_units = p.multiProcessorCount;
    info->wavefront_size = p.warpSize;
    info->clock_khz = p.clockRate;
    info->memory_clock_khz = p.memoryClockRate;
    info->memory_bus_bits = p.memoryBusWidth;
    info->hbm_bytes = p.totalGlobalMem;
    info->lds_bytes_per_cu = p.maxSharedMemoryPerMultiProcessor;
    info->l2_bytes = p.l2CacheSize;
    return HX_OK;
}

hx_status hx_ctx_create(int dev, const hx_ctx_opts* opts, hx_ctx* out) {
    if (!out) return HX_ERR_ARG;
    hx_ctx_opts o{};
    if (opts) o = *opts;
    if (o.compute_streams < 0 || o.compute_streams > 16) return HX_ERR_ARG;
    Ctx* c = new Ctx();
    c->check = o.check != 0;
    c->timing = o.timing != 0;
    c->events.emplace_back();  // slot 0 unused
    c->buffers.emplace_back();
    c->plans.emplace_back();
    if (const char* inj = getenv("HX_FAULT_INJECT")) c->inject_seq = strtoull(inj, nullptr, 10);
    if (dev >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n == 0) { delete c; return HX_ERR_NO_DEVICE; }
        if (dev >= n) { delete c; return HX_ERR_ARG; }
        if (hipSetDevice(dev) != hipSuccess) { delete c; return HX_ERR_HIP; }
        c->device = dev;
        c->host_only = false;
        // Default: leave the copy streams hardware queues of their own.  HIP maps
        // streams onto GPU_MAX_HW_QUEUES queues (4 unless set); streams sharing
        // a queue serialise, which stalls copies behind waiting kernels.
        int hwq = 4;
        if (const char* q = getenv("GPU_MAX_HW_QUEUES")) hwq = std::max(1, atoi(q));
        c->ncompute = o.compute_streams ? o.compute_streams : std::max(1, hwq - 2);
        for (int i = 0; i < c->ncompute + 2; ++i) {
            hipStream_t s = nullptr;
            if (i == 0 && o.external_stream) {
                s = static_cast<hipStream_t>(o.external_stream);
                c->external0 = true;
            } else if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                for (size_t k = (c->external0 ? 1 : 0); k < c->streams.size(); ++k)
                    hipStreamDestroy(c->streams[k]);
                delete c;
                return HX_ERR_HIP;
            }
            c->streams.push_back(s);
        }
        c->h2d = c->ncompute;
        c->d2h = c->ncompute + 1;
        c->stream_tail.assign(c->streams.size(), 0);
        // the device address of the allocation-free loss's scratch (an error
        // here only disables that entry point, which then reports it)
        if (hx::scratch_init(dev) != hipSuccess) hipGetLastError();
    }
    *out = reinterpret_cast<hx_ctx>(c);
    return HX_OK;
}

hx_status hx_ctx_synchronize(hx_ctx ctx) {
    Ctx* c = C(ctx);
    if (!c) return HX_ERR_INVALID;
    std::vector<hipStream_t> ss;
    {
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only) return HX_OK;
        if (hx_status s = c->no_capture("hx_ctx_synchronize")) return s;
        hipSetDevice(c->device);
        ss = c->streams;
    }
    hx_status st = HX_OK;
    for (hipStream_t s : ss)
        if (hipStreamSynchronize(s) != hipSuccess) st = HX_ERR_HIP;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->sweep();
    return st;
}

hx_status hx_ctx_destroy(hx_ctx ctx) {
    Ctx* c = C(ctx);
    if (!c) return HX_ERR_INVALID;
    if (c->worker.joinable()) {
        {
            std::lock_guard<std::recursive_mutex> lk(c->mu);
            c->worker_stop = true;
        }
        c->cv.notify_all();
        c->worker.join();
    }
    if (!c->host_only) {
        hipSetDevice(c->device);
        if (c->capturing) {
            // an open capture is abandoned: end it, drop the graph
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(c->streams[0], &g) == hipSuccess && g) hipGraphDestroy(g);
            hipGetLastError();
            c->capturing = false;
        }
        for (hipStream_t s : c->streams) hipStreamSynchronize(s);
    }
    for (Plan& p : c->plans)
        if (p.live && p.destroy) p.destroy(p.impl);
    for (Buffer& b : c->buffers)
        if (b.live && b.owned && b.ptr) hipFree(b.ptr);
    for (auto& z : c->zombies) hipFree(z.ptr);
    for (void* h : c->host_allocs) hipHostFree(h);
    for (Event& e : c->events) {
        if (e.hev) hipEventDestroy(e.hev);
        if (e.hev_start) hipEventDestroy(e.hev_start);
    }
    for (hipEvent_t h : c->hev_pool) hipEventDestroy(h);
    for (size_t k = (c->external0 ? 1 : 0); k < c->streams.size(); ++k)
        hipStreamDestroy(c->streams[k]);
    delete c;
    return HX_OK;
}

hx_status hx_last_error(hx_ctx ctx, char* buf, size_t len) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!buf || len == 0) return HX_ERR_ARG;
    snprintf(buf, len, "%s", c->last_error.c_str());
    return HX_OK;
}

// ------------------------------------------------------------------ buffers
static hx_status add_buffer(Ctx* c, void* p, size_t bytes, bool owned, hx_buffer* out) {
    uint32_t slot;
    if (!c->free_buffers.empty()) {
        slot = c->free_buffers.back();
        c->free_buffers.pop_back();
    } else {
        slot = (uint32_t)c->buffers.size();
        c->buffers.emplace_back();
    }
    Buffer& b = c->buffers[slot];
    b.gen = ((b.gen + 1) & 0xFFFFFFu) ? b.gen + 1 : 1;
    b.live = true;
    b.owned = owned;
    b.ptr = p;
    b.bytes = bytes;
    b.uses.clear();
    *out = make_handle(HK_BUFFER, b.gen, slot);
    return HX_OK;
}

hx_status hx_buffer_create(hx_ctx ctx, size_t bytes, hx_buffer* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!out) return HX_ERR_ARG;
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    hipSetDevice(c->device);
    void* p = nullptr;
    if (bytes > 0 && hipMalloc(&p, bytes) != hipSuccess) {
        hipGetLastError();
        return c->fail(HX_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return add_buffer(c, p, bytes, true, out);
}

hx_status hx_buffer_wrap(hx_ctx ctx, void* dev_ptr, size_t bytes, hx_buffer* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!out || (!dev_ptr && bytes)) return HX_ERR_ARG;
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    return add_buffer(c, dev_ptr, bytes, false, out);
}

hx_status hx_buffer_destroy(hx_ctx ctx, hx_buffer h) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (hx_status s_ = c->no_capture("hx_buffer_destroy")) return s_;
    Buffer* b = c->get_buffer(h);
    if (!b) return HX_ERR_INVALID;
    b->live = false;
    uint32_t slot = handle_slot(h);
    std::vector<uint32_t> uses;
    uses.swap(b->uses);
    if (b->owned && b->ptr) {
        c->zombies.push_back(Ctx::Zombie{b->ptr, uses});
    } else {
        for (uint32_t u : uses) c->unref_event(u);
    }
    b->ptr = nullptr;
    c->free_buffers.push_back(slot);
    c->sweep();
    return HX_OK;
}

hx_status hx_buffer_ptr(hx_ctx ctx, hx_buffer h, void** p, size_t* bytes) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    Buffer* b = c->get_buffer(h);
    if (!b) return HX_ERR_INVALID;
    if (p) *p = b->ptr;
    if (bytes) *bytes = b->bytes;
    return HX_OK;
}

hx_status hx_host_alloc(hx_ctx ctx, size_t bytes, void** out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!out || bytes == 0) return HX_ERR_ARG;
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    hipSetDevice(c->device);
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        hipGetLastError();
        return c->fail(HX_ERR_OOM, "hipHostMalloc failed");
    }
    c->host_allocs.push_back(p);
    *out = p;
    return HX_OK;
}

hx_status hx_host_free(hx_ctx ctx, void* p) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (hx_status s_ = c->no_capture("hx_host_free")) return s_;
    auto it = std::find(c->host_allocs.begin(), c->host_allocs.end(), p);
    if (it == c->host_allocs.end()) return HX_ERR_ARG;
    c->host_allocs.erase(it);
    hipHostFree(p);
    return HX_OK;
}

// ------------------------------------------------------------------- copies
hx_status hx_copy_async(hx_ctx ctx, const hx_copy_desc* d, const hx_event* deps, int ndeps,
                        hx_event* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    return hx::copy_async_locked(c, d, deps, ndeps, out);
}

}  // extern "C"

hx_status hx::copy_async_locked(Ctx* c, const hx_copy_desc* d, const hx_event* deps, int ndeps,
                                hx_event* out) {
    if (!d || !out) return c->fail(HX_ERR_ARG, "null argument");
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    hipSetDevice(c->device);
    std::vector<Access> acc;
    Access a{};
    char* dev = nullptr;
    const size_t bytes = d->bytes;
    if (d->dir == HX_H2D || d->dir == HX_D2H) {
        if (!d->host && bytes) return c->fail(HX_ERR_ARG, "null host pointer");
        hx_status s = resolve_range(c, d->buf, d->offset, bytes, &dev, &a, d->dir == HX_H2D);
        if (s) return s;
        acc.push_back(a);
        void* host = d->host;
        if (d->dir == HX_H2D) {
            return c->submit(SC_H2D, deps, ndeps, acc, "copy H2D",
                             [=](hipStream_t st) {
                                 return bytes ? hipMemcpyAsync(dev, host, bytes,
                                                               hipMemcpyHostToDevice, st)
                                              : hipSuccess;
                             },
                             out);
        }
        return c->submit(SC_D2H, deps, ndeps, acc, "copy D2H",
                         [=](hipStream_t st) {
                             return bytes ? hipMemcpyAsync(host, dev, bytes,
                                                           hipMemcpyDeviceToHost, st)
                                          : hipSuccess;
                         },
                         out);
    }
    if (d->dir == HX_D2D) {
        char* src = nullptr;
        Access b{};
        hx_status s = resolve_range(c, d->buf, d->offset, bytes, &dev, &a, true);
        if (s) return s;
        s = resolve_range(c, d->src_buf, d->src_offset, bytes, &src, &b, false);
        if (s) return s;
        if (a.buf_slot == b.buf_slot && a.lo < b.hi && b.lo < a.hi)
            return c->fail(HX_ERR_ARG, "overlapping D2D ranges");
        acc.push_back(a);
        acc.push_back(b);
        // aligned ranges take the library's one-pass vector copy kernel, the
        // rest hipMemcpyAsync
        const bool vec = ((reinterpret_cast<uintptr_t>(dev) | reinterpret_cast<uintptr_t>(src) |
                           bytes) & 15u) == 0;
        return c->submit(SC_COMPUTE, deps, ndeps, acc, "copy D2D",
                         [=](hipStream_t st) {
                             if (!bytes) return hipSuccess;
                             if (vec) return launch_copy16(dev, src, bytes, st);
                             return hipMemcpyAsync(dev, src, bytes, hipMemcpyDeviceToDevice, st);
                         },
                         out);
    }
    return c->fail(HX_ERR_ARG, "bad copy direction");
}

void hx::release_locked(Ctx* c, hx_event ev) {
    Event* e = c->get_event(ev);
    if (!e) return;
    e->user_ref = false;
    c->maybe_free_event(handle_slot(ev));
}

extern "C" {

// ------------------------------------------------------------------- events
hx_status hx_when_all(hx_ctx ctx, const hx_event* evs, int n, hx_event* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    return hx::when_all_locked(c, evs, n, out);
}

}  // extern "C"

hx_status hx::when_all_locked(Ctx* c, const hx_event* evs, int n, hx_event* out) {
    if (!out || n < 0 || (n > 0 && !evs)) return HX_ERR_ARG;
    std::vector<uint32_t> slots;
    for (int i = 0; i < n; ++i) {
        if (evs[i] == 0) continue;
        if (!c->get_event(evs[i])) return c->fail(HX_ERR_INVALID, "invalid event in when_all");
        slots.push_back(handle_slot(evs[i]));
    }
    uint32_t slot = c->new_event(slots.empty() ? EK_DONE : EK_COMPOSITE);
    Event& e = c->events[slot];
    for (uint32_t s : slots) {
        e.deps.push_back(s);
        c->ref_event(s);
    }
    if (c->check) {
        std::vector<uint64_t> dseq;
        for (uint32_t s : slots) dseq.push_back(c->events[s].seq);
        c->check_op(c->events[slot].seq, dseq, {}, "when_all");
    }
    *out = c->handle_of(slot);
    return HX_OK;
}

extern "C" {

hx_status hx_event_query(hx_ctx ctx, hx_event ev, hx_status* state) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!state) return HX_ERR_ARG;
    if (ev == 0) { *state = HX_OK; return HX_OK; }
    if (!c->get_event(ev)) return HX_ERR_INVALID;
    if (!c->host_only) hipSetDevice(c->device);
    *state = c->refresh(handle_slot(ev));
    return HX_OK;
}

hx_status hx_wait(hx_ctx ctx, hx_event ev, int64_t timeout_ns) {
    Ctx* c = C(ctx);
    if (!c) return HX_ERR_INVALID;
    if (ev == 0) return HX_OK;
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    std::unique_lock<std::recursive_mutex> lk(c->mu);
    if (!c->get_event(ev)) return HX_ERR_INVALID;
    if (c->capturing && c->has_captured_leaf(handle_slot(ev)))
        return c->fail(HX_ERR_ARG, "an operation of a graph being captured cannot be waited on");
    if (!c->host_only) hipSetDevice(c->device);
    const uint32_t slot = handle_slot(ev);
    c->ref_event(slot);  // keep the slot alive while unlocked
    hx_status result;
    for (;;) {
        hx_status s = c->refresh(slot);
        if (s != HX_PENDING) { result = s; break; }
        if (timeout_ns >= 0 &&
            std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count() >=
                timeout_ns) {
            result = HX_ERR_TIMEOUT;
            break;
        }
        // Block on the GPU events that are already queued; poll the rest.
        std::vector<uint32_t> leaves;
        c->collect_leaves(slot, leaves);
        hipEvent_t hev = nullptr;
        uint32_t hslot = 0;
        for (uint32_t l : leaves) {
            const Event& le = c->events[l];
            if (le.kind == EK_GPU && le.status == HX_PENDING) { hev = le.hev; hslot = l; break; }
        }
        if (hev && timeout_ns < 0) {
            c->ref_event(hslot);
            lk.unlock();
            hipEventSynchronize(hev);
            lk.lock();
            c->refresh(hslot);
            c->unref_event(hslot);
        } else {
            c->cv.wait_for(lk, std::chrono::microseconds(hev ? 20 : 200));
        }
    }
    if (result == HX_OK && c->check) c->mark_joined(c->events[slot].seq);
    c->unref_event(slot);
    return result;
}

hx_status hx_event_release(hx_ctx ctx, hx_event ev) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (ev == 0) return HX_OK;
    Event* e = c->get_event(ev);
    if (!e) return HX_ERR_INVALID;
    e->user_ref = false;
    c->maybe_free_event(handle_slot(ev));
    return HX_OK;
}

hx_status hx_event_elapsed(hx_ctx ctx, hx_event a, hx_event b, double* ms) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!ms) return HX_ERR_ARG;
    if (!c->timing) return c->fail(HX_ERR_UNSUPPORTED, "context created without timing");
    Event* ea = c->get_event(a);
    Event* eb = c->get_event(b);
    if (!ea || !eb) return HX_ERR_INVALID;
    if (ea->kind != EK_GPU || eb->kind != EK_GPU) return c->fail(HX_ERR_ARG, "not GPU events");
    if (c->refresh(handle_slot(a)) != HX_OK || c->refresh(handle_slot(b)) != HX_OK)
        return c->fail(HX_ERR_ARG, "events not complete");
    float f = 0;
    if (hipEventElapsedTime(&f, ea->hev, eb->hev) != hipSuccess) return HX_ERR_HIP;
    *ms = f;
    return HX_OK;
}

hx_status hx_event_span(hx_ctx ctx, hx_event ev, hx_event ref, double* start_ms, double* end_ms) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!start_ms || !end_ms) return HX_ERR_ARG;
    if (!c->timing) return c->fail(HX_ERR_UNSUPPORTED, "context created without timing");
    Event* e = c->get_event(ev);
    Event* r = c->get_event(ref);
    if (!e || !r) return HX_ERR_INVALID;
    if (e->kind != EK_GPU || !e->hev_start || r->kind != EK_GPU)
        return c->fail(HX_ERR_ARG, "not a timed GPU operation");
    if (c->refresh(handle_slot(ev)) != HX_OK || c->refresh(handle_slot(ref)) != HX_OK)
        return c->fail(HX_ERR_ARG, "events not complete");
    float a = 0, b = 0;
    if (hipEventElapsedTime(&a, r->hev, e->hev_start) != hipSuccess) return HX_ERR_HIP;
    if (hipEventElapsedTime(&b, r->hev, e->hev) != hipSuccess) return HX_ERR_HIP;
    *start_ms = a;
    *end_ms = b;
    return HX_OK;
}

hx_status hx_user_event_create(hx_ctx ctx, hx_event* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!out) return HX_ERR_ARG;
    uint32_t slot = c->new_event(EK_USER);
    if (c->check) c->check_op(c->events[slot].seq, {}, {}, "user event");
    *out = c->handle_of(slot);
    return HX_OK;
}

hx_status hx_user_event_set(hx_ctx ctx, hx_event ev, hx_status status) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    Event* e = c->get_event(ev);
    if (!e) return HX_ERR_INVALID;
    if (e->kind != EK_USER) return c->fail(HX_ERR_ARG, "not a user event");
    if (e->status != HX_PENDING) return c->fail(HX_ERR_ARG, "user event already set");
    if (status > 0) return HX_ERR_ARG;
    if (!c->host_only) hipSetDevice(c->device);
    e->status = status;
    c->resolve_waiters(handle_slot(ev));
    return HX_OK;
}

hx_status hx_event_record_stream(hx_ctx ctx, void* stream, hx_event* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (hx_status s_ = c->no_capture("hx_event_record_stream")) return s_;
    if (!out) return HX_ERR_ARG;
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    hipSetDevice(c->device);
    uint32_t slot = c->new_event(EK_GPU);
    Event& e = c->events[slot];
    e.hev = c->take_hev();
    if (hipEventRecord(e.hev, static_cast<hipStream_t>(stream)) != hipSuccess) {
        e.kind = EK_DONE;
        e.status = HX_ERR_HIP;
    }
    e.stream = -1;
    e.enqueued = true;
    if (c->check) c->check_op(e.seq, {}, {}, "foreign stream");
    *out = c->handle_of(slot);
    return HX_OK;
}

hx_status hx_stream_wait_event(hx_ctx ctx, void* stream, hx_event ev) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (hx_status s_ = c->no_capture("hx_stream_wait_event")) return s_;
    if (ev == 0) return HX_OK;
    if (!c->get_event(ev)) return HX_ERR_INVALID;
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    hipSetDevice(c->device);
    std::vector<uint32_t> leaves;
    c->collect_leaves(handle_slot(ev), leaves);
    for (uint32_t l : leaves) {
        hx_status s = c->refresh(l);
        if (s < 0) return HX_ERR_DEP_FAILED;
        if (!leaf_ready(c->events[l]))
            return c->fail(HX_ERR_ARG, "event still held on the host (unset user event)");
    }
    for (uint32_t l : leaves) {
        const Event& le = c->events[l];
        if (le.kind == EK_GPU && le.status == HX_PENDING)
            hipStreamWaitEvent(static_cast<hipStream_t>(stream), le.hev, 0);
    }
    return HX_OK;
}

hx_status hx_host_task(hx_ctx ctx, hx_host_fn fn, void* user, const hx_event* deps, int ndeps,
                       hx_event* out) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (hx_status s_ = c->no_capture("hx_host_task")) return s_;
    if (!out || !fn) return c->fail(HX_ERR_ARG, "null function or output event");
    if (ndeps < 0 || (ndeps > 0 && !deps)) return c->fail(HX_ERR_ARG, "bad dependency list");
    std::vector<uint32_t> dslots;
    for (int i = 0; i < ndeps; ++i) {
        if (deps[i] == 0) continue;
        if (!c->get_event(deps[i])) return c->fail(HX_ERR_INVALID, "invalid dependency event");
        dslots.push_back(handle_slot(deps[i]));
    }
    uint32_t slot = c->new_event(EK_HOST);
    Event& e = c->events[slot];
    const uint64_t seq = e.seq;
    if (seq == c->inject_seq) {
        e.kind = EK_DONE;
        e.status = HX_ERR_INJECTED;
        c->last_error = "injected failure at operation " + std::to_string(seq) + " (host task)";
        *out = c->handle_of(slot);
        return HX_OK;
    }
    e.hfn = fn;
    e.huser = user;
    for (uint32_t d : dslots) {
        c->events[slot].deps.push_back(d);
        c->ref_event(d);
    }
    if (c->check) {
        std::vector<uint64_t> dseq;
        for (uint32_t d : dslots) dseq.push_back(c->events[d].seq);
        c->check_op(seq, dseq, {}, "host task");
    }
    c->host_tasks.push_back(slot);
    c->ref_event(slot);
    c->start_worker();
    c->cv.notify_all();
    *out = c->handle_of(slot);
    return HX_OK;
}

hx_status hx_debug_next_seq(hx_ctx ctx, uint64_t* seq) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!seq) return HX_ERR_ARG;
    *seq = c->next_seq;
    return HX_OK;
}

hx_status hx_debug_inject(hx_ctx ctx, uint64_t seq) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    c->inject_seq = seq;
    return HX_OK;
}

hx_status hx_hazard_count(hx_ctx ctx, int64_t* count) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!count) return HX_ERR_ARG;
    if (!c->check) return c->fail(HX_ERR_UNSUPPORTED, "context created without check");
    *count = c->hazard_count;
    return HX_OK;
}

hx_status hx_hazard_report(hx_ctx ctx, char* buf, size_t len) {
    Ctx* c = C(ctx);
    CTX_OR_FAIL(c);
    if (!buf || len == 0) return HX_ERR_ARG;
    if (!c->check) return c->fail(HX_ERR_UNSUPPORTED, "context created without check");
    snprintf(buf, len, "%s", c->hazard_text.c_str());
    return HX_OK;
}

}  // extern "C"
