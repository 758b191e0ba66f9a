// Runtime-compiled programs (the paper's program object, Sec. IV and
// Listing 2: source text compiled at run time, kernels run with arguments,
// grid and block as future-returning operations).  hiprtc compiles HIP C++
// for the context's device; the code object is loaded as a HIP module.
#include <hip/hiprtc.h>

#include <array>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hx_runtime.hpp"

using namespace hx;

namespace {

enum { PLAN_PROGRAM = 3 };

struct Program {
    std::string source, name, log;
    std::vector<char> code;
    hipModule_t module = nullptr;
    std::map<std::string, hipFunction_t> fns;
    bool built = false;
    int device = -1;
};

void destroy_program(void* p) {
    Program* pr = static_cast<Program*>(p);
    if (pr->module) {
        hipSetDevice(pr->device);
        hipModuleUnload(pr->module);
    }
    delete pr;
}

// The architecture name of the context's device up to its feature suffix
// ("gfx950:sramecc+:xnack-" -> "gfx950"); gfx950 for a host-only context.
std::string device_arch(Ctx* c) {
    if (c->host_only) return "gfx950";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return "gfx950";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

Program* get_program(Ctx* c, hx_program h) {
    Plan* p = c->get_plan(h, PLAN_PROGRAM);
    return p ? static_cast<Program*>(p->impl) : nullptr;
}

hx_status lookup(Ctx* c, Program* pr, const char* kernel, hipFunction_t* fn) {
    if (!pr->built || !pr->module) return c->fail(HX_ERR_ARG, "the program is not built and loaded");
    if (!kernel) return c->fail(HX_ERR_ARG, "null kernel name");
    auto it = pr->fns.find(kernel);
    if (it != pr->fns.end()) {
        *fn = it->second;
        return HX_OK;
    }
    hipSetDevice(c->device);
    hipFunction_t f = nullptr;
    if (hipModuleGetFunction(&f, pr->module, kernel) != hipSuccess || !f) {
        hipGetLastError();
        return c->fail(HX_ERR_ARG, std::string("no kernel named ") + kernel + " in the program");
    }
    pr->fns[kernel] = f;
    *fn = f;
    return HX_OK;
}

}  // namespace

extern "C" {

hx_status hx_program_create(hx_ctx ctx, const char* source, const char* name, hx_program* prog) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!source || !prog) return c->fail(HX_ERR_ARG, "null source or output");
    auto* pr = new Program();
    pr->source = source;
    pr->name = name ? name : "program.hip";
    pr->device = c->device;
    *prog = c->add_plan(PLAN_PROGRAM, pr, destroy_program);
    return HX_OK;
}

hx_status hx_program_build(hx_ctx ctx, hx_program prog, const char* const* options, int nopts) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Program* pr = get_program(c, prog);
    if (!pr) return c->fail(HX_ERR_INVALID, "invalid program handle");
    if (pr->built) return c->fail(HX_ERR_ARG, "the program is already built");
    if (nopts < 0 || (nopts > 0 && !options)) return c->fail(HX_ERR_ARG, "bad option list");
    const std::string arch = "--offload-arch=" + device_arch(c);
    std::vector<const char*> opts = {arch.c_str(), "-O3",       "-Xclang",
                                     "-target-feature", "-Xclang", "-packed-fp32-ops"};
    for (int i = 0; i < nopts; ++i) {
        if (!options[i]) return c->fail(HX_ERR_ARG, "null option string");
        opts.push_back(options[i]);
    }
    hiprtcProgram rp = nullptr;
    if (hiprtcCreateProgram(&rp, pr->source.c_str(), pr->name.c_str(), 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return c->fail(HX_ERR_HIP, "hiprtcCreateProgram failed");
    const hiprtcResult cr = hiprtcCompileProgram(rp, (int)opts.size(), opts.data());
    size_t ls = 0;
    pr->log.clear();
    if (hiprtcGetProgramLogSize(rp, &ls) == HIPRTC_SUCCESS && ls > 1) {
        pr->log.resize(ls);
        hiprtcGetProgramLog(rp, &pr->log[0]);
        pr->log.resize(strnlen(pr->log.c_str(), ls));
    }
    if (cr != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&rp);
        return c->fail(HX_ERR_ARG, "the program does not compile: " +
                                       std::string(hiprtcGetErrorString(cr)) + "\n" + pr->log);
    }
    size_t cs = 0;
    hiprtcGetCodeSize(rp, &cs);
    pr->code.resize(cs);
    if (cs) hiprtcGetCode(rp, pr->code.data());
    hiprtcDestroyProgram(&rp);
    if (!c->host_only) {
        hipSetDevice(c->device);
        if (hipModuleLoadData(&pr->module, pr->code.data()) != hipSuccess) {
            hipGetLastError();
            pr->module = nullptr;
            return c->fail(HX_ERR_HIP, "the code object does not load on the device");
        }
    }
    pr->built = true;
    return HX_OK;
}

hx_status hx_program_log(hx_ctx ctx, hx_program prog, char* buf, size_t len, size_t* needed) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Program* pr = get_program(c, prog);
    if (!pr) return c->fail(HX_ERR_INVALID, "invalid program handle");
    if (needed) *needed = pr->log.size() + 1;
    if (buf && len) {
        const size_t n = std::min(len - 1, pr->log.size());
        memcpy(buf, pr->log.data(), n);
        buf[n] = '\0';
    }
    return HX_OK;
}

hx_status hx_program_function(hx_ctx ctx, hx_program prog, const char* kernel, void** function) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!function) return c->fail(HX_ERR_ARG, "null output");
    Program* pr = get_program(c, prog);
    if (!pr) return c->fail(HX_ERR_INVALID, "invalid program handle");
    hipFunction_t f = nullptr;
    hx_status s = lookup(c, pr, kernel, &f);
    if (s) return s;
    *function = reinterpret_cast<void*>(f);
    return HX_OK;
}

hx_status hx_program_run(hx_ctx ctx, hx_program prog, const char* kernel, const hx_kernel_arg* args,
                         int nargs, const uint32_t grid[3], const uint32_t block[3],
                         uint32_t shared_bytes, const hx_event* deps, int ndeps, hx_event* out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out || !grid || !block) return c->fail(HX_ERR_ARG, "null grid, block or output");
    if (nargs < 0 || (nargs > 0 && !args)) return c->fail(HX_ERR_ARG, "bad argument list");
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    Program* pr = get_program(c, prog);
    if (!pr) return c->fail(HX_ERR_INVALID, "invalid program handle");
    c->capture_plan(prog);
    hipFunction_t fn = nullptr;
    hx_status s = lookup(c, pr, kernel, &fn);
    if (s) return s;
    for (int d = 0; d < 3; ++d)
        if (grid[d] == 0 || block[d] == 0) return c->fail(HX_ERR_ARG, "grid and block must be >= 1");
    if ((uint64_t)block[0] * block[1] * block[2] > 1024)
        return c->fail(HX_ERR_ARG, "more than 1024 work-items per group");
    // Each parameter's bytes, held by the enqueued closure until it runs.
    std::vector<std::array<uint8_t, 16>> vals(nargs);
    std::vector<Access> acc;
    for (int i = 0; i < nargs; ++i) {
        const hx_kernel_arg& a = args[i];
        vals[i].fill(0);
        if (a.kind == HX_ARG_BUFFER) {
            if (a.access < 1 || a.access > 3)
                return c->fail(HX_ERR_ARG, "argument " + std::to_string(i) +
                                               ": access must be READ, WRITE or both");
            Buffer* b = c->get_buffer(a.buffer);
            if (!b) return c->fail(HX_ERR_INVALID, "argument " + std::to_string(i) +
                                                       ": invalid buffer");
            if (a.offset > b->bytes)
                return c->fail(HX_ERR_RANGE, "argument " + std::to_string(i) +
                                                 ": offset beyond the buffer");
            char* p = nullptr;
            Access ac{};
            s = resolve_range(c, a.buffer, a.offset, b->bytes - a.offset, &p, &ac,
                              (a.access & HX_ACCESS_WRITE) != 0);
            if (s) return s;
            acc.push_back(ac);
            memcpy(vals[i].data(), &p, sizeof(p));
        } else if (a.kind == HX_ARG_VALUE) {
            if (a.size < 1 || a.size > 16)
                return c->fail(HX_ERR_ARG, "argument " + std::to_string(i) +
                                               ": value size must be 1..16 bytes");
            memcpy(vals[i].data(), a.value, a.size);
        } else {
            return c->fail(HX_ERR_ARG, "argument " + std::to_string(i) + ": unknown kind");
        }
    }
    const uint32_t g0 = grid[0], g1 = grid[1], g2 = grid[2];
    const uint32_t b0 = block[0], b1 = block[1], b2 = block[2];
    std::string what = std::string("program kernel ") + kernel;
    return c->submit(
        SC_COMPUTE, deps, ndeps, acc, what,
        [fn, vals, g0, g1, g2, b0, b1, b2, shared_bytes](hipStream_t st) mutable -> hipError_t {
            std::vector<void*> params(vals.size());
            for (size_t i = 0; i < vals.size(); ++i) params[i] = vals[i].data();
            return hipModuleLaunchKernel(fn, g0, g1, g2, b0, b1, b2, shared_bytes, st,
                                         params.empty() ? nullptr : params.data(), nullptr);
        },
        out);
}

hx_status hx_program_destroy(hx_ctx ctx, hx_program prog) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return HX_ERR_INVALID;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Plan* p = c->get_plan(prog, PLAN_PROGRAM);
    if (!p) return HX_ERR_INVALID;
    if (hx_status s = c->no_capture("hx_program_destroy")) return s;
    if (p->graph_refs > 0)
        return c->fail(HX_ERR_ARG, "a captured graph still uses this program: destroy the graph "
                                   "first");
    if (!c->host_only)
        for (hipStream_t s : c->streams) hipStreamSynchronize(s);
    if (p->destroy) p->destroy(p->impl);
    p->live = false;
    p->impl = nullptr;
    return HX_OK;
}

}  // extern "C"
