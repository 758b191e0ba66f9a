// Variable-coefficient heat: single steps, the checkpointed forward and
// backward schedules, and the FP64 reductions, as hx operations.
//
// Checkpointing: with segment length S (default ceil(sqrt(T))) the forward run
// keeps u_{kS} for k = 1 .. nseg-1 (u_0 is the caller's input itself).  The
// backward run walks the segments from the last: it recomputes the segment's
// states u_{kS+1} .. u_{kS+S-1} from its checkpoint into a store of S-1 states,
// then runs the adjoint steps t = kS+S-1 .. kS, each reading u_t and
// lam_{t+1}, writing lam_t and adding the step's conductivity gradient into a
// per-segment accumulator of the run dtype; at the end of the segment the
// accumulator is folded into the FP64 total and cleared.  Memory: nseg-1 + S-1
// + 2 states instead of T.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "hx_internal.h"
#include "hx_runtime.hpp"

using namespace hx;

namespace {

size_t esz(int dt) { return dt == HX_F64 ? 8 : 4; }

struct Sched {
    int S = 1, nseg = 1;
};

Sched schedule(int steps, int ckpt) {
    Sched s;
    s.S = ckpt > 0 ? ckpt : std::max(1, (int)std::ceil(std::sqrt((double)std::max(steps, 1))));
    s.nseg = std::max(1, (steps + s.S - 1) / s.S);
    return s;
}

// Resolve a whole-state operand (cells * es bytes at `count` consecutive states).
hx_status state_range(Ctx* c, hx_buffer b, size_t bytes, int count, bool write, char** p,
                      std::vector<Access>& acc) {
    if (count <= 0) { *p = nullptr; return HX_OK; }
    Access a{};
    hx_status s = resolve_range(c, b, 0, bytes * (size_t)count, p, &a, write);
    if (s) return s;
    acc.push_back(a);
    return HX_OK;
}

hx_status check_common(Ctx* c, int dtype, int64_t nx, int64_t ny) {
    if (c->host_only) return c->fail(HX_ERR_NO_DEVICE, "host-only context");
    if (dtype != HX_F32 && dtype != HX_F64) return c->fail(HX_ERR_ARG, "bad dtype");
    if (nx <= 0 || ny <= 0) return c->fail(HX_ERR_ARG, "nx and ny must be positive");
    hipSetDevice(c->device);
    return HX_OK;
}

}  // namespace

#define LOCK_CTX(ctx)                                  \
    Ctx* c = reinterpret_cast<Ctx*>(ctx);              \
    if (!c) return HX_ERR_INVALID;                     \
    std::lock_guard<std::recursive_mutex> lk_(c->mu)

extern "C" {

hx_status hx_heat_vc_step(hx_ctx ctx, int dtype, int64_t nx, int64_t ny, double dt, hx_buffer u,
                          hx_buffer kappa, hx_buffer out_buf, const hx_event* deps, int ndeps,
                          hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, nx, ny);
    if (s) return s;
    const size_t bytes = (size_t)nx * ny * esz(dtype);
    std::vector<Access> acc;
    char *pu, *pk, *po;
    if ((s = state_range(c, u, bytes, 1, false, &pu, acc))) return s;
    if ((s = state_range(c, kappa, bytes, 1, false, &pk, acc))) return s;
    if ((s = state_range(c, out_buf, bytes, 1, true, &po, acc))) return s;
    if (po == pu) return c->fail(HX_ERR_ARG, "out must differ from u");
    VCArgs v{pu, pk, nullptr, po, nullptr, nx, ny, dt, 0};
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "heat_vc_step",
                     [=](hipStream_t st) { return launch_vc_step(dtype, false, v, st); }, out);
}

hx_status hx_heat_vc_adjoint_step(hx_ctx ctx, int dtype, int64_t nx, int64_t ny, double dt,
                                  hx_buffer u_t, hx_buffer lam_next, hx_buffer kappa,
                                  hx_buffer lam_out, hx_buffer gacc, const hx_event* deps,
                                  int ndeps, hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, nx, ny);
    if (s) return s;
    const size_t bytes = (size_t)nx * ny * esz(dtype);
    std::vector<Access> acc;
    char *pu, *pl, *pk, *po, *pg;
    if ((s = state_range(c, u_t, bytes, 1, false, &pu, acc))) return s;
    if ((s = state_range(c, lam_next, bytes, 1, false, &pl, acc))) return s;
    if ((s = state_range(c, kappa, bytes, 1, false, &pk, acc))) return s;
    if ((s = state_range(c, lam_out, bytes, 1, true, &po, acc))) return s;
    if ((s = state_range(c, gacc, bytes, 1, true, &pg, acc))) return s;
    if (po == pl) return c->fail(HX_ERR_ARG, "lam_out must differ from lam_next");
    VCArgs v{pu, pk, pl, po, pg, nx, ny, dt, 0};
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "heat_vc_adjoint_step",
                     [=](hipStream_t st) { return launch_vc_step(dtype, true, v, st); }, out);
}

hx_status hx_heat_vc_forward(hx_ctx ctx, const hx_vc_args* a, const hx_event* deps, int ndeps,
                             hx_event* out) {
    LOCK_CTX(ctx);
    if (!a || !out) return c->fail(HX_ERR_ARG, "null argument");
    hx_status s = check_common(c, a->dtype, a->nx, a->ny);
    if (s) return s;
    if (a->steps < 0 || a->ckpt < 0) return c->fail(HX_ERR_ARG, "negative steps or ckpt");
    const Sched sc = schedule(a->steps, a->ckpt);
    const int T = a->steps;
    const size_t bytes = (size_t)a->nx * a->ny * esz(a->dtype);
    std::vector<Access> acc;
    char *pu0, *pk, *puT, *pck = nullptr, *pw = nullptr;
    if ((s = state_range(c, a->u0, bytes, 1, false, &pu0, acc))) return s;
    if ((s = state_range(c, a->kappa, bytes, 1, false, &pk, acc))) return s;
    if ((s = state_range(c, a->uT, bytes, 1, true, &puT, acc))) return s;
    if ((s = state_range(c, a->ckpts, bytes, sc.nseg - 1, true, &pck, acc))) return s;
    if ((s = state_range(c, a->work, bytes, T > 1 ? 2 : 0, true, &pw, acc))) return s;
    const int dt = a->dtype;
    const int64_t nx = a->nx, ny = a->ny;
    const double tau = a->dt;
    const int rows = a->rows_per_block;
    const int S = sc.S;
    auto loc = [=](int t) -> char* {
        if (t == 0) return pu0;
        if (t == T) return puT;
        if (t % S == 0) return pck + (size_t)(t / S - 1) * bytes;
        return pw + (size_t)(t % 2) * bytes;
    };
    // Aligned grids run each stretch between kept states (u0, the checkpoints,
    // uT) in fused passes of up to kVcFusedMax steps, as even as the stretch
    // allows, ping-ponging through the two work states; the others step by
    // step.  Both give the same bits.
    VCArgs probe{pu0, pk, nullptr, puT, nullptr, nx, ny, tau, rows};
    const bool fused = vc_fused_supported(dt, probe) &&
                       (T <= 1 || (((uintptr_t)pw & 15u) == 0 && (bytes & 15u) == 0)) &&
                       (sc.nseg <= 1 || (((uintptr_t)pck & 15u) == 0));
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "heat_vc_forward",
                     [=](hipStream_t st) -> hipError_t {
                         if (T == 0)
                             return hipMemcpyAsync(puT, pu0, bytes, hipMemcpyDeviceToDevice, st);
                         if (!fused) {
                             for (int t = 0; t < T; ++t) {
                                 VCArgs v{loc(t), pk, nullptr, loc(t + 1), nullptr, nx, ny, tau,
                                          rows};
                                 hipError_t e = launch_vc_step(dt, false, v, st);
                                 if (e != hipSuccess) return e;
                             }
                             return hipSuccess;
                         }
                         for (int t0 = 0; t0 < T; t0 += S) {
                             const int t1 = std::min(t0 + S, T);
                             const int L = t1 - t0;
                             const int np = (L + kVcFusedMax - 1) / kVcFusedMax;
                             char* src = loc(t0);
                             for (int j = 0; j < np; ++j) {
                                 const int d = L / np + (j < L % np ? 1 : 0);
                                 char* dst = j + 1 == np ? loc(t1) : pw + (size_t)(j % 2) * bytes;
                                 VCArgs v{src, pk, nullptr, dst, nullptr, nx, ny, tau, rows};
                                 hipError_t e = launch_vc_forward(dt, d, v, st);
                                 if (e != hipSuccess) return e;
                                 src = dst;
                             }
                         }
                         return hipSuccess;
                     },
                     out);
}

hx_status hx_heat_vc_backward(hx_ctx ctx, const hx_vc_args* a, const hx_event* deps, int ndeps,
                              hx_event* out) {
    LOCK_CTX(ctx);
    if (!a || !out) return c->fail(HX_ERR_ARG, "null argument");
    hx_status s = check_common(c, a->dtype, a->nx, a->ny);
    if (s) return s;
    if (a->steps < 0 || a->ckpt < 0) return c->fail(HX_ERR_ARG, "negative steps or ckpt");
    const Sched sc = schedule(a->steps, a->ckpt);
    const int T = a->steps;
    const int S = sc.S;
    const int64_t cells = a->nx * a->ny;
    const size_t bytes = (size_t)cells * esz(a->dtype);
    std::vector<Access> acc;
    char *pu0, *pk, *pck = nullptr, *pw = nullptr, *pseg = nullptr, *plT, *pl0, *pg64, *pga;
    if ((s = state_range(c, a->u0, bytes, 1, false, &pu0, acc))) return s;
    if ((s = state_range(c, a->kappa, bytes, 1, false, &pk, acc))) return s;
    if ((s = state_range(c, a->ckpts, bytes, sc.nseg - 1, false, &pck, acc))) return s;
    if ((s = state_range(c, a->work, bytes, T > 1 ? 2 : 0, true, &pw, acc))) return s;
    if ((s = state_range(c, a->seg, bytes, S - 1, true, &pseg, acc))) return s;
    if ((s = state_range(c, a->lamT, bytes, 1, false, &plT, acc))) return s;
    if ((s = state_range(c, a->lam0, bytes, 1, true, &pl0, acc))) return s;
    if ((s = state_range(c, a->gk64, (size_t)cells * 8, 1, true, &pg64, acc))) return s;
    if ((s = state_range(c, a->gacc, bytes, 1, true, &pga, acc))) return s;
    const int dt = a->dtype;
    const int64_t nx = a->nx, ny = a->ny;
    const double tau = a->dt;
    const int rows = a->rows_per_block;
    const int nseg = sc.nseg;
    auto lam_in = [=](int t) -> const char* {  // lam_{t+1}
        return (t + 1 == T) ? plT : pw + (size_t)((t + 1) % 2) * bytes;
    };
    auto lam_out = [=](int t) -> char* { return t == 0 ? pl0 : pw + (size_t)(t % 2) * bytes; };
    // Aligned grids recompute each segment's states in fused passes that store
    // every level (one read of the state and of kappa per pass instead of per
    // step); the others step by step.  Both give the same bits.
    VCArgs probe{pu0, pk, nullptr, pseg ? pseg : pu0, nullptr, nx, ny, tau, rows};
    const bool fused = vc_fused_supported(dt, probe) && (bytes & 15u) == 0 &&
                       (!pseg || ((uintptr_t)pseg & 15u) == 0) &&
                       (sc.nseg <= 1 || ((uintptr_t)pck & 15u) == 0);
    // ... and run the reverse sweep in fused passes of up to four adjoint
    // steps with their gradient terms (lam moving between the two work slots,
    // the last pass into lam0)
    auto al16 = [](const void* q) { return ((uintptr_t)q & 15u) == 0; };
    const bool fused_adj = fused && al16(plT) && al16(pl0) && al16(pga) && (T <= 1 || al16(pw));
    return c->submit(
        SC_COMPUTE, deps, ndeps, acc, "heat_vc_backward",
        [=](hipStream_t st) -> hipError_t {
            hipError_t e = launch_fill(1, pg64, cells, 0.0, st);
            if (e != hipSuccess) return e;
            if ((e = launch_fill(dt, pga, cells, 0.0, st)) != hipSuccess) return e;
            if (T == 0) return hipMemcpyAsync(pl0, plT, bytes, hipMemcpyDeviceToDevice, st);
            const char* cur = plT;  // the fused sweep's lam_{t+1}
            for (int k = nseg - 1; k >= 0; --k) {
                const int t0 = k * S;
                const int t1 = std::min(T, t0 + S);
                const char* uck = (k == 0) ? pu0 : pck + (size_t)(k - 1) * bytes;
                auto ut = [=](int t) -> const char* {
                    return t == t0 ? uck : pseg + (size_t)(t - t0 - 1) * bytes;
                };
                if (fused && t1 - t0 > 1) {  // recompute the segment, fused
                    const int nst = t1 - t0 - 1;  // states t0+1 .. t1-1, slots 0 .. nst-1
                    const int np = (nst + kVcFusedMax - 1) / kVcFusedMax;
                    const char* src = uck;
                    for (int j = 0, done = 0; j < np; ++j) {
                        const int d = nst / np + (j < nst % np ? 1 : 0);
                        char* mid = pseg + (size_t)done * bytes;
                        char* dst = pseg + (size_t)(done + d - 1) * bytes;
                        VCArgs v{src, pk, nullptr, dst, nullptr, nx, ny, tau, rows};
                        if ((e = launch_vc_forward(dt, d, v, st, d > 1 ? mid : nullptr,
                                                   (int64_t)bytes)) != hipSuccess)
                            return e;
                        src = dst;
                        done += d;
                    }
                } else {
                    for (int t = t0 + 1; t < t1; ++t) {  // recompute the segment
                        VCArgs v{ut(t - 1), pk, nullptr, pseg + (size_t)(t - t0 - 1) * bytes,
                                 nullptr, nx, ny, tau, rows};
                        if ((e = launch_vc_step(dt, false, v, st)) != hipSuccess) return e;
                    }
                }
                if (fused_adj) {  // reverse sweep, fused
                    // at most two steps per FP64 pass: deeper FP64 passes need
                    // more than the 512 registers a wave can hold and spill
                    // hundreds of them to scratch (any depth gives the same bits)
                    const int L = t1 - t0;
                    const int dmax = dt == HX_F32 ? kVcFusedMax : 2;
                    const int np = (L + dmax - 1) / dmax;
                    int tb = t1 - 1;
                    for (int j = 0; j < np; ++j) {
                        const int d = L / np + (j < L % np ? 1 : 0);
                        const void* us[kVcFusedMax] = {};
                        for (int q = 0; q < d; ++q) us[q] = ut(tb - q);
                        char* dst = tb - d + 1 == 0 ? pl0 : (cur == pw ? pw + bytes : pw);
                        VCArgs v{nullptr, pk, cur, dst, pga, nx, ny, tau, rows};
                        // the first pass starts the segment's accumulator at
                        // zero, the last folds it into the FP64 total
                        if ((e = launch_vc_adjoint(
                                 dt, d, v, us, st, j == 0,
                                 j + 1 == np ? reinterpret_cast<double*>(pg64) : nullptr)) !=
                            hipSuccess)
                            return e;
                        cur = dst;
                        tb -= d;
                    }
                    continue;  // folded
                } else {
                    for (int t = t1 - 1; t >= t0; --t) {  // reverse sweep
                        VCArgs v{ut(t), pk, lam_in(t), lam_out(t), pga, nx, ny, tau, rows};
                        if ((e = launch_vc_step(dt, true, v, st)) != hipSuccess) return e;
                    }
                }
                if ((e = launch_fold(dt, pga, reinterpret_cast<double*>(pg64), cells, st)) !=
                    hipSuccess)
                    return e;
            }
            return hipSuccess;
        },
        out);
}

hx_status hx_launch_loss(hx_ctx ctx, int dtype, int64_t n, hx_buffer u, hx_buffer y,
                         hx_buffer resid, hx_buffer out64, hx_buffer work, const hx_event* deps,
                         int ndeps, hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, n, 1);
    if (s) return s;
    const size_t bytes = (size_t)n * esz(dtype);
    std::vector<Access> acc;
    char *pu, *py, *pr = nullptr, *po, *pw;
    if ((s = state_range(c, u, bytes, 1, false, &pu, acc))) return s;
    if ((s = state_range(c, y, bytes, 1, false, &py, acc))) return s;
    if (resid && (s = state_range(c, resid, bytes, 1, true, &pr, acc))) return s;
    if ((s = state_range(c, out64, 8, 1, true, &po, acc))) return s;
    if ((s = state_range(c, work, (size_t)reduce_blocks(n) * 8, 1, true, &pw, acc))) return s;
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "loss",
                     [=](hipStream_t st) {
                         return launch_reduce(dtype, 0, pu, py, pr, n,
                                              reinterpret_cast<double*>(pw),
                                              reinterpret_cast<double*>(po), st);
                     },
                     out);
}

hx_status hx_launch_loss_noalloc(hx_ctx ctx, int dtype, int64_t n, hx_buffer u, hx_buffer y,
                                 hx_buffer resid, hx_buffer out64, const hx_event* deps,
                                 int ndeps, hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, n, 1);
    if (s) return s;
    if (reduce_blocks(n) > kLossScratch)
        return c->fail(HX_ERR_RANGE, "the reduction needs more partial sums than the scratch "
                                     "holds (" + std::to_string(kLossScratch) + ")");
    double* pw = scratch_of(c->device);
    if (!pw) return c->fail(HX_ERR_HIP, "the device address of the loss scratch is unknown");
    const size_t bytes = (size_t)n * esz(dtype);
    std::vector<Access> acc;
    char *pu, *py, *pr = nullptr, *po;
    if ((s = state_range(c, u, bytes, 1, false, &pu, acc))) return s;
    if ((s = state_range(c, y, bytes, 1, false, &py, acc))) return s;
    if (resid && (s = state_range(c, resid, bytes, 1, true, &pr, acc))) return s;
    if ((s = state_range(c, out64, 8, 1, true, &po, acc))) return s;
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "loss (no allocation)",
                     [=](hipStream_t st) {
                         return launch_reduce(dtype, 0, pu, py, pr, n, pw,
                                              reinterpret_cast<double*>(po), st);
                     },
                     out);
}

hx_status hx_launch_dot(hx_ctx ctx, int dtype, int64_t n, hx_buffer a, hx_buffer b,
                        hx_buffer out64, hx_buffer work, const hx_event* deps, int ndeps,
                        hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, n, 1);
    if (s) return s;
    const size_t bytes = (size_t)n * esz(dtype);
    std::vector<Access> acc;
    char *pa, *pb, *po, *pw;
    if ((s = state_range(c, a, bytes, 1, false, &pa, acc))) return s;
    if ((s = state_range(c, b, bytes, 1, false, &pb, acc))) return s;
    if ((s = state_range(c, out64, 8, 1, true, &po, acc))) return s;
    if ((s = state_range(c, work, (size_t)reduce_blocks(n) * 8, 1, true, &pw, acc))) return s;
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "dot",
                     [=](hipStream_t st) {
                         return launch_reduce(dtype, 1, pa, pb, nullptr, n,
                                              reinterpret_cast<double*>(pw),
                                              reinterpret_cast<double*>(po), st);
                     },
                     out);
}

hx_status hx_launch_scale(hx_ctx ctx, int dtype, int64_t n, hx_buffer x, hx_buffer s64,
                          hx_buffer y, const hx_event* deps, int ndeps, hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, n, 1);
    if (s) return s;
    const size_t bytes = (size_t)n * esz(dtype);
    std::vector<Access> acc;
    char *px, *ps, *py;
    if ((s = state_range(c, x, bytes, 1, false, &px, acc))) return s;
    if ((s = state_range(c, s64, 8, 1, false, &ps, acc))) return s;
    if ((s = state_range(c, y, bytes, 1, true, &py, acc))) return s;
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "scale",
                     [=](hipStream_t st) {
                         return launch_scale(dtype, px, reinterpret_cast<const double*>(ps), py, n,
                                             st);
                     },
                     out);
}

hx_status hx_launch_cast64(hx_ctx ctx, int dtype, int64_t n, hx_buffer src64, hx_buffer dst,
                           const hx_event* deps, int ndeps, hx_event* out) {
    LOCK_CTX(ctx);
    if (!out) return c->fail(HX_ERR_ARG, "null output event");
    hx_status s = check_common(c, dtype, n, 1);
    if (s) return s;
    std::vector<Access> acc;
    char *ps, *pd;
    if ((s = state_range(c, src64, (size_t)n * 8, 1, false, &ps, acc))) return s;
    if ((s = state_range(c, dst, (size_t)n * esz(dtype), 1, true, &pd, acc))) return s;
    return c->submit(SC_COMPUTE, deps, ndeps, acc, "cast64",
                     [=](hipStream_t st) {
                         return launch_cast64(dtype, reinterpret_cast<const double*>(ps), pd, n,
                                              st);
                     },
                     out);
}

hx_status hx_vc_schedule(int steps, int ckpt, int* segment_length, int* segments) {
    if (steps < 0 || ckpt < 0 || !segment_length || !segments) return HX_ERR_ARG;
    const Sched s = schedule(steps, ckpt);
    *segment_length = s.S;
    *segments = s.nseg;
    return HX_OK;
}

}  // extern "C"
