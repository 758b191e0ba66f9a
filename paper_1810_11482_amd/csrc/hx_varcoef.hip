// Variable-coefficient heat step, its adjoint, and the FP64 reductions of the
// gradient path, for gfx950.
//
// Forward step (h = 1, zero-Dirichlet): v_c = u_c + dt * sum_f kappa_f (u_n - u_c)
// over the west, east, north and south faces, kappa_f = (kappa_c + kappa_n) / 2
// on interior faces; a face on the domain edge has kappa_f = kappa_c and a ghost
// u_n = 0.  Writing the ghost as (u = 0, kappa = kappa_c) makes the interior
// formula exact at the edge too, since (kappa_c + kappa_c) / 2 = kappa_c.
//
// Adjoint step (loss L = 0.5 ||u_T - y||^2, lam_T = u_T - y): the face rule is
// symmetric, so lam_t = A^T lam_{t+1} = A lam_{t+1} is the forward formula
// applied to lam, and in the same pass the conductivity gradient gains
//   -dt * [ sum_{interior f} (u_n - u_c)(lam_n - lam_c) / 2 + sum_{edge f} u_c lam_c ]
// with u = u_t and lam = lam_{t+1}.
//
// Mapping: a wave owns a strip of 64*C columns (C = 4 adjacent cells per lane)
// and streams a chunk of rows top to bottom, keeping the rows above, at and
// below the current one of every field in registers, so each field is read from
// HBM once per step.  West/east neighbours come from DPP wave shifts; the two
// cells just outside the strip are loaded per row by lanes 0 and 63.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "hx_internal.h"

namespace hx {
namespace {

constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

constexpr int C = 4;  // cells per lane
constexpr int S = 64 * C;

// One row of one field as seen by a lane: its C cells plus the cells just west
// and east of them.  Cells outside the domain are replaced by `ghost`.
template <typename T>
struct Row {
    T c[C];
    T w, e;
};

// Raw loads of one row of one field for the lane's cells [xl, xl + C) plus,
// in lanes 0 and 63, the cells just outside the strip.  Issued one row ahead of
// use so that their latency overlaps the arithmetic of the current row.
template <typename T>
struct Raw {
    T c[C];
    T edge;     // lane 0: cell x0 - 1; lane 63: cell x0 + S
    bool rowin;
};

// VEC (every row 16-byte aligned, nx a multiple of C): the same number of
// loads for every row of every wave -- one vector per lane from a clamped
// address plus one cell per lane for the strip edges, outside values replaced
// by 0 afterwards -- so no load sits under a branch and the compiler's wait
// counts cover only the row being consumed, not the one in flight.
template <typename T, bool VEC>
__device__ __forceinline__ void fetch_row(const T* __restrict__ f, int64_t y, int64_t ny, int64_t nx,
                                          int64_t x0, int64_t xl, int lane, bool vec, Raw<T>& r) {
    if constexpr (VEC) {
        typedef T V2 __attribute__((ext_vector_type(16 / sizeof(T))));
        typedef __attribute__((address_space(1))) const V2 GV2;
        typedef __attribute__((address_space(1))) const T GT;
        constexpr int VN = 16 / sizeof(T);
        r.rowin = y >= 0 && y < ny;
        const T* row = f + (y < 0 ? 0 : (y >= ny ? ny - 1 : y)) * nx;
        const bool lin = xl + C <= nx;  // the lane's cells are wholly inside or outside
        const int64_t xv = lin ? xl : nx - C;
#pragma unroll
        for (int q = 0; q < C / VN; ++q) {
            const V2 x = *((GV2*)(row + xv) + q);
#pragma unroll
            for (int e = 0; e < VN; ++e) r.c[q * VN + e] = lin ? x[e] : T(0);
        }
        const int64_t xe = (lane == 0) ? x0 - 1 : (lane == 63 ? x0 + S : xv);
        const bool ein = (lane == 0 || lane == 63) && xe >= 0 && xe < nx;
        const T ev = *((GT*)row + (ein ? xe : xv));
        r.edge = ein ? ev : T(0);
        return;
    }
    r.rowin = y >= 0 && y < ny;
    if (r.rowin && vec) {
        typedef T V2 __attribute__((ext_vector_type(16 / sizeof(T))));
        const V2* p = reinterpret_cast<const V2*>(f + y * nx + xl);
        constexpr int VN = 16 / sizeof(T);
#pragma unroll
        for (int q = 0; q < C / VN; ++q) {
            const V2 x = p[q];
#pragma unroll
            for (int e = 0; e < VN; ++e) r.c[q * VN + e] = x[e];
        }
    } else {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int64_t x = xl + j;
            r.c[j] = (r.rowin && x >= 0 && x < nx) ? f[y * nx + x] : T(0);
        }
    }
    r.edge = T(0);
    const int64_t xe = (lane == 0) ? x0 - 1 : x0 + S;
    if ((lane == 0 || lane == 63) && r.rowin && xe >= 0 && xe < nx) r.edge = f[y * nx + xe];
}

// Row as used by the arithmetic: rows outside the domain become the ghost
// `gc`; west/east neighbours across lanes come from DPP wave shifts.
template <typename T>
__device__ __forceinline__ void finish_row(const Raw<T>& raw, const T (&gc)[C], int lane, Row<T>& r) {
#pragma unroll
    for (int j = 0; j < C; ++j) r.c[j] = raw.rowin ? raw.c[j] : gc[j];
    const T fromw = dpp_move<DPP_WAVE_SHR1>(r.c[C - 1]);
    const T frome = dpp_move<DPP_WAVE_SHL1>(r.c[0]);
    r.w = lane == 0 ? raw.edge : fromw;
    r.e = lane == 63 ? raw.edge : frome;
}

struct VCDev {
    const void* u;      // state (forward input; adjoint: u_t)
    const void* kappa;
    const void* lam;    // adjoint: lam_{t+1}
    void* out;          // forward: u_{t+1}; adjoint: lam_t
    void* gacc;         // adjoint: per-segment conductivity-gradient accumulator (T)
    int64_t nx, ny;
    double dt;
    int rows;
    int aligned;        // every row starts 16-byte aligned
};

// Weighted face sum sum_f kappa_f (f_n - f_c) for the lane's C cells of row y.
template <typename T>
__device__ __forceinline__ void face_sum(const Row<T>& fm, const Row<T>& f0, const Row<T>& fp,
                                         const Row<T>& km, const Row<T>& k0, const Row<T>& kp,
                                         int64_t xl, int64_t nx, T (&acc)[C]) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const T fc = f0.c[j];
        const T kc = k0.c[j];
        const int64_t x = xl + j;
        const T fw = j > 0 ? f0.c[j - 1] : f0.w;
        const T fe = j + 1 < C ? f0.c[j + 1] : f0.e;
        // west/east ghosts: u = 0 (loaded as 0), kappa = kappa_c
        const T kw = (x - 1 >= 0) ? (j > 0 ? k0.c[j - 1] : k0.w) : kc;
        const T ke = (x + 1 < nx) ? (j + 1 < C ? k0.c[j + 1] : k0.e) : kc;
        const T fW = (x - 1 >= 0) ? fw : T(0);
        const T fE = (x + 1 < nx) ? fe : T(0);
        const T kfw = (kc + kw) * T(0.5);
        const T kfe = (kc + ke) * T(0.5);
        const T kfn = (kc + km.c[j]) * T(0.5);
        const T kfs = (kc + kp.c[j]) * T(0.5);
        T a = kfw * (fW - fc);
        a = fmaT(kfe, fE - fc, a);
        a = fmaT(kfn, fm.c[j] - fc, a);
        a = fmaT(kfs, fp.c[j] - fc, a);
        acc[j] = a;
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int BUF_DWORD3 = 0x00020000;  // raw 32-bit buffer (gfx9 family)
constexpr uint32_t OOB_OFFSET = 0x7ffffff0u;

// VEC stores of one lane's C cells of row y through a bounds-checked buffer
// resource: a lane whose cells lie past nx stores at an out-of-range offset,
// which the hardware drops, so the store is never under a branch.
template <typename T>
__device__ __forceinline__ void store_row(__amdgpu_buffer_rsrc_t rs, uint32_t lane_off, int64_t y,
                                          int64_t nx, const T (&v)[C]) {
    typedef T V2 __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int VN = 16 / sizeof(T);
    const uint32_t row = (uint32_t)(y * nx * (int64_t)sizeof(T));
#pragma unroll
    for (int q = 0; q < C / VN; ++q) {
        V2 x;
#pragma unroll
        for (int e = 0; e < VN; ++e) x[e] = v[q * VN + e];
        u32x4 bits;
        __builtin_memcpy(&bits, &x, sizeof(bits));
        __builtin_amdgcn_raw_buffer_store_b128(bits, rs, (int)(lane_off + row + q * 16), 0, 0);
    }
}

// store_row of a row that is stored only when `ok` (wave-uniform): otherwise
// every lane stores to the out-of-range offset, so no branch splits the
// caller's code
template <typename T, int AUX = 0>
__device__ __forceinline__ void store_row_if(__amdgpu_buffer_rsrc_t rs, uint32_t lane_off, bool ok,
                                             int64_t y, int64_t nx, const T (&v)[C]) {
    typedef T V2 __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int VN = 16 / sizeof(T);
    const uint32_t off = ok ? lane_off + (uint32_t)(y * nx * (int64_t)sizeof(T)) : OOB_OFFSET;
#pragma unroll
    for (int q = 0; q < C / VN; ++q) {
        V2 x;
#pragma unroll
        for (int e = 0; e < VN; ++e) x[e] = v[q * VN + e];
        u32x4 bits;
        __builtin_memcpy(&bits, &x, sizeof(bits));
        __builtin_amdgcn_raw_buffer_store_b128(bits, rs, (int)(off + q * 16), 0, AUX);
    }
}

template <typename T, bool ADJ, bool VEC>
__global__ __launch_bounds__(256) void k_vc_step(VCDev a, int64_t nstrips, int64_t nwaves) {
    const int wpg = blockDim.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * wpg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    const int64_t strip = wave % nstrips, chunk = wave / nstrips;
    const int64_t nx = a.nx, ny = a.ny;
    const int64_t x0 = strip * S;
    const int64_t xl = x0 + (int64_t)lane * C;
    const int64_t y0 = chunk * a.rows;
    const int64_t y1 = (y0 + a.rows < ny) ? y0 + a.rows : ny;
    const bool vec = VEC || ((x0 + S <= nx) && a.aligned);
    const T dt = static_cast<T>(a.dt);
    const T* U = static_cast<const T*>(a.u);
    const T* K = static_cast<const T*>(a.kappa);
    const T* L = static_cast<const T*>(a.lam);
    T* O = static_cast<T*>(a.out);
    T* G = static_cast<T*>(a.gacc);
    const T zero[C] = {T(0), T(0), T(0), T(0)};

    Row<T> um, u0, up, km, k0, kp, lm, l0, lp;
    Raw<T> rk, ru, rl, rg;
    // (used by the VEC form only)
    const int bytes = VEC ? (int)(ny * nx * (int64_t)sizeof(T)) : 0;
    const __amdgpu_buffer_rsrc_t rso = __builtin_amdgcn_make_buffer_rsrc(O, (short)0, bytes, BUF_DWORD3);
    const __amdgpu_buffer_rsrc_t rsg = __builtin_amdgcn_make_buffer_rsrc(G, (short)0, bytes, BUF_DWORD3);
    const uint32_t lane_off = (xl + C <= nx) ? (uint32_t)(xl * (int64_t)sizeof(T)) : OOB_OFFSET;
    // rows y0 and y0-1 (kappa ghosts of row y0-1 are kappa of row y0)
    fetch_row<T, VEC>(K, y0, ny, nx, x0, xl, lane, vec, rk);
    finish_row<T>(rk, zero, lane, k0);
    fetch_row<T, VEC>(K, y0 - 1, ny, nx, x0, xl, lane, vec, rk);
    finish_row<T>(rk, k0.c, lane, km);
    fetch_row<T, VEC>(U, y0 - 1, ny, nx, x0, xl, lane, vec, ru);
    finish_row<T>(ru, zero, lane, um);
    fetch_row<T, VEC>(U, y0, ny, nx, x0, xl, lane, vec, ru);
    finish_row<T>(ru, zero, lane, u0);
    if (ADJ) {
        fetch_row<T, VEC>(L, y0 - 1, ny, nx, x0, xl, lane, vec, rl);
        finish_row<T>(rl, zero, lane, lm);
        fetch_row<T, VEC>(L, y0, ny, nx, x0, xl, lane, vec, rl);
        finish_row<T>(rl, zero, lane, l0);
    }
    // the accumulator row y0 (adjoint, VEC) and the field rows y0+1 in flight
    if (VEC && ADJ) fetch_row<T, VEC>(G, y0, ny, nx, x0, xl, lane, vec, rg);
    fetch_row<T, VEC>(K, y0 + 1, ny, nx, x0, xl, lane, vec, rk);
    fetch_row<T, VEC>(U, y0 + 1, ny, nx, x0, xl, lane, vec, ru);
    if (ADJ) fetch_row<T, VEC>(L, y0 + 1, ny, nx, x0, xl, lane, vec, rl);
    for (int64_t y = y0; y < y1; ++y) {
        // row y+1 arrives; row y+2 goes in flight (VEC: unconditionally, the
        // rows past the chunk are clamped reads of the last row)
        finish_row<T>(rk, k0.c, lane, kp);
        finish_row<T>(ru, zero, lane, up);
        if (ADJ) finish_row<T>(rl, zero, lane, lp);
        T gr[C];
        if (VEC && ADJ) {
#pragma unroll
            for (int j = 0; j < C; ++j) gr[j] = rg.c[j];
        }
        if (VEC || y + 1 < y1) {
            if (VEC && ADJ) fetch_row<T, VEC>(G, y + 1, ny, nx, x0, xl, lane, vec, rg);
            fetch_row<T, VEC>(K, y + 2, ny, nx, x0, xl, lane, vec, rk);
            fetch_row<T, VEC>(U, y + 2, ny, nx, x0, xl, lane, vec, ru);
            if (ADJ) fetch_row<T, VEC>(L, y + 2, ny, nx, x0, xl, lane, vec, rl);
        }
        // rows outside the domain carry ghost kappa = kappa of the row y cell
        if (y - 1 < 0) {
#pragma unroll
            for (int j = 0; j < C; ++j) km.c[j] = k0.c[j];
        }
        T acc[C];
        if (!ADJ) {
            face_sum<T>(um, u0, up, km, k0, kp, xl, nx, acc);
            if constexpr (VEC) {
                T o[C];
#pragma unroll
                for (int j = 0; j < C; ++j) o[j] = fmaT(dt, acc[j], u0.c[j]);
                store_row<T>(rso, lane_off, y, nx, o);
            } else {
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    const int64_t x = xl + j;
                    if (x < nx) O[y * nx + x] = fmaT(dt, acc[j], u0.c[j]);
                }
            }
        } else {
            face_sum<T>(lm, l0, lp, km, k0, kp, xl, nx, acc);
            T o[C], gn[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int64_t x = xl + j;
                const T uc = u0.c[j], lc = l0.c[j];
                const T prod = uc * lc;
                const T hw = (x - 1 >= 0) ? ((j > 0 ? u0.c[j - 1] : u0.w) - uc) *
                                                ((j > 0 ? l0.c[j - 1] : l0.w) - lc) * T(0.5)
                                          : prod;
                const T he = (x + 1 < nx) ? ((j + 1 < C ? u0.c[j + 1] : u0.e) - uc) *
                                                ((j + 1 < C ? l0.c[j + 1] : l0.e) - lc) * T(0.5)
                                          : prod;
                const T hn = (y - 1 >= 0) ? (um.c[j] - uc) * (lm.c[j] - lc) * T(0.5) : prod;
                const T hs = (y + 1 < ny) ? (up.c[j] - uc) * (lp.c[j] - lc) * T(0.5) : prod;
                const T g = ((hw + he) + (hn + hs));
                if constexpr (VEC) {
                    o[j] = fmaT(dt, acc[j], lc);
                    gn[j] = fmaT(-dt, g, gr[j]);
                } else if (x < nx) {
                    O[y * nx + x] = fmaT(dt, acc[j], lc);
                    G[y * nx + x] = fmaT(-dt, g, G[y * nx + x]);
                }
            }
            if constexpr (VEC) {
                store_row<T>(rso, lane_off, y, nx, o);
                store_row<T>(rsg, lane_off, y, nx, gn);
            }
        }
        um = u0; u0 = up;
        km = k0; k0 = kp;
        if (ADJ) { lm = l0; l0 = lp; }
    }
}

// acc -> fp64 total, and acc reset to 0 (the fold of one checkpoint segment)
template <typename T>
__global__ void k_fold(T* __restrict__ acc, double* __restrict__ total, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        total[i] += (double)acc[i];
        acc[i] = T(0);
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T>
__global__ void k_cast64(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = (T)src[i];
}

// out = x * s, s a device FP64 scalar
template <typename T>
__global__ void k_scale(const T* __restrict__ x, const double* __restrict__ s, T* __restrict__ out,
                        int64_t n) {
    const double f = *s;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (T)((double)x[i] * f);
}

// Deterministic FP64 block reduction: every block writes one partial sum
// (wave DPP-free shuffle tree then LDS), a second one-block pass adds the
// partials in index order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <int MODE, typename T>  // MODE 0: 0.5*(a-b)^2 (+ residual), 1: a*b
__global__ __launch_bounds__(256) void k_reduce(const T* __restrict__ a, const T* __restrict__ b,
                                                T* __restrict__ resid, int64_t n,
                                                double* __restrict__ partial) {
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (MODE == 0) {
            const T d = a[i] - b[i];
            if (resid) resid[i] = d;
            s += (double)d * (double)d;
        } else {
            s += (double)a[i] * (double)b[i];
        }
    }
    __shared__ double ws[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += ws[w];
        partial[blockIdx.x] = MODE == 0 ? 0.5 * t : t;
    }
}

__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ partial, int nblocks,
                                                double* __restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += partial[i];
    __shared__ double ws[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += ws[w];
        *out = t;
    }
}

unsigned grid_for(int64_t n) {
    int64_t g = (n + 1023) / 1024;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// Row rings of the fused passes.  A pass streams rows base, base+1, ... (base
// = the pass's first row); the ring entry of row rho sits in slot
// (rho - base) mod 3 (field rows) or mod 6 (face rows, accumulator rows).  The
// row loop is unrolled six times with the phase as a constant, so every slot
// index is known at compile time: the rings live in registers and a row
// advances by renaming, not by register moves.  Rows in flight (PF per
// field) take slot t mod PF.
template <int P>
struct Phase {
    static constexpr int value = P;
};
__host__ __device__ constexpr int m3(int x) { return (x % 3 + 3) % 3; }
__host__ __device__ constexpr int m6(int x) { return (x % 6 + 6) % 6; }
constexpr int PF = 2;     // rows in flight per field (a divisor of 6)
constexpr int ST_NT = 2;  // buffer-store cache policy: nontemporal (the adjoint's two row
                          // stores per row: measured 4-7 % faster than cached stores)

// The dispatcher hands consecutive workgroups to the eight XCDs in turn, and
// each XCD has its own L2.  A fused pass's neighbouring waves (adjacent
// strips of one chunk) share the 128-byte lines at their strip edges; this
// bijection of [0, n) gives every XCD a contiguous range of workgroups, so
// that neighbouring strips mostly run under one L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
    constexpr uint32_t X = 8;
    const uint32_t q = n / X, r = n % X, x = b % X;
    return x * q + (x < r ? x : r) + b / X;
}

// Face conductivities of one row for a lane's C cells, as the single step
// forms them: the east face of cell j, (kappa_j + kappa_{j+1}) / 2, in e[j]
// (kappa_{j+1} = kappa_j on the domain's east edge) and cell 0's west face in
// e[C]; the west face of cell j > 0 is e[j - 1], the same sum with its
// operands swapped, hence the same value.  The south faces of the row above,
// (kappa_{rho-1} + kappa_rho) / 2, in s: the north face of row rho is the
// south face of row rho - 1.  Rows outside the domain are clamped reads of the
// edge row, so the edge faces come out as (kappa + kappa) / 2 = kappa.
template <typename T>
__device__ __forceinline__ void row_faces(const T (&kc)[C], const T (&ka)[C], bool wok, bool eok,
                                          T (&e)[C + 1], T (&s)[C]) {
    const T kel = dpp_move<DPP_WAVE_SHL1>(kc[0]);
    const T kwl = dpp_move<DPP_WAVE_SHR1>(kc[C - 1]);
#pragma unroll
    for (int j = 0; j + 1 < C; ++j) e[j] = (kc[j] + kc[j + 1]) * T(0.5);
    e[C - 1] = (kc[C - 1] + (eok ? kel : kc[C - 1])) * T(0.5);
    e[C] = (kc[0] + (wok ? kwl : kc[0])) * T(0.5);
#pragma unroll
    for (int j = 0; j < C; ++j) s[j] = (ka[j] + kc[j]) * T(0.5);
}

// D fused forward steps (temporal blocking), for aligned grids (every row
// 16-byte aligned, nx a multiple of C, under 2 GiB).  A wave owns 64*C
// columns, of which lanes 1..62 are its output: the strips overlap by one
// lane on each side, and the outer lanes' values go stale one column per step
// (from lanes 0 and 63 inward), which D <= C steps keep out of lanes 1..62.
// Rows stream top to bottom once: input row i (u and kappa) enters level 0;
// level k (1..D) then produces row i - k from level k-1's rows i-k-1 .. i-k+1,
// so u and kappa are read once and u written once per D steps.  The face
// conductivities of a row are formed once, when its kappa row arrives, and
// serve all D levels.  Lanes hold C whole cells inside or outside the domain
// (nx a multiple of C), so only a lane's outer cells can border the domain's
// west or east edge, and only those two take the edge rule; a level's rows
// outside the domain are set to 0 (the ghost value), which gives the north and
// south edge rule without a test per cell.  The arithmetic, and its order, is
// the single step's (k_vc_step), so a fused pass gives the same bits as D
// single steps.  MID: levels 1..D-1 are stored too, level k into mid + (k - 1)
// * mid_stride bytes (the states between the pass's input and its output, as
// the checkpointed backward sweep recomputes them): one read of u and kappa and
// D writes for D steps.
template <typename T, int D, bool MID>
__global__ __launch_bounds__(256) void k_vc_fwd(VCDev a, int64_t nstrips, int64_t nwaves,
                                                void* mid, int64_t mid_stride) {
    static_assert(D >= 1 && D <= C && D <= 5, "the halo lane covers at most C steps");
    typedef T V2 __attribute__((ext_vector_type(16 / sizeof(T))));
    typedef __attribute__((address_space(1))) const V2 GV2;
    constexpr int VN = 16 / sizeof(T);
    constexpr int W = S - 2 * C;  // output columns per strip
    const int wpg = blockDim.x >> 6;
    const int64_t wave = (int64_t)xcd_block(blockIdx.x, gridDim.x) * wpg +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    const int64_t strip = wave % nstrips, chunk = wave / nstrips;
    const int64_t nx = a.nx, ny = a.ny;
    const int64_t xl = strip * W - C + (int64_t)lane * C;  // this lane's first column
    const int64_t y0 = chunk * a.rows;
    const int64_t y1 = (y0 + a.rows < ny) ? y0 + a.rows : ny;
    const T dt = static_cast<T>(a.dt);
    const T* U = static_cast<const T*>(a.u);
    const T* K = static_cast<const T*>(a.kappa);
    const bool lin = xl >= 0 && xl + C <= nx;  // the lane's cells: all inside or all outside
    const int64_t xv = lin ? xl : 0;
    const bool wok = xl >= 1;       // cell 0's west face is interior
    const bool eok = xl + C < nx;   // cell C-1's east face is interior
    // row y of f for this lane, from a clamped row address (values of lanes
    // outside the domain are never used).  A pass reads each row once (a
    // chunk's halo rows twice); nontemporal loads measured faster where the
    // pass stores one row per row read (5.3 against 4.4 TB/s), cached loads
    // where it stores every level (MID)
    auto raw = [&](const T* f, int64_t y, T (&v)[C]) {
        const T* row = f + (y < 0 ? 0 : (y >= ny ? ny - 1 : y)) * nx;
#pragma unroll
        for (int q = 0; q < C / VN; ++q) {
            const V2 x = MID ? *((GV2*)(row + xv) + q)
                             : __builtin_nontemporal_load((GV2*)(row + xv) + q);
#pragma unroll
            for (int e = 0; e < VN; ++e) v[q * VN + e] = x[e];
        }
    };
    const int bytes = (int)(ny * nx * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rso =
        __builtin_amdgcn_make_buffer_rsrc(a.out, (short)0, bytes, BUF_DWORD3);
    const bool store_lane = lane >= 1 && lane <= 62 && lin;
    const uint32_t lane_off = store_lane ? (uint32_t)(xl * (int64_t)sizeof(T)) : OOB_OFFSET;
    __amdgpu_buffer_rsrc_t rsm[D > 1 ? D - 1 : 1];
    if constexpr (MID)
#pragma unroll
        for (int k = 0; k + 1 < D; ++k)
            rsm[k] = __builtin_amdgcn_make_buffer_rsrc(static_cast<char*>(mid) + k * mid_stride,
                                                       (short)0, bytes, BUF_DWORD3);

    T fr[D][3][C];    // level k's rows (level 0: u)
    T kr[3][C];       // kappa rows
    T ef[6][C + 1];   // east faces of a row, and cell 0's west face
    T sf[6][C];       // south faces of a row
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int j = 0; j < C; ++j) fr[k][m][j] = T(0);
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int j = 0; j <= C; ++j) {
            if (m < 3 && j < C) kr[m][j] = T(0);
            ef[m][j] = T(0);
            if (j < C) sf[m][j] = T(0);
        }
    const int64_t base = y0 - D;
    const int64_t nt = y1 - y0 + 2 * D;  // rows base .. y1 + D - 1 enter level 0
    T upf[PF][C], kpf[PF][C];            // rows in flight: row base + t in slot t mod PF
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        raw(U, base + m, upf[m]);
        raw(K, base + m, kpf[m]);
    }
    auto body = [&](auto ph, int64_t t) __attribute__((always_inline)) {
        constexpr int P = decltype(ph)::value;  // t mod 6
        constexpr int Q = P % PF;
        const int64_t i = base + t;
        const bool iin = i >= 0 && i < ny;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            fr[0][m3(P)][j] = iin ? upf[Q][j] : T(0);
            kr[m3(P)][j] = kpf[Q][j];
        }
        // row i+PF in flight (rows past the domain are clamped reads)
        raw(U, i + PF, upf[Q]);
        raw(K, i + PF, kpf[Q]);
        row_faces<T>(kr[m3(P)], kr[m3(P - 1)], wok, eok, ef[m6(P)], sf[m6(P - 1)]);
        T out[C];
#pragma unroll
        for (int k = 1; k <= D; ++k) {
            const int64_t r = i - k;  // the row level k produces
            const T* fm = fr[k - 1][m3(P - k - 1)];
            const T* f0 = fr[k - 1][m3(P - k)];
            const T* fp = fr[k - 1][m3(P - k + 1)];
            const T* e = ef[m6(P - k)];
            const T* fn = sf[m6(P - k - 1)];
            const T* fs = sf[m6(P - k)];
            const T fwl = dpp_move<DPP_WAVE_SHR1>(f0[C - 1]);
            const T fel = dpp_move<DPP_WAVE_SHL1>(f0[0]);
            T v[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const T fc = f0[j];
                const T fW = j > 0 ? f0[j - 1] : (wok ? fwl : T(0));
                const T fE = j + 1 < C ? f0[j + 1] : (eok ? fel : T(0));
                const T kfw = j > 0 ? e[j - 1] : e[C];
                T acc = kfw * (fW - fc);
                acc = fmaT(e[j], fE - fc, acc);
                acc = fmaT(fn[j], fm[j] - fc, acc);
                acc = fmaT(fs[j], fp[j] - fc, acc);
                v[j] = fmaT(dt, acc, fc);
            }
            if (k < D) {
                const bool rin = r >= 0 && r < ny;
#pragma unroll
                for (int j = 0; j < C; ++j) fr[k][m3(P - k)][j] = rin ? v[j] : T(0);
                if constexpr (MID)
                    store_row_if<T>(rsm[k - 1], lane_off, r >= y0 && r < y1, r, nx, v);
            } else {
#pragma unroll
                for (int j = 0; j < C; ++j) out[j] = v[j];
            }
        }
        const int64_t r = i - D;
        store_row_if<T>(rso, lane_off, r >= y0 && r < y1, r, nx, out);
    };
    // whole groups of six rows (one exit keeps the rings in registers): the
    // up to five rows past the pass's last are clamped reads and not stored
    for (int64_t t = 0; t < nt; t += 6) {
        body(Phase<0>{}, t);
        body(Phase<1>{}, t + 1);
        body(Phase<2>{}, t + 2);
        body(Phase<3>{}, t + 3);
        body(Phase<4>{}, t + 4);
        body(Phase<5>{}, t + 5);
    }
}


// D fused adjoint steps with their conductivity-gradient terms (temporal
// blocking of the reverse sweep), for the grids k_vc_fwd takes.  Steps
// t = tb, tb-1, ..., tb-D+1: level 0 is lam_{tb+1} (input rows), level k
// (1..D) produces lam_t, t = tb+1-k, from level k-1's rows and kappa, and adds
// -dt g_t to the accumulator, g_t from u_t (us.p[k-1], read row by row into a
// three-row ring per level) and lam_{t+1} (level k-1).  Rows stream top to
// bottom once: per row, lam, kappa and the accumulator are read once and
// written once (lam at level D only), each u_t read once: (D + 3) reads and 2
// writes per D steps instead of 6 reads and writes per step.  The
// accumulator row of row r enters at level 1 and leaves after level D, taking
// the D terms in the single step's order (t descending) with its fma, and
// lam's arithmetic is the single step's: the same bits as D single adjoint
// steps.  Faces, rings and edge rules as in k_vc_fwd; a gradient term across
// an edge face reads u_c lam_c, as the single step's.  ZIN: the pass opens a
// checkpoint segment, whose accumulator starts at zero (not read).  FOLD: the
// pass closes the segment: the accumulator's rows are added to the FP64 total
// (as the fold of a segment does) instead of being stored.
struct UStates {
    const void* p[4];
};

template <typename T, int D, bool ZIN, bool FOLD>
__global__ __launch_bounds__(256) void k_vc_adj(VCDev a, UStates us, double* __restrict__ total,
                                                int64_t nstrips, int64_t nwaves) {
    static_assert(D >= 1 && D <= C && D <= 4, "the halo lane covers at most C steps");
    typedef T V2 __attribute__((ext_vector_type(16 / sizeof(T))));
    typedef __attribute__((address_space(1))) const V2 GV2;
    constexpr int VN = 16 / sizeof(T);
    constexpr int W = S - 2 * C;  // output columns per strip
    const int wpg = blockDim.x >> 6;
    const int64_t wave = (int64_t)xcd_block(blockIdx.x, gridDim.x) * wpg +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & 63;
    const int64_t strip = wave % nstrips, chunk = wave / nstrips;
    const int64_t nx = a.nx, ny = a.ny;
    const int64_t xl = strip * W - C + (int64_t)lane * C;  // this lane's first column
    const int64_t y0 = chunk * a.rows;
    const int64_t y1 = (y0 + a.rows < ny) ? y0 + a.rows : ny;
    const T dt = static_cast<T>(a.dt);
    const T* L = static_cast<const T*>(a.lam);
    const T* K = static_cast<const T*>(a.kappa);
    const T* G = static_cast<const T*>(a.gacc);
    const bool lin = xl >= 0 && xl + C <= nx;  // the lane's cells: all inside or all outside
    const int64_t xv = lin ? xl : 0;
    const bool wok = xl >= 1;       // cell 0's west face is interior
    const bool eok = xl + C < nx;   // cell C-1's east face is interior
    auto raw = [&](const T* f, int64_t y, T (&v)[C]) {
        const T* row = f + (y < 0 ? 0 : (y >= ny ? ny - 1 : y)) * nx;
#pragma unroll
        for (int q = 0; q < C / VN; ++q) {
            const V2 x = *((GV2*)(row + xv) + q);
#pragma unroll
            for (int e = 0; e < VN; ++e) v[q * VN + e] = x[e];
        }
    };
    const int bytes = (int)(ny * nx * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rso =
        __builtin_amdgcn_make_buffer_rsrc(a.out, (short)0, bytes, BUF_DWORD3);
    const __amdgpu_buffer_rsrc_t rsg =
        __builtin_amdgcn_make_buffer_rsrc(a.gacc, (short)0, bytes, BUF_DWORD3);
    const bool store_lane = lane >= 1 && lane <= 62 && lin;
    const uint32_t lane_off = store_lane ? (uint32_t)(xl * (int64_t)sizeof(T)) : OOB_OFFSET;

    T lr[D][3][C];    // lam of level k (level 0: lam_{tb+1})
    T ur[D][3][C];    // u_t read by level k + 1
    T kr[3][C];       // kappa rows
    T ef[6][C + 1];   // east faces of a row, and cell 0's west face
    T sf[6][C];       // south faces of a row
    T gr[6][C];       // accumulator rows, from level 1 to level D
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int j = 0; j < C; ++j) lr[k][m][j] = ur[k][m][j] = T(0);
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int j = 0; j <= C; ++j) {
            if (m < 3 && j < C) kr[m][j] = T(0);
            ef[m][j] = T(0);
            if (j < C) sf[m][j] = gr[m][j] = T(0);
        }
    const int64_t base = y0 - D;
    const int64_t nt = y1 - y0 + 2 * D;  // rows base .. y1 + D - 1 enter level 0
    // rows in flight, in slot t mod PF for the iteration t that consumes them
    T lpf[PF][C], kpf[PF][C], gpf[PF][C], upf[PF][D][C];
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        raw(L, base + m, lpf[m]);
        raw(K, base + m, kpf[m]);
        if (!ZIN) raw(G, base + m - 1, gpf[m]);
#pragma unroll
        for (int k = 0; k < D; ++k) raw(static_cast<const T*>(us.p[k]), base + m - k, upf[m][k]);
    }
    auto body = [&](auto ph, int64_t t) __attribute__((always_inline)) {
        constexpr int P = decltype(ph)::value;  // t mod 6
        constexpr int Q = P % PF;
        const int64_t i = base + t;
        const bool iin = i >= 0 && i < ny;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            lr[0][m3(P)][j] = iin ? lpf[Q][j] : T(0);
            kr[m3(P)][j] = kpf[Q][j];
            gr[m6(P - 1)][j] = ZIN ? T(0) : gpf[Q][j];
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
            for (int j = 0; j < C; ++j) ur[k][m3(P - k)][j] = upf[Q][k][j];
        // the rows PF ahead in flight (rows past the domain are clamped reads)
        raw(L, i + PF, lpf[Q]);
        raw(K, i + PF, kpf[Q]);
        if (!ZIN) raw(G, i + PF - 1, gpf[Q]);
#pragma unroll
        for (int k = 0; k < D; ++k) raw(static_cast<const T*>(us.p[k]), i + PF - k, upf[Q][k]);
        row_faces<T>(kr[m3(P)], kr[m3(P - 1)], wok, eok, ef[m6(P)], sf[m6(P - 1)]);
        T out[C];
#pragma unroll
        for (int k = 1; k <= D; ++k) {
            const int64_t r = i - k;  // the row level k produces
            const T* fm = lr[k - 1][m3(P - k - 1)];
            const T* f0 = lr[k - 1][m3(P - k)];
            const T* fp = lr[k - 1][m3(P - k + 1)];
            const T* um = ur[k - 1][m3(P - k - 1)];
            const T* u0 = ur[k - 1][m3(P - k)];
            const T* up = ur[k - 1][m3(P - k + 1)];
            const T* e = ef[m6(P - k)];
            const T* fn = sf[m6(P - k - 1)];
            const T* fs = sf[m6(P - k)];
            T* g = gr[m6(P - k)];
            const bool nin = r - 1 >= 0, sin = r + 1 < ny;
            const T fwl = dpp_move<DPP_WAVE_SHR1>(f0[C - 1]);
            const T fel = dpp_move<DPP_WAVE_SHL1>(f0[0]);
            const T uwl = dpp_move<DPP_WAVE_SHR1>(u0[C - 1]);
            const T uel = dpp_move<DPP_WAVE_SHL1>(u0[0]);
            T v[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const T fc = f0[j];
                const T uc = u0[j];
                const bool wi = j > 0 || wok, ei = j + 1 < C || eok;
                const T fW = j > 0 ? f0[j - 1] : (wok ? fwl : T(0));
                const T fE = j + 1 < C ? f0[j + 1] : (eok ? fel : T(0));
                const T uw = j > 0 ? u0[j - 1] : uwl;
                const T ue = j + 1 < C ? u0[j + 1] : uel;
                const T kfw = j > 0 ? e[j - 1] : e[C];
                const T dW = fW - fc, dE = fE - fc, dN = fm[j] - fc, dS = fp[j] - fc;
                T acc = kfw * dW;
                acc = fmaT(e[j], dE, acc);
                acc = fmaT(fn[j], dN, acc);
                acc = fmaT(fs[j], dS, acc);
                v[j] = fmaT(dt, acc, fc);
                // the step's conductivity-gradient term, as the single step
                const T prod = uc * fc;
                const T hw = wi ? (uw - uc) * dW * T(0.5) : prod;
                const T he = ei ? (ue - uc) * dE * T(0.5) : prod;
                const T hn = nin ? (um[j] - uc) * dN * T(0.5) : prod;
                const T hs = sin ? (up[j] - uc) * dS * T(0.5) : prod;
                const T gt = ((hw + he) + (hn + hs));
                g[j] = fmaT(-dt, gt, g[j]);
            }
            if (k < D) {
                const bool rin = r >= 0 && r < ny;
#pragma unroll
                for (int j = 0; j < C; ++j) lr[k][m3(P - k)][j] = rin ? v[j] : T(0);
            } else {
#pragma unroll
                for (int j = 0; j < C; ++j) out[j] = v[j];
            }
        }
        const int64_t r = i - D;
        const bool rout = r >= y0 && r < y1;
        store_row_if<T, ST_NT>(rso, lane_off, rout, r, nx, out);
        if constexpr (FOLD) {
            if (rout && store_lane) {
                double* tp = total + r * nx + xl;
#pragma unroll
                for (int j = 0; j < C; ++j) tp[j] += (double)gr[m6(P - D)][j];
            }
        } else {
            store_row_if<T, ST_NT>(rsg, lane_off, rout, r, nx, gr[m6(P - D)]);
        }
    };
    // whole groups of six rows (one exit keeps the rings in registers): the
    // up to five rows past the pass's last are clamped reads and not stored
    for (int64_t t = 0; t < nt; t += 6) {
        body(Phase<0>{}, t);
        body(Phase<1>{}, t + 1);
        body(Phase<2>{}, t + 2);
        body(Phase<3>{}, t + 3);
        body(Phase<4>{}, t + 4);
        body(Phase<5>{}, t + 5);
    }
}

}  // namespace

hipError_t launch_vc_step(int dtype, bool adjoint, const VCArgs& v, hipStream_t st) {
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const int es = dtype == 0 ? 4 : 8;
    const bool aligned = ((v.nx * es) % 16 == 0) && al(v.u) && al(v.kappa) &&
                         (!v.lam || al(v.lam)) && al(v.out) && (!v.gacc || al(v.gacc));
    // VEC: aligned rows, whole lane chunks (nx a multiple of C) and a grid
    // under 2 GiB (32-bit buffer offsets)
    const bool vecform = aligned && v.nx % C == 0 && v.nx * v.ny * es < (int64_t(1) << 31);
    VCDev a{v.u, v.kappa, v.lam, v.out, v.gacc, v.nx, v.ny, v.dt, v.rows > 0 ? v.rows : 64,
            aligned ? 1 : 0};
    const int64_t nstrips = (v.nx + S - 1) / S;
    const int64_t nchunks = (v.ny + a.rows - 1) / a.rows;
    const int64_t nwaves = nstrips * nchunks;
    const int wpg = 4;
    const dim3 block(64 * wpg), grid((unsigned)((nwaves + wpg - 1) / wpg));
#define HX_VC_LAUNCH(T, ADJ, VEC) \
    hipLaunchKernelGGL((k_vc_step<T, ADJ, VEC>), grid, block, 0, st, a, nstrips, nwaves)
    if (dtype == 0) {
        if (adjoint) { if (vecform) HX_VC_LAUNCH(float, true, true); else HX_VC_LAUNCH(float, true, false); }
        else { if (vecform) HX_VC_LAUNCH(float, false, true); else HX_VC_LAUNCH(float, false, false); }
    } else {
        if (adjoint) { if (vecform) HX_VC_LAUNCH(double, true, true); else HX_VC_LAUNCH(double, true, false); }
        else { if (vecform) HX_VC_LAUNCH(double, false, true); else HX_VC_LAUNCH(double, false, false); }
    }
#undef HX_VC_LAUNCH
    return hipGetLastError();
}

bool vc_fused_supported(int dtype, const VCArgs& v) {
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const int es = dtype == 0 ? 4 : 8;
    return v.nx % C == 0 && (v.nx * es) % 16 == 0 && al(v.u) && al(v.kappa) && al(v.out) &&
           v.nx * v.ny * es < (int64_t(1) << 31) && v.nx > 0 && v.ny > 0;
}

// The fused kernel for (dtype, steps, variant): variant bit 0 = MID (forward)
// or ZIN (adjoint), bit 1 = FOLD (adjoint).
template <typename T>
const void* fused_kernel(bool adjoint, int steps, int variant) {
#define HX_VC_FWD_K(D) (variant & 1) ? (const void*)k_vc_fwd<T, D, true> : (const void*)k_vc_fwd<T, D, false>
#define HX_VC_ADJ_K(D)                                                                   \
    variant == 3   ? (const void*)k_vc_adj<T, D, true, true>                             \
    : variant == 1 ? (const void*)k_vc_adj<T, D, true, false>                            \
    : variant == 2 ? (const void*)k_vc_adj<T, D, false, true>                            \
                   : (const void*)k_vc_adj<T, D, false, false>
    switch (steps) {
        case 1: return adjoint ? (HX_VC_ADJ_K(1)) : (HX_VC_FWD_K(1));
        case 2: return adjoint ? (HX_VC_ADJ_K(2)) : (HX_VC_FWD_K(2));
        case 3: return adjoint ? (HX_VC_ADJ_K(3)) : (HX_VC_FWD_K(3));
        case 4: return adjoint ? (HX_VC_ADJ_K(4)) : (HX_VC_FWD_K(4));
        default: return nullptr;
    }
#undef HX_VC_FWD_K
#undef HX_VC_ADJ_K
}

// Rows per chunk when the caller leaves the choice to the library: enough
// chunks that strips x chunks waves fill the device's resident wave slots for
// this kernel once (one round of waves: no partly filled second round), at
// least 16 rows.  A wave streams its chunk plus 2D halo rows, so taller
// chunks also recompute fewer rows.  The result does not depend on the chunk
// height.
int fill_rows(const void* k, int64_t nstrips, int64_t ny) {
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void*, int>, int64_t>> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 64;
    }
    int64_t slots = 0;
    {
        std::lock_guard<std::mutex> g(mu);
        for (const auto& e : cache)
            if (e.first.first == k && e.first.second == dev) slots = e.second;
    }
    if (slots == 0) {
        int cus = 0, blocks = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, 256, 0) != hipSuccess ||
            cus < 1 || blocks < 1) {
            (void)hipGetLastError();
            return 64;
        }
        slots = (int64_t)cus * blocks * 4;  // four waves per workgroup
        std::lock_guard<std::mutex> g(mu);
        cache.push_back({{k, dev}, slots});
    }
    const int64_t chunks = std::max<int64_t>(1, slots / nstrips);
    const int64_t rows = std::max<int64_t>(16, (ny + chunks - 1) / chunks);
    return (int)std::min<int64_t>(rows, int64_t(1) << 30);
}

hipError_t launch_fused(const void* k, VCDev a, int rows_req, void* arg3, void* arg4,
                        bool adjoint, hipStream_t st) {
    if (!k) return hipErrorInvalidValue;
    int64_t nstrips = (a.nx + (S - 2 * C) - 1) / (S - 2 * C);
    a.rows = rows_req > 0 ? rows_req : fill_rows(k, nstrips, a.ny);
    int64_t nwaves = nstrips * ((a.ny + a.rows - 1) / a.rows);
    const int wpg = 4;
    const int64_t groups = (nwaves + wpg - 1) / wpg;
    if (groups >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    // forward: (a, nstrips, nwaves, mid, mid_stride); adjoint: (a, us, total, nstrips, nwaves)
    void* fargs[] = {&a, &nstrips, &nwaves, arg3, arg4};
    void* aargs[] = {&a, arg3, arg4, &nstrips, &nwaves};
    return hipLaunchKernel(k, dim3((unsigned)groups), dim3(64 * wpg), adjoint ? aargs : fargs, 0, st);
}

hipError_t launch_vc_forward(int dtype, int steps, const VCArgs& v, hipStream_t st, void* mid,
                             int64_t mid_stride) {
    if (steps < 1 || steps > C || !vc_fused_supported(dtype, v)) return hipErrorInvalidValue;
    const int es = dtype == 0 ? 4 : 8;
    if (mid && (((reinterpret_cast<uintptr_t>(mid) | (uintptr_t)mid_stride) & 15u) ||
                mid_stride < v.nx * v.ny * es))
        return hipErrorInvalidValue;
    VCDev a{v.u, v.kappa, nullptr, v.out, nullptr, v.nx, v.ny, v.dt, 0, 1};
    const int variant = mid ? 1 : 0;
    const void* k = dtype == 0 ? fused_kernel<float>(false, steps, variant)
                               : fused_kernel<double>(false, steps, variant);
    return launch_fused(k, a, v.rows, &mid, &mid_stride, false, st);
}

hipError_t launch_vc_adjoint(int dtype, int steps, const VCArgs& v, const void* const* ustates,
                             hipStream_t st, bool zero_in, double* fold_total) {
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    if (steps < 1 || steps > C || steps > 4 || !v.lam || !v.gacc || !al(v.lam) || !al(v.gacc) ||
        !al(fold_total) || !vc_fused_supported(dtype, v))
        return hipErrorInvalidValue;
    UStates us{};
    for (int k = 0; k < steps; ++k) {
        if (!ustates[k] || !al(ustates[k])) return hipErrorInvalidValue;
        us.p[k] = ustates[k];
    }
    VCDev a{nullptr, v.kappa, v.lam, v.out, v.gacc, v.nx, v.ny, v.dt, 0, 1};
    const int variant = (zero_in ? 1 : 0) | (fold_total ? 2 : 0);
    const void* k = dtype == 0 ? fused_kernel<float>(true, steps, variant)
                               : fused_kernel<double>(true, steps, variant);
    return launch_fused(k, a, v.rows, &us, &fold_total, true, st);
}

hipError_t launch_fold(int dtype, void* acc, double* total, int64_t n, hipStream_t st) {
    if (dtype == 0) hipLaunchKernelGGL((k_fold<float>), dim3(grid_for(n)), dim3(256), 0, st, (float*)acc, total, n);
    else hipLaunchKernelGGL((k_fold<double>), dim3(grid_for(n)), dim3(256), 0, st, (double*)acc, total, n);
    return hipGetLastError();
}

hipError_t launch_fill(int dtype, void* p, int64_t n, double v, hipStream_t st) {
    if (dtype == 0) hipLaunchKernelGGL((k_fill<float>), dim3(grid_for(n)), dim3(256), 0, st, (float*)p, n, (float)v);
    else hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(n)), dim3(256), 0, st, (double*)p, n, v);
    return hipGetLastError();
}

hipError_t launch_cast64(int dtype, const double* src, void* dst, int64_t n, hipStream_t st) {
    if (dtype == 0) hipLaunchKernelGGL((k_cast64<float>), dim3(grid_for(n)), dim3(256), 0, st, src, (float*)dst, n);
    else hipLaunchKernelGGL((k_cast64<double>), dim3(grid_for(n)), dim3(256), 0, st, src, (double*)dst, n);
    return hipGetLastError();
}

hipError_t launch_scale(int dtype, const void* x, const double* s, void* out, int64_t n,
                        hipStream_t st) {
    if (dtype == 0) hipLaunchKernelGGL((k_scale<float>), dim3(grid_for(n)), dim3(256), 0, st, (const float*)x, s, (float*)out, n);
    else hipLaunchKernelGGL((k_scale<double>), dim3(grid_for(n)), dim3(256), 0, st, (const double*)x, s, (double*)out, n);
    return hipGetLastError();
}

int reduce_blocks(int64_t n) { return (int)grid_for(n); }

// Scratch of the allocation-free loss (hx_launch_loss_noalloc): the partial
// sums of one reduction, one per workgroup (grid_for caps the grid at
// kLossScratch).  Every GPU the library runs on holds its own copy until the
// process ends.  Host code never uses the array's name as an address: it uses
// the device address that hipGetSymbolAddress returns, once per device, with
// that device current (scratch_init, from hx_ctx_create).
static __device__ __align__(256) double scratch[kLossScratch];

namespace {
std::mutex scratch_mu;
double* scratch_dev[kMaxDevices];  // per device: the address of `scratch` there
}  // namespace

hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    scratch_dev[device] = static_cast<double*>(p);
    return hipSuccess;
}

double* scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_dev[device];
}

hipError_t launch_reduce(int dtype, int mode, const void* a, const void* b, void* resid, int64_t n,
                         double* partial, double* out, hipStream_t st) {
    const unsigned g = grid_for(n);
    if (dtype == 0) {
        if (mode == 0) hipLaunchKernelGGL((k_reduce<0, float>), dim3(g), dim3(256), 0, st, (const float*)a, (const float*)b, (float*)resid, n, partial);
        else hipLaunchKernelGGL((k_reduce<1, float>), dim3(g), dim3(256), 0, st, (const float*)a, (const float*)b, (float*)nullptr, n, partial);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_reduce<0, double>), dim3(g), dim3(256), 0, st, (const double*)a, (const double*)b, (double*)resid, n, partial);
        else hipLaunchKernelGGL((k_reduce<1, double>), dim3(g), dim3(256), 0, st, (const double*)a, (const double*)b, (double*)nullptr, n, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, st, partial, (int)g, out);
    return hipGetLastError();
}

}  // namespace hx
