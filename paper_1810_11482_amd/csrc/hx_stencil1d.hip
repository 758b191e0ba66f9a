// 1D explicit heat stencil with temporal blocking, for gfx950.
//
// Operation: u'_i = u_i + r (u_{i-1} - 2 u_i + u_{i+1}) (the 3-point stencil of
// the paper's Sec. V-A.1 in heat form), `steps` steps fused per pass.
//
// Mapping.  Every wave owns a tile of 64*C consecutive cells held in registers,
// C per lane and lane-contiguous (lane l holds cells l*C .. l*C+C-1 of the
// tile).  The outer `halo` cells on each side are context: they are loaded,
// advanced with the rest and discarded, so after `steps` <= halo steps the
// inner 64*C - 2*halo cells are exact and are written.  A step needs, per lane,
// only the last cell of the lane below and the first cell of the lane above;
// both come from a single DPP wave shift (wave_shr:1 / wave_shl:1), so the
// whole time loop runs out of registers with no barrier, and waves are fully
// independent.  HBM is read and written only in coalesced order, through a
// wave-private LDS area that transposes to and from the lane-contiguous
// layout.  HBM traffic per pass is one read and one write of every cell plus
// 2*halo/(64*C) of re-read context.
//
// Arithmetic.  For 0 <= r <= 3/8 the tile is advanced in the rescaled form
// w' = fma(r/(1-2r), l + rt, w) with a periodic rescale (set_rate_1d): one add
// and one fma per cell-step.  Other rates use s = l + rt; d = fma(-2, c, s);
// c' = fma(r, d, c).  Either way the result of a pass depends only on its step
// count, not on the tile geometry.
#include <hip/hip_runtime.h>

#include "hx_internal.h"

namespace hx {
namespace {

enum { BC_PERIODIC = 0, BC_DIRICHLET0 = 1, BC_GHOST = 2 };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct V16;
template <> struct V16<float> { typedef f32x4 t; enum { N = 4 }; };
template <> struct V16<double> { typedef f64x2 t; enum { N = 2 }; };

// DPP controls of the wave-wide shifts: lane i reads lane i-1 (shr) or i+1 (shl);
// the lane with no source reads 0.
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

// Value of cell g (any integer) of segment s at the start of the pass.
template <typename T>
__device__ __forceinline__ T load_cell(const Seg1D& s, int64_t g) {
    const T* in = static_cast<const T*>(s.in);
    if (g >= 0 && g < s.n) return in[g];
    if (g < 0) {
        if (s.bc_lo == BC_PERIODIC) {
            // 32-bit remainder where it fits (every segment under 2^31 cells)
            int64_t m = (s.n < (int64_t(1) << 31) && g > -(int64_t(1) << 31))
                            ? (int64_t)((int32_t)g % (int32_t)s.n)
                            : g % s.n;
            if (m < 0) m += s.n;
            return in[m];
        }
        if (s.bc_lo == BC_GHOST && g >= -(int64_t)s.hw)
            return static_cast<const T*>(s.halo_lo)[s.hw + g];
        return T(0);
    }
    if (s.bc_hi == BC_PERIODIC)
        return in[(g < (int64_t(1) << 31)) ? (int64_t)((uint32_t)g % (uint32_t)s.n) : g % s.n];
    if (s.bc_hi == BC_GHOST && g - s.n < (int64_t)s.hw)
        return static_cast<const T*>(s.halo_hi)[g - s.n];
    return T(0);
}

// One step of a whole wave tile, in place on the lane-contiguous registers a.
// The cell left of a lane's first comes from the lane below, the cell right of
// its last from the lane above (DPP wave shifts of the old values).  The
// neighbour sum of cell j+1 is formed from the old a[j] before a[j] is
// overwritten, so one array and two short-lived temporaries suffice and the
// register assignment is the same after every step (no register moves).  Per
// cell: s = l + rt; d = fma(-2, c, s); c' = fma(r, d, c).  Cells outside a
// zero-Dirichlet end are reset to 0 after the step.
template <typename T, int C>
__device__ __forceinline__ void step_tile(T (&a)[C], T k, bool zero_lo, bool zero_hi,
                                          int64_t lbase, int64_t n) {
    const T left = dpp_move<DPP_WAVE_SHR1>(a[C - 1]);
    const T right = dpp_move<DPP_WAVE_SHL1>(a[0]);
    T s_cur = left + (C > 1 ? a[1] : right);
#pragma unroll
    for (int j = 0; j < C; ++j) {
        T s_next = T(0);
        if (j + 1 < C) s_next = a[j] + (j + 2 < C ? a[j + 2] : right);
        const T d = fmaT(T(-2), a[j], s_cur);
        a[j] = fmaT(k, d, a[j]);
        s_cur = s_next;
    }
    if (zero_lo || zero_hi) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int64_t g = lbase + j;
            if ((zero_lo && g < 0) || (zero_hi && g >= n)) a[j] = T(0);
        }
    }
}

// One step of the rescaled form (see set_rate_1d): w' = w + b (w_l + w_r).
// Same register discipline as step_tile: one add and one fma per cell.
template <typename T, int C>
__device__ __forceinline__ void step_tile_scaled(T (&a)[C], T b, bool zero_lo, bool zero_hi,
                                                 int64_t lbase, int64_t n) {
    const T left = dpp_move<DPP_WAVE_SHR1>(a[C - 1]);
    const T right = dpp_move<DPP_WAVE_SHL1>(a[0]);
    T s_cur = left + (C > 1 ? a[1] : right);
#pragma unroll
    for (int j = 0; j < C; ++j) {
        T s_next = T(0);
        if (j + 1 < C) s_next = a[j] + (j + 2 < C ? a[j + 2] : right);
        a[j] = fmaT(b, s_cur, a[j]);
        s_cur = s_next;
    }
    if (zero_lo || zero_hi) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int64_t g = lbase + j;
            if ((zero_lo && g < 0) || (zero_hi && g >= n)) a[j] = T(0);
        }
    }
}

template <typename T, int C>
__device__ __forceinline__ void scale_tile(T (&a)[C], T f) {
#pragma unroll
    for (int j = 0; j < C; ++j) a[j] *= f;
}

// Segment pointers arrive as generic addresses; the tile's vector accesses go
// through the global address space explicitly, so they compile to global
// (not flat) instructions, which the LDS counters do not wait on.
template <typename VT>
__device__ __forceinline__ VT gload_nt(const VT* p, int64_t i) {
    typedef __attribute__((address_space(1))) const VT GVT;
    return __builtin_nontemporal_load((GVT*)p + i);
}
template <typename VT>
__device__ __forceinline__ void gstore_nt(VT x, VT* p, int64_t i) {
    typedef __attribute__((address_space(1))) VT GVT;
    __builtin_nontemporal_store(x, (GVT*)p + i);
}

__device__ __forceinline__ bool aligned16(const void* p) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Position of tile cell i in the wave's LDS staging area: lane chunks of C
// cells, each followed by one vector of padding so that the transposed reads
// (lane j reading chunk j) spread over all banks.
template <typename T, int C>
__device__ __forceinline__ int lds_pos(int i) {
    constexpr int VN = V16<T>::N;
    return (i / C) * (C + VN) + (i % C);
}

// A tile's pass is four phases, so that a persistent wave can overlap the
// next tile's HBM reads with the current tile's steps:
//   tile_fetch:  HBM -> registers, coalesced (lane l holds the vectors
//                VN*(l + 64k), k = 0 .. C/VN-1, of the tile);
//   tile_stage:  registers -> wave-private LDS -> lane-contiguous registers
//                (lane l holds cells l*C .. l*C+C-1);
//   tile_steps:  the time loop, registers only;
//   tile_store:  registers -> LDS -> HBM, coalesced, inner cells only.
// HBM is touched only in coalesced order.  LDS accesses of one wave execute in
// order, so the wave needs no barrier between writing and reading its area.
struct TileGeom {
    int64_t o0, base;   // first output cell, first held cell
    bool interior;      // the whole tile lies inside [0, n)
};

template <int C>
__device__ __forceinline__ TileGeom tile_geom(const Seg1D& s, int64_t tile, int halo) {
    TileGeom g;
    const int64_t wout = 64LL * C - 2LL * halo;
    g.o0 = tile * wout - s.shift;
    g.base = g.o0 - halo;
    g.interior = g.base >= 0 && g.base + 64LL * C <= s.n;
    return g;
}

// Vector fetch of a tile that lies inside the segment with a 16-byte aligned
// start (every tile but the segment's ends, given the grid shift).
template <typename T>
__device__ __forceinline__ bool tile_fast(const Seg1D& s, const TileGeom& tg) {
    return tg.interior && aligned16(static_cast<const T*>(s.in) + tg.base);
}

template <typename T, int C>
__device__ __forceinline__ void tile_fetch(const Seg1D& s, const TileGeom& tg, T (&pf)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    const int lane = threadIdx.x & 63;
    const VT* src = reinterpret_cast<const VT*>(static_cast<const T*>(s.in) + tg.base);
#pragma unroll
    for (int k = 0; k < C / VN; ++k) {
        const VT x = gload_nt(src, lane + 64 * k);
#pragma unroll
        for (int e = 0; e < VN; ++e) pf[k * VN + e] = x[e];
    }
}

// Any other tile: cell by cell (boundary rules included) straight into the
// wave's LDS area, in the same positions tile_stage writes.  Kept out of line:
// it is rare and its boundary arithmetic would otherwise inflate the register
// allocation of the whole tile loop.
template <typename T, int C>
__device__ __forceinline__ void tile_fill_slow(const Seg1D& s, int64_t base,
                                                         bool interior, T* __restrict__ lds) {
    const int lane = threadIdx.x & 63;
    const T* in = static_cast<const T*>(s.in);
    // a rolled loop: the path is rare, and unrolled its 64-bit addresses would
    // set the register allocation of the whole kernel
#pragma unroll 1
    for (int j = 0; j < C; ++j) {
        const int i = lane + 64 * j;
        lds[lds_pos<T, C>(i)] = interior ? in[base + i] : load_cell<T>(s, base + i);
    }
}

template <typename T, int C>
__device__ __forceinline__ void tile_read(const T* __restrict__ lds, T (&v)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < C / VN; ++q) {
        const VT x = *reinterpret_cast<const VT*>(lds + lane * (C + VN) + q * VN);
#pragma unroll
        for (int e = 0; e < VN; ++e) v[q * VN + e] = x[e];
    }
}

template <typename T, int C>
__device__ __forceinline__ void tile_stage(const T (&pf)[C], T* __restrict__ lds, T (&v)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < C / VN; ++k) {
        VT x;
#pragma unroll
        for (int e = 0; e < VN; ++e) x[e] = pf[k * VN + e];
        *reinterpret_cast<VT*>(lds + lds_pos<T, C>(VN * (lane + 64 * k))) = x;
    }
    __builtin_amdgcn_wave_barrier();
    tile_read<T, C>(lds, v);
}

// SC selects the rescaled update (every segment the kernel runs has
// period > 0) or the direct one; the two are separate instantiations so that
// each keeps its own, smaller register allocation.
template <typename T, int C, bool SC>
__device__ __forceinline__ void tile_steps(const Seg1D& s, const TileGeom& tg, int steps,
                                           T (&v)[C]) {
    constexpr int W = 64 * C;
    const int lane = threadIdx.x & 63;
    const int64_t n = s.n;
    const int64_t lbase = tg.base + (int64_t)lane * C;
    const bool zero_lo = s.bc_lo == BC_DIRICHLET0 && tg.base < 0;
    const bool zero_hi = s.bc_hi == BC_DIRICHLET0 && tg.base + W > n;
    if constexpr (SC) {
        const T b = static_cast<T>(s.beta);
        const T ap = static_cast<T>(s.alpha_p);
        int since = 0;
        for (int t = 0; t < steps; ++t) {
            step_tile_scaled<T, C>(v, b, zero_lo, zero_hi, lbase, n);
            if (++since == s.period) {
                since = 0;
                scale_tile<T, C>(v, ap);
            }
        }
        if (since) scale_tile<T, C>(v, static_cast<T>(s.alpha_rem));
    } else {
        const T k = static_cast<T>(s.r);
        for (int t = 0; t < steps; ++t) step_tile<T, C>(v, k, zero_lo, zero_hi, lbase, n);
    }
}

// Cell-by-cell store of the inner cells of a boundary or unaligned tile from
// the wave's LDS area.
template <typename T, int C>
__device__ __forceinline__ void tile_store_slow(const Seg1D& s, int64_t o0, int64_t base,
                                                          int halo, const T* __restrict__ lds) {
    const int lane = threadIdx.x & 63;
    const int64_t n = s.n;
    const int64_t wout = 64LL * C - 2LL * halo;
    T* out = static_cast<T*>(s.out);
    const int64_t ostart = o0 > 0 ? o0 : 0;
    const int64_t oend = (o0 + wout < n) ? o0 + wout : n;
#pragma unroll 1
    for (int j = 0; j < C; ++j) {
        const int i = lane + 64 * j;
        const int64_t g = base + i;
        if (g >= ostart && g < oend) out[g] = lds[lds_pos<T, C>(i)];
    }
}

template <typename T, int C>
__device__ __forceinline__ void tile_store(const Seg1D& s, const TileGeom& tg, int halo,
                                           T* __restrict__ lds, const T (&v)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    constexpr int W = 64 * C;
    const int lane = threadIdx.x & 63;
    T* out = static_cast<T*>(s.out);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < C / VN; ++q) {
        VT x;
#pragma unroll
        for (int e = 0; e < VN; ++e) x[e] = v[q * VN + e];
        *reinterpret_cast<VT*>(lds + lane * (C + VN) + q * VN) = x;
    }
    __builtin_amdgcn_wave_barrier();
    if (tg.interior && aligned16(out + tg.base)) {
        VT* dst = reinterpret_cast<VT*>(out + tg.base);
#pragma unroll
        for (int kk = 0; kk < C / VN; ++kk) {
            const int i = VN * (lane + 64 * kk);
            if (i >= halo && i < W - halo)
                gstore_nt(*reinterpret_cast<const VT*>(lds + lds_pos<T, C>(i)), dst,
                          lane + 64 * kk);
        }
    } else {
        tile_store_slow<T, C>(s, tg.o0, tg.base, halo, lds);
    }
    // the next tile's LDS writes must follow the reads above
    __builtin_amdgcn_wave_barrier();
}

// Advance tile `tile` of segment `s` by `steps` steps: the phases in a row.
template <typename T, int C, bool SC>
__device__ __forceinline__ void tile1d(const Seg1D& s, int64_t tile, int steps, int halo,
                                       T* __restrict__ lds) {
    static_assert(C % V16<T>::N == 0, "cells per lane must be a multiple of the vector width");
    const TileGeom tg = tile_geom<C>(s, tile, halo);
    T v[C];
    if (tile_fast<T>(s, tg)) {
        T pf[C];
        tile_fetch<T, C>(s, tg, pf);
        tile_stage<T, C>(pf, lds, v);
    } else {
        tile_fill_slow<T, C>(s, tg.base, tg.interior, lds);
        __builtin_amdgcn_wave_barrier();
        tile_read<T, C>(lds, v);
    }
    tile_steps<T, C, SC>(s, tg, steps, v);
    tile_store<T, C>(s, tg, halo, lds, v);
}

// Dynamic LDS of the tile kernels: `wpg` wave areas of 64*(C + VN) cells.
extern __shared__ __attribute__((aligned(16))) unsigned char hx_lds1d[];

template <typename T, int C>
__device__ __forceinline__ T* wave_lds() {
    constexpr int VN = V16<T>::N;
    return reinterpret_cast<T*>(hx_lds1d) +
           __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * (64 * (C + VN));
}

template <typename T, int C, bool SC>
__global__ __launch_bounds__(256) void k_stencil1d(Seg1D s, int steps, int halo, int64_t ntiles) {
    const int wpg = blockDim.x >> 6;
    const int64_t tile = (int64_t)blockIdx.x * wpg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tile >= ntiles) return;
    tile1d<T, C, SC>(s, tile, steps, halo, wave_lds<T, C>());
}

// Segment and tile of table entry t: computed when every segment has per_seg
// tiles (the table is in segment order), else read from the table.
__device__ __forceinline__ void locate_tile(const uint32_t* __restrict__ tseg,
                                            const uint32_t* __restrict__ tidx, int64_t t,
                                            int64_t per_seg, uint32_t& si, uint32_t& ti) {
    if (per_seg > 0) {
        // the tile table is uint32-indexed, so 32-bit division suffices
        si = (uint32_t)t / (uint32_t)per_seg;
        ti = (uint32_t)t - si * (uint32_t)per_seg;
    } else {
        si = __builtin_amdgcn_readfirstlane(tseg[t]);
        ti = __builtin_amdgcn_readfirstlane(tidx[t]);
    }
}

// Persistent, software-pipelined form: `gridDim.x * wpg` waves stride over the
// tile table, and each wave issues the HBM reads of its next tile (into
// registers) before running the current tile's steps, so the reads' latency
// hides behind the arithmetic instead of behind other waves only.  `segs` is
// the segment table (TAB), or unused for a single segment passed by value in
// `s0` (!TAB); the two are separate instantiations so that the segment's fields
// stay in scalar registers either way.
template <typename T, int C, bool SC, bool TAB>
__global__ __launch_bounds__(256) void k_stencil1d_pipe(Seg1D s0, const Seg1D* __restrict__ segs,
                                                        const uint32_t* __restrict__ tseg,
                                                        const uint32_t* __restrict__ tidx,
                                                        int64_t ntiles, int steps, int halo,
                                                        int64_t per_seg) {
    const int wpg = blockDim.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * wpg;
    int64_t t = (int64_t)blockIdx.x * wpg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= ntiles) return;
    T* lds = wave_lds<T, C>();
    // The segment and geometry of a tile are recomputed from its index where
    // needed (scalar work), so that only the tile index, the prefetch flag and
    // the prefetched registers are carried from one iteration to the next.
    auto seg_of = [&](int64_t tt, uint32_t& ti) -> const Seg1D& {
        uint32_t si = 0;
        ti = (uint32_t)tt;
        if constexpr (TAB) {
            locate_tile(tseg, tidx, tt, per_seg, si, ti);
            return segs[si];
        } else {
            return s0;
        }
    };
    T pf[C], v[C];
    bool fast;
    {
        uint32_t ti;
        const Seg1D& s = seg_of(t, ti);
        const TileGeom tg = tile_geom<C>(s, ti, halo);
        fast = tile_fast<T>(s, tg);
        if (fast) tile_fetch<T, C>(s, tg, pf);
    }
#pragma clang loop unroll(disable)
    for (;;) {
        uint32_t ti;
        const Seg1D& s = seg_of(t, ti);
        const TileGeom tg = tile_geom<C>(s, ti, halo);
        if (fast) {
            tile_stage<T, C>(pf, lds, v);
        } else {
            tile_fill_slow<T, C>(s, tg.base, tg.interior, lds);
            __builtin_amdgcn_wave_barrier();
            tile_read<T, C>(lds, v);
        }
        const int64_t tn = t + nwaves;
        const bool more = tn < ntiles;
        bool fastn = false;
        if (more) {
            uint32_t tin;
            const Seg1D& sn = seg_of(tn, tin);
            const TileGeom tgn = tile_geom<C>(sn, tin, halo);
            fastn = tile_fast<T>(sn, tgn);
            if (fastn) tile_fetch<T, C>(sn, tgn, pf);  // overlaps the steps below
        }
        tile_steps<T, C, SC>(s, tg, steps, v);
        tile_store<T, C>(s, tg, halo, lds, v);
        if (!more) break;
        t = tn;
        fast = fastn;
    }
}

template <typename T>
size_t lds_bytes(const Geom1D& g) {
    return (size_t)g.wpg * 64 * (g.cpl + V16<T>::N) * sizeof(T);
}

// One tile per wave (the grid covers the whole tile table): the hardware
// dispatcher does the load balancing, and with no loop around the tile the
// register allocation matches the single-segment kernel.
// When every segment has the same tile count `per_seg` (a batch of equal
// partitions), the tile's segment and index are computed instead of loaded, so
// a wave's first HBM access does not wait behind two table lookups.
template <typename T, int C, bool SC>
__global__ __launch_bounds__(256) void k_stencil1d_flat(const Seg1D* __restrict__ segs,
                                                        const uint32_t* __restrict__ tseg,
                                                        const uint32_t* __restrict__ tidx,
                                                        int64_t ntiles, int steps, int halo,
                                                        int64_t per_seg) {
    const int wpg = blockDim.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * wpg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= ntiles) return;
    uint32_t si, ti;
    locate_tile(tseg, tidx, t, per_seg, si, ti);
    tile1d<T, C, SC>(segs[si], ti, steps, halo, wave_lds<T, C>());
}

#define HX_CPL_SWITCH(KERNEL, ...)                                                    \
    switch (g.cpl) {                                                                  \
    case 8: hipLaunchKernelGGL((KERNEL<T, 8, SC>), __VA_ARGS__); break;                \
    case 16: hipLaunchKernelGGL((KERNEL<T, 16, SC>), __VA_ARGS__); break;              \
    case 32: hipLaunchKernelGGL((KERNEL<T, 32, SC>), __VA_ARGS__); break;              \
    case 64: hipLaunchKernelGGL((KERNEL<T, 64, SC>), __VA_ARGS__); break;              \
    default: return hipErrorInvalidValue;                                             \
    }

#define HX_CPL_SWITCH4(KERNEL, B, ...)                                                \
    switch (g.cpl) {                                                                  \
    case 8: hipLaunchKernelGGL((KERNEL<T, 8, SC, B>), __VA_ARGS__); break;             \
    case 16: hipLaunchKernelGGL((KERNEL<T, 16, SC, B>), __VA_ARGS__); break;           \
    case 32: hipLaunchKernelGGL((KERNEL<T, 32, SC, B>), __VA_ARGS__); break;           \
    case 64: hipLaunchKernelGGL((KERNEL<T, 64, SC, B>), __VA_ARGS__); break;           \
    default: return hipErrorInvalidValue;                                             \
    }

template <typename T, bool SC>
hipError_t launch_pipe(const Seg1D& s0, const Seg1D* segs, const uint32_t* tseg,
                       const uint32_t* tidx, int64_t ntiles, const Geom1D& g, int64_t grid_waves,
                       int64_t per_seg, hipStream_t st) {
    const dim3 block(64 * g.wpg);
    const dim3 grid((unsigned)((grid_waves + g.wpg - 1) / g.wpg));
    const size_t sh = lds_bytes<T>(g);
    if (segs) {
        HX_CPL_SWITCH4(k_stencil1d_pipe, true, grid, block, sh, st, s0, segs, tseg, tidx, ntiles,
                       g.steps, g.halo, per_seg)
    } else {
        HX_CPL_SWITCH4(k_stencil1d_pipe, false, grid, block, sh, st, s0, segs, tseg, tidx, ntiles,
                       g.steps, g.halo, per_seg)
    }
    return hipGetLastError();
}

template <typename T, bool SC>
hipError_t launch_single_sc(const Seg1D& s, const Geom1D& g, hipStream_t st) {
    const int64_t ntiles = tiles_1d(s, g);
    const dim3 block(64 * g.wpg);
    const dim3 grid((unsigned)((ntiles + g.wpg - 1) / g.wpg));
    const size_t sh = lds_bytes<T>(g);
    HX_CPL_SWITCH(k_stencil1d, grid, block, sh, st, s, g.steps, g.halo, ntiles)
    return hipGetLastError();
}

template <typename T>
hipError_t launch_single(const Seg1D& s0, const Geom1D& g, hipStream_t st) {
    Seg1D s = s0;
    s.shift = tile_shift(s.in, sizeof(T));
    set_rate_1d(s, g.steps);
    return s.period > 0 ? launch_single_sc<T, true>(s, g, st) : launch_single_sc<T, false>(s, g, st);
}

template <typename T, bool SC>
hipError_t launch_batched_sc(const Seg1D* segs, const uint32_t* tseg, const uint32_t* tidx,
                             int64_t ntiles, const Geom1D& g, int64_t grid_waves, int64_t per_seg,
                             hipStream_t st) {
    if (grid_waves > 0 && grid_waves < ntiles)
        return launch_pipe<T, SC>(Seg1D{}, segs, tseg, tidx, ntiles, g, grid_waves, per_seg, st);
    const dim3 block(64 * g.wpg);
    const size_t sh = lds_bytes<T>(g);
    const dim3 grid((unsigned)((ntiles + g.wpg - 1) / g.wpg));
    HX_CPL_SWITCH(k_stencil1d_flat, grid, block, sh, st, segs, tseg, tidx, ntiles, g.steps,
                  g.halo, per_seg)
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batched(const Seg1D* segs, const uint32_t* tseg, const uint32_t* tidx,
                          int64_t ntiles, const Geom1D& g, int64_t grid_waves, int64_t per_seg,
                          bool scaled, hipStream_t st) {
    return scaled ? launch_batched_sc<T, true>(segs, tseg, tidx, ntiles, g, grid_waves, per_seg, st)
                  : launch_batched_sc<T, false>(segs, tseg, tidx, ntiles, g, grid_waves, per_seg,
                                                st);
}

#undef HX_CPL_SWITCH
#undef HX_CPL_SWITCH4

}  // namespace

hipError_t launch_stencil1d(int dtype, const Seg1D& seg, const Geom1D& g, hipStream_t stream) {
    return dtype == 0 ? launch_single<float>(seg, g, stream) : launch_single<double>(seg, g, stream);
}

hipError_t launch_stencil1d_batched(int dtype, const Seg1D* segs_dev, const uint32_t* tile_seg,
                                    const uint32_t* tile_idx, int64_t ntiles, const Geom1D& g,
                                    int64_t grid_waves, int64_t per_seg, bool scaled,
                                    hipStream_t stream) {
    return dtype == 0 ? launch_batched<float>(segs_dev, tile_seg, tile_idx, ntiles, g, grid_waves,
                                              per_seg, scaled, stream)
                      : launch_batched<double>(segs_dev, tile_seg, tile_idx, ntiles, g,
                                               grid_waves, per_seg, scaled, stream);
}

}  // namespace hx
