// 2D explicit five-point heat stencil with temporal blocking, for gfx950.
//
// Operation: u'_ij = u_ij + r (u_{i-1,j} + u_{i+1,j} + u_{i,j-1} + u_{i,j+1}
// - 4 u_ij) on a row-major band of ny x nx cells (the Sec. V-A.1 stencil
// extended to a grid), D steps fused per pass, zero-Dirichlet on the left and
// right edges, top and bottom either zero-Dirichlet or supplied by halo rows.
//
// Mapping (2.5D streaming with a register pipeline).  A wave owns a strip of
// 64*C columns (C adjacent columns per lane) and a chunk of R output rows.  It
// streams the strip's input rows from R0 - D to R1 + D - 1 once, top to
// bottom.  Time level k (1..D) keeps the previous two rows it received from
// level k-1 in registers (a three-slot ring per level, rotated by unrolling
// the row loop three times); each new level-(k-1) row lets level k produce the
// row above it.  A row therefore enters from HBM once, climbs all D levels inside
// registers, and leaves to HBM once: a pass costs one read and one write per
// cell plus the 2*D halo rows per chunk and 2*H halo columns per strip, whatever
// D is.  West/east neighbours across lanes come from DPP wave shifts; north and
// south neighbours are the pipeline's own rows, so there is no LDS and no
// barrier.  Outer context columns (H >= D per side) go stale one column per
// level and are never stored.
//
// Per cell-step: a = n + s; b = w + e; t = a + b; d = fma(-4, c, t);
// c' = fma(r, d, c) -- the same rounding in every geometry.
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

__device__ __forceinline__ bool aligned16(const void* p) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Pointer to band row y (any integer), or null when the row is a zero ghost.
template <typename T>
__device__ __forceinline__ const T* row_ptr(const Band2D& b, int64_t y) {
    if (y >= 0 && y < b.ny) return static_cast<const T*>(b.in) + y * b.nx;
    if (y < 0) {
        if (b.bc_top == BC_GHOST && y >= -(int64_t)b.hw)
            return static_cast<const T*>(b.halo_top) + (b.hw + y) * b.nx;
        return nullptr;
    }
    if (b.bc_bot == BC_GHOST && y - b.ny < (int64_t)b.hw)
        return static_cast<const T*>(b.halo_bot) + (y - b.ny) * b.nx;
    return nullptr;
}

// True for a row that is a zero-Dirichlet ghost at every time level.
__device__ __forceinline__ bool zero_row(const Band2D& b, int64_t y) {
    return (y < 0 && b.bc_top != BC_GHOST) || (y >= b.ny && b.bc_bot != BC_GHOST);
}

// Per-wave constants of a strip/chunk.
struct Strip {
    int64_t xl;      // first column of this lane
    int64_t x0;      // first output column of the strip
    int64_t wout;    // output columns of the strip
    int64_t y0, y1;  // output rows [y0, y1)
    bool xin;        // whole strip inside [0, nx)
    bool vec;        // vector loads/stores possible
    int lane;
};

// One row step of the pipeline for a row index whose position in the 3-row
// rotation is M: row yy enters level 0 in slot M of every level's ring, the
// rows of level l in slots M+1 and M+2 (mod 3) are the two before it, and
// level l+1 receives its new row (yy - l - 1) in its own slot M.  All slot
// indices are compile-time constants, so rotating the rows costs no moves.
// Load row y of the band (or its zero ghost) for this lane's columns.
template <typename T, int C>
__device__ __forceinline__ void load_row2d(const Band2D& b, const Strip& w, int64_t y, T (&dst)[C],
                                           const bool (&colok)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    const T* rp = row_ptr<T>(b, y);
    if (rp == nullptr) {
#pragma unroll
        for (int j = 0; j < C; ++j) dst[j] = T(0);
    } else if (w.vec) {
        const VT* src = reinterpret_cast<const VT*>(rp + w.xl);
#pragma unroll
        for (int q = 0; q < C / VN; ++q) {
            const VT x = __builtin_nontemporal_load(src + q);
#pragma unroll
            for (int e = 0; e < VN; ++e) dst[q * VN + e] = x[e];
        }
    } else {
#pragma unroll
        for (int j = 0; j < C; ++j) dst[j] = colok[j] ? rp[w.xl + j] : T(0);
    }
}

// One row step of the pipeline for a row index whose position in the 3-row
// rotation is M: row yy (already loaded, in `pf0`) enters level 0 in slot M of
// every level's ring, the rows of level l in slots M+1 and M+2 (mod 3) are the
// two before it, and level l+1 receives its new row (yy - l - 1) in its own
// slot M.  All slot indices are compile-time constants, so rotating the rows
// costs no moves.  Rows are prefetched two ahead: the loads of row yy+2 are
// issued before the arithmetic of row yy, so their latency overlaps it.
template <typename T, int C, int D, int M>
__device__ __forceinline__ void row_step(const Band2D& b, const Strip& w, int halo, int64_t yy,
                                         T (&R)[D][3][C], const bool (&colok)[C], T k,
                                         T (&pf0)[C], T (&pf1)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    constexpr int S = 64 * C;
    constexpr int OLD = (M + 1) % 3, NEW = (M + 2) % 3;
    // ---- level 0: row yy from the prefetch queue; queue row yy+2
#pragma unroll
    for (int j = 0; j < C; ++j) {
        R[0][M][j] = pf0[j];
        pf0[j] = pf1[j];
    }
    load_row2d<T, C>(b, w, yy + 2, pf1, colok);
    // ---- levels 1..D
    T last[C];
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const int64_t yo = yy - l - 1;  // row produced at level l+1
        const T* cn = R[l][NEW];        // row yo at level l (centre)
        const T* no = R[l][OLD];        // row yo - 1 (north)
        const T* so = R[l][M];          // row yo + 1 (south)
        const T left = dpp_move<DPP_WAVE_SHR1>(cn[C - 1]);
        const T right = dpp_move<DPP_WAVE_SHL1>(cn[0]);
        T nw[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const T c = cn[j];
            const T we = (j > 0 ? cn[j - 1] : left) + (j + 1 < C ? cn[j + 1] : right);
            const T ns = no[j] + so[j];
            const T t = ns + we;
            const T d = fmaT(T(-4), c, t);
            nw[j] = fmaT(k, d, c);
        }
        if (zero_row(b, yo)) {
#pragma unroll
            for (int j = 0; j < C; ++j) nw[j] = T(0);
        } else if (!w.xin) {
#pragma unroll
            for (int j = 0; j < C; ++j) nw[j] = colok[j] ? nw[j] : T(0);
        }
        if (l + 1 < D) {
#pragma unroll
            for (int j = 0; j < C; ++j) R[l + 1 < D ? l + 1 : 0][M][j] = nw[j];
        } else {
#pragma unroll
            for (int j = 0; j < C; ++j) last[j] = nw[j];
        }
    }
    // ---- row yy - D at level D: store if it is an output row of this wave
    const int64_t yo = yy - D;
    if (yo >= w.y0 && yo < w.y1) {
        T* orow = static_cast<T*>(b.out) + yo * b.nx;
        if (w.vec) {
            VT* dst = reinterpret_cast<VT*>(orow + w.xl);
#pragma unroll
            for (int q = 0; q < C / VN; ++q) {
                const int lc = w.lane * C + q * VN;
                if (lc >= halo && lc < S - halo) {
                    VT x;
#pragma unroll
                    for (int e = 0; e < VN; ++e) x[e] = last[q * VN + e];
                    __builtin_nontemporal_store(x, dst + q);
                }
            }
        } else {
            const int64_t xs = w.x0 > 0 ? w.x0 : 0;
            const int64_t xe = (w.x0 + w.wout < b.nx) ? w.x0 + w.wout : b.nx;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int64_t x = w.xl + j;
                if (x >= xs && x < xe) orow[x] = last[j];
            }
        }
    }
}

template <typename T, int C, int D>
__global__ __launch_bounds__(256) void k_stencil2d(Band2D b, int rows, int halo, int64_t nstrips,
                                                   int64_t nwaves) {
    constexpr int VN = V16<T>::N;
    constexpr int S = 64 * C;
    static_assert(C % VN == 0, "columns per lane must be a multiple of the vector width");
    const int wpg = blockDim.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * wpg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    Strip w;
    w.lane = threadIdx.x & 63;
    const int64_t strip = wave % nstrips;
    const int64_t chunk = wave / nstrips;
    w.wout = S - 2 * halo;
    w.x0 = strip * w.wout;
    const int64_t xb = w.x0 - halo;  // first column held by lane 0
    w.xl = xb + (int64_t)w.lane * C;
    w.y0 = chunk * rows;
    w.y1 = (w.y0 + rows < b.ny) ? w.y0 + rows : b.ny;
    w.xin = xb >= 0 && xb + S <= b.nx;
    w.vec = w.xin && b.aligned;
    const T k = static_cast<T>(b.r);

    // column mask for edge strips (cells outside [0, nx) are zero ghosts)
    bool colok[C];
#pragma unroll
    for (int j = 0; j < C; ++j) colok[j] = (w.xl + j >= 0) && (w.xl + j < b.nx);

    T R[D][3][C];
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int j = 0; j < C; ++j) R[l][m][j] = T(0);

    const int64_t yend = w.y1 + D;
    T pf0[C], pf1[C];
    load_row2d<T, C>(b, w, w.y0 - D, pf0, colok);
    load_row2d<T, C>(b, w, w.y0 - D + 1, pf1, colok);
    for (int64_t yy = w.y0 - D; yy < yend; yy += 3) {
        row_step<T, C, D, 0>(b, w, halo, yy, R, colok, k, pf0, pf1);
        if (yy + 1 >= yend) break;
        row_step<T, C, D, 1>(b, w, halo, yy + 1, R, colok, k, pf0, pf1);
        if (yy + 2 >= yend) break;
        row_step<T, C, D, 2>(b, w, halo, yy + 2, R, colok, k, pf0, pf1);
    }
}

template <typename T, int C, int D>
hipError_t launch_cd(const Band2D& b, const Geom2D& g, hipStream_t st) {
    const int64_t wout = 64LL * C - 2LL * g.halo;
    const int64_t nstrips = (b.nx + wout - 1) / wout;
    const int64_t nchunks = (b.ny + g.rows - 1) / g.rows;
    const int64_t nwaves = nstrips * nchunks;
    const dim3 block(64 * g.wpg);
    const dim3 grid((unsigned)((nwaves + g.wpg - 1) / g.wpg));
    hipLaunchKernelGGL((k_stencil2d<T, C, D>), grid, block, 0, st, b, g.rows, g.halo, nstrips,
                       nwaves);
    return hipGetLastError();
}

template <typename T, int C, bool DEEP>
hipError_t launch_c(const Band2D& b, const Geom2D& g, hipStream_t st) {
    if constexpr (DEEP) {
        switch (g.steps) {
        case 10: return launch_cd<T, C, 10>(b, g, st);
        case 12: return launch_cd<T, C, 12>(b, g, st);
        case 16: return launch_cd<T, C, 16>(b, g, st);
        default: break;
        }
    }
    switch (g.steps) {
    case 1: return launch_cd<T, C, 1>(b, g, st);
    case 2: return launch_cd<T, C, 2>(b, g, st);
    case 3: return launch_cd<T, C, 3>(b, g, st);
    case 4: return launch_cd<T, C, 4>(b, g, st);
    case 5: return launch_cd<T, C, 5>(b, g, st);
    case 6: return launch_cd<T, C, 6>(b, g, st);
    case 7: return launch_cd<T, C, 7>(b, g, st);
    case 8: return launch_cd<T, C, 8>(b, g, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool stencil2d_supported(int dtype, int cpl, int steps) {
    const bool small = steps >= 1 && steps <= 8;
    const bool deep = steps == 10 || steps == 12 || steps == 16;
    if (dtype == 0 && cpl == 4) return small || deep;
    if (dtype == 0 && cpl == 8) return small;
    return dtype == 1 && cpl == 4 && small;
}

hipError_t launch_stencil2d(int dtype, const Band2D& b, const Geom2D& g, hipStream_t stream) {
    if (!stencil2d_supported(dtype, g.cpl, g.steps)) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (g.cpl == 4) return launch_c<float, 4, true>(b, g, stream);
        return launch_c<float, 8, false>(b, g, stream);
    }
    return launch_c<double, 4, false>(b, g, stream);
}

}  // namespace hx
