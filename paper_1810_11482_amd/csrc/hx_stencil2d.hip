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
// Per cell-step: t = (n + s) + (w + e), then for 0 <= r <= 7/32 the rescaled
// update w' = fma(r/(1-4r), t, w) (set_rate_2d), otherwise d = fma(-4, c, t);
// c' = fma(r, d, c).  A pass's result depends on its depth only, not on the
// tile geometry.
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

// The per-cell update of one level: direct (k = r) or rescaled (SC: b =
// r/(1-4r), and the level's row is multiplied by ap at every rescale level,
// by arem at the last one when the depth is not a multiple of the period;
// `mask` has bit l set for the levels l+1 that rescale).
template <typename T>
struct Rate2 {
    T k, b, ap, arem;
    uint32_t mask;
    bool tail;
};

template <typename T, int D, bool SC>
__device__ __forceinline__ Rate2<T> make_rate(const Band2D& band) {
    Rate2<T> rt;
    rt.k = static_cast<T>(band.r);
    rt.b = static_cast<T>(band.beta);
    rt.ap = static_cast<T>(band.alpha_p);
    rt.arem = static_cast<T>(band.alpha_rem);
    rt.mask = 0;
    rt.tail = false;
    if constexpr (SC) {
        const int p = band.period;
        for (int l = 0; l < D; ++l)
            if ((l + 1) % p == 0) rt.mask |= 1u << l;
        rt.tail = (D % p) != 0;
        if (rt.tail) rt.mask |= 1u << (D - 1);
    }
    return rt;
}

template <typename T, bool SC>
__device__ __forceinline__ T update(const Rate2<T>& rt, T c, T t) {
    if constexpr (SC) {
        return fmaT(rt.b, t, c);
    } else {
        const T d = fmaT(T(-4), c, t);
        return fmaT(rt.k, d, c);
    }
}

template <typename T, int C, int D, bool SC>
__device__ __forceinline__ void rescale_level(const Rate2<T>& rt, int l, T* v) {
    if constexpr (SC) {
        if ((rt.mask >> l) & 1u) {
            const T f = (l + 1 == D && rt.tail) ? rt.arem : rt.ap;
#pragma unroll
            for (int j = 0; j < C; ++j) v[j] *= f;
        }
    }
}

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
            const VT x = src[q];
#pragma unroll
            for (int e = 0; e < VN; ++e) dst[q * VN + e] = x[e];
        }
    } else {
#pragma unroll
        for (int j = 0; j < C; ++j) dst[j] = colok[j] ? rp[w.xl + j] : T(0);
    }
}

// Level-0 rows live in a ring of Q rows (Q a multiple of 3): rows yy-2 .. yy
// are the pipeline's input window and rows yy+1 .. yy+Q-3 are loads in flight,
// so Q-3 rows are prefetched ahead of their use.  Row y sits in slot
// (y - ystart) mod Q.
constexpr int ring_rows() { return 6; }

// One row step of the pipeline for the row yy whose ring position is M
// (compile-time, the row loop is unrolled Q times): the load of row yy+Q-3 is
// issued into the slot of row yy-3, no longer needed; then level l+1 (l =
// 0..D-1) produces row yy-l-1 from its three level-l rows.  Level 0 reads the
// Q-row ring, levels 1..D-1 keep their last three rows in a three-slot ring
// at position M mod 3.  Every slot index is a compile-time constant, so
// rotating rows costs no register moves.
//
// EDGE = false is the interior form: the wave's strip lies inside [0, nx) and
// none of the rows it produces is a zero-Dirichlet ghost, so no cell is masked
// and each level is straight-line code (which also lets the compiler fold the
// DPP shifts into the adds).
template <typename T, int C, int D, int Q, int M, bool EDGE, bool SC>
__device__ __forceinline__ void row_step(const Band2D& b, const Strip& w, int halo, int64_t yy,
                                         int64_t yend, T (&Z)[Q][C], T (&R)[D][3][C],
                                         const bool (&colok)[C], const Rate2<T>& rt) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    constexpr int S = 64 * C;
    constexpr int M3 = M % 3, OLD = (M3 + 1) % 3, NEW = (M3 + 2) % 3;
    if (yy + Q - 3 < yend) load_row2d<T, C>(b, w, yy + Q - 3, Z[(M + Q - 3) % Q], colok);
    T last[C];
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const int64_t yo = yy - l - 1;  // row produced at level l+1
        const T* cn = l == 0 ? Z[(M + Q - 1) % Q] : R[l][NEW];  // row yo at level l
        const T* no = l == 0 ? Z[(M + Q - 2) % Q] : R[l][OLD];  // row yo - 1
        const T* so = l == 0 ? Z[M] : R[l][M3];                 // row yo + 1
        const T left = dpp_move<DPP_WAVE_SHR1>(cn[C - 1]);
        const T right = dpp_move<DPP_WAVE_SHL1>(cn[0]);
        T nw[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const T c = cn[j];
            const T we = (j > 0 ? cn[j - 1] : left) + (j + 1 < C ? cn[j + 1] : right);
            const T ns = no[j] + so[j];
            const T t = ns + we;
            nw[j] = update<T, SC>(rt, c, t);
        }
        if constexpr (EDGE) {
            if (zero_row(b, yo)) {
#pragma unroll
                for (int j = 0; j < C; ++j) nw[j] = T(0);
            } else if (!w.xin) {
#pragma unroll
                for (int j = 0; j < C; ++j) nw[j] = colok[j] ? nw[j] : T(0);
            }
        }
        rescale_level<T, C, D, SC>(rt, l, nw);
        if (l + 1 < D) {
#pragma unroll
            for (int j = 0; j < C; ++j) R[l + 1 < D ? l + 1 : 0][M3][j] = nw[j];
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

// ---------------------------------------------------------------------------
// Static-count form, for bands whose rows are all 16-byte aligned and whose
// size is under 2 GiB (32-bit buffer offsets).  Every row step issues exactly
// one vector load per lane (the prefetch; rows past the chunk are clamped to
// its last row) and, once the pipeline is full, exactly one vector store per
// lane.  Lanes that must not store (halo columns, columns past nx) store
// through a buffer resource with an out-of-range offset, which the hardware
// drops, so no memory operation sits under a branch or an exec mask.  With
// straight-line memory operations the compiler's wait counts cover only the
// row being consumed, and Q-3 rows stay in flight behind the arithmetic.
//
// EDGE waves (a strip reaching past [0, nx), or rows that are zero-Dirichlet
// ghosts) run the same code plus selects: zero rows and columns outside
// [0, nx) are loaded from a valid clamped address and replaced by 0, and every
// level re-zeroes them.
template <typename T, int C>
struct FastIO {
    const T* in;
    const T* top;
    const T* bot;
    int64_t nx, ny, hw;
    int64_t ylo, yhi;                   // clamp range of level-0 rows
    int64_t xload[C / V16<T>::N];       // column of each lane vector's load (clamped into the row)
    bool top_ghost, bot_ghost;          // top/bottom rows come from halo buffers
    __amdgpu_buffer_rsrc_t out;         // the band's output, bounds-checked
    uint32_t off[C / V16<T>::N];        // byte offset of each lane vector, or out of range
    bool colin[C / V16<T>::N];          // lane vector inside [0, nx)
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int BUF_DWORD3 = 0x00020000;  // raw 32-bit buffer (gfx9 family)
constexpr uint32_t OOB_OFFSET = 0x7ffffff0u;

// Row y is a zero ghost: outside the band on a zero-Dirichlet side, or past
// the supplied halo rows.
template <typename T, int C>
__device__ __forceinline__ bool zero_row_fast(const FastIO<T, C>& io, int64_t y) {
    return (y < 0 && (!io.top_ghost || y < -io.hw)) ||
           (y >= io.ny && (!io.bot_ghost || y >= io.ny + io.hw));
}

template <typename T, int C, bool EDGE>
__device__ __forceinline__ void load_fast(const FastIO<T, C>& io, int64_t y, T (&dst)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    y = y < io.ylo ? io.ylo : (y > io.yhi ? io.yhi : y);
    const bool zr = EDGE && zero_row_fast(io, y);
    const int64_t ys = zr ? 0 : y;
    const T* rp = ys < 0 ? io.top + (io.hw + ys) * io.nx
                         : (ys < io.ny ? io.in + ys * io.nx : io.bot + (ys - io.ny) * io.nx);
#pragma unroll
    for (int q = 0; q < C / VN; ++q) {
        const VT x = *(reinterpret_cast<const VT*>(rp + io.xload[q]));
#pragma unroll
        for (int e = 0; e < VN; ++e)
            dst[q * VN + e] = (EDGE && (zr || !io.colin[q])) ? T(0) : x[e];
    }
}

template <typename T, int C>
__device__ __forceinline__ void store_fast(const FastIO<T, C>& io, int64_t y, const T (&v)[C]) {
    typedef typename V16<T>::t VT;
    constexpr int VN = V16<T>::N;
    const uint32_t row = (uint32_t)(y * io.nx * (int64_t)sizeof(T));
#pragma unroll
    for (int q = 0; q < C / VN; ++q) {
        VT x;
#pragma unroll
        for (int e = 0; e < VN; ++e) x[e] = v[q * VN + e];
        u32x4 bits;
        __builtin_memcpy(&bits, &x, sizeof(bits));
        __builtin_amdgcn_raw_buffer_store_b128(bits, io.out, (int)(io.off[q] + row), 0, 0);
    }
}

template <typename T, int C, int D, int Q, int M, bool STORE, bool EDGE, bool SC>
__device__ __forceinline__ void row_step_fast(const FastIO<T, C>& io, int64_t yy, T (&Z)[Q][C],
                                              T (&R)[D][3][C], const Rate2<T>& rt) {
    constexpr int VN = V16<T>::N;
    constexpr int M3 = M % 3, OLD = (M3 + 1) % 3, NEW = (M3 + 2) % 3;
    load_fast<T, C, EDGE>(io, yy + Q - 3, Z[(M + Q - 3) % Q]);
    T last[C];
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const T* cn = l == 0 ? Z[(M + Q - 1) % Q] : R[l][NEW];
        const T* no = l == 0 ? Z[(M + Q - 2) % Q] : R[l][OLD];
        const T* so = l == 0 ? Z[M] : R[l][M3];
        const T left = dpp_move<DPP_WAVE_SHR1>(cn[C - 1]);
        const T right = dpp_move<DPP_WAVE_SHL1>(cn[0]);
        T* dst = l + 1 < D ? R[l + 1 < D ? l + 1 : 0][M3] : last;
        const bool zr = EDGE && zero_row_fast(io, yy - l - 1);
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const T c = cn[j];
            const T we = (j > 0 ? cn[j - 1] : left) + (j + 1 < C ? cn[j + 1] : right);
            const T ns = no[j] + so[j];
            const T t = ns + we;
            const T v = update<T, SC>(rt, c, t);
            dst[j] = (EDGE && (zr || !io.colin[j / VN])) ? T(0) : v;
        }
        rescale_level<T, C, D, SC>(rt, l, dst);
    }
    if constexpr (STORE) store_fast<T, C>(io, yy - D, last);
}

// N consecutive row steps starting at ring position M.  Steps that store
// stop at the chunk's end.
template <typename T, int C, int D, int Q, int M, int N, bool STORE, bool EDGE, bool SC>
__device__ __forceinline__ void steps_fast(const FastIO<T, C>& io, int64_t& yy, int64_t yend,
                                           T (&Z)[Q][C], T (&R)[D][3][C], const Rate2<T>& rt) {
    if constexpr (N > 0) {
        if (STORE && yy >= yend) return;
        row_step_fast<T, C, D, Q, M, STORE, EDGE, SC>(io, yy, Z, R, rt);
        ++yy;
        steps_fast<T, C, D, Q, (M + 1) % Q, N - 1, STORE, EDGE, SC>(io, yy, yend, Z, R, rt);
    }
}

// Rows ystart .. ystart+2D-1 fill the pipeline (nothing to store yet); from
// then on every row step stores row yy - D, an output row of the chunk.
template <typename T, int C, int D, int Q, bool EDGE, bool SC>
__device__ __forceinline__ void stream_rows_fast(const FastIO<T, C>& io, int64_t ystart,
                                                 int64_t yend, T (&Z)[Q][C], T (&R)[D][3][C],
                                                 const Rate2<T>& rt) {
    constexpr int W = 2 * D, WF = W / Q, WR = W % Q;
#pragma unroll
    for (int m = 0; m < Q - 3; ++m) load_fast<T, C, EDGE>(io, ystart + m, Z[m]);
    int64_t yy = ystart;
    for (int i = 0; i < WF; ++i)
        steps_fast<T, C, D, Q, 0, Q, false, EDGE, SC>(io, yy, yend, Z, R, rt);
    steps_fast<T, C, D, Q, 0, WR, false, EDGE, SC>(io, yy, yend, Z, R, rt);
    while (yy < yend) steps_fast<T, C, D, Q, WR, Q, true, EDGE, SC>(io, yy, yend, Z, R, rt);
}

// The row loop of the general form, unrolled Q times so that every ring slot
// index is a compile-time constant.
template <typename T, int C, int D, int Q, bool EDGE, bool SC>
__device__ __forceinline__ void stream_rows(const Band2D& b, const Strip& w, int halo,
                                            int64_t ystart, int64_t yend, T (&Z)[Q][C],
                                            T (&R)[D][3][C], const bool (&colok)[C],
                                            const Rate2<T>& k) {
#pragma unroll
    for (int m = 0; m < Q - 3; ++m) {
        if (ystart + m < yend) {
            load_row2d<T, C>(b, w, ystart + m, Z[m], colok);
        } else {
#pragma unroll
            for (int j = 0; j < C; ++j) Z[m][j] = T(0);
        }
    }
    for (int64_t yy = ystart; yy < yend; yy += Q) {
        row_step<T, C, D, Q, 0, EDGE, SC>(b, w, halo, yy, yend, Z, R, colok, k);
        if (yy + 1 >= yend) break;
        row_step<T, C, D, Q, 1, EDGE, SC>(b, w, halo, yy + 1, yend, Z, R, colok, k);
        if (yy + 2 >= yend) break;
        row_step<T, C, D, Q, 2, EDGE, SC>(b, w, halo, yy + 2, yend, Z, R, colok, k);
        if (yy + 3 >= yend) break;
        row_step<T, C, D, Q, 3 % Q, EDGE, SC>(b, w, halo, yy + 3, yend, Z, R, colok, k);
        if (yy + 4 >= yend) break;
        row_step<T, C, D, Q, 4 % Q, EDGE, SC>(b, w, halo, yy + 4, yend, Z, R, colok, k);
        if (yy + 5 >= yend) break;
        row_step<T, C, D, Q, 5 % Q, EDGE, SC>(b, w, halo, yy + 5, yend, Z, R, colok, k);
        if constexpr (Q > 6) {
            if (yy + 6 >= yend) break;
            row_step<T, C, D, Q, 6 % Q, EDGE, SC>(b, w, halo, yy + 6, yend, Z, R, colok, k);
            if (yy + 7 >= yend) break;
            row_step<T, C, D, Q, 7 % Q, EDGE, SC>(b, w, halo, yy + 7, yend, Z, R, colok, k);
            if (yy + 8 >= yend) break;
            row_step<T, C, D, Q, 8 % Q, EDGE, SC>(b, w, halo, yy + 8, yend, Z, R, colok, k);
        }
    }
}

// FAST = true: the static-count form (the host checks alignment and size);
// FAST = false: the general form with per-row boundary handling.
// One launch advances up to kMaxBands bands of one grid (same nx, r and
// depth) by one pass: band k owns waves [first[k], first[k+1]), each wave a
// (strip, chunk) of that band.  The set travels as the kernel argument.
struct BandSet {
    Band2D b[kMaxBands];
    int64_t first[kMaxBands + 1];
    int n;
};

// The dispatcher hands consecutive workgroups to the eight XCDs in turn, and
// each XCD has its own L2.  Neighbouring waves (adjacent strips of one chunk)
// share the lines at their strip edges; this bijection of [0, n) gives every
// XCD a contiguous range of workgroups, so that neighbouring strips mostly run
// under one L2 (measured 1.5-2 % faster on the 16384^2 pass).
__device__ __forceinline__ uint32_t xcd_block2d(uint32_t b, uint32_t n) {
    constexpr uint32_t X = 8;
    const uint32_t q = n / X, r = n % X, x = b % X;
    return x * q + (x < r ? x : r) + b / X;
}

template <typename T, int C, int D, bool FAST, bool SC>
__global__ __launch_bounds__(256) void k_stencil2d(BandSet set, int rows, int halo,
                                                   int64_t nstrips) {
    constexpr int VN = V16<T>::N;
    constexpr int S = 64 * C;
    constexpr int Q = ring_rows();
    static_assert(C % VN == 0, "columns per lane must be a multiple of the vector width");
    static_assert(Q % 3 == 0 && Q >= 6, "the level-0 ring must be a multiple of 3 rows");
    const int wpg = blockDim.x >> 6;
    const int64_t wave = (int64_t)xcd_block2d(blockIdx.x, gridDim.x) * wpg +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= set.first[set.n]) return;
    int kb = 0;
    while (kb + 1 < set.n && wave >= set.first[kb + 1]) ++kb;
    const Band2D& b = set.b[kb];
    const int64_t wl = wave - set.first[kb];
    Strip w;
    w.lane = threadIdx.x & 63;
    const int64_t strip = wl % nstrips;
    const int64_t chunk = wl / nstrips;
    w.wout = S - 2 * halo;
    w.x0 = strip * w.wout;
    const int64_t xb = w.x0 - halo;  // first column held by lane 0
    w.xl = xb + (int64_t)w.lane * C;
    w.y0 = chunk * rows;
    w.y1 = (w.y0 + rows < b.ny) ? w.y0 + rows : b.ny;
    w.xin = xb >= 0 && xb + S <= b.nx;
    w.vec = w.xin && b.aligned;
    const Rate2<T> k = make_rate<T, D, SC>(b);

    // Rows above the first streamed row only feed rows that are never stored;
    // they start as zeros so that no stale register value is ever read.
    T R[D][3][C];
    T Z[Q][C];
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int j = 0; j < C; ++j) R[l][m][j] = T(0);
#pragma unroll
    for (int m = Q - 2; m < Q; ++m)
#pragma unroll
        for (int j = 0; j < C; ++j) Z[m][j] = T(0);

    const int64_t ystart = w.y0 - D;
    const int64_t yend = w.y1 + D;
    // Waves whose strip and rows stay clear of the zero-Dirichlet edges take
    // the interior variant.
    const bool edge = !w.xin || (ystart - D < 0 && b.bc_top != BC_GHOST) ||
                      (yend > b.ny && b.bc_bot != BC_GHOST);
    if constexpr (FAST) {
        FastIO<T, C> io;
        io.in = static_cast<const T*>(b.in);
        io.top = static_cast<const T*>(b.halo_top);
        io.bot = static_cast<const T*>(b.halo_bot);
        io.nx = b.nx;
        io.ny = b.ny;
        io.hw = b.hw;
        io.ylo = ystart;
        io.yhi = yend - 1;
        io.top_ghost = b.bc_top == BC_GHOST;
        io.bot_ghost = b.bc_bot == BC_GHOST;
        io.out = __builtin_amdgcn_make_buffer_rsrc(b.out, (short)0,
                                                   (int)(b.ny * b.nx * (int64_t)sizeof(T)),
                                                   BUF_DWORD3);
        // nx is a multiple of the vector width here, so a lane vector is
        // either wholly inside [0, nx) or wholly outside; one outside loads a
        // clamped address and is replaced by zeros
#pragma unroll
        for (int q = 0; q < C / VN; ++q) {
            const int64_t x = w.xl + q * VN;
            const int lc = w.lane * C + q * VN;
            io.colin[q] = x >= 0 && x < b.nx;
            io.xload[q] = x < 0 ? 0 : (x + VN > b.nx ? b.nx - VN : x);
            io.off[q] = (lc >= halo && lc < S - halo && io.colin[q])
                            ? (uint32_t)(x * (int64_t)sizeof(T))
                            : OOB_OFFSET;
        }
        if (edge) {
            stream_rows_fast<T, C, D, Q, true, SC>(io, ystart, yend, Z, R, k);
        } else {
            stream_rows_fast<T, C, D, Q, false, SC>(io, ystart, yend, Z, R, k);
        }
    } else {
        // column mask for edge strips (cells outside [0, nx) are zero ghosts)
        bool colok[C];
#pragma unroll
        for (int j = 0; j < C; ++j) colok[j] = (w.xl + j >= 0) && (w.xl + j < b.nx);
        if (edge)
            stream_rows<T, C, D, Q, true, SC>(b, w, halo, ystart, yend, Z, R, colok, k);
        else
            stream_rows<T, C, D, Q, false, SC>(b, w, halo, ystart, yend, Z, R, colok, k);
    }
}

template <typename T, int C, int D>
hipError_t launch_cd(const Band2D* bands, int n, const Geom2D& g, hipStream_t st) {
    constexpr int VN = V16<T>::N;
    const int64_t wout = 64LL * C - 2LL * g.halo;
    const int64_t nstrips = (bands[0].nx + wout - 1) / wout;
    BandSet set{};
    set.n = n;
    bool fast = true, sc = true;
    int64_t total = 0;
    for (int k = 0; k < n; ++k) {
        Band2D bb = bands[k];
        set_rate_2d(bb, D);
        fast = fast && bb.aligned && bb.nx % VN == 0 && bb.nx >= VN &&
               bb.ny * bb.nx * (int64_t)sizeof(T) < (int64_t(1) << 31);
        sc = sc && bb.period > 0;
        set.b[k] = bb;
        set.first[k] = total;
        total += nstrips * ((bb.ny + g.rows - 1) / g.rows);
    }
    set.first[n] = total;
    const dim3 block(64 * g.wpg);
    const dim3 grid((unsigned)((total + g.wpg - 1) / g.wpg));
    if (fast && sc)
        hipLaunchKernelGGL((k_stencil2d<T, C, D, true, true>), grid, block, 0, st, set, g.rows,
                           g.halo, nstrips);
    else if (fast)
        hipLaunchKernelGGL((k_stencil2d<T, C, D, true, false>), grid, block, 0, st, set, g.rows,
                           g.halo, nstrips);
    else if (sc)
        hipLaunchKernelGGL((k_stencil2d<T, C, D, false, true>), grid, block, 0, st, set, g.rows,
                           g.halo, nstrips);
    else
        hipLaunchKernelGGL((k_stencil2d<T, C, D, false, false>), grid, block, 0, st, set, g.rows,
                           g.halo, nstrips);
    return hipGetLastError();
}

template <typename T, int C, bool DEEP>
hipError_t launch_c(const Band2D* b, int n, const Geom2D& g, hipStream_t st) {
    if constexpr (DEEP) {
        switch (g.steps) {
        case 10: return launch_cd<T, C, 10>(b, n, g, st);
        case 12: return launch_cd<T, C, 12>(b, n, g, st);
        case 16: return launch_cd<T, C, 16>(b, n, g, st);
        default: break;
        }
    }
    switch (g.steps) {
    case 1: return launch_cd<T, C, 1>(b, n, g, st);
    case 2: return launch_cd<T, C, 2>(b, n, g, st);
    case 3: return launch_cd<T, C, 3>(b, n, g, st);
    case 4: return launch_cd<T, C, 4>(b, n, g, st);
    case 5: return launch_cd<T, C, 5>(b, n, g, st);
    case 6: return launch_cd<T, C, 6>(b, n, g, st);
    case 7: return launch_cd<T, C, 7>(b, n, g, st);
    case 8: return launch_cd<T, C, 8>(b, n, g, st);
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

hipError_t launch_stencil2d_bands(int dtype, const Band2D* b, int n, const Geom2D& g,
                                  hipStream_t stream) {
    if (!stencil2d_supported(dtype, g.cpl, g.steps) || n < 1 || n > kMaxBands)
        return hipErrorInvalidValue;
    for (int k = 1; k < n; ++k)
        if (b[k].nx != b[0].nx) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (g.cpl == 4) return launch_c<float, 4, true>(b, n, g, stream);
        return launch_c<float, 8, false>(b, n, g, stream);
    }
    return launch_c<double, 4, false>(b, n, g, stream);
}

hipError_t launch_stencil2d(int dtype, const Band2D& b, const Geom2D& g, hipStream_t stream) {
    return launch_stencil2d_bands(dtype, &b, 1, g, stream);
}

}  // namespace hx
