// Propagator form of a fused 1D pass (f32) on the MFMA units.
//
// The explicit heat step u' = u + r (u_{i-1} - 2 u_i + u_{i+1}) (the 3-point
// stencil of Sec. V-A.1 in heat form) is linear and shift-invariant, so D steps
// of it are one convolution of the state with the D-step propagator
// p = [r, 1-2r, r] convolved with itself D times (2D+1 taps, p_j for
// |j| <= D).  On a periodic segment, or a segment whose halos hold the D cells
// each side reaches, u^(D)_i = sum_j p_j u_{i+j} is exactly the result of D
// steps; only the rounding differs from stepping.  The taps come from the host
// in FP64, rounded once to f32.
//
// The convolution is a banded Toeplitz product, evaluated as dense 32x32x16
// bf16 MFMA tiles:
//   * a wave walks a contiguous span of its segment, 1024 cells per
//     iteration: 32 "streams" of 32 consecutive cells (the N dimension);
//   * each stream's output rows 0..31 (the M dimension) need the window of
//     cells [-OD, -OD + 16 NC) around it, taken in NC chunks of 16 (the K
//     dimension); A_c[m][k] = p_{16c + k - OD - m} (zero outside the band),
//     B_c[k][s] = u[32 s - OD + 16 c + k];
//   * every f32 operand is split exactly into three bf16 terms
//     (x = hi + mid + lo, below), and the six products hi*hi, hi*mid, mid*hi,
//     hi*lo, lo*hi, mid*mid are accumulated in f32: the dropped terms are
//     below 2^-20 of each product (|mid| < 2^-7 |x|, |lo| < 2^-14 |x|), so the
//     pass keeps f32 accuracy (measured within 4e-7 of the FP64 result,
//     against about 3e-6 for 50 stepped f32 updates);
//   * the taps fall off like a Gaussian of variance 2rD, so the outer chunks
//     of the window meet taps far below f32 resolution: each chunk takes only
//     the product levels whose omission would exceed 2^-30 of the taps' total
//     magnitude (prop1d_levels), which skips 18 of the 54 products per
//     iteration at r = 1/4, D = 50;
//   * that pruning adds an absolute error, at most E (prop1d_err_bound) times
//     the largest |x| of the block's window, which is not small against an
//     output far below that largest value (a cell next to a spike, or a zero
//     crossing).  So every block checks its outputs: unless each is finite
//     and at least 2^21 E times the window's largest finite |x|, its products
//     are not stored and the wave advances the block by plain f32 stepping
//     instead, after its other blocks (step_block, in LDS).  Every output therefore carries only
//     relative errors of f32 size, or is the stepped result, and a non-finite
//     input reaches exactly the outputs that stepping reaches.
// Data path per iteration: the wave loads the next 1024 cells with coalesced
// 16-byte loads (two iterations ahead), splits them once into three bf16
// planes in an LDS ring of three 1024-cell slots (64-byte rows, 16-byte units
// XOR-swizzled so that 8 consecutive rows hit distinct banks), and reads each
// stream's window chunks from the ring as B operands.  A wave holds 18 KiB of
// LDS, so two waves share each SIMD.  The outputs of an iteration leave at the
// start of the next one, before its loads: transposed through the ring slot
// that is dead at that point, so that every store instruction writes 1 KiB of
// consecutive cells (the matrix-core layout would scatter 32-byte pieces at a
// 128-byte stride, which measured 13 % slower on the memory path alone), and
// issued before the loads, so the wait for those loads never waits for stores
// issued just before.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "hx_internal.h"

namespace hx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kPlane = 96 * 64;  // bytes of one bf16 plane: 3 slots x 32 rows x 64 bytes
constexpr int kSlot = 32 * 64;   // bytes of one 1024-cell slot within a plane

__device__ __forceinline__ uint32_t fbits(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float bitsf(uint32_t b) { return __builtin_bit_cast(float, b); }

// Exact split of two f32 values into packed bf16 pairs (element 0 in the low
// half).  hi keeps the top 8 significand bits (truncation), mid the next 8 of
// the exact remainder x - hi, lo the last 8 of the exact remainder (x - hi) -
// mid, which therefore is a bf16 value: x == hi + mid + lo.
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t& h, uint32_t& m,
                                           uint32_t& l) {
    const uint32_t b0 = fbits(x0), b1 = fbits(x1);
    const float r0 = x0 - bitsf(b0 & 0xffff0000u), r1 = x1 - bitsf(b1 & 0xffff0000u);
    const uint32_t c0 = fbits(r0), c1 = fbits(r1);
    const float s0 = r0 - bitsf(c0 & 0xffff0000u), s1 = r1 - bitsf(c1 & 0xffff0000u);
    h = (b1 & 0xffff0000u) | (b0 >> 16);
    m = (c1 & 0xffff0000u) | (c0 >> 16);
    l = (fbits(s1) & 0xffff0000u) | (fbits(s0) >> 16);
}

struct Split8 {
    u32x4 h, m, l;
};

__device__ __forceinline__ Split8 split8(const float v[8]) {
    Split8 s;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        uint32_t h, m, l;
        split_pair(v[2 * p], v[2 * p + 1], h, m, l);
        s.h[p] = h;
        s.m[p] = m;
        s.l[p] = l;
    }
    return s;
}

__device__ __forceinline__ f32x16 mfma(u32x4 a, u32x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Byte offset of 16-byte unit `unit` (0..3) of ring row `row` within a plane.
__device__ __forceinline__ int swz(int row, int unit) {
    return row * 64 + ((unit ^ ((row >> 1) & 3)) << 4);
}

template <bool NT = false>
__device__ __forceinline__ f32x4 gload(const float* p) {
    typedef __attribute__((address_space(1))) const f32x4 G;
    if (NT) return __builtin_nontemporal_load((G*)p);
    return *(G*)p;
}

template <bool NT = false>
__device__ __forceinline__ void gstore(f32x4 v, float* p) {
    typedef __attribute__((address_space(1))) f32x4 G;
    if (NT)
        __builtin_nontemporal_store(v, (G*)p);
    else
        *(G*)p = v;
}

// Four cells starting at segment cell c (a multiple of 4): from the segment,
// the left source (halo or wrap) or the right source, clamped into what each
// holds.  Cells beyond the sources' reach only meet zero taps; clamping keeps
// their reads in bounds and finite.
template <bool INTERIOR, bool NT = false>
__device__ __forceinline__ f32x4 load4(const PropSeg& s, int64_t c) {
    if (INTERIOR) return gload<NT>(s.in + c);
    const bool lo = c < 0, hi = c >= s.n;
    const int64_t cl = c < -s.lo_av ? -s.lo_av : c;
    const int64_t ch = c - s.n > s.hi_av - 4 ? s.hi_av - 4 : c - s.n;
    const float* p = lo ? s.lo_base + cl : (hi ? s.hi_base + ch : s.in + c);
    return gload<NT>(p);
}

// One cell c of a segment from the same sources as load4, clamped cell by
// cell (the stepping path below).
__device__ __forceinline__ float load1(const PropSeg& s, int64_t c) {
    if (c < 0) return s.lo_base[c < -s.lo_av ? -s.lo_av : c];
    if (c >= s.n) {
        const int64_t h = c - s.n;
        return s.hi_base[h > s.hi_av - 1 ? s.hi_av - 1 : h];
    }
    return s.in[c];
}

// The stepping path of one block: its 1024 cells from c0 advanced D steps of
// u' = u + r ((u_{i-1} - 2 u_i) + u_{i+1}) in f32, over the block's window of
// 64 cells each side (D <= 64), held in 1152 floats of LDS that the caller no
// longer needs (`cell(i)` is window cell i).  Lane l steps window cells
// 18 l .. 18 l + 17 in place: each step reads the two neighbours across its
// ends first, then updates its cells in order carrying the old left value; the
// cells within D of the window's ends go stale and are never stored.  It
// serves the blocks whose products fail the accuracy check, after the wave's
// other blocks, so it is rare and kept simple (loops not unrolled): every cell
// is one 4-byte load and one 4-byte store.  WAVE: the caller's workgroup has
// other waves, which do not take part: the steps are ordered by wave-level
// barriers (the wave's LDS operations execute in order) instead of the
// workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE = false>
__device__ __forceinline__ void block_sync() {
    if (WAVE)
        wave_sync();
    else
        __syncthreads();
}

template <bool WAVE = false, typename Cell>
__device__ __forceinline__ void step_block(const PropSeg& s, int64_t c0, int D, Cell cell) {
    const int l = threadIdx.x & 63;
    const float r = s.r;
    const int b = 18 * l;
    block_sync<WAVE>();
#pragma unroll 1
    for (int t = 0; t < 18; ++t) cell(b + t) = load1(s, c0 - 64 + b + t);
    block_sync<WAVE>();
    for (int k = 0; k < D; ++k) {
        const float lf = l > 0 ? cell(b - 1) : 0.f;
        const float rt = l < 63 ? cell(b + 18) : 0.f;
        block_sync<WAVE>();
        float prev = lf, cur = cell(b);
#pragma unroll 1
        for (int t = 0; t < 18; ++t) {
            const float nx = t < 17 ? cell(b + t + 1) : rt;
            cell(b + t) = cur + r * ((prev - 2.f * cur) + nx);
            prev = cur;
            cur = nx;
        }
        block_sync<WAVE>();
    }
#pragma unroll 1
    for (int t = 0; t < 18; ++t) {
        const int64_t c = c0 - 64 + b + t;
        if (c >= c0 && c < c0 + 1024 && c < s.n) s.out[c] = cell(b + t);
    }
    block_sync<WAVE>();
}

// True on every lane when some output of the block fails the accuracy check:
// non-finite (including NaN), or below thr in magnitude.
__device__ __forceinline__ bool block_fails(const f32x16& y, float thr) {
    bool bad = false;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const float a = fabsf(y[e]);
        bad = bad || !(a <= 3.402823466e38f) || a < thr;
    }
    return __ballot(bad) != 0;
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

// The A operands of window chunks [S0, NC - S0): lane (m = i, g) holds the
// taps of k = 8g .. 8g+7, split into three bf16 levels.
template <int NC, int S0>
__device__ __forceinline__ void prop_taps(const float* coef, int D, int OD, Split8 (&A)[NC]) {
    const int l = threadIdx.x, i = l & 31, g = l >> 5;
#pragma unroll
    for (int c = S0; c < NC - S0; ++c) {
        float a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = 16 * c + 8 * g + e - OD - i;
            const float v = coef[j < -D ? 0 : (j > D ? 2 * D : j + D)];
            a[e] = (j >= -D && j <= D) ? v : 0.f;
        }
        A[c] = split8(a);
    }
}

// Chunks [S0, NC - S0) of the window are materialised: the outer S0 chunks on
// each side take no products for any segment of the launch.
template <int NC, int S0, bool INTERIOR>
__device__ __forceinline__ void prop_wave(const PropSeg& s, int64_t blk0, int ni, int D, int OD,
                                          char* lds, uint16_t* fails) {
    const int l = threadIdx.x, i = l & 31, g = l >> 5;
    const uint32_t lv = s.levels;
    Split8 A[NC];
    prop_taps<NC, S0>(s.coef, D, OD, A);
    // Ring: segment m (relative to the span) lives in slot (m + 1) % 3.  At
    // iteration k (ring phase ph = k % 3) the window of stream i, chunk c,
    // starts X = 16c + 8g - OD cells from the stream, i.e. ring row
    // 32 (ph + 1) + i + floor(X / 32), 16-byte unit (X mod 32) / 8.
    int roff[3][NC];
#pragma unroll
    for (int ph = 0; ph < 3; ++ph)
#pragma unroll
        for (int c = S0; c < NC - S0; ++c) {
            const int X = 16 * c + 8 * g - OD;
            int t = 32 * ph + 32 + i + (X >> 5);
            t = t < 0 ? t + 96 : (t >= 96 ? t - 96 : t);
            roff[ph][c] = swz(t, (X & 31) >> 3);
        }
    // This lane's four 8-byte pieces of a slot: cells 256 j + 4 l .. +3.
    int woff[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) woff[j] = swz(8 * j + (l >> 3), (l & 7) >> 1) + 8 * (l & 1);
    // smx[slot]: the largest finite |x| of the slot's 1024 cells
    float smx[3] = {0.f, 0.f, 0.f};
    auto put = [&](int slot, const f32x4 v[4]) {
        float mx = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float a = fabsf(v[j][e]);
                mx = (a <= 3.402823466e38f && a > mx) ? a : mx;
            }
        smx[slot] = __builtin_bit_cast(
            float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, wave_max(mx))));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t h0, m0, l0, h1, m1, l1;
            split_pair(v[j][0], v[j][1], h0, m0, l0);
            split_pair(v[j][2], v[j][3], h1, m1, l1);
            char* p = lds + slot * kSlot + woff[j];
            *reinterpret_cast<u32x2*>(p) = u32x2{h0, h1};
            *reinterpret_cast<u32x2*>(p + kPlane) = u32x2{m0, m1};
            *reinterpret_cast<u32x2*>(p + 2 * kPlane) = u32x2{l0, l1};
        }
    };
    const int64_t c_span = 1024 * blk0;
    auto fetch = [&](int m, f32x4 v[4]) {  // cells of relative segment m
        const int64_t c0 = c_span + 1024 * (int64_t)m + 4 * l;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = load4<INTERIOR>(s, c0 + 256 * j);
    };
    {
        f32x4 v[4];
        fetch(-1, v);
        put(0, v);
        fetch(0, v);
        put(1, v);
    }
    f32x4 St[2][4];
    fetch(ni < 1 ? ni : 1, St[0]);
    fetch(ni < 2 ? ni : 2, St[1]);
    // Output transposition.  Lane (i, g) ends an iteration with rows
    // 8q + 4g .. +3 (q = 0..3) of stream i; written through LDS and read back,
    // lane l holds cells 256 j + 4 l .. +3 (j = 0..3) of the block, so every
    // store instruction writes 1 KiB of consecutive cells.  The block goes
    // through the ring slot whose segment is dead at the start of an iteration
    // (planes h and m of it: 1024 cells as 32 rows of 128 bytes, 16-byte units
    // XOR-swizzled by row).
    auto tpos = [](int row, int unit) {
        return (row < 16 ? 0 : kPlane) + (row & 15) * 128 + ((unit ^ (row & 7)) << 4);
    };
    int wt[4], rd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wt[q] = tpos(i, 2 * q + g);
#pragma unroll
    for (int j = 0; j < 4; ++j) rd[j] = tpos(8 * j + (l >> 3), l & 7);
    f32x16 yprev = {};
    auto store = [&](int slot, const f32x16& y, int kb) {  // kb: the block y belongs to
        char* t = lds + slot * kSlot;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<f32x4*>(t + wt[q]) =
                f32x4{y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]};
        f32x4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = *reinterpret_cast<const f32x4*>(t + rd[j]);
        const int64_t o = c_span + 1024 * (int64_t)kb + 4 * l;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (o + 256 * j < s.n) gstore(v[j], s.out + o + 256 * j);
    };
    // The block's window lies in the three slots of the ring (segments kb - 1,
    // kb, kb + 1): its outputs pass the check against their largest finite
    // |x|, or the block goes on the wave's list (`fails`, at most 256 entries:
    // a span has at most 256 blocks) and is stepped after the span, when the
    // registers of the pipeline are free.
    int nfail = 0;
    auto emit = [&](int slot, const f32x16& y, int kb) {
        const float M = fmaxf(fmaxf(smx[0], smx[1]), smx[2]);
        if (block_fails(y, s.chk * M)) {
            if (l == 0) fails[nfail] = (uint16_t)kb;
            ++nfail;
        } else {
            store(slot, y, kb);
        }
    };
    for (int k0 = 0; k0 < ni; k0 += 6) {
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const int k = k0 + u, ph = u % 3, sb = u & 1;
            if (k >= ni) break;
            // the previous block's outputs go out through slot (k + 2) % 3 (its
            // segment, k - 2, is dead); then segment k+1, fetched two
            // iterations ago, goes into the same slot
            if (k > 0) emit((ph + 2) % 3, yprev, k - 1);
            __builtin_amdgcn_sched_barrier(0);
            put((ph + 2) % 3, St[sb]);
            __builtin_amdgcn_sched_barrier(0);
            fetch(k + 3 < ni ? k + 3 : ni, St[sb]);
            __builtin_amdgcn_sched_barrier(0);
            f32x16 a0 = {}, a1 = {};
            // window chunks, each read one chunk ahead; a chunk multiplies only
            // the product levels it takes (uniform per wave)
            u32x4 bh = *reinterpret_cast<const u32x4*>(lds + roff[ph][S0]);
            u32x4 bm = *reinterpret_cast<const u32x4*>(lds + roff[ph][S0] + kPlane);
            u32x4 bl = *reinterpret_cast<const u32x4*>(lds + roff[ph][S0] + 2 * kPlane);
#pragma unroll
            for (int c = S0; c < NC - S0; ++c) {
                const int L = (lv >> (2 * c)) & 3;
                u32x4 nh = bh, nm = bm, nl = bl;
                if (c + 1 < NC - S0) {
                    const char* p = lds + roff[ph][c + 1];
                    nh = *reinterpret_cast<const u32x4*>(p);
                    nm = *reinterpret_cast<const u32x4*>(p + kPlane);
                    nl = *reinterpret_cast<const u32x4*>(p + 2 * kPlane);
                }
                if (L >= 1) a1 = mfma(A[c].h, bh, a1);
                if (L >= 2) {
                    a0 = mfma(A[c].h, bm, a0);
                    a1 = mfma(A[c].m, bh, a1);
                }
                if (L >= 3) {
                    a0 = mfma(A[c].l, bh, a0);
                    a1 = mfma(A[c].h, bl, a1);
                    a0 = mfma(A[c].m, bm, a0);
                }
                bh = nh;
                bm = nm;
                bl = nl;
            }
            yprev = a0 + a1;
        }
    }
    // the last block, through the slot that iteration ni would have refilled
    emit((ni + 2) % 3, yprev, ni - 1);
    // the listed blocks, stepped in plane 0 of the ring (4.5 of its 6 KiB)
    __syncthreads();
    for (int f = 0; f < nfail; ++f)
        step_block(s, c_span + 1024 * (int64_t)fails[f], D,
                   [&](int i) -> float& { return reinterpret_cast<float*>(lds)[i]; });
}

template <int NC, int S0>
__global__ __launch_bounds__(64) void k_prop1d(const PropSeg* __restrict__ segs,
                                               const PropWave* __restrict__ waves, int D, int OD) {
    __shared__ __attribute__((aligned(16))) char lds[3 * kPlane];
    __shared__ uint16_t fails[kSpanMax];
    const PropWave w = waves[blockIdx.x];
    const PropSeg s = segs[w.seg];
    if (w.interior)
        prop_wave<NC, S0, true>(s, w.blk0, (int)w.ni, D, OD, lds, fails);
    else
        prop_wave<NC, S0, false>(s, w.blk0, (int)w.ni, D, OD, lds, fails);
}

// Interleaved walk (every segment of the launch has the same n and the same
// taps).  The blocks of all segments are numbered back to back, block b of
// the launch being block b mod bps of segment b / bps (bps = blocks per
// segment), and wave w of a persistent grid of nw waves takes blocks w,
// w + nw, w + 2 nw, ...: at any moment the grid reads and writes one narrow
// band of the arrays instead of nw bands far apart, which measured 9 % more
// HBM bandwidth for the same bytes than contiguous spans.  A block is read
// with the 64 cells on each side that its windows reach (12.5 % more read
// requests; the counters put about 14 % more bytes fetched than the block's
// own, because the neighbouring blocks run on other XCDs, and placing them on
// one XCD measured slower).  Loads are ordinary cached loads and stores are
// nontemporal: the launch measured 4 % faster than with nontemporal loads,
// and ordinary stores were no faster.
//
// Because a block's whole window (1152 cells) is loaded at once, it can share
// one scale: the window's largest finite |x| is brought into [2^14, 2^15) by
// an exact power of two 2^ex, and every cell is split into two fp16 terms,
// x 2^ex = hi + lo (round to nearest each, so the pair holds x to 2^-22 of
// itself, or, below fp16's normal range, to an absolute 2^-25 at that scale,
// i.e. 2^-39 of the largest).  The taps are split the same way at their own
// scale 2^texp.  These absolute floors and the pruning of product levels are
// what the check after the products bounds (as in the span walk: a block
// whose outputs are not all finite and at least 2^21 E times the window's
// largest is stepped instead, in the window's LDS).  A product
// then takes three 32x32x16 fp16 MFMAs (hi*hi, hi*lo, lo*hi; the dropped
// lo*lo is below 2^-22 of it) instead of the six of the bf16 split, which
// halves the matrix-core work (17 instead of 36 products per block at
// r = 1/4, D = 50, with the fp16 levels' pruning) and the power it draws on
// high-entropy data, where the six-product form ran into the card's power
// limit.  The result is scaled back by 2^-(ex + texp).  A non-finite cell is
// left out of the scale; the outputs it reaches through the products fail the
// check.
constexpr int kWPlane = 36 * 64;  // bytes of one fp16 plane of the 1152-cell window

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma16(u32x4 a, u32x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t hbits(_Float16 x) {
    return (uint32_t)__builtin_bit_cast(uint16_t, x);
}

// Two f32 values scaled by 2^e (exact) and split into packed fp16 pairs
// (element 0 in the low half): x 2^e = hi + lo, both rounded to nearest.
__device__ __forceinline__ void split16_pair(float x0, float x1, int e, uint32_t& h,
                                             uint32_t& l) {
    const float s0 = ldexpf(x0, e), s1 = ldexpf(x1, e);
    const _Float16 h0 = (_Float16)s0, h1 = (_Float16)s1;
    const _Float16 l0 = (_Float16)(s0 - (float)h0), l1 = (_Float16)(s1 - (float)h1);
    h = hbits(h0) | (hbits(h1) << 16);
    l = hbits(l0) | (hbits(l1) << 16);
}

struct Split8h {
    u32x4 h, l;
};

// Up to 7 materialised window chunks the kernel fits three waves per SIMD
// (168 registers): one accumulator, and each block's outputs leave at the end
// of its own iteration, so no result is held across iterations.  Measured at
// the headline shape, three waves per SIMD ran the same work 3.6 % faster on
// average and without the dip in clocks that two waves per SIMD met a few
// milliseconds into sustained launches.
template <int NC, int S0>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NC - 2 * S0 <= 7 ? 3 : 1, 8)))
void k_prop1d_il(const PropSeg* __restrict__ segs, uint32_t nblocks, uint32_t bps, int D, int OD) {
    __shared__ __attribute__((aligned(16))) char lds[2 * kWPlane];
    __shared__ uint16_t fails[kIlMax];  // this wave's blocks that failed the check
    const int l = threadIdx.x, i = l & 31, g = l >> 5;
    const uint32_t w = blockIdx.x, nw = gridDim.x;
    if (w >= nblocks) return;
    const int nk = (int)((nblocks - 1 - w) / nw) + 1;  // at most kIlMax (the host's grid)
    int nfail = 0;
    const uint32_t lv = segs[0].levels16;
    const int texp = segs[0].texp;
    const float chk = segs[0].chk;
    // A operands: lane (m = i, g) holds the taps of k = 8g .. 8g+7, scaled by
    // 2^texp and split into two fp16 terms
    Split8h A[NC];
    {
        const float* coef = segs[0].coef;
#pragma unroll
        for (int c = S0; c < NC - S0; ++c) {
            float a[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int j = 16 * c + 8 * g + e - OD - i;
                const float v = coef[j < -D ? 0 : (j > D ? 2 * D : j + D)];
                a[e] = (j >= -D && j <= D) ? v : 0.f;
            }
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                uint32_t h, lo;
                split16_pair(a[2 * p], a[2 * p + 1], texp, h, lo);
                A[c].h[p] = h;
                A[c].l[p] = lo;
            }
        }
    }
    // Window row r holds cells 32 (r - 2) .. +31 of the block.  The window of
    // stream i, chunk c, starts X = 16c + 8g - OD cells from the stream: row
    // 2 + i + floor(X / 32), 16-byte unit (X mod 32) / 8.
    int roff[NC];
#pragma unroll
    for (int c = S0; c < NC - S0; ++c) {
        const int X = 16 * c + 8 * g - OD;
        roff[c] = swz(2 + i + (X >> 5), (X & 31) >> 3);
    }
    // This lane's 8-byte pieces of the window: block cells 256 j + 4 l .. +3
    // (j = 0..3) and context cells 4 q .. +3 (q = l mod 16) of the left 64
    // (lanes with l mod 32 < 16) or the right 64 (the others).
    int woff[5];
#pragma unroll
    for (int j = 0; j < 4; ++j) woff[j] = swz(2 + 8 * j + (l >> 3), (l & 7) >> 1) + 8 * (l & 1);
    const int q = l & 15;
    const bool left = (l & 31) < 16;
    woff[4] = swz((left ? 0 : 34) + (q >> 3), (q & 7) >> 1) + 8 * (q & 1);
    // split the window into the two planes at the window's own scale; sets
    // that scale's exponent and the check's threshold (zero for a window with
    // no nonzero finite cell, whose outputs are exact)
    auto put = [&](const f32x4 v[5], int& ex_out, float& thr) {
        float mx = 0.f;
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float a = fabsf(v[j][e]);
                mx = (a <= 3.402823466e38f && a > mx) ? a : mx;  // finite only
            }
        mx = wave_max(mx);
        const int ex = __builtin_amdgcn_readfirstlane(
            mx > 0.f ? 15 - __builtin_amdgcn_frexp_expf(mx) : 0);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            uint32_t h0, l0, h1, l1;
            split16_pair(v[j][0], v[j][1], ex, h0, l0);
            split16_pair(v[j][2], v[j][3], ex, h1, l1);
            char* p = lds + woff[j];
            *reinterpret_cast<u32x2*>(p) = u32x2{h0, h1};
            *reinterpret_cast<u32x2*>(p + kWPlane) = u32x2{l0, l1};
        }
        ex_out = ex;
        thr = mx > 0.f ? chk : 0.f;
    };
    auto fetch = [&](int k, f32x4 v[5]) {
        const uint32_t b = w + (uint32_t)k * nw;
        const uint32_t sg = b / bps;
        const PropSeg& s = segs[sg];
        const int64_t c0 = 1024 * (int64_t)(b - sg * bps);
        const int64_t cx = (left ? c0 - 64 : c0 + 1024) + 4 * q;
        if (c0 >= 1024 && c0 + 1024 + 64 <= s.n) {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = gload(s.in + c0 + 256 * j + 4 * l);
            v[4] = gload(s.in + cx);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = load4<false>(s, c0 + 256 * j + 4 * l);
            v[4] = load4<false>(s, cx);
        }
    };
    // Output transposition, as in the span walk, through the two planes of
    // the window (32 rows of 128 bytes, 16-byte units XOR-swizzled by row).
    // The stores follow the fetch of block k + 2, so the wait for that
    // fetch's predecessors never waits for them.
    auto tpos = [](int row, int unit) {
        return (row < 16 ? 0 : kWPlane) + (row & 15) * 128 + ((unit ^ (row & 7)) << 4);
    };
    int wt[4], rd[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) wt[e] = tpos(i, 2 * e + g);
#pragma unroll
    for (int j = 0; j < 4; ++j) rd[j] = tpos(8 * j + (l >> 3), l & 7);
    auto store = [&](int k, const f32x16& y, int ex) {
        const int sc = -(ex + texp);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            *reinterpret_cast<f32x4*>(lds + wt[e]) =
                f32x4{ldexpf(y[4 * e], sc), ldexpf(y[4 * e + 1], sc), ldexpf(y[4 * e + 2], sc),
                      ldexpf(y[4 * e + 3], sc)};
        f32x4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = *reinterpret_cast<const f32x4*>(lds + rd[j]);
        const uint32_t b = w + (uint32_t)k * nw;
        const uint32_t sg = b / bps;
        const PropSeg& s = segs[sg];
        const int64_t o = 1024 * (int64_t)(b - sg * bps) + 4 * l;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (o + 256 * j < s.n) gstore<true>(v[j], s.out + o + 256 * j);
    };
    f32x4 St[2][5];
    fetch(0, St[0]);
    fetch(nk > 1 ? 1 : 0, St[1]);
    for (int k0 = 0; k0 < nk; k0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = k0 + u;
            if (k >= nk) break;
            // block k (fetched two iterations ago) takes the window, then
            // block k + 2 is fetched into the registers it leaves
            int ex;
            float thr;
            put(St[u], ex, thr);
            __builtin_amdgcn_sched_barrier(0);
            fetch(k + 2 < nk ? k + 2 : nk - 1, St[u]);
            __builtin_amdgcn_sched_barrier(0);
            f32x16 acc = {};
            u32x4 bh = *reinterpret_cast<const u32x4*>(lds + roff[S0]);
            u32x4 bl = *reinterpret_cast<const u32x4*>(lds + roff[S0] + kWPlane);
#pragma unroll
            for (int c = S0; c < NC - S0; ++c) {
                const int L = (lv >> (2 * c)) & 3;
                u32x4 nh = bh, nl = bl;
                if (c + 1 < NC - S0) {
                    const char* p = lds + roff[c + 1];
                    nh = *reinterpret_cast<const u32x4*>(p);
                    nl = *reinterpret_cast<const u32x4*>(p + kWPlane);
                }
                if (L >= 1) acc = mfma16(A[c].h, bh, acc);
                if (L >= 2) {
                    acc = mfma16(A[c].h, bl, acc);
                    acc = mfma16(A[c].l, bh, acc);
                }
                bh = nh;
                bl = nl;
            }
            // the outputs leave through the window, whose reads are all issued;
            // a block that fails the check is stepped instead
            __builtin_amdgcn_sched_barrier(0);
            if (block_fails(acc, thr)) {
                if (l == 0) fails[nfail] = (uint16_t)k;
                ++nfail;
            } else {
                store(k, acc, ex);
            }
        }
    }
    // the listed blocks, stepped now that the pipeline's registers are free
    __syncthreads();
    for (int f = 0; f < nfail; ++f) {
        const uint32_t b = w + (uint32_t)fails[f] * nw;
        const uint32_t sg = b / bps;
        step_block(segs[sg], 1024 * (int64_t)(b - sg * bps), D,
                   [&](int c) -> float& { return reinterpret_cast<float*>(lds)[c]; });
    }
}


// Block walk (every segment of the launch has the same n and the same taps,
// as in the interleaved walk): one workgroup of one wave per 1024-cell block,
// blockIdx.x the block within its segment and blockIdx.y the segment, so the
// grid covers every block once and the hardware dispatcher, not a persistent
// loop, keeps the memory system busy.  A persistent grid moved the same bytes
// at 5.3-5.5 TB/s in a probe without arithmetic, one wave per block at
// 5.9-6.0 TB/s.
//
// A wave that lives for one block cannot build its tap operands from the taps
// (56 values per lane to select, scale and split).  The plan builds them once
// (prop1d_bw_table): the two fp16 terms of the scaled taps, in eight copies
// shifted by one element each, so that the 8 consecutive taps a lane's A
// operand holds for a chunk are one aligned 16-byte unit of one copy.  Each
// wave stages the table (5 KiB, L2-resident) in LDS while its window loads are
// in flight, and reads its A operands from there with the B operands.  The
// lanes of an 8-lane group read 8 distinct copies, and the odd stride of a copy
// (U units of 16 bytes) puts their units in distinct banks.
//
// Everything else is the interleaved walk's arithmetic, in the same order, so
// the two give the same bits: the window's shared power-of-two scale, the
// two-term fp16 split of every cell (here with the packed conversion), the
// products chunk by chunk, the accuracy check, and the stepped fallback for a
// block that fails it (right away, in the window's LDS).
constexpr int bw_units(int NC, int S0) { return 2 * (NC - S0) + 3; }

// x 2^e for two f32 values split into packed fp16 pairs: x 2^e = hi + lo,
// each rounded to nearest (the packed form of split16_pair).
__device__ __forceinline__ void split16_pk(float x0, float x1, int e, uint32_t& h, uint32_t& l) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 s = {ldexpf(x0, e), ldexpf(x1, e)};
    const h2 hi = __builtin_convertvector(s, h2);
    const f2 rem = s - __builtin_convertvector(hi, f2);
    h = __builtin_bit_cast(uint32_t, hi);
    l = __builtin_bit_cast(uint32_t, __builtin_convertvector(rem, h2));
}

template <int NC, int S0, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_prop1d_bw(const PropSeg* __restrict__ segs, const u32x4* __restrict__ tab, int D, int OD,
                 int64_t bps) {
    constexpr int U = bw_units(NC, S0);
    constexpr int kUnits = 16 * U;                     // 16-byte units of the table
    constexpr int kLoads = (kUnits + 64 * W - 1) / (64 * W);  // per work-item
    // W waves per workgroup (blocks W x + w of the segment): they share one
    // staged table, and the context cells of a block that are its
    // neighbours' own cells are read by the same CU
    __shared__ __attribute__((aligned(16))) char lds_all[W * 2 * kWPlane + 16 * kUnits];
    char* const tl = lds_all + W * 2 * kWPlane;
    const int wv = threadIdx.x >> 6;
    char* const lds = lds_all + wv * 2 * kWPlane;
    const int l = threadIdx.x & 63, i = l & 31, g = l >> 5;
    const PropSeg& s = segs[blockIdx.y];
    const int64_t blk = (int64_t)blockIdx.x * W + wv;
    const bool live = W == 1 || blk < bps;  // a wave past the segment's end only stages the table
    const int64_t c0 = 1024 * blk;
    const uint32_t lv = s.levels16;
    // the table first, so that waiting for it leaves the window's loads in flight
    u32x4 T[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int u = (int)threadIdx.x + 64 * W * k;
        if (k + 1 < kLoads || u < kUnits) T[k] = tab[u];
    }
    // the window: this lane's 16-byte pieces of the block (cells 256 j + 4 l)
    // and of the left or right 64 context cells, as in the interleaved walk.
    // The block's own cells are read nontemporally (about 1 % faster than
    // cached loads); the context cells, which the neighbouring blocks read as
    // their own, with cached loads
    const int q = l & 15;
    const bool left = (l & 31) < 16;
    f32x4 v[5] = {};
    if (live) {
        const int64_t cx = (left ? c0 - 64 : c0 + 1024) + 4 * q;
        if (c0 >= 1024 && c0 + 1024 + 64 <= s.n) {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = gload<true>(s.in + c0 + 256 * j + 4 * l);
            v[4] = gload(s.in + cx);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = load4<false>(s, c0 + 256 * j + 4 * l);
            v[4] = load4<false>(s, cx);
        }
    }
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int u = (int)threadIdx.x + 64 * W * k;
        if (k + 1 < kLoads || u < kUnits) *reinterpret_cast<u32x4*>(tl + 16 * u) = T[k];
    }
    // the window's scale: its largest |x| if all are finite (a NaN or an
    // infinity makes the maximum non-finite), else the largest finite one
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) mx = __builtin_elementwise_maximum(mx, fabsf(v[j][e]));
    if (__ballot(!(mx <= 3.402823466e38f))) {
        mx = 0.f;
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float a = fabsf(v[j][e]);
                mx = (a <= 3.402823466e38f && a > mx) ? a : mx;
            }
    }
    mx = wave_max(mx);
    const int ex = __builtin_amdgcn_readfirstlane(
        mx > 0.f ? 15 - __builtin_amdgcn_frexp_expf(mx) : 0);
    const float thr = mx > 0.f ? s.chk : 0.f;
    // the two fp16 planes of the window (the interleaved walk's layout)
    {
        int woff[5];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            woff[j] = swz(2 + 8 * j + (l >> 3), (l & 7) >> 1) + 8 * (l & 1);
        woff[4] = swz((left ? 0 : 34) + (q >> 3), (q & 7) >> 1) + 8 * (q & 1);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            uint32_t h0, l0, h1, l1;
            split16_pk(v[j][0], v[j][1], ex, h0, l0);
            split16_pk(v[j][2], v[j][3], ex, h1, l1);
            char* p = lds + woff[j];
            *reinterpret_cast<u32x2*>(p) = u32x2{h0, h1};
            *reinterpret_cast<u32x2*>(p + kWPlane) = u32x2{l0, l1};
        }
    }
    __syncthreads();
    if (!live) return;
    // A operand of chunk c for lane (m = i, g): taps 16c + 8g - OD - i + 0..7,
    // unit (d - d mod 8) / 8 of copy d mod 8, d = 16c + 8g + 31 - i (the table
    // starts at tap -OD - 31); one chunk further is two units further on
    const int d0 = 16 * S0 + 8 * g + 31 - i;
    const char* ta = tl + 16 * ((d0 & 7) * U + (d0 >> 3));
    f32x16 acc = {};
    {
        int roff[NC];
#pragma unroll
        for (int c = S0; c < NC - S0; ++c) {
            const int X = 16 * c + 8 * g - OD;
            roff[c] = swz(2 + i + (X >> 5), (X & 31) >> 3);
        }
        u32x4 bh = *reinterpret_cast<const u32x4*>(lds + roff[S0]);
        u32x4 bl = *reinterpret_cast<const u32x4*>(lds + roff[S0] + kWPlane);
        u32x4 ah = *reinterpret_cast<const u32x4*>(ta);
        u32x4 al = *reinterpret_cast<const u32x4*>(ta + 16 * 8 * U);
#pragma unroll
        for (int c = S0; c < NC - S0; ++c) {
            const int L = (lv >> (2 * c)) & 3;
            u32x4 nbh = bh, nbl = bl, nah = ah, nal = al;
            if (c + 1 < NC - S0) {
                const char* p = lds + roff[c + 1];
                const char* pa = ta + 32 * (c + 1 - S0);
                nbh = *reinterpret_cast<const u32x4*>(p);
                nbl = *reinterpret_cast<const u32x4*>(p + kWPlane);
                nah = *reinterpret_cast<const u32x4*>(pa);
                nal = *reinterpret_cast<const u32x4*>(pa + 16 * 8 * U);
            }
            if (L >= 1) acc = mfma16(ah, bh, acc);
            if (L >= 2) {
                acc = mfma16(ah, bl, acc);
                acc = mfma16(al, bh, acc);
            }
            bh = nbh;
            bl = nbl;
            ah = nah;
            al = nal;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // the accuracy check: every output finite and at least thr in magnitude
    float mn = fabsf(acc[0]), mo = mn;
#pragma unroll
    for (int e = 1; e < 16; ++e) {
        mn = __builtin_elementwise_minimum(mn, fabsf(acc[e]));
        mo = __builtin_elementwise_maximum(mo, fabsf(acc[e]));
    }
    if (__ballot(!(mn >= thr) || !(mo <= 3.402823466e38f))) {
        step_block<(W > 1)>(s, c0, D,
                            [&](int c) -> float& { return reinterpret_cast<float*>(lds)[c]; });
        return;
    }
    // the outputs, scaled back and transposed through the window's planes
    // (whose reads are all issued) so that each store writes 1 KiB of cells
    auto tpos = [](int row, int unit) {
        return (row < 16 ? 0 : kWPlane) + (row & 15) * 128 + ((unit ^ (row & 7)) << 4);
    };
    const int sc = -(ex + s.texp);
#pragma unroll
    for (int e = 0; e < 4; ++e)
        *reinterpret_cast<f32x4*>(lds + tpos(i, 2 * e + g)) =
            f32x4{ldexpf(acc[4 * e], sc), ldexpf(acc[4 * e + 1], sc),
                  ldexpf(acc[4 * e + 2], sc), ldexpf(acc[4 * e + 3], sc)};
    f32x4 o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = *reinterpret_cast<const f32x4*>(lds + tpos(8 * j + (l >> 3), l & 7));
    const int64_t oc = c0 + 4 * l;
    if (c0 + 1024 <= s.n) {
#pragma unroll
        for (int j = 0; j < 4; ++j) gstore<true>(o[j], s.out + oc + 256 * j);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (oc + 256 * j < s.n) gstore<true>(o[j], s.out + oc + 256 * j);
    }
}

}  // namespace

// The kernel instantiation for depth D and `skip` dropped chunks per side
// (nullptr when there is none), for the walk `walk` (PROP_SPAN, PROP_IL or
// PROP_BW, the last with `wpg` = 1 or 4 waves per workgroup).
static const void* prop1d_kernel(int D, int skip, int walk = PROP_SPAN, int wpg = 1) {
    if (walk == PROP_BW && wpg != 1 && wpg != 4) return nullptr;
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC) || skip < 0 || NC - 2 * skip < 1) return nullptr;
    switch (NC * 4 + (skip > 2 ? 2 : skip)) {
#define HX_PROP_CASE(N, S)                                                      \
    case N * 4 + S:                                                             \
        return walk == PROP_IL ? reinterpret_cast<const void*>(&k_prop1d_il<N, S>)           \
               : walk != PROP_BW ? reinterpret_cast<const void*>(&k_prop1d<N, S>)       \
               : wpg == 4 ? reinterpret_cast<const void*>(&k_prop1d_bw<N, S, 4>)        \
                          : reinterpret_cast<const void*>(&k_prop1d_bw<N, S, 1>);
#define HX_PROP_CASES(N) HX_PROP_CASE(N, 0) HX_PROP_CASE(N, 1) HX_PROP_CASE(N, 2)
        HX_PROP_CASE(3, 0)
        HX_PROP_CASE(3, 1)
        HX_PROP_CASE(4, 0)
        HX_PROP_CASE(4, 1)
        HX_PROP_CASES(5)
        HX_PROP_CASES(6)
        HX_PROP_CASES(7)
        HX_PROP_CASES(8)
        HX_PROP_CASES(9)
        HX_PROP_CASES(10)
#undef HX_PROP_CASES
#undef HX_PROP_CASE
    default:
        return nullptr;
    }
}

int prop1d_waves_per_cu(int D, int skip, int walk) {
    const void* k = prop1d_kernel(D, skip, walk);
    int blocks = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, 64, 0) != hipSuccess) {
        hipGetLastError();
        return 4;
    }
    return blocks > 0 ? blocks : 1;
}

hipError_t launch_prop1d(const PropSeg* segs_dev, const PropWave* waves_dev, int64_t nwaves, int D,
                         int skip, hipStream_t stream) {
    int OD = 0, NC = 0;
    const void* k = prop1d_kernel(D, skip);
    if (!k || !prop1d_geometry(D, &OD, &NC) || nwaves <= 0 || nwaves >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    void* args[] = {&segs_dev, &waves_dev, &D, &OD};
    return hipLaunchKernel(k, dim3((unsigned)nwaves), dim3(64), args, 0, stream);
}

hipError_t launch_prop1d_il(const PropSeg* segs_dev, int64_t nblocks, int64_t bps, int64_t nwaves,
                            int D, int skip, hipStream_t stream) {
    int OD = 0, NC = 0;
    const void* k = prop1d_kernel(D, skip, PROP_IL);
    if (!k || !prop1d_geometry(D, &OD, &NC) || nblocks <= 0 || nblocks >= (int64_t(1) << 32) ||
        bps <= 0 || nblocks % bps != 0 || nwaves <= 0 || nwaves > nblocks ||
        (nblocks + nwaves - 1) / nwaves > kIlMax)
        return hipErrorInvalidValue;
    uint32_t nb = (uint32_t)nblocks, bp = (uint32_t)bps;
    void* args[] = {&segs_dev, &nb, &bp, &D, &OD};
    return hipLaunchKernel(k, dim3((unsigned)nwaves), dim3(64), args, 0, stream);
}

size_t prop1d_bw_table_bytes(int D, int skip) {
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC) || skip < 0 || NC - 2 * skip < 1) return 0;
    return (size_t)256 * bw_units(NC, std::min(skip, 2));
}

// Copy c (0..7) of level v (0 = hi, 1 = lo), unit u, element e holds that term
// of tap j = -OD - 31 + c + 8 u + e (zero outside [-D, D]), the tap scaled by
// 2^texp and split as split16_pair splits it: round to nearest fp16 for hi,
// then the rounded exact remainder for lo.
std::vector<uint16_t> prop1d_bw_table(const float* taps, int D, int skip, int texp) {
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC) || skip < 0 || NC - 2 * skip < 1) return {};
    const int U = bw_units(NC, std::min(skip, 2));
    std::vector<uint16_t> t((size_t)2 * 8 * U * 8);
    for (int c = 0; c < 8; ++c)
        for (int u = 0; u < U; ++u)
            for (int e = 0; e < 8; ++e) {
                const int j = -OD - 31 + c + 8 * u + e;
                const float p = (j >= -D && j <= D) ? taps[j + D] : 0.f;
                const float sc = std::ldexp(p, texp);
                const _Float16 hi = (_Float16)sc;
                const _Float16 lo = (_Float16)(sc - (float)hi);
                t[((size_t)(0 * 8 + c) * U + u) * 8 + e] = __builtin_bit_cast(uint16_t, hi);
                t[((size_t)(1 * 8 + c) * U + u) * 8 + e] = __builtin_bit_cast(uint16_t, lo);
            }
    return t;
}

hipError_t launch_prop1d_bw(const PropSeg* segs_dev, const void* tab_dev, int64_t nsegs,
                            int64_t bps, int wpg, int D, int skip, hipStream_t stream) {
    int OD = 0, NC = 0;
    const void* k = prop1d_kernel(D, skip, PROP_BW, wpg);
    if (!k || !prop1d_geometry(D, &OD, &NC) || !tab_dev || nsegs <= 0 || nsegs > 65535 ||
        bps <= 0 || bps >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    void* args[] = {&segs_dev, &tab_dev, &D, &OD, &bps};
    const int64_t groups = (bps + wpg - 1) / wpg;
    return hipLaunchKernel(k, dim3((unsigned)groups, (unsigned)nsegs), dim3(64 * wpg), args, 0,
                           stream);
}

}  // namespace hx
