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
//     below 2^-24 of each product, so the pass keeps f32 accuracy (measured
//     within 4e-7 of the FP64 result, against about 3e-6 for 50 stepped f32
//     updates);
//   * the taps fall off like a Gaussian of variance 2rD, so the outer chunks
//     of the window meet taps far below f32 resolution: each chunk takes only
//     the product levels whose omission would exceed 2^-30 of the taps' total
//     magnitude (prop1d_levels), which skips 18 of the 54 products per
//     iteration at r = 1/4, D = 50.
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

__device__ __forceinline__ f32x4 gload(const float* p) {
    typedef __attribute__((address_space(1))) const f32x4 G;
    return *(G*)p;
}

__device__ __forceinline__ void gstore(f32x4 v, float* p) {
    typedef __attribute__((address_space(1))) f32x4 G;
    *(G*)p = v;
}

// Four cells starting at segment cell c (a multiple of 4): from the segment,
// the left source (halo or wrap) or the right source, clamped into what each
// holds.  Cells beyond the sources' reach only meet zero taps; clamping keeps
// their reads in bounds and finite.
template <bool INTERIOR>
__device__ __forceinline__ f32x4 load4(const PropSeg& s, int64_t c) {
    if (INTERIOR) return gload(s.in + c);
    const bool lo = c < 0, hi = c >= s.n;
    const int64_t cl = c < -s.lo_av ? -s.lo_av : c;
    const int64_t ch = c - s.n > s.hi_av - 4 ? s.hi_av - 4 : c - s.n;
    const float* p = lo ? s.lo_base + cl : (hi ? s.hi_base + ch : s.in + c);
    return gload(p);
}

// Chunks [S0, NC - S0) of the window are materialised: the outer S0 chunks on
// each side take no products for any segment of the launch.
template <int NC, int S0, bool INTERIOR>
__device__ __forceinline__ void prop_wave(const PropSeg& s, int64_t blk0, int ni, int D, int OD,
                                          char* lds) {
    const int l = threadIdx.x, i = l & 31, g = l >> 5;
    const uint32_t lv = s.levels;
    // A operands: lane (m = i, g) holds taps for k = 8g..8g+7 of chunk c
    Split8 A[NC];
#pragma unroll
    for (int c = S0; c < NC - S0; ++c) {
        float a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = 16 * c + 8 * g + e - OD - i;
            const float v = s.coef[j < -D ? 0 : (j > D ? 2 * D : j + D)];
            a[e] = (j >= -D && j <= D) ? v : 0.f;
        }
        A[c] = split8(a);
    }
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
    auto put = [&](int slot, const f32x4 v[4]) {
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
    for (int k0 = 0; k0 < ni; k0 += 6) {
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const int k = k0 + u, ph = u % 3, sb = u & 1;
            if (k >= ni) break;
            // the previous block's outputs go out through slot (k + 2) % 3 (its
            // segment, k - 2, is dead); then segment k+1, fetched two
            // iterations ago, goes into the same slot
            if (k > 0) store((ph + 2) % 3, yprev, k - 1);
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
    store((ni + 2) % 3, yprev, ni - 1);
}

template <int NC, int S0>
__global__ __launch_bounds__(64) void k_prop1d(const PropSeg* __restrict__ segs,
                                               const PropWave* __restrict__ waves, int D, int OD) {
    __shared__ __attribute__((aligned(16))) char lds[3 * kPlane];
    const PropWave w = waves[blockIdx.x];
    const PropSeg s = segs[w.seg];
    if (w.interior)
        prop_wave<NC, S0, true>(s, w.blk0, (int)w.ni, D, OD, lds);
    else
        prop_wave<NC, S0, false>(s, w.blk0, (int)w.ni, D, OD, lds);
}

}  // namespace

// The kernel instantiation for depth D and `skip` dropped chunks per side
// (nullptr when there is none).
static const void* prop1d_kernel(int D, int skip) {
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC) || skip < 0 || NC - 2 * skip < 1) return nullptr;
    switch (NC * 4 + (skip > 2 ? 2 : skip)) {
#define HX_PROP_CASE(N, S) \
    case N * 4 + S:        \
        return reinterpret_cast<const void*>(&k_prop1d<N, S>);
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

int prop1d_waves_per_cu(int D, int skip) {
    const void* k = prop1d_kernel(D, skip);
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

}  // namespace hx
