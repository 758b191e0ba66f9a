// Internal declarations shared by the hx runtime (host C++) and the HIP kernel
// translation units.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

namespace hx {

// One 1D segment: a contiguous run of n cells advanced `steps` steps from `in`
// into `out`.  Cells outside [0, n) come from the boundary rule of each side.
struct Seg1D {
    const void* in;
    void* out;
    const void* halo_lo;   // GHOST left: hw cells, halo_lo[hw-1] is cell -1
    const void* halo_hi;   // GHOST right: hw cells, halo_hi[0] is cell n
    int64_t n;
    double r;
    int32_t bc_lo, bc_hi;  // hx_bc values
    int32_t hw;            // halo width of the GHOST sides
    int32_t shift;         // tile grid offset: tiles start at t*wout - shift, chosen so
                           // that interior tiles of `in` start 16-byte aligned
    // Rescaled update, filled by set_rate_1d for the pass's step count:
    // period > 0 selects it, 0 the direct form.
    int32_t period;        // steps between rescales
    double beta;           // r / (1 - 2r)
    double alpha_p;        // (1 - 2r)^period
    double alpha_rem;      // (1 - 2r)^(steps mod period)
};

// Rescaled form of the step.  With a = 1 - 2r the step is
// u' = a u + r (u_l + u_r); carrying w = u / a^k after k steps turns it into
// w' = w + (r/a)(w_l + w_r), one add and one fma per cell instead of three
// operations.  The state is multiplied by a^period every `period` steps and by
// a^(steps mod period) at the end, so it never grows beyond 2^16 times u.
// Used for 1/4 <= a <= 1 (0 <= r <= 3/8); other rates take the direct form.
inline void set_rate_1d(Seg1D& s, int steps) {
    const double a = 1.0 - 2.0 * s.r;
    s.period = 0;
    s.beta = s.alpha_p = s.alpha_rem = 1.0;
    if (!(a >= 0.25 && a <= 1.0)) return;
    int p = 0;
    double ap = 1.0;
    while (p < 32 && ap * a >= 1.0 / 65536.0) {
        ap *= a;
        ++p;
    }
    double ar = 1.0;
    for (int i = 0; i < (steps > 0 ? steps % p : 0); ++i) ar *= a;
    s.period = p;
    s.beta = s.r / a;
    s.alpha_p = ap;
    s.alpha_rem = ar;
}

// Tile-grid shift that makes in + (t*wout - shift - halo) 16-byte aligned for
// every t (wout and halo are multiples of the vector width).
inline int32_t tile_shift(const void* in, int esize) {
    const int vn = 16 / esize;
    return (int32_t)((reinterpret_cast<uintptr_t>(in) / esize) % vn);
}

// Launch geometry of the 1D tile kernel: each wave owns 64*cpl cells, of which
// the outer `halo` on each side are recomputed context and 64*cpl - 2*halo are
// written.  halo >= steps and a multiple of the 16-byte vector width.
struct Geom1D {
    int cpl;        // cells per lane: 8, 16, 32, 64
    int steps;      // time steps fused in this pass
    int halo;       // context cells per side
    int wpg;        // waves per workgroup
};

inline int64_t tile_out_1d(const Geom1D& g) { return 64LL * g.cpl - 2LL * g.halo; }
inline int64_t tiles_1d(const Seg1D& s, const Geom1D& g) {
    const int64_t w = tile_out_1d(g);
    return (s.n + s.shift + w - 1) / w;
}

// dtype: 0 = f32, 1 = f64.  Returns hipSuccess or the launch error.
hipError_t launch_stencil1d(int dtype, const Seg1D& seg, const Geom1D& g, hipStream_t stream);

// Batched 1D: segments described in device memory; `ntiles` entries of
// (segment index, tile index within the segment) in device memory.  With
// grid_waves >= ntiles (or <= 0) every wave takes one tile, otherwise
// `grid_waves` persistent waves stride over the table, each prefetching its
// next tile while it advances the current one.  per_seg > 0 means every segment has exactly per_seg
// tiles in segment order, so the table need not be read.  scaled: every
// segment has period > 0 (set_rate_1d for g.steps), so the rescaled update runs.
hipError_t launch_stencil1d_batched(int dtype, const Seg1D* segs_dev, const uint32_t* tile_seg,
                                    const uint32_t* tile_idx, int64_t ntiles, const Geom1D& g,
                                    int64_t grid_waves, int64_t per_seg, bool scaled,
                                    hipStream_t stream);

// Propagator form of a fused 1D pass (f32, MFMA): D steps as one convolution
// with the D-step propagator.  A segment reads cell c < 0 at lo_base + c
// (clamped to c >= -lo_av) and cell c >= n at hi_base + (c - n) (clamped to
// c - n <= hi_av - 4): for a halo-fed segment these are the halos, for a
// periodic one the segment itself.  n, lo_av and hi_av are multiples of 4 and
// every base is 16-byte aligned.
struct PropSeg {
    const float* in;
    float* out;
    const float* lo_base;
    const float* hi_base;
    const float* coef;     // 2D+1 taps, coef[D + j] = p_j
    int64_t n;
    int64_t lo_av, hi_av;
    // Bits 2c..2c+1: how many magnitude levels of the split products window
    // chunk c takes: 0 none, 1 hi*hi, 2 also hi*mid and mid*hi, 3 all six.
    // Chosen from the taps the chunk meets (prop1d_levels).
    uint32_t levels;
    // The same for the two-term fp16 split of the interleaved walk: 0 none,
    // 1 hi*hi, 2 also hi*lo and lo*hi (prop1d_levels16).
    uint32_t levels16;
    // fp16 split: the taps are scaled by 2^texp so that the largest lies in
    // [2^14, 2^15).
    int32_t texp;
    float r;               // the segment's rate (the stepping path of a block)
    // Accuracy check of a block's products (prop1d_err_bound): the absolute
    // error the split and the pruning can add is at most E times the largest
    // finite |x| of the block's window; a block whose every output y has
    // |y| >= 2^21 E M keeps those terms within 2^-21 |y|, any other block
    // (or one with a non-finite output) is advanced by stepping instead.  Span
    // walk: chk = 2^21 E (times the window's M in the kernel); interleaved
    // walk: chk = 2^21 E 2^(15 + texp), the same bound in the scaled units of
    // its products (where M < 2^15).
    float chk;
    int32_t pad;
};

// One wave's work: iterations blk0 .. blk0+ni-1 (1024 cells each) of segment
// `seg`; interior = every cell it reads lies in [0, n).
struct PropWave {
    uint32_t seg, blk0, ni, interior;
};

// Window of the propagator kernel for depth D: offset OD (the window starts OD
// cells before a stream, a multiple of 8 >= D) and NC 16-cell chunks.
// Supported for 1 <= D <= 64.
inline bool prop1d_geometry(int D, int* OD, int* NC) {
    if (D < 1 || D > 64) return false;
    *OD = 8 * ((D + 7) / 8);
    *NC = (32 + D + *OD + 15) / 16;
    return true;
}

// Product levels per window chunk for taps p[0..2D] (p[D + j] = p_j): a chunk
// keeps the levels whose omitted products stay below 2^-30 of the taps' total
// magnitude.  The products of level k are about 2^-8k of the chunk's largest
// tap t and there are at most three per level and 16 taps per row, so a chunk
// is skipped when 16 t <= 2^-30 S, keeps hi*hi alone when 48 t 2^-8 <= 2^-30 S,
// levels 0-1 when 48 t 2^-16 <= 2^-30 S, and all six products otherwise
// (S = sum |p_j|).
inline uint32_t prop1d_levels(const double* p, int D) {
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC)) return 0;
    double S = 0.0;
    for (int j = 0; j <= 2 * D; ++j) S += p[j] < 0 ? -p[j] : p[j];
    const double eps = S / 1073741824.0;  // 2^-30 S
    uint32_t mask = 0;
    for (int c = 0; c < NC; ++c) {
        double t = 0.0;
        for (int j = 16 * c - OD - 31; j <= 16 * c - OD + 15; ++j) {
            if (j < -D || j > D) continue;
            const double a = p[j + D] < 0 ? -p[j + D] : p[j + D];
            if (a > t) t = a;
        }
        uint32_t L = 3;
        if (16.0 * t <= eps) L = 0;
        else if (48.0 * t / 256.0 <= eps) L = 1;
        else if (48.0 * t / 65536.0 <= eps) L = 2;
        mask |= L << (2 * c);
    }
    return mask;
}

// Product levels per window chunk for the interleaved walk's two-term fp16
// split (each operand x = hi + lo to 22 bits, the product keeping hi*hi, hi*lo
// and lo*hi, so it carries a relative error of about 3 * 2^-22 of itself).
// The pruning bound is set below that: a chunk is skipped when its omission,
// at most 16 t per row, is within 2^-26 S, and keeps hi*hi alone when the two
// cross terms, at most 2 * 16 t 2^-11, are (t: the chunk's largest |tap|,
// S = sum |p_j|).
inline uint32_t prop1d_levels16(const double* p, int D) {
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC)) return 0;
    double S = 0.0;
    for (int j = 0; j <= 2 * D; ++j) S += p[j] < 0 ? -p[j] : p[j];
    const double eps = S / 67108864.0;  // 2^-26 S
    uint32_t mask = 0;
    for (int c = 0; c < NC; ++c) {
        double t = 0.0;
        for (int j = 16 * c - OD - 31; j <= 16 * c - OD + 15; ++j) {
            if (j < -D || j > D) continue;
            const double a = p[j + D] < 0 ? -p[j + D] : p[j + D];
            if (a > t) t = a;
        }
        uint32_t L = 2;
        if (16.0 * t <= eps) L = 0;
        else if (32.0 * t / 2048.0 <= eps) L = 1;
        mask |= L << (2 * c);
    }
    return mask;
}

// Bound E on the absolute error that the operand split and the level pruning
// add to an output, in units of the largest finite |x| of the block's window
// (the relative parts, at most a few 2^-22 of each product, are not counted
// here).  Per output row m of a stream, a chunk at level 0 omits its products
// entirely; at the fp16 split (fp16 = true), level 1 omits the two cross terms
// (at most 2^-10 of |p_j x_j|); at the bf16 split, level 1 omits all but
// hi*hi (below 2^-5 of it) and level 2 the terms of order 2^-14 and smaller
// (below 2^-12).  The fp16 split adds two absolute floors: a data term below
// fp16's subnormal spacing (2^-25 at a scale that puts the window's largest in
// [2^14, 2^15), i.e. 2^-39 of it, per unit of tap mass) and a tap term below
// 2^-25 at the taps' scale 2^texp, per tap.
inline double prop1d_err_bound(const double* p, int D, uint32_t levels, bool fp16, int texp) {
    int OD = 0, NC = 0;
    if (!prop1d_geometry(D, &OD, &NC)) return 0.0;
    double S = 0.0;
    for (int j = 0; j <= 2 * D; ++j) S += p[j] < 0 ? -p[j] : p[j];
    double E = 0.0;
    for (int m = 0; m < 32; ++m) {
        double e = 0.0;
        for (int c = 0; c < NC; ++c) {
            const uint32_t L = (levels >> (2 * c)) & 3;
            const double f = L == 0 ? 1.0
                             : fp16 ? (L == 1 ? 1.0 / 1024.0 : 0.0)
                                    : (L == 1 ? 1.0 / 32.0 : (L == 2 ? 1.0 / 4096.0 : 0.0));
            if (f == 0.0) continue;
            for (int k = 0; k < 16; ++k) {
                const int j = 16 * c + k - OD - m;
                if (j < -D || j > D) continue;
                e += f * (p[j + D] < 0 ? -p[j + D] : p[j + D]);
            }
        }
        E = e > E ? e : E;
    }
    if (fp16) E += S * __builtin_ldexp(1.0, -39) + (2 * D + 1) * __builtin_ldexp(1.0, -25 - texp);
    return E;
}

// Exponent e with max|p_j| 2^e in [2^14, 2^15) (0 for all-zero taps).
inline int32_t prop1d_tap_exp(const double* p, int D) {
    double t = 0.0;
    for (int j = 0; j <= 2 * D; ++j) t = (p[j] < 0 ? -p[j] : p[j]) > t ? (p[j] < 0 ? -p[j] : p[j]) : t;
    if (!(t > 0.0)) return 0;
    int e = 0;
    while (t * __builtin_ldexp(1.0, e) >= 32768.0) --e;
    while (t * __builtin_ldexp(1.0, e) < 16384.0) ++e;
    return e;
}

// skip: window chunks on each side that no segment of the launch multiplies
// (level 0 in every segment's mask); at most 2 are dropped from the kernel.
// A block whose products fail the accuracy check (PropSeg::chk) is advanced
// by f32 stepping in the same launch, by its wave after the wave's other
// blocks: a wave lists at most kSpanMax blocks (span walk: the most blocks a
// wave walks) or kIlMax (interleaved walk: the grid must have at least
// ceil(nblocks / kIlMax) waves).
constexpr int kSpanMax = 256;
constexpr int kIlMax = 128;
hipError_t launch_prop1d(const PropSeg* segs_dev, const PropWave* waves_dev, int64_t nwaves, int D,
                         int skip, hipStream_t stream);
// The walks of the propagator pass: contiguous spans of blocks per wave, the
// interleaved persistent grid, and one wave per block.
enum { PROP_SPAN = 0, PROP_IL = 1, PROP_BW = 2 };
// Waves of that walk's kernel resident per CU (registers and LDS permitting).
int prop1d_waves_per_cu(int D, int skip, int walk = PROP_SPAN);
// Interleaved walk of the same pass: `nblocks` 1024-cell blocks, bps per
// segment (every segment has the same n and the same taps, those of segs[0]);
// a persistent grid of nwaves <= nblocks waves, wave w taking blocks w,
// w + nwaves, ...  nblocks < 2^32 and a multiple of bps.
hipError_t launch_prop1d_il(const PropSeg* segs_dev, int64_t nblocks, int64_t bps, int64_t nwaves,
                            int D, int skip, hipStream_t stream);
// Block walk of the same pass: one wave per block, bps blocks in each of
// `nsegs` segments (same n and taps, as the interleaved walk; nsegs <= 65535,
// bps < 2^31), `wpg` (1 or 4) waves per workgroup on consecutive blocks, the
// tap operands read from `tab_dev`, the table prop1d_bw_table builds for
// (taps, D, skip, texp) of segs[0] (prop1d_bw_table_bytes of device memory,
// 16-byte aligned).
size_t prop1d_bw_table_bytes(int D, int skip);
std::vector<uint16_t> prop1d_bw_table(const float* taps, int D, int skip, int texp);
hipError_t launch_prop1d_bw(const PropSeg* segs_dev, const void* tab_dev, int64_t nsegs,
                            int64_t bps, int wpg, int D, int skip, hipStream_t stream);

// One 2D band: ny rows of nx cells, row-major, advanced `steps` steps from in
// into out.  Rows outside [0, ny) come from the top/bottom rule; columns
// outside [0, nx) are zero-Dirichlet.
struct Band2D {
    const void* in;
    void* out;
    const void* halo_top;  // GHOST top: hw rows, its last row is row -1
    const void* halo_bot;  // GHOST bottom: hw rows, its first row is row ny
    int64_t nx, ny;
    double r;
    int32_t bc_top, bc_bot;
    int32_t hw;
    int32_t aligned;       // every row of in/out/halos starts 16-byte aligned
    // Rescaled update (set_rate_2d for the pass's depth): period > 0 selects it.
    int32_t period;        // levels between rescales
    double beta;           // r / (1 - 4r)
    double alpha_p;        // (1 - 4r)^period
    double alpha_rem;      // (1 - 4r)^(steps mod period)
};

// The 2D analogue of set_rate_1d: u' = a u + r (u_n + u_s + u_w + u_e) with
// a = 1 - 4r becomes w' = w + (r/a)(w_n + w_s + w_w + w_e) on w = u / a^k
// (three adds and one fma per cell-level instead of five operations), with
// rescales every `period` levels and at the end, so w never exceeds 2^16 u.
// Used for 1/8 <= a <= 1 (0 <= r <= 7/32); other rates take the direct form.
inline void set_rate_2d(Band2D& b, int steps) {
    const double a = 1.0 - 4.0 * b.r;
    b.period = 0;
    b.beta = b.alpha_p = b.alpha_rem = 1.0;
    if (!(a >= 0.125 && a <= 1.0)) return;
    int p = 0;
    double ap = 1.0;
    while (p < 32 && ap * a >= 1.0 / 65536.0) {
        ap *= a;
        ++p;
    }
    double ar = 1.0;
    for (int i = 0; i < (steps > 0 ? steps % p : 0); ++i) ar *= a;
    b.period = p;
    b.beta = b.r / a;
    b.alpha_p = ap;
    b.alpha_rem = ar;
}

struct Geom2D {
    int cpl;    // columns per lane: 4 (or 8 for f32 with steps <= 8)
    int steps;  // fused time levels of this pass
    int halo;   // context columns per side (>= steps, multiple of the vector width)
    int rows;   // output rows per wave
    int wpg;    // waves per workgroup
};

bool stencil2d_supported(int dtype, int cpl, int steps);
hipError_t launch_stencil2d(int dtype, const Band2D& b, const Geom2D& g, hipStream_t stream);
// Up to kMaxBands bands of one grid (same nx, r, depth g.steps) in one launch.
constexpr int kMaxBands = 16;
hipError_t launch_stencil2d_bands(int dtype, const Band2D* bands, int n, const Geom2D& g,
                                  hipStream_t stream);

// One variable-coefficient step (forward: out = A u; adjoint: out = A^T lam
// and gacc += the step's conductivity gradient) on an ny x nx grid.
struct VCArgs {
    const void* u;
    const void* kappa;
    const void* lam;
    void* out;
    void* gacc;
    int64_t nx, ny;
    double dt;
    int rows;
};

hipError_t launch_vc_step(int dtype, bool adjoint, const VCArgs& v, hipStream_t stream);
// `steps` (1..4) forward steps fused in one pass, u -> out (the same bits as
// that many single steps); for grids whose rows are 16-byte aligned with nx a
// multiple of 4 and under 2 GiB (vc_fused_supported), else hipErrorInvalidValue.
constexpr int kVcFusedMax = 4;
bool vc_fused_supported(int dtype, const VCArgs& v);
// mid (16-byte aligned, stride a multiple of 16 of at least one state):
// also store the states after steps 1 .. steps-1 at mid + (k-1) * mid_stride.
hipError_t launch_vc_forward(int dtype, int steps, const VCArgs& v, hipStream_t stream,
                             void* mid = nullptr, int64_t mid_stride = 0);
// `steps` (1..4) adjoint steps t = tb .. tb-steps+1 fused in one pass: v.lam
// (lam_{tb+1}) -> v.out (lam_{tb+1-steps}), adding each step's
// conductivity-gradient term to v.gacc in the single steps' order (the same
// bits as that many launch_vc_step adjoint steps); ustates[k] is u_t of step
// t = tb - k.  zero_in: the accumulator starts at zero (not read);
// fold_total: add the accumulator to this FP64 total (the segment's fold)
// instead of storing it.  The grids vc_fused_supported takes, lam, gacc, the
// total and the states 16-byte aligned, else hipErrorInvalidValue.
hipError_t launch_vc_adjoint(int dtype, int steps, const VCArgs& v, const void* const* ustates,
                             hipStream_t stream, bool zero_in = false,
                             double* fold_total = nullptr);
hipError_t launch_fold(int dtype, void* acc, double* total, int64_t n, hipStream_t stream);
hipError_t launch_fill(int dtype, void* p, int64_t n, double v, hipStream_t stream);
hipError_t launch_cast64(int dtype, const double* src, void* dst, int64_t n, hipStream_t stream);
hipError_t launch_scale(int dtype, const void* x, const double* s, void* out, int64_t n,
                        hipStream_t stream);
int reduce_blocks(int64_t n);
// The allocation-free loss's scratch: kLossScratch doubles per device in a
// static device array.  scratch_init (with `device` current; once per device,
// from hx_ctx_create) looks up its device address; scratch_of returns it, or
// nullptr before scratch_init succeeded on that device.
constexpr int kLossScratch = 4096;
constexpr int kMaxDevices = 64;
hipError_t scratch_init(int device);
double* scratch_of(int device);
// mode 0: out = 0.5 sum (a-b)^2 (resid = a - b if non-null); mode 1: out = sum a*b.
hipError_t launch_reduce(int dtype, int mode, const void* a, const void* b, void* resid, int64_t n,
                         double* partial, double* out, hipStream_t stream);

// Halo copy descriptor on the device: `rows` runs of row_bytes (a multiple of
// 4), run k at src + k*src_pitch -> dst + k*dst_pitch.
struct HaloDev {
    const void* src;
    void* dst;
    int64_t rows, row_bytes, src_pitch, dst_pitch;
};

// Device-to-device copy of `bytes` (a multiple of 16, both ends 16-byte
// aligned, under 2^43 bytes): one 16-byte nontemporal vector per thread.
// hipErrorInvalidValue for anything else (the caller then uses hipMemcpyAsync).
hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t stream);

// first_run[i] = runs of descriptors 0..i-1 (device arrays of nd entries).
hipError_t launch_halo(const HaloDev* descs, const int64_t* first_run, int nd, int64_t total_runs,
                       hipStream_t stream);

}  // namespace hx
