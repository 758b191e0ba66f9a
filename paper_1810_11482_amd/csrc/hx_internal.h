// Internal declarations shared by the hx runtime (host C++) and the HIP kernel
// translation units.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

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
    int32_t pad_;
};

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

// dtype: 0 = f32, 1 = f64.  Returns hipSuccess or the launch error.
hipError_t launch_stencil1d(int dtype, const Seg1D& seg, const Geom1D& g, hipStream_t stream);

// Batched 1D: `nseg` segments described in device memory; `tiles` entries of
// (segment index, tile index within the segment) in device memory.  The grid is
// persistent: `grid_waves` waves stride over the tile list.
hipError_t launch_stencil1d_batched(int dtype, const Seg1D* segs_dev, const uint32_t* tile_seg,
                                    const uint32_t* tile_idx, int64_t ntiles, const Geom1D& g,
                                    int64_t grid_waves, hipStream_t stream);

}  // namespace hx
