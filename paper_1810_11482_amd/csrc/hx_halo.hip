// Halo pack/unpack, and the device-to-device copy kernel.
//
// Halo pack/unpack: one launch copies every descriptor's runs (a run is a
// contiguous byte range; descriptors with a pitch gather or scatter columns),
// so all partitions' halos move between state buffers and ghost slots in a
// single kernel.  Each wave takes one (descriptor, run) pair and copies it with
// 16-byte accesses when the addresses allow, 4-byte accesses otherwise.
#include <hip/hip_runtime.h>

#include "hx_internal.h"

namespace hx {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_halo(const HaloDev* __restrict__ d,
                                              const int64_t* __restrict__ first_run, int nd,
                                              int64_t total_runs) {
    const int wpg = blockDim.x >> 6;
    const int64_t run = (int64_t)blockIdx.x * wpg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (run >= total_runs) return;
    const int lane = threadIdx.x & 63;
    // descriptor owning this run: binary search over the prefix of run counts
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_run[mid] <= run) lo = mid; else hi = mid - 1;
    }
    const HaloDev h = d[lo];
    const int64_t r = run - first_run[lo];
    const char* src = static_cast<const char*>(h.src) + r * h.src_pitch;
    char* dst = static_cast<char*>(h.dst) + r * h.dst_pitch;
    const int64_t nb = h.row_bytes;
    if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | (uintptr_t)nb) & 15u) == 0) {
        const u32x4* s = reinterpret_cast<const u32x4*>(src);
        u32x4* t = reinterpret_cast<u32x4*>(dst);
        for (int64_t i = lane; i < nb / 16; i += 64) t[i] = s[i];
    } else {
        const unsigned* s = reinterpret_cast<const unsigned*>(src);
        unsigned* t = reinterpret_cast<unsigned*>(dst);
        for (int64_t i = lane; i < nb / 4; i += 64) t[i] = s[i];
    }
}

// Device-to-device copy of a 16-byte-aligned range: every thread moves one
// 16-byte vector with a nontemporal load and store, 256 threads (4 KiB) per
// workgroup, one pass (no loop): the pattern that measured the highest copy
// bandwidth on MI355X; the grid's tail workgroup checks the bound.
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src,
                                                u32x4* __restrict__ dst, int64_t nvec) {
    typedef __attribute__((address_space(1))) const u32x4 G;
    typedef __attribute__((address_space(1))) u32x4 GW;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nvec) __builtin_nontemporal_store(__builtin_nontemporal_load((G*)(src + i)),
                                              (GW*)(dst + i));
}

}  // namespace

hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | bytes) & 15u) ||
        bytes / 16 / 256 >= (size_t(1) << 31))
        return hipErrorInvalidValue;
    const int64_t nvec = (int64_t)(bytes / 16);
    const dim3 block(256), grid((unsigned)((nvec + 255) / 256));
    hipLaunchKernelGGL(k_copy16, grid, block, 0, st, static_cast<const u32x4*>(src),
                       static_cast<u32x4*>(dst), nvec);
    return hipGetLastError();
}

hipError_t launch_halo(const HaloDev* descs, const int64_t* first_run, int nd, int64_t total_runs,
                       hipStream_t st) {
    if (total_runs == 0) return hipSuccess;
    const int wpg = 4;
    const dim3 block(64 * wpg), grid((unsigned)((total_runs + wpg - 1) / wpg));
    hipLaunchKernelGGL(k_halo, grid, block, 0, st, descs, first_run, nd, total_runs);
    return hipGetLastError();
}

}  // namespace hx
