// device_common.hpp -- launch geometry and lane helpers shared by the kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace afs {
namespace dev {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcds = 8;

// Workgroups are handed to the 8 XCDs round-robin.  Renumber them so that each
// XCD receives one contiguous range of logical blocks (and with it a contiguous
// range of restart columns, whose x rows then stay in that XCD's L2).
__device__ __forceinline__ uint32_t xcd_block()
{
    const uint32_t nb = gridDim.x;
    const uint32_t i = blockIdx.x;
    const uint32_t xcd = i % kXcds, idx = i / kXcds;
    const uint32_t base = nb / kXcds, extra = nb % kXcds;
    return xcd * base + (xcd < extra ? xcd : extra) + idx;
}

__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

inline dim3 grid_for_waves(int64_t items)
{
    return dim3((unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock));
}

// One dispatch covers fewer than 2^32 work-items (its grid size is a 32-bit
// count).  Launchers of one-wave-per-item kernels therefore split the items into
// launches of at most kMaxLaunchWaves waves; each kernel adds its launch's first
// item (item0) to the item it derives from the block and wave index.
constexpr int64_t kMaxLaunchWaves = int64_t(1) << 24;

template <class Launch>
hipError_t for_launch_chunks(int64_t items, Launch launch)
{
    for (int64_t first = 0; first < items; first += kMaxLaunchWaves) {
        const int64_t count = items - first < kMaxLaunchWaves ? items - first : kMaxLaunchWaves;
        launch(first, count);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Partial assignments (one row of fixed [n_partial][n] per slice of the restart
// columns): restart b of B belongs to slice b * n_partial / B, so the slices are
// as even as B allows.  fixed == nullptr fixes nothing.
__device__ __forceinline__ bool is_fixed(const uint8_t *fixed, int n_partial, int n, int B, int v, int b)
{
    if (!fixed) return false;
    const int p = n_partial > 1 ? (int)(((int64_t)b * n_partial) / B) : 0;
    return fixed[(int64_t)p * n + v] != 0;
}

}  // namespace dev
}  // namespace afs
