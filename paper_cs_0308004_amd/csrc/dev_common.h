// Device-side helpers shared by the libdpg kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dpg {

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X
// (workgroup p runs on XCD p % 8).  Remap the dispatch index so that each XCD
// works through one contiguous range of tiles: neighbouring tiles then share
// that XCD's L2, which is where partial cache lines of a stream get merged.
__device__ __forceinline__ int64_t xcd_tile(int64_t p, int64_t n, int remap) {
    if (!remap) return p;
    const int64_t x = p & 7, slot = p >> 3, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + slot;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << __lane_id()) - 1;
}

// Lanes of the wave holding the same value of `key` (nbits low bits), among
// the lanes in `active`.  One ballot per key bit.
__device__ __forceinline__ uint64_t match_lanes(uint32_t key, int nbits, uint64_t active) {
    uint64_t m = active;
    for (int bit = 0; bit < nbits; ++bit) {
        const bool set = (key >> bit) & 1u;
        const uint64_t b = __ballot(set);
        m &= set ? b : ~b;
    }
    return m;
}

// Read `v` from lane `src_lane` of the wave.
__device__ __forceinline__ int32_t lane_read(int32_t v, int src_lane) {
    return __shfl(v, src_lane, 64);
}

}  // namespace dpg
