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

// s[j] = f(j) for j in [0, cnt), spread over the workgroup's 256 lanes.  Each
// lane evaluates f four rows at a time without branches (rows past cnt repeat
// row cnt - 1) and then stores the rows that exist, so the global loads inside
// f are issued back to back instead of one per loop trip.
template <typename F>
__device__ __forceinline__ void stage_rows(int32_t *s, int cnt, F f) {
    for (int j0 = 0; j0 < cnt; j0 += 4 * 256) {
        int32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = f(min(j0 + (int)threadIdx.x + k * 256, cnt - 1));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = j0 + (int)threadIdx.x + k * 256;
            if (j < cnt) s[j] = v[k];
        }
    }
}

// Read `v` from lane `src_lane` of the wave.
__device__ __forceinline__ int32_t lane_read(int32_t v, int src_lane) {
    return __shfl(v, src_lane, 64);
}

}  // namespace dpg
