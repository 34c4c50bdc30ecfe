// DPG Phase III (Section 2.1, Figure 1's gather) staged through LDS.
//
// The partition distribute cuts the rid list into tiles of T rids and leaves
// the records of tile t in INTERNAL as one contiguous segment per run: run b's
// share starts at off[t][b] (the column-scanned count matrix) and ends where
// tile t + 1's share of run b starts (or at the end of run b for the last
// tile).  With local slots, the distribute also wrote for every rid its slot
// in the tile's segments laid end to end in run order.
//
// One workgroup per tile copies the tile's segments into LDS with coalesced
// loads, then writes the tile's output rows in rid-list order, each read from
// its slot in LDS.  Each LDS slot finds its segment by a binary search over
// the segments' starts, narrowed first by a table that holds, for every 64th
// slot, the segment containing it: a wave's 64 consecutive slots then search
// only the few segments of their own 64-slot cell.  Every global access is then coalesced,
// where the cached gather spends one cache-line request per small record.
// Used for records of 4, 8 and 16 bytes, where a tile fits the LDS.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kGatherThreads = 1024;
constexpr int kGatherPer = 8;  // elements per thread per round, all loads in flight together
constexpr int kOutVec = 4;     // 16-byte output vectors per thread per round (VEC)
constexpr int kMaxGatherTile = 65535;  // segment starts are held as uint16

template <typename E>
__device__ __forceinline__ void put16(u32x4 &o, int j, const E &v) {
    if constexpr (sizeof(E) == 4) {
        o[j] = v;
    } else {
        o[2 * j] = v.x;
        o[2 * j + 1] = v.y;
    }
}

// Stages the records of distribute tile t in LDS: the tile's run segments of
// INTERNAL (run d's share starts at off[t][d] and ends where tile t + 1's
// share starts, or at the end of run d) are copied, laid end to end in run
// order, to the start of smem with coalesced loads.  Returns V, the number of
// records staged; the caller synchronises before reading them.  LDS layout
// after the T * WE records: an int32 and a uint16 table over the 2^nbits
// runs, then the 64-slot cell table (gather_lds_bytes).
template <typename E, int WE>
__device__ __forceinline__ int stage_tile(const E *__restrict__ internal, int T, int nbits, int64_t t, int64_t nT,
                                          const int32_t *__restrict__ off, const int32_t *__restrict__ bucket_off,
                                          char *smem) {
    constexpr int W = kGatherThreads / 64;
    const int nb = 1 << nbits;
    E *s_rec = (E *)smem;                                         // T * WE elements
    int32_t *s_base = (int32_t *)(smem + sizeof(E) * (size_t)T * WE);  // INTERNAL start, then start - LDS start
    uint16_t *s_start = (uint16_t *)(s_base + nb);                // segment length, then start in s_rec
    int32_t *s_cell = (int32_t *)(s_start + nb);                  // segment of slot 64c, c <= ceil(V / 64)
    __shared__ int32_t s_wsum[W];
    __shared__ int32_t s_total;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < nb; d += kGatherThreads) {
        const int32_t o = off[t * nb + d];
        const int32_t next = t + 1 < nT ? off[(t + 1) * nb + d] : bucket_off[d + 1];
        s_base[d] = o;
        s_start[d] = (uint16_t)(next - o);
    }
    __syncthreads();
    // exclusive prefix of the segment lengths: wave w scans the w-th slice,
    // then every slice is offset by the totals before it
    {
        const int per_w = (nb + W - 1) / W;
        const int d_lo = min(wave * per_w, nb), d_hi = min(d_lo + per_w, nb);
        int32_t carry = 0;
        for (int d0 = d_lo; d0 < d_hi; d0 += 64) {
            const int d = d0 + lane;
            const int32_t c = d < d_hi ? s_start[d] : 0;
            int32_t inc = c;
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) {
                const int32_t y = __shfl_up(inc, s, 64);
                if (lane >= s) inc += y;
            }
            if (d < d_hi) s_start[d] = (uint16_t)(carry + inc - c);
            carry += __shfl(inc, 63, 64);
        }
        if (lane == 0) s_wsum[wave] = carry;
        __syncthreads();
        int32_t before = 0, all = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            before += v < wave ? s_wsum[v] : 0;
            all += s_wsum[v];
        }
        for (int d = d_lo + lane; d < d_hi; d += 64) {
            const int32_t st = s_start[d] + before;
            s_start[d] = (uint16_t)st;
            s_base[d] -= st;  // INTERNAL index of slot q in segment d: s_base[d] + q
        }
        if (threadIdx.x == 0) s_total = all;
    }
    __syncthreads();
    const int V = s_total;  // records of valid rids in this tile (<= cnt)
    // cell table: for c < ceil(V / 64) the segment holding slot 64c, and
    // after the last cell the segment holding slot V - 1 (largest d with
    // s_start[d] <= slot: that segment is non-empty and holds the slot)
    const int n_cell = (V + 63) >> 6;
    for (int c = threadIdx.x; c <= n_cell && V > 0; c += kGatherThreads) {
        const int q = min(c << 6, V - 1);
        int d = 0;
        for (int step = nb >> 1; step > 0; step >>= 1)
            if (s_start[d + step] <= q) d += step;
        s_cell[c] = d;
    }
    __syncthreads();
    // segments -> LDS
    const int total_in = V * WE;
    for (int x0 = 0; x0 < total_in; x0 += kGatherThreads * kGatherPer) {
        int q[kGatherPer], d[kGatherPer], hi[kGatherPer];
        int span = 0;
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            q[k] = min(x0 + (int)threadIdx.x + k * kGatherThreads, total_in - 1) / WE;
            const int c = q[k] >> 6;
            d[k] = s_cell[c];
            hi[k] = s_cell[c + 1];
            span = max(span, hi[k] - d[k]);
        }
        // largest d in [s_cell[c], s_cell[c + 1]] with s_start[d] <= slot
        // (binary lifting, clamped to the range; the searches interleaved)
        for (int step = span > 0 ? 1 << (31 - __clz(span)) : 0; step > 0; step >>= 1) {
#pragma unroll
            for (int k = 0; k < kGatherPer; ++k) {
                const int e = min(d[k] + step, hi[k]);
                if (s_start[e] <= q[k]) d[k] = e;
            }
        }
        E v[kGatherPer];
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            const int x = min(x0 + (int)threadIdx.x + k * kGatherThreads, total_in - 1);
            const int w = x - q[k] * WE;
            v[k] = internal[(int64_t)(s_base[d[k]] + q[k]) * WE + w];
        }
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            const int x = x0 + (int)threadIdx.x + k * kGatherThreads;
            if (x < total_in) s_rec[x] = v[k];
        }
    }
    return V;
}

// VEC: records of 4 or 8 bytes (WE == 1) written as 16-byte vectors of
// consecutive output rows (dst and the slot array 16-byte aligned).
template <typename E, int WE, bool NT, bool VEC>
__global__ __launch_bounds__(kGatherThreads) void k_gather_lds(const E *__restrict__ internal,
                                                               const int32_t *__restrict__ slot, E *__restrict__ dst,
                                                               int64_t n, int T, int nbits, int64_t nT,
                                                               const int32_t *__restrict__ off,
                                                               const int32_t *__restrict__ bucket_off, int remap) {
    extern __shared__ __align__(16) char smem[];
    E *s_rec = (E *)smem;  // T * WE elements
    const int64_t t = xcd_tile(blockIdx.x, nT, remap);
    const int64_t base = t * T;
    const int cnt = (int)min((int64_t)T, n - base);
    const int V = stage_tile<E, WE>(internal, T, nbits, t, nT, off, bucket_off, smem);
    __syncthreads();
    // LDS -> output rows in rid-list order (invalid rids: slot 0, undefined row)
    const int total_out = cnt * WE;
    E *out = dst + base * WE;
    int done = 0;  // output elements written by the vector loop
    if constexpr (VEC) {
        static_assert(WE == 1 && (sizeof(E) == 4 || sizeof(E) == 8), "16-byte vectors of whole records");
        constexpr int VO = 16 / (int)sizeof(E);  // rows per vector
        typedef int32_t i32v __attribute__((ext_vector_type(VO)));
        const int nvec = cnt / VO;
        const i32v *slot_v = (const i32v *)(slot + base);
        u32x4 *out_v = (u32x4 *)out;
        for (int y0 = 0; y0 < nvec; y0 += kGatherThreads * kOutVec) {
            i32v q[kOutVec];
#pragma unroll
            for (int k = 0; k < kOutVec; ++k) q[k] = slot_v[min(y0 + (int)threadIdx.x + k * kGatherThreads, nvec - 1)];
#pragma unroll
            for (int k = 0; k < kOutVec; ++k) {
                const int y = y0 + (int)threadIdx.x + k * kGatherThreads;
                if (y < nvec) {
                    u32x4 o = {0u, 0u, 0u, 0u};
#pragma unroll
                    for (int j = 0; j < VO; ++j) {
                        const int qq = min(max((int)q[k][j], 0), max(V - 1, 0));
                        put16(o, j, V > 0 ? s_rec[qq] : E{});
                    }
                    if constexpr (NT) __builtin_nontemporal_store(o, out_v + y);
                    else out_v[y] = o;
                }
            }
        }
        done = nvec * VO;
    }
    for (int y0 = done; y0 < total_out; y0 += kGatherThreads * kGatherPer) {
        int32_t q[kGatherPer];
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            const int y = min(y0 + (int)threadIdx.x + k * kGatherThreads, total_out - 1);
            q[k] = slot[base + y / WE];
        }
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            const int y = y0 + (int)threadIdx.x + k * kGatherThreads;
            if (y < total_out) {
                const int e = y / WE, w = y - e * WE;
                const int qq = min(max(q[k], 0), max(V - 1, 0));
                const E val = V > 0 ? s_rec[qq * WE + w] : E{};
                if constexpr (NT) __builtin_nontemporal_store(val, out + y);
                else out[y] = val;
            }
        }
    }
}

template <typename E, int WE, bool VEC>
static dpg_status launch_gather_lds_t(const RetrievePlan &p, const void *internal, const int32_t *slot, void *dst,
                                      const int32_t *off, const int32_t *bucket_off, int remap, hipStream_t stream) {
    const size_t lds = gather_lds_bytes(p.part_tile, (int)sizeof(E) * WE, p.part_nbits);
    const bool nt = (double)p.n_rids * p.rec_bytes > 256.0 * 1024 * 1024;
    const int64_t nT = (p.n_rids + p.part_tile - 1) / p.part_tile;
    if (nT > 0x7fffffffLL || p.part_tile > kMaxGatherTile || p.part_tile % 64 != 0) return DPG_ERR_UNSUPPORTED;
#define DPG_LAUNCH_GLDS(NTV)                                                                                      \
    do {                                                                                                          \
        if (lds > 64 * 1024)                                                                                      \
            DPG_HIP(hipFuncSetAttribute((const void *)k_gather_lds<E, WE, NTV, VEC>,                             \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));                   \
        hipLaunchKernelGGL((k_gather_lds<E, WE, NTV, VEC>), dim3((unsigned)nT), dim3(kGatherThreads), lds, stream, \
                           (const E *)internal, slot, (E *)dst, p.n_rids, p.part_tile, p.part_nbits, nT, off,     \
                           bucket_off, remap);                                                                    \
    } while (0)
    if (nt) DPG_LAUNCH_GLDS(true);
    else DPG_LAUNCH_GLDS(false);
#undef DPG_LAUNCH_GLDS
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

dpg_status launch_gather_lds(dpg_ctx *ctx, const RetrievePlan &p, void *ws, void *dst, hipStream_t stream) {
    if (!p.gather_lds || (p.dist_mode != DIST_PARTITION && p.dist_mode != DIST_SAMPLED) || p.part_tile <= 0)
        return DPG_ERR_UNSUPPORTED;
    if (p.n_rids <= 0) return DPG_OK;
    char *w = (char *)ws;
    const PartPlan pp = dist_partition(p);
    if (pp.tile != p.part_tile) return DPG_ERR_UNSUPPORTED;
    const int32_t *off = (const int32_t *)(w + p.off_part + pp.off_cnt);
    const int32_t *bucket_off = (const int32_t *)(w + p.off_part + pp.off_bucket);
    const int32_t *slot = (const int32_t *)(w + p.off_inv);
    const void *internal = w + p.off_internal;
    const double M = (double)p.n_rids, R = p.rec_bytes;
    ProfScope prof(ctx, K_GATHER_LDS, 4.0 * M + 2.0 * R * M, stream);
    const int remap = xcd_remap_flag(ctx);
    const bool a16 = ((uintptr_t)dst % 16) == 0, a8 = ((uintptr_t)dst % 8) == 0;
    const bool vec = a16 && ((uintptr_t)slot % 16) == 0;  // tiles start at multiples of 64 rows
    switch (p.rec_bytes) {
        case 4:
            if (vec) return launch_gather_lds_t<uint32_t, 1, true>(p, internal, slot, dst, off, bucket_off, remap, stream);
            return launch_gather_lds_t<uint32_t, 1, false>(p, internal, slot, dst, off, bucket_off, remap, stream);
        case 8:
            if (vec) return launch_gather_lds_t<u32x2, 1, true>(p, internal, slot, dst, off, bucket_off, remap, stream);
            if (a8) return launch_gather_lds_t<u32x2, 1, false>(p, internal, slot, dst, off, bucket_off, remap, stream);
            return launch_gather_lds_t<uint32_t, 2, false>(p, internal, slot, dst, off, bucket_off, remap, stream);
        case 16:
            if (a16) return launch_gather_lds_t<u32x4, 1, false>(p, internal, slot, dst, off, bucket_off, remap, stream);
            return launch_gather_lds_t<uint32_t, 4, false>(p, internal, slot, dst, off, bucket_off, remap, stream);
    }
    return DPG_ERR_UNSUPPORTED;
}

}  // namespace dpg
