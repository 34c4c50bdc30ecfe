// Record copy by index: dst[k] = src[idx[k]].
//
// One kernel serves three roles:
//   * direct retrieval (idx = the rid list; Section 1's "standard approach"),
//   * the DPG probe when source runs are read through the caches
//     (idx = the RID runs, dst = INTERNAL; Section 2.1, Phase II),
//   * the DPG gather (idx = slot of each rid in INTERNAL, src = INTERNAL;
//     Section 2.1, Phase III).
//
// Layout: a workgroup owns a tile of consecutive outputs.  The tile's indices
// are staged in LDS, then the tile's (record, element) pairs are flattened over
// the 256 lanes, so each wave's loads cover whole records and its stores are
// one contiguous span of dst.  Every thread issues all of its loads before its
// first store, keeping PER independent loads in flight.
#include "dev_common.h"
#include "dpg_internal.h"

namespace dpg {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr double kStreamingStoreBytes = 256.0 * 1024 * 1024;

__host__ __device__ constexpr int gcd_int(int a, int b) {
    while (b) {
        const int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Records per tile: at most `raw`, and a multiple of 256 / gcd(R, 256) so that
// every tile's output starts on a 256-byte boundary.  Streaming stores of
// partial 128-byte lines are several times slower than whole lines on MI355X.
__host__ __device__ constexpr int aligned_tile(int raw, int rec_bytes) {
    const int step = 256 / gcd_int(rec_bytes, 256);
    const int t = raw / step * step;
    return t > 0 ? t : raw;
}

// TR > 0 (records of a fixed WE only): tiles of TR records, PER elements per
// lane as needed (the last lanes of a tile repeat its last element); TR must
// be a multiple of the 256-byte alignment step.
template <typename E, int WE, int TR = 0>
struct GatherShape {
    static constexpr int kEDw = sizeof(E) / 4;
    static constexpr int kInRange = (WE > 0 && WE * kEDw >= 16 && WE * kEDw <= 64);
    static constexpr int PER = TR > 0 ? (TR * WE + 255) / 256 : kInRange ? WE : 32 / kEDw;  // elements per thread
    static constexpr int TILE = TR > 0 ? TR : WE > 0 ? aligned_tile((256 * PER) / WE, WE * (int)sizeof(E)) : 0;
    static_assert(TR == 0 || (WE > 0 && aligned_tile(TR, WE * (int)sizeof(E)) == TR), "tile breaks the alignment");
};

template <typename E, int WE, bool NT, int TR = 0>
__device__ __forceinline__ void gather_tile(const E *__restrict__ src, const int32_t *__restrict__ idx,
                                            E *__restrict__ dst, int64_t n, int64_t limit, int we_rt,
                                            uint32_t magic, int tile_rt, int remap) {
    extern __shared__ int32_t s_idx[];
    using S = GatherShape<E, WE, TR>;
    constexpr int PER = S::PER;
    const int we = WE > 0 ? WE : we_rt;
    const int tile = WE > 0 ? S::TILE : tile_rt;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x, remap);
    const int64_t base = t * tile;
    const int cnt = (int)min((int64_t)tile, n - base);
    // An index outside [0, limit) reads record 0 instead (undefined result, no
    // out-of-bounds access).
#pragma unroll 8
    for (int j = threadIdx.x; j < cnt; j += 256) {
        const int32_t r = idx[base + j];
        s_idx[j] = (r >= 0 && (int64_t)r < limit) ? r : 0;
    }
    __syncthreads();
    const int total = cnt * we;
    // Every lane loads unconditionally (lanes past the tile repeat its last
    // element), so the loads carry no branches and all PER stay in flight.
    int64_t off[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = min(threadIdx.x + k * 256, total - 1);
        int j;
        if constexpr (WE > 0) j = e / WE;
        else j = (int)__umulhi((uint32_t)e, magic);
        off[k] = (int64_t)s_idx[j] * we + (e - j * we);
    }
    E v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) v[k] = src[off[k]];
    E *out = dst + base * we;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        if (e < total) {
            if constexpr (NT) __builtin_nontemporal_store(v[k], out + e);
            else out[e] = v[k];
        }
    }
}

// Three kernel symbols for the three roles, so profiles tell them apart.
#define DPG_GATHER_KERNEL(NAME)                                                                              \
    template <typename E, int WE, bool NT, int TR>                                                           \
    __global__ __launch_bounds__(256) void NAME(const E *__restrict__ src, const int32_t *__restrict__ idx, \
                                                E *__restrict__ dst, int64_t n, int64_t limit, int we_rt,    \
                                                uint32_t magic, int tile_rt, int remap) {                    \
        gather_tile<E, WE, NT, TR>(src, idx, dst, n, limit, we_rt, magic, tile_rt, remap);                  \
    }
DPG_GATHER_KERNEL(k_direct_gather)
DPG_GATHER_KERNEL(k_probe_cached)
DPG_GATHER_KERNEL(k_gather_phase)
#undef DPG_GATHER_KERNEL

// Two-phase DPG (the probe scatters): dst[pos[k]] = src[run[k]] for k in run
// order.  The same flattened tile as the gather, with the tile's positions
// staged beside its indices; only the first *n_valid entries are live (the
// distribute drops invalid rids), and a position outside [0, n_dst) is skipped.
template <typename E, int WE, bool NT>
__global__ __launch_bounds__(256) void k_probe_scatter(const E *__restrict__ src, const int32_t *__restrict__ run,
                                                       const int32_t *__restrict__ pos,
                                                       const int32_t *__restrict__ n_valid, E *__restrict__ dst,
                                                       int64_t n_dst, int64_t limit, int we_rt, uint32_t magic,
                                                       int tile_rt, int remap) {
    extern __shared__ int32_t s_tab[];
    using S = GatherShape<E, WE>;
    constexpr int PER = S::PER;
    const int we = WE > 0 ? WE : we_rt;
    const int tile = WE > 0 ? S::TILE : tile_rt;
    int32_t *s_run = s_tab, *s_pos = s_tab + tile;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x, remap);
    const int64_t base = t * tile;
    const int64_t live = min((int64_t)*n_valid, n_dst);
    const int cnt = (int)min((int64_t)tile, live - base);
    if (cnt <= 0) return;
#pragma unroll 8
    for (int j = threadIdx.x; j < cnt; j += 256) {
        const int32_t r = run[base + j];
        const int32_t q = pos[base + j];
        s_run[j] = (r >= 0 && (int64_t)r < limit) ? r : 0;
        s_pos[j] = (q >= 0 && (int64_t)q < n_dst) ? q : -1;
    }
    __syncthreads();
    const int total = cnt * we;
    int64_t off[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = min(threadIdx.x + k * 256, total - 1);
        int j;
        if constexpr (WE > 0) j = e / WE;
        else j = (int)__umulhi((uint32_t)e, magic);
        off[k] = (int64_t)s_run[j] * we + (e - j * we);
    }
    E v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) v[k] = src[off[k]];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        if (e < total) {
            int j;
            if constexpr (WE > 0) j = e / WE;
            else j = (int)__umulhi((uint32_t)e, magic);
            const int32_t q = s_pos[j];
            if (q >= 0) {
                E *o = dst + (int64_t)q * we + (e - j * we);
                if constexpr (NT) __builtin_nontemporal_store(v[k], o);
                else *o = v[k];
            }
        }
    }
}

template <typename E, int WE>
static dpg_status launch_scatter_t(const void *src, const int32_t *run, const int32_t *pos, const int32_t *n_valid,
                                   void *dst, int64_t n, int64_t limit, int we, int remap, bool nt,
                                   hipStream_t stream) {
    using S = GatherShape<E, WE>;
    int tile;
    uint32_t magic = 0;
    if constexpr (WE > 0) {
        tile = S::TILE;
    } else {
        tile = aligned_tile((256 * S::PER) / we, we * (int)sizeof(E));
        if (tile < 1 || we < 2) return DPG_ERR_UNSUPPORTED;
        magic = (uint32_t)((0x100000000ull + (uint64_t)we - 1) / (uint64_t)we);
    }
    const int64_t grid = (n + tile - 1) / tile;
    if (grid > 0x7fffffffLL) return DPG_ERR_UNSUPPORTED;
    const size_t lds = 2 * (size_t)tile * sizeof(int32_t);
    if (nt)
        hipLaunchKernelGGL((k_probe_scatter<E, WE, true>), dim3((unsigned)grid), dim3(256), lds, stream, (const E *)src,
                           run, pos, n_valid, (E *)dst, n, limit, we, magic, tile, remap);
    else
        hipLaunchKernelGGL((k_probe_scatter<E, WE, false>), dim3((unsigned)grid), dim3(256), lds, stream,
                           (const E *)src, run, pos, n_valid, (E *)dst, n, limit, we, magic, tile, remap);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

dpg_status launch_probe_scatter(dpg_ctx *ctx, const void *src, int64_t limit, const int32_t *run, const int32_t *pos,
                                const int32_t *n_valid, void *dst, int64_t n, int rec_bytes, hipStream_t stream) {
    if (n <= 0) return DPG_OK;
    const double M = (double)n, R = rec_bytes;
    ProfScope prof(ctx, K_PROBE_SCATTER, 8.0 * M + 2.0 * R * M, stream);
    const int remap = xcd_remap_flag(ctx);
    // the same rule as the gather: streaming stores for outputs larger than
    // the Infinity Cache
    const bool nt = (double)n * rec_bytes > kStreamingStoreBytes;
    const uintptr_t al = (uintptr_t)src | (uintptr_t)dst;
    if (rec_bytes % 16 == 0 && al % 16 == 0) {
        const int we = rec_bytes / 16;
        if (we == 1) return launch_scatter_t<u32x4, 1>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
        return launch_scatter_t<u32x4, 0>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
    }
    if (rec_bytes % 8 == 0 && al % 8 == 0) {
        const int we = rec_bytes / 8;
        if (we == 1) return launch_scatter_t<u32x2, 1>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
        return launch_scatter_t<u32x2, 0>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
    }
    const int we = rec_bytes / 4;
    if (we == 1) return launch_scatter_t<uint32_t, 1>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
    if (we == 25) return launch_scatter_t<uint32_t, 25>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
    return launch_scatter_t<uint32_t, 0>(src, run, pos, n_valid, dst, n, limit, we, remap, nt, stream);
}

template <typename E, int WE, int TR = 0>
static dpg_status launch_gather_t(int role, const void *src, const int32_t *idx, void *dst, int64_t n,
                                  int64_t limit, int we, int remap, hipStream_t stream) {
    using S = GatherShape<E, WE, TR>;
    int tile;
    uint32_t magic = 0;
    if constexpr (WE > 0) {
        tile = S::TILE;
    } else {
        tile = aligned_tile((256 * S::PER) / we, we * (int)sizeof(E));
        if (tile < 1 || we < 2) return DPG_ERR_UNSUPPORTED;
        magic = (uint32_t)((0x100000000ull + (uint64_t)we - 1) / (uint64_t)we);
    }
    const int64_t grid = (n + tile - 1) / tile;
    if (grid > 0x7fffffffLL) return DPG_ERR_UNSUPPORTED;
    const size_t lds = (size_t)tile * sizeof(int32_t);
    // Outputs larger than the Infinity Cache are written with nontemporal
    // stores: they will not be read again before being evicted.
    const bool nt = (double)n * we * sizeof(E) > kStreamingStoreBytes;
#define DPG_LAUNCH_ROLE(KERNEL)                                                                                    \
    do {                                                                                                           \
        if (nt)                                                                                                    \
            hipLaunchKernelGGL((KERNEL<E, WE, true, TR>), dim3((unsigned)grid), dim3(256), lds, stream,             \
                               (const E *)src, idx, (E *)dst, n, limit, we, magic, tile, remap);                  \
        else                                                                                                       \
            hipLaunchKernelGGL((KERNEL<E, WE, false, TR>), dim3((unsigned)grid), dim3(256), lds, stream,            \
                               (const E *)src, idx, (E *)dst, n, limit, we, magic, tile, remap);                  \
    } while (0)
    if (role == K_PROBE_CACHED) DPG_LAUNCH_ROLE(k_probe_cached);
    else if (role == K_GATHER_PHASE) DPG_LAUNCH_ROLE(k_gather_phase);
    else DPG_LAUNCH_ROLE(k_direct_gather);
#undef DPG_LAUNCH_ROLE
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

dpg_status launch_gather(dpg_ctx *ctx, int kernel_id, const void *src, int64_t limit, const int32_t *idx,
                         void *dst, int64_t n, int rec_bytes, double alg_bytes, hipStream_t stream) {
    if (n <= 0) return DPG_OK;
    ProfScope prof(ctx, kernel_id, alg_bytes, stream);
    const int remap = xcd_remap_flag(ctx);
    const uintptr_t al = (uintptr_t)src | (uintptr_t)dst;
    if (rec_bytes % 16 == 0 && al % 16 == 0) {
        const int we = rec_bytes / 16;
        switch (we) {
            case 1: return launch_gather_t<u32x4, 1>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            case 2: return launch_gather_t<u32x4, 2>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            case 4: return launch_gather_t<u32x4, 4>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            case 8: return launch_gather_t<u32x4, 8>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            case 16: return launch_gather_t<u32x4, 16>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            default: return launch_gather_t<u32x4, 0>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
        }
    }
    if (rec_bytes % 8 == 0 && al % 8 == 0) {
        const int we = rec_bytes / 8;
        if (we == 1) return launch_gather_t<u32x2, 1>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
        return launch_gather_t<u32x2, 0>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
    }
    const int we = rec_bytes / 4;
    switch (we) {
        case 1: return launch_gather_t<uint32_t, 1>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
        case 3: return launch_gather_t<uint32_t, 3>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
        case 25:
            // 100-byte records: tiles measured at 2^26 records -- 64 rows for
            // random reads, 128 for the probe's region-local reads, 192 for
            // the gather's reads from the run streams (256 rows: 1-2% slower)
            if (kernel_id == K_PROBE_CACHED)
                return launch_gather_t<uint32_t, 25, 128>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            if (kernel_id == K_GATHER_PHASE)
                return launch_gather_t<uint32_t, 25, 192>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
            return launch_gather_t<uint32_t, 25, 64>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
        default: return launch_gather_t<uint32_t, 0>(kernel_id, src, idx, dst, n, limit, we, remap, stream);
    }
}

// Plain streaming copy: the practical read + write ceiling against which the
// copy phases are measured.  Each workgroup copies one contiguous tile of
// 256 * PER 16-byte vectors; a lane issues its PER loads before its first
// store.  Stores are nontemporal unless asked otherwise.
template <int PER, bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                      int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * (256 * PER) + threadIdx.x;
    u32x4 v[PER];
    if (base + (int64_t)(PER - 1) * 256 < n) {
#pragma unroll
        for (int k = 0; k < PER; ++k) v[k] = src[base + k * 256];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if constexpr (NT) __builtin_nontemporal_store(v[k], dst + base + k * 256);
            else dst[base + k * 256] = v[k];
        }
        return;
    }
    for (int k = 0; k < PER; ++k) {
        const int64_t i = base + k * 256;
        if (i < n) {
            if constexpr (NT) __builtin_nontemporal_store(src[i], dst + i);
            else dst[i] = src[i];
        }
    }
}

dpg_status launch_stream_copy(dpg_ctx *ctx, const void *src, void *dst, size_t bytes, int per, bool nt,
                              hipStream_t stream) {
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return DPG_OK;
    ProfScope prof(ctx, K_STREAM_COPY, 2.0 * (double)bytes, stream);
    const int64_t grid = (n + 256 * per - 1) / (256 * per);
    if (grid > 0x7fffffffLL) return DPG_ERR_UNSUPPORTED;
#define DPG_LAUNCH_COPY(P)                                                                                    \
    do {                                                                                                      \
        if (nt)                                                                                               \
            hipLaunchKernelGGL((k_stream_copy<P, true>), dim3((unsigned)grid), dim3(256), 0, stream,          \
                               (const u32x4 *)src, (u32x4 *)dst, n);                                          \
        else                                                                                                  \
            hipLaunchKernelGGL((k_stream_copy<P, false>), dim3((unsigned)grid), dim3(256), 0, stream,         \
                               (const u32x4 *)src, (u32x4 *)dst, n);                                          \
    } while (0)
    switch (per) {
        case 2: DPG_LAUNCH_COPY(2); break;
        case 4: DPG_LAUNCH_COPY(4); break;
        case 8: DPG_LAUNCH_COPY(8); break;
        case 16: DPG_LAUNCH_COPY(16); break;
        default: return DPG_ERR_INVALID_ARG;
    }
#undef DPG_LAUNCH_COPY
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

dpg_status launch_fill_i32(dpg_ctx *ctx, int32_t *p, int64_t n, int32_t value, hipStream_t stream) {
    if (n <= 0) return DPG_OK;
    ProfScope prof(ctx, K_FILL, 4.0 * n, stream);
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)grid), dim3(256), 0, stream, p, n, value);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

// Every id in [0, limit)?  Sets *flag to 1 otherwise (vector atomic).
__global__ __launch_bounds__(256) void k_check_ids(const int32_t *__restrict__ ids, int64_t n, int64_t limit,
                                                   int32_t *flag) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t v = ids[i];
        bad |= (v < 0) | ((int64_t)v >= limit);
    }
    if (__any(bad) && __lane_id() == 0) atomicOr(flag, 1);
}

dpg_status check_ids(dpg_ctx *ctx, const int32_t *ids, int64_t n, int64_t limit, int32_t *flag_dev,
                     hipStream_t stream, bool *bad) {
    *bad = false;
    if (n <= 0) return DPG_OK;
    dpg_status st = launch_fill_i32(ctx, flag_dev, 1, 0, stream);
    if (st != DPG_OK) return st;
    {
        ProfScope prof(ctx, K_CHECK_IDS, 4.0 * n, stream);
        int64_t grid = (n + 255) / 256;
        if (grid > (int64_t)ctx->n_cu * 16) grid = (int64_t)ctx->n_cu * 16;
        hipLaunchKernelGGL(k_check_ids, dim3((unsigned)grid), dim3(256), 0, stream, ids, n, limit, flag_dev);
        DPG_HIP(hipGetLastError());
    }
    DPG_HIP(hipMemcpyAsync(ctx->host_flag, flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    DPG_HIP(hipStreamSynchronize(stream));
    *bad = (*ctx->host_flag != 0);
    return DPG_OK;
}

}  // namespace dpg
