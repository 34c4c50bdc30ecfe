// DPG Phase II, Probe, with the source run staged in LDS (Section 2.1: "one
// loads the i-th INPUT run entirely into cache").
//
// Work item = (run b, chunk of at most P entries of RID run b).  The workgroup
// reads source records [b*L, min((b+1)*L, n_src)) into LDS with coalesced
// loads, stages its chunk of RID run b, then writes INTERNAL[k] =
// region[rid_run[k] - b*L] for its slots k in order -- INTERNAL is written
// sequentially, the source is read sequentially, the random access stays in
// LDS.  Runs longer than P (duplicates, skew; Section 2.3) get several items,
// each loading the region again.
#include "dev_common.h"
#include "dpg_internal.h"

namespace dpg {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename E, int WE>
__global__ __launch_bounds__(256) void k_probe_lds(const E *__restrict__ src, int64_t n_src, int we_rt,
                                                   uint32_t magic, const int32_t *__restrict__ run,
                                                   const int32_t *__restrict__ run_off,
                                                   const int32_t *__restrict__ item_off, int B, int shift, int P,
                                                   E *__restrict__ internal, int region_elems_off) {
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_bucket;
    int32_t *s_run = (int32_t *)smem;
    E *region = (E *)(smem + region_elems_off);
    const int we = WE > 0 ? WE : we_rt;
    const int32_t item = (int32_t)blockIdx.x;
    if (item >= item_off[B]) return;
    if (threadIdx.x == 0) {
        int lo = 0, hi = B - 1;  // largest b with item_off[b] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        s_bucket = lo;
    }
    __syncthreads();
    const int b = s_bucket;
    const int64_t k0 = (int64_t)run_off[b] + (int64_t)(item - item_off[b]) * P;
    const int64_t k1 = min(k0 + P, (int64_t)run_off[b + 1]);
    const int cnt = (int)(k1 - k0);
    const int64_t r0 = (int64_t)b << shift;
    const int64_t rlen = min((int64_t)1 << shift, n_src - r0);
#pragma unroll 8
    for (int j = threadIdx.x; j < cnt; j += 256) {
        const int64_t loc = (int64_t)run[k0 + j] - r0;
        s_run[j] = (loc >= 0 && loc < rlen) ? (int32_t)loc : 0;
    }
    const E *rs = src + r0 * we;
    const int relems = (int)(rlen * we);
#pragma unroll 8
    for (int e = threadIdx.x; e < relems; e += 256) region[e] = rs[e];
    __syncthreads();
    E *out = internal + k0 * we;
    const int total = cnt * we;
    for (int e = threadIdx.x; e < total; e += 256) {
        int j;
        if constexpr (WE > 0) j = e / WE;
        else j = (int)__umulhi((uint32_t)e, magic);
        const int w = e - j * we;
        out[e] = region[s_run[j] * we + w];
    }
}

// The same phase for records of one element (4, 8 or 16 bytes): a workgroup
// of 1024 threads stages a region of up to 128 KiB with 16-byte loads, then
// every thread takes one rid at a time (kProbeWideBatch loads in flight),
// reads its record from LDS and writes INTERNAL in order.  The rids are not
// staged, so a work item can cover a whole run of up to 32768 rids and the
// region is loaded once per run.
constexpr int kProbeWideThreads = 1024;
constexpr int kProbeWideBatch = 16;

template <typename E, bool NT>
__global__ __launch_bounds__(kProbeWideThreads) void k_probe_lds_wide(
    const E *__restrict__ src, int64_t n_src, const int32_t *__restrict__ run, const int32_t *__restrict__ run_off,
    const int32_t *__restrict__ item_off, int B, int shift, int P, E *__restrict__ internal, int src_a16) {
    extern __shared__ __align__(16) char smem[];
    E *region = (E *)smem;
    __shared__ int s_bucket;
    const int32_t item = (int32_t)blockIdx.x;
    if (item >= item_off[B]) return;
    if (threadIdx.x == 0) {
        int lo = 0, hi = B - 1;  // largest b with item_off[b] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        s_bucket = lo;
    }
    __syncthreads();
    const int b = s_bucket;
    const int64_t k0 = (int64_t)run_off[b] + (int64_t)(item - item_off[b]) * P;
    const int64_t k1 = min(k0 + P, (int64_t)run_off[b + 1]);
    const int cnt = (int)(k1 - k0);
    const int64_t r0 = (int64_t)b << shift;
    const int rlen = (int)min((int64_t)1 << shift, n_src - r0);
    // the region: 16-byte loads when src_a16 (the source and every region
    // start are 16-byte aligned), then the elements of a ragged tail
    {
        const int n16 = src_a16 ? (int)(((int64_t)rlen * sizeof(E)) / 16) : 0;
        const u32x4 *s16 = (const u32x4 *)(src + r0);
        u32x4 *d16 = (u32x4 *)region;
#pragma unroll 4
        for (int e = threadIdx.x; e < n16; e += kProbeWideThreads) d16[e] = s16[e];
        for (int e = n16 * (int)(16 / sizeof(E)) + threadIdx.x; e < rlen; e += kProbeWideThreads)
            region[e] = src[r0 + e];
    }
    __syncthreads();
    for (int j0 = 0; j0 < cnt; j0 += kProbeWideThreads * kProbeWideBatch) {
        int32_t rr[kProbeWideBatch];
#pragma unroll
        for (int k = 0; k < kProbeWideBatch; ++k)
            rr[k] = run[k0 + min(j0 + (int)threadIdx.x + k * kProbeWideThreads, cnt - 1)];
#pragma unroll
        for (int k = 0; k < kProbeWideBatch; ++k) {
            const int j = j0 + (int)threadIdx.x + k * kProbeWideThreads;
            if (j < cnt) {
                const int64_t loc = (int64_t)rr[k] - r0;
                const E v = region[(loc >= 0 && loc < rlen) ? (int)loc : 0];
                if constexpr (NT) __builtin_nontemporal_store(v, internal + k0 + j);
                else internal[k0 + j] = v;
            }
        }
    }
}

template <typename E>
static dpg_status launch_probe_wide_t(const RetrievePlan &p, const void *src, void *ws, hipStream_t stream) {
    char *w = (char *)ws;
    const int32_t *run = (const int32_t *)(w + p.off_run);
    const int32_t *run_off = (const int32_t *)(w + p.off_bucket);
    const int32_t *item_off = (const int32_t *)(w + p.off_items);
    E *internal = (E *)(w + p.off_internal);
    const int P = p.probe_chunk;
    const size_t lds = ((size_t)1 << p.log2_run) * sizeof(E);
    if (lds > kProbeWideRegionBytes) return DPG_ERR_UNSUPPORTED;
    // 16-byte staging when src and every region start are 16-byte aligned
    const int a16 = ((uintptr_t)src) % 16 == 0 && (((size_t)1 << p.log2_run) * sizeof(E)) % 16 == 0;
    const int B = 1 << p.part_nbits;
    const int64_t grid = p.n_runs + (p.n_rids + P - 1) / P;
    if (grid > 0x7fffffffLL) return DPG_ERR_UNSUPPORTED;
    const bool nt = (double)p.n_rids * sizeof(E) > 256.0 * 1024 * 1024;
    const void *fn = nt ? (const void *)k_probe_lds_wide<E, true> : (const void *)k_probe_lds_wide<E, false>;
    if (lds > 64 * 1024) DPG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (nt)
        hipLaunchKernelGGL((k_probe_lds_wide<E, true>), dim3((unsigned)grid), dim3(kProbeWideThreads), lds, stream,
                           (const E *)src, p.n_src, run, run_off, item_off, B, p.log2_run, P, internal, a16);
    else
        hipLaunchKernelGGL((k_probe_lds_wide<E, false>), dim3((unsigned)grid), dim3(kProbeWideThreads), lds, stream,
                           (const E *)src, p.n_src, run, run_off, item_off, B, p.log2_run, P, internal, a16);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

template <typename E, int WE>
static dpg_status launch_probe_t(const RetrievePlan &p, const void *src, void *ws, int we, hipStream_t stream) {
    char *w = (char *)ws;
    const int32_t *run = (const int32_t *)(w + p.off_run);
    const int32_t *run_off = (const int32_t *)(w + p.off_bucket);
    const int32_t *item_off = (const int32_t *)(w + p.off_items);
    E *internal = (E *)(w + p.off_internal);
    const int P = p.probe_chunk;
    const int region_off = (int)align_up((size_t)P * sizeof(int32_t), 16);
    const size_t lds = region_off + ((size_t)1 << p.log2_run) * p.rec_bytes;
    const uint32_t magic = we >= 2 ? (uint32_t)((0x100000000ull + (uint64_t)we - 1) / (uint64_t)we) : 0;
    if constexpr (WE == 0) {
        if (we < 2) return DPG_ERR_UNSUPPORTED;
    }
    const int64_t grid = p.n_runs + (p.n_rids + P - 1) / P;
    if (grid > 0x7fffffffLL) return DPG_ERR_UNSUPPORTED;
    if (lds > 64 * 1024) {
        DPG_HIP(hipFuncSetAttribute((const void *)k_probe_lds<E, WE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
    }
    hipLaunchKernelGGL((k_probe_lds<E, WE>), dim3((unsigned)grid), dim3(256), lds, stream, (const E *)src, p.n_src,
                       we, magic, run, run_off, item_off, (int)p.n_runs, p.log2_run, P, internal, region_off);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

dpg_status launch_probe_lds(dpg_ctx *ctx, const RetrievePlan &p, const void *src, void *ws, hipStream_t stream) {
    const double R = p.rec_bytes, M = (double)p.n_rids;
    const double touched = (double)(p.n_src < p.n_rids ? p.n_src : p.n_rids);
    ProfScope prof(ctx, K_PROBE_LDS, 4.0 * M + R * touched + R * M, stream);
    if (p.probe_wide) {
        if (p.dist_mode != DIST_PARTITION) return DPG_ERR_UNSUPPORTED;
        switch (p.rec_bytes) {
            case 4: return launch_probe_wide_t<uint32_t>(p, src, ws, stream);
            case 8: return launch_probe_wide_t<u32x2>(p, src, ws, stream);
            case 16: return launch_probe_wide_t<u32x4>(p, src, ws, stream);
        }
        return DPG_ERR_UNSUPPORTED;
    }
    const uintptr_t al = (uintptr_t)src | (uintptr_t)((char *)ws + p.off_internal);
    if (p.rec_bytes % 16 == 0 && al % 16 == 0) {
        const int we = p.rec_bytes / 16;
        if (we == 1) return launch_probe_t<u32x4, 1>(p, src, ws, we, stream);
        if (we == 4) return launch_probe_t<u32x4, 4>(p, src, ws, we, stream);
        return launch_probe_t<u32x4, 0>(p, src, ws, we, stream);
    }
    if (p.rec_bytes % 8 == 0 && al % 8 == 0) {
        const int we = p.rec_bytes / 8;
        if (we == 1) return launch_probe_t<u32x2, 1>(p, src, ws, we, stream);
        return launch_probe_t<u32x2, 0>(p, src, ws, we, stream);
    }
    const int we = p.rec_bytes / 4;
    if (we == 1) return launch_probe_t<uint32_t, 1>(p, src, ws, we, stream);
    if (we == 25) return launch_probe_t<uint32_t, 25>(p, src, ws, we, stream);
    return launch_probe_t<uint32_t, 0>(p, src, ws, we, stream);
}

}  // namespace dpg
