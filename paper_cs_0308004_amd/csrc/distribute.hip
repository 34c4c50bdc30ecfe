// DPG Phase I, Distribute (Section 2.1; Figure 1).
//
// The rid list is cut into tiles of T consecutive rids.  The run of rid r is
// b = r >> log2(L).  Three steps, each coalesced:
//   1. k_dist_hist     per tile, an LDS histogram over the B runs -> cnt[t][b]
//   2. column scan     off[t][b] = (rids in runs < b) + (rids of run b in tiles < t);
//                      this is the "set bucket boundaries" step of the count
//                      bucket sort of Section 5.3, also giving run_off[b]
//   3. k_dist_scatter  one wave per tile walks its rids in list order and
//                      appends each to its run: run[pos] = r, inv[i] = pos.
// Appending in list order keeps every run in RID order, as Figure 1 does;
// inv[i] names the INTERNAL slot that will hold the record of the i-th rid, so
// the gather needs no search and does not depend on the order inside a run.
// When B fits one 8-bit digit the distribute is instead one partition pass
// (partition.hip) whose order inside a run is unspecified; inv keeps the
// result exact.
//
// A rid outside [0, n_src) is skipped (its inv is 0), so no kernel of the
// pipeline can address memory outside its buffers even on invalid input.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

__global__ __launch_bounds__(256) void k_dist_hist(const int32_t *__restrict__ rids, int64_t n, int64_t n_src,
                                                   int shift, int B, int T, int32_t *__restrict__ cnt) {
    extern __shared__ int32_t h[];
    for (int b = threadIdx.x; b < B; b += 256) h[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * T;
    const int64_t end = min(base + T, n);
    constexpr int kBatch = 8;
    for (int64_t i0 = base + threadIdx.x; i0 < end; i0 += 256 * kBatch) {
        int32_t rv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t i = i0 + (int64_t)u * 256;
            rv[u] = i < end ? rids[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (rv[u] >= 0 && (int64_t)rv[u] < n_src) atomicAdd(&h[rv[u] >> shift], 1);
    }
    __syncthreads();
    int32_t *row = cnt + (int64_t)blockIdx.x * B;
    for (int b = threadIdx.x; b < B; b += 256) row[b] = h[b];
}

// One wave per tile.  The running append position of every run lives in LDS;
// rids are staged in LDS a chunk at a time (all loads of a chunk in flight at
// once), and each step's 64 rids are ranked among equal runs with ballots, so
// the append order is the rid-list order.
constexpr int kScatterChunk = 1024;

__global__ __launch_bounds__(64) void k_dist_scatter(const int32_t *__restrict__ rids, int64_t n, int64_t n_src,
                                                     int shift, int nbits, int B, int T, int64_t nT,
                                                     const int32_t *__restrict__ off, int32_t *__restrict__ run,
                                                     int32_t *__restrict__ inv, int remap) {
    extern __shared__ int32_t smem[];
    int32_t *cur = smem;
    int32_t *s_rid = smem + ((B + 3) & ~3);
    const int64_t t = xcd_tile(blockIdx.x, nT, remap);
    const int lane = threadIdx.x;
    const int32_t *row = off + t * B;
    for (int b = lane; b < B; b += 64) cur[b] = row[b];
    const int64_t base = t * T;
    const int64_t end = min(base + T, n);
    for (int64_t c0 = base; c0 < end; c0 += kScatterChunk) {
        const int n_c = (int)min((int64_t)kScatterChunk, end - c0);
        int32_t staged[kScatterChunk / 64];
#pragma unroll
        for (int k = 0; k < kScatterChunk / 64; ++k) {
            const int j = lane + k * 64;
            staged[k] = j < n_c ? rids[c0 + j] : -1;
        }
#pragma unroll
        for (int k = 0; k < kScatterChunk / 64; ++k) s_rid[lane + k * 64] = staged[k];
        __syncthreads();
        for (int j0 = 0; j0 < n_c; j0 += 64) {
            const int j = j0 + lane;
            const int64_t i = c0 + j;
            const bool in_list = j < n_c;
            const int32_t r = s_rid[j];
            const bool valid = in_list && r >= 0 && (int64_t)r < n_src;
            const uint32_t b = valid ? ((uint32_t)r >> shift) : 0u;
            const uint64_t act = __ballot(valid);
            const uint64_t peers = match_lanes(b, nbits, act);
            const int leader = peers ? (__ffsll((unsigned long long)peers) - 1) : 0;
            int32_t head = 0;
            if (valid && lane == leader) head = cur[b];
            head = lane_read(head, leader);
            if (valid) {
                const int32_t pos = head + __popcll(peers & lanemask_lt());
                run[pos] = r;
                inv[i] = pos;
                if (lane == leader) cur[b] = head + __popcll(peers);
            } else if (in_list) {
                inv[i] = 0;
            }
            __syncthreads();
        }
    }
}

dpg_status launch_distribute(dpg_ctx *ctx, const RetrievePlan &p, const int32_t *rids, void *ws,
                             hipStream_t stream, bool local_inv) {
    char *w = (char *)ws;
    if (local_inv && p.dist_mode != DIST_PARTITION) return DPG_ERR_UNSUPPORTED;
    if (p.dist_mode == DIST_PARTITION) {
        const PartPlan pp = plan_partition(p.n_rids, p.part_nbits, 4, false);
        int32_t *item_off = p.probe == DPG_PROBE_LDS ? (int32_t *)(w + p.off_items) : nullptr;
        return launch_partition(ctx, pp, rids, nullptr, w + p.off_run, nullptr, (int32_t *)(w + p.off_inv),
                                p.log2_run, (uint64_t)p.n_src, w + p.off_part, stream, nullptr, item_off,
                                p.probe == DPG_PROBE_LDS ? p.probe_chunk : 0, /*stable=*/false, local_inv);
    }
    int32_t *cnt = (int32_t *)(w + p.off_cnt);
    int32_t *csum = (int32_t *)(w + p.off_csum);
    int32_t *total = (int32_t *)(w + p.off_total);
    int32_t *run_off = (int32_t *)(w + p.off_bucket);
    int32_t *item_off = p.probe == DPG_PROBE_LDS ? (int32_t *)(w + p.off_items) : nullptr;
    int32_t *run = (int32_t *)(w + p.off_run);
    int32_t *inv = (int32_t *)(w + p.off_inv);
    const int B = (int)p.n_runs, T = p.dist_tile, shift = p.log2_run;
    const int64_t nT = p.n_tiles, nC = p.n_chunks, M = p.n_rids;
    const int nbits = bit_length((uint64_t)(B - 1));
    const size_t lds = (size_t)B * sizeof(int32_t);
    {
        ProfScope prof(ctx, K_DIST_HIST, 4.0 * M + 4.0 * nT * B, stream);
        hipLaunchKernelGGL(k_dist_hist, dim3((unsigned)nT), dim3(256), lds, stream, rids, M, p.n_src, shift, B, T,
                           cnt);
        DPG_HIP(hipGetLastError());
    }
    dpg_status st = launch_column_scan(ctx, cnt, nT, B, csum, nC, total, run_off, item_off,
                                       p.probe == DPG_PROBE_LDS ? p.probe_chunk : 0, stream);
    if (st != DPG_OK) return st;
    {
        ProfScope prof(ctx, K_DIST_SCATTER, 12.0 * M + 4.0 * nT * B, stream);
        const size_t lds_scatter = (size_t)((B + 3) & ~3) * sizeof(int32_t) + kScatterChunk * sizeof(int32_t);
        hipLaunchKernelGGL(k_dist_scatter, dim3((unsigned)nT), dim3(64), lds_scatter, stream, rids, M, p.n_src, shift,
                           nbits, B, T, nT, cnt, run, inv, xcd_remap_flag(ctx));
        DPG_HIP(hipGetLastError());
    }
    return DPG_OK;
}

}  // namespace dpg
