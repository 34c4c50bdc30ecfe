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
#include <algorithm>

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

// Sample for the splitters of the skew-balanced runs: n_sample rids at evenly
// spaced list positions (an rid out of range is clamped into it: only the
// balance of the runs depends on the sample).
__global__ __launch_bounds__(256) void k_dist_sample(const int32_t *__restrict__ rids, int64_t m, int64_t n_src,
                                                     int64_t s, uint32_t *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= s) return;
    const int64_t r = rids[k * m / s];  // k < s and m below 2^31: no overflow
    out[k] = (uint32_t)(r < 0 ? 0 : (r >= n_src ? n_src - 1 : r));
}

// split[b] = the last sampled rid of the b-th of B equal shares of the sorted
// sample, b < B - 1: run b then holds the rids in (split[b-1], split[b]].
__global__ __launch_bounds__(256) void k_dist_splitters(const uint32_t *__restrict__ sorted, int64_t s, int B,
                                                        uint32_t *__restrict__ split) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B - 1) return;
    int64_t at = (int64_t)(b + 1) * s / B - 1;
    if (at < 0) at = 0;
    split[b] = sorted[at];
}

// Phase I with runs balanced by a sample (Section 2.3, data skew): sample the
// rids, sort the sample (stable 8-bit passes over the bytes an rid can
// occupy), take B - 1 splitters that cut it into equal shares, then one
// partition pass of the rids by splitter.
static dpg_status launch_distribute_sampled(dpg_ctx *ctx, const RetrievePlan &p, const int32_t *rids, char *w,
                                            hipStream_t stream, bool local_inv) {
    const int64_t s = p.n_sample, M = p.n_rids;
    const int B = (int)p.n_runs;
    uint32_t *a = (uint32_t *)(w + p.off_sample), *b = (uint32_t *)(w + p.off_sample2);
    uint32_t *split = (uint32_t *)(w + p.off_split);
    hipLaunchKernelGGL(k_dist_sample, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, stream, rids, M, p.n_src, s,
                       a);
    DPG_HIP(hipGetLastError());
    const PartPlan sp = plan_partition(s, 8, 4, false);
    const int passes = std::max(1, (bit_length((uint64_t)(p.n_src > 1 ? p.n_src - 1 : 1)) + 7) / 8);
    for (int k = 0; k < passes; ++k) {
        const dpg_status st =
            launch_partition(ctx, sp, a, nullptr, b, nullptr, nullptr, 8 * k, 0, w + p.off_spart, stream, nullptr);
        if (st != DPG_OK) return st;
        std::swap(a, b);
    }
    if (B > 1) {
        hipLaunchKernelGGL(k_dist_splitters, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, a, s, B, split);
        DPG_HIP(hipGetLastError());
    }
    const PartPlan pp = dist_partition(p);
    return launch_partition(ctx, pp, rids, nullptr, w + p.off_run, nullptr, (int32_t *)(w + p.off_inv), 0,
                            (uint64_t)p.n_src, w + p.off_part, stream, nullptr, nullptr, 0, /*stable=*/false,
                            local_inv, 1u, split, B - 1);
}

// Run boundaries of a list sorted by run (the two-pass distribute's output):
// run_off[b] = first position whose run is >= b, for b in [0, B], over the
// first *n_valid entries.  Each position k writes the boundaries of the runs
// after its predecessor's up to its own; the last position also closes the
// runs after its own.
__global__ __launch_bounds__(256) void k_run_bounds(const int32_t *__restrict__ run, int64_t M,
                                                    const int32_t *__restrict__ n_valid, int shift, int B,
                                                    int32_t *__restrict__ run_off) {
    const int64_t nv = min((int64_t)*n_valid, M);
    if (nv == 0) {
        for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b <= B; b += (int64_t)gridDim.x * 256)
            run_off[b] = 0;
        return;
    }
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nv; k += (int64_t)gridDim.x * 256) {
        const int r = min(run[k] >> shift, B - 1);
        const int rp = k > 0 ? min(run[k - 1] >> shift, B - 1) : -1;
        for (int b = rp + 1; b <= r; ++b) run_off[b] = (int32_t)k;
        if (k == nv - 1)
            for (int b = r + 1; b <= B; ++b) run_off[b] = (int32_t)nv;
    }
}

// Work items of the LDS probe: items[b] = ceil(len(run b) / P), scanned later.
__global__ __launch_bounds__(256) void k_run_items(const int32_t *__restrict__ run_off, int B, int P,
                                                   int32_t *__restrict__ items) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < B) items[b] = (run_off[b + 1] - run_off[b] + P - 1) / P;
}

// Phase I in two passes (the multi-pass DPG of Section 7): the rids are
// partitioned by the fine bits of their run index (unstable), then that list
// by the coarse bits (stable), so the final list is in run order; inv_f and
// inv_c record both moves.  An rid out of range is dropped by the first pass;
// the second pass treats the unwritten tail of the first pass's output the
// same way, so every later index stays in its buffer.
static dpg_status launch_distribute_two_pass(dpg_ctx *ctx, const RetrievePlan &p, const int32_t *rids, char *w,
                                             hipStream_t stream) {
    const int64_t M = p.n_rids;
    const PartPlan pf = plan_partition(M, p.lg_fine, 4, false);
    const PartPlan pc = plan_partition(M, p.lg_coarse, 4, false);
    if (p.probe == DPG_PROBE_LDS) {
        // the first pass leaves the slots of dropped rids unwritten; filled
        // with an invalid rid, they are dropped by the second pass too, so
        // that its output is exactly the valid rids in run order (the run
        // boundaries below rely on that order)
        dpg_status st = launch_fill_i32(ctx, (int32_t *)(w + p.off_run_f), M, (int32_t)p.n_src, stream);
        if (st != DPG_OK) return st;
    }
    dpg_status st = launch_partition(ctx, pf, rids, nullptr, w + p.off_run_f, nullptr, (int32_t *)(w + p.off_inv_f),
                                     p.log2_run, (uint64_t)p.n_src, w + p.off_part, stream, nullptr, nullptr, 0,
                                     /*stable=*/false);
    if (st != DPG_OK) return st;
    st = launch_partition(ctx, pc, w + p.off_run_f, nullptr, w + p.off_run, nullptr, (int32_t *)(w + p.off_inv_c),
                          p.log2_run + p.lg_fine, (uint64_t)p.n_src, w + p.off_part2, stream, nullptr, nullptr, 0,
                          /*stable=*/true);
    if (st != DPG_OK || p.probe != DPG_PROBE_LDS) return st;
    // the LDS probe needs every run's boundaries: the list is in run order,
    // so they are where the run changes; then each run's work items
    const int B = (int)p.n_runs;
    const int32_t *n_valid = (const int32_t *)(w + p.off_part2 + pc.off_bucket) + (1 << p.lg_coarse);
    int32_t *run_off = (int32_t *)(w + p.off_bucket);
    int32_t *items = (int32_t *)(w + p.off_items);
    {
        ProfScope prof(ctx, K_RUN_BOUNDS, 8.0 * M + 8.0 * B, stream);
        const int64_t grid = std::min<int64_t>((M + 255) / 256, (int64_t)ctx->n_cu * 16);
        hipLaunchKernelGGL(k_run_bounds, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(256), 0, stream,
                           (const int32_t *)(w + p.off_run), M, n_valid, p.log2_run, B, run_off);
        DPG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_run_items, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, run_off, B,
                           p.probe_chunk, items);
        DPG_HIP(hipGetLastError());
    }
    return launch_scan_1d(ctx, items, B, (int32_t *)(w + p.off_scan), items + B, stream);
}

dpg_status launch_distribute(dpg_ctx *ctx, const RetrievePlan &p, const int32_t *rids, void *ws,
                             hipStream_t stream, bool local_inv) {
    char *w = (char *)ws;
    if (local_inv && p.dist_mode != DIST_PARTITION && p.dist_mode != DIST_SAMPLED) return DPG_ERR_UNSUPPORTED;
    if (p.dist_mode == DIST_SAMPLED) return launch_distribute_sampled(ctx, p, rids, w, stream, local_inv);
    if (p.dist_mode == DIST_TWO_PASS) return launch_distribute_two_pass(ctx, p, rids, w, stream);
    if (p.dist_mode == DIST_PARTITION && p.scatter) {
        // two-phase DPG: the runs, and beside each rid its list position
        const PartPlan pp = dist_partition(p);
        return launch_partition(ctx, pp, rids, nullptr, w + p.off_run, nullptr, nullptr, p.log2_run,
                                (uint64_t)p.n_src, w + p.off_part, stream, nullptr, nullptr, 0, /*stable=*/false,
                                false, 1u, nullptr, 0, (uint32_t *)(w + p.off_inv));
    }
    if (p.dist_mode == DIST_PARTITION) {
        const PartPlan pp = dist_partition(p);
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
