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
// Appending in list order keeps every run in RID order (the stability the
// gather of Phase III relies on); inv[i] names the INTERNAL slot that will hold
// the record of the i-th rid, so the gather needs no search.
//
// A rid outside [0, n_src) is skipped (its inv is 0), so no kernel of the
// pipeline can address memory outside its buffers even on invalid input.
#include "dev_common.h"
#include "dpg_internal.h"

namespace dpg {

constexpr int kScanChunkRows = 32;

__global__ __launch_bounds__(256) void k_dist_hist(const int32_t *__restrict__ rids, int64_t n, int64_t n_src,
                                                   int shift, int B, int T, int32_t *__restrict__ cnt) {
    extern __shared__ int32_t h[];
    for (int b = threadIdx.x; b < B; b += 256) h[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * T;
    const int64_t end = min(base + T, n);
#pragma unroll 4
    for (int64_t i = base + threadIdx.x; i < end; i += 256) {
        const int32_t r = rids[i];
        if (r >= 0 && (int64_t)r < n_src) atomicAdd(&h[r >> shift], 1);
    }
    __syncthreads();
    int32_t *row = cnt + (int64_t)blockIdx.x * B;
    for (int b = threadIdx.x; b < B; b += 256) row[b] = h[b];
}

// csum[b][c] = sum of cnt[t][b] over the rows t of chunk c.
__global__ __launch_bounds__(256) void k_scan_chunks(const int32_t *__restrict__ cnt, int64_t nT, int B,
                                                     int32_t *__restrict__ csum, int64_t nC) {
    const int64_t c = blockIdx.x;
    const int b = blockIdx.y * 256 + threadIdx.x;
    if (b >= B) return;
    const int64_t t0 = c * kScanChunkRows, t1 = min(t0 + kScanChunkRows, nT);
    int32_t s = 0;
    for (int64_t t = t0; t < t1; ++t) s += cnt[t * B + b];
    csum[(int64_t)b * nC + c] = s;
}

__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// One wave per run b: exclusive scan of csum[b][*] in place, total[b] = sum.
__global__ __launch_bounds__(256) void k_scan_cols(int32_t *__restrict__ csum, int64_t nC, int B,
                                                   int32_t *__restrict__ total) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= B) return;
    int32_t *col = csum + (int64_t)b * nC;
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < nC; c0 += 64) {
        const int64_t c = c0 + lane;
        const int32_t v = c < nC ? col[c] : 0;
        const int32_t inc = wave_inclusive_scan(v);
        if (c < nC) col[c] = carry + inc - v;
        carry += __shfl(inc, 63, 64);
    }
    if (lane == 0) total[b] = carry;
}

// Exclusive scans over the runs: run_off[b] (b = 0..B) and, for the LDS probe,
// item_off[b] = sum over b' < b of ceil(total[b'] / chunk).
__global__ __launch_bounds__(1024) void k_scan_base(const int32_t *__restrict__ total, int B,
                                                    int32_t *__restrict__ run_off, int32_t *__restrict__ item_off,
                                                    int chunk) {
    __shared__ int32_t wsum[2][16];
    __shared__ int32_t carry[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (int b0 = 0; b0 < B; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const int32_t v = b < B ? total[b] : 0;
        const int32_t u = (b < B && chunk > 0) ? (v + chunk - 1) / chunk : 0;
        const int32_t iv = wave_inclusive_scan(v), iu = wave_inclusive_scan(u);
        if (lane == 63) { wsum[0][wave] = iv; wsum[1][wave] = iu; }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int32_t a = lane < 16 ? wsum[0][lane] : 0;
            const int32_t c = lane < 16 ? wsum[1][lane] : 0;
            const int32_t sa = wave_inclusive_scan(a), sc = wave_inclusive_scan(c);
            if (lane < 16) { wsum[0][lane] = sa - a; wsum[1][lane] = sc - c; }
        }
        __syncthreads();
        if (b < B) {
            run_off[b] = carry[0] + wsum[0][wave] + iv - v;
            if (item_off) item_off[b] = carry[1] + wsum[1][wave] + iu - u;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] += wsum[0][15] + iv;
            carry[1] += wsum[1][15] + iu;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        run_off[B] = carry[0];
        if (item_off) item_off[B] = carry[1];
    }
}

// cnt[t][b] <- run_off[b] + rids of run b in tiles before t.
__global__ __launch_bounds__(256) void k_scan_apply(int32_t *__restrict__ cnt, int64_t nT, int B,
                                                    const int32_t *__restrict__ csum, int64_t nC,
                                                    const int32_t *__restrict__ run_off) {
    const int64_t c = blockIdx.x;
    const int b = blockIdx.y * 256 + threadIdx.x;
    if (b >= B) return;
    int32_t run = run_off[b] + csum[(int64_t)b * nC + c];
    const int64_t t0 = c * kScanChunkRows, t1 = min(t0 + kScanChunkRows, nT);
    for (int64_t t = t0; t < t1; ++t) {
        const int32_t v = cnt[t * B + b];
        cnt[t * B + b] = run;
        run += v;
    }
}

// One wave per tile.  The running append position of every run lives in LDS;
// the 64 rids of a step are ranked among equal runs with ballots, so the
// append order is the rid-list order.
__global__ __launch_bounds__(64) void k_dist_scatter(const int32_t *__restrict__ rids, int64_t n, int64_t n_src,
                                                     int shift, int nbits, int B, int T, int64_t nT,
                                                     const int32_t *__restrict__ off, int32_t *__restrict__ run,
                                                     int32_t *__restrict__ inv, int remap) {
    extern __shared__ int32_t cur[];
    const int64_t t = xcd_tile(blockIdx.x, nT, remap);
    const int lane = threadIdx.x;
    const int32_t *row = off + t * B;
    for (int b = lane; b < B; b += 64) cur[b] = row[b];
    __syncthreads();
    const int64_t base = t * T;
    const int64_t end = min(base + T, n);
    int32_t r_next = (base + lane < end) ? rids[base + lane] : -1;
    for (int64_t i0 = base; i0 < end; i0 += 64) {
        const int64_t i = i0 + lane;
        const int32_t r = r_next;
        r_next = (i + 64 < end) ? rids[i + 64] : -1;
        const bool in_list = i < end;
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

dpg_status launch_distribute(dpg_ctx *ctx, const RetrievePlan &p, const int32_t *rids, void *ws,
                             hipStream_t stream) {
    char *w = (char *)ws;
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
    const unsigned gy = (unsigned)((B + 255) / 256);
    {
        ProfScope prof(ctx, K_DIST_HIST, 4.0 * M + 4.0 * nT * B, stream);
        hipLaunchKernelGGL(k_dist_hist, dim3((unsigned)nT), dim3(256), lds, stream, rids, M, p.n_src, shift, B, T,
                           cnt);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_CHUNKS, 4.0 * nT * B + 4.0 * nC * B, stream);
        hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nC, gy), dim3(256), 0, stream, cnt, nT, B, csum, nC);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_COLS, 8.0 * nC * B, stream);
        hipLaunchKernelGGL(k_scan_cols, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, stream, csum, nC, B, total);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_BASE, 12.0 * B, stream);
        hipLaunchKernelGGL(k_scan_base, dim3(1), dim3(1024), 0, stream, total, B, run_off, item_off,
                           p.probe == DPG_PROBE_LDS ? p.probe_chunk : 0);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_APPLY, 8.0 * nT * B + 4.0 * nC * B, stream);
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nC, gy), dim3(256), 0, stream, cnt, nT, B, csum, nC,
                           run_off);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_DIST_SCATTER, 12.0 * M + 4.0 * nT * B, stream);
        hipLaunchKernelGGL(k_dist_scatter, dim3((unsigned)nT), dim3(64), lds, stream, rids, M, p.n_src, shift,
                           nbits, B, T, nT, cnt, run, inv, xcd_remap_flag(ctx));
        DPG_HIP(hipGetLastError());
    }
    return DPG_OK;
}

}  // namespace dpg
