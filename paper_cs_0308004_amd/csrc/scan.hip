// Column scan of a (tiles x buckets) count matrix, the "set bucket
// boundaries" step of a count bucket sort (Section 5.3): for every tile t and
// bucket b, off[t][b] = (elements in buckets < b) + (elements of bucket b in
// tiles < t), computed in place over the row-major count matrix, plus the
// bucket offsets bucket_off[0..B].  Every kernel reads and writes whole rows,
// so all accesses are coalesced.
#include "dev_common.h"
#include "dpg_internal.h"

namespace dpg {

constexpr int kScanChunkRows = 32;

// csum[b][c] = sum of cnt[t][b] over the rows t of chunk c.
__global__ __launch_bounds__(256) void k_scan_chunks(const int32_t *__restrict__ cnt, int64_t nT, int B,
                                                     int32_t *__restrict__ csum, int64_t nC,
                                                     const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
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
                                                   int32_t *__restrict__ total, const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
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
                                                    int chunk, const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
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
                                                    const int32_t *__restrict__ run_off,
                                                    const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
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

// ---------------------------------------------------------------------------
// Exclusive scan of one int32 array in place: per-block sums, one workgroup
// scanning the block sums, then each block rescans its chunk with its offset.
// ---------------------------------------------------------------------------
constexpr int kScan1dThreads = 1024;
constexpr int kScan1dPer = 16;
constexpr int64_t kScan1dChunk = (int64_t)kScan1dThreads * kScan1dPer;

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *s_w, int32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t inc = wave_inclusive_scan(v);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int32_t w = lane < kScan1dThreads / 64 ? s_w[lane] : 0;
        const int32_t sw = wave_inclusive_scan(w);
        if (lane < kScan1dThreads / 64) s_w[lane] = sw - w;
        if (lane == 63) *total = sw;
    }
    __syncthreads();
    const int32_t r = s_w[wave] + inc - v;
    __syncthreads();
    return r;
}

// block_sums[b] = sum of chunk b (kScan1dChunk elements; each thread sums kScan1dPer consecutive ones)
__global__ __launch_bounds__(kScan1dThreads) void k_scan1d_reduce(const int32_t *__restrict__ a, int64_t n,
                                                                  int32_t *__restrict__ block_sums) {
    __shared__ int32_t s_w[kScan1dThreads / 64];
    __shared__ int32_t s_tot;
    const int64_t base = (int64_t)blockIdx.x * kScan1dChunk + (int64_t)threadIdx.x * kScan1dPer;
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScan1dPer; ++k) sum += base + k < n ? a[base + k] : 0;
    (void)block_exclusive_scan(sum, s_w, &s_tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_tot;
}

// One workgroup: exclusive scan of block_sums in place; *total = sum.
__global__ __launch_bounds__(kScan1dThreads) void k_scan1d_blocks(int32_t *__restrict__ block_sums, int64_t nb,
                                                                  int32_t *__restrict__ total) {
    __shared__ int32_t s_w[kScan1dThreads / 64];
    __shared__ int32_t s_tot;
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScan1dThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int32_t v = b < nb ? block_sums[b] : 0;
        const int32_t ex = block_exclusive_scan(v, s_w, &s_tot);
        if (b < nb) block_sums[b] = carry + ex;
        carry += s_tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScan1dThreads) void k_scan1d_apply(int32_t *__restrict__ a, int64_t n,
                                                                 const int32_t *__restrict__ block_sums) {
    __shared__ int32_t s_w[kScan1dThreads / 64];
    __shared__ int32_t s_tot;
    const int64_t base = (int64_t)blockIdx.x * kScan1dChunk + (int64_t)threadIdx.x * kScan1dPer;
    int32_t v[kScan1dPer];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScan1dPer; ++k) {
        v[k] = base + k < n ? a[base + k] : 0;
        sum += v[k];
    }
    int32_t run = block_sums[blockIdx.x] + block_exclusive_scan(sum, s_w, &s_tot);
#pragma unroll
    for (int k = 0; k < kScan1dPer; ++k) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
}

size_t scan_1d_scratch_bytes(int64_t n) {
    return (size_t)((n + kScan1dChunk - 1) / kScan1dChunk + 1) * sizeof(int32_t);
}

dpg_status launch_scan_1d(dpg_ctx *ctx, int32_t *a, int64_t n, int32_t *scratch, int32_t *total,
                          hipStream_t stream) {
    if (n <= 0) return launch_fill_i32(ctx, total, 1, 0, stream);
    const int64_t nb = (n + kScan1dChunk - 1) / kScan1dChunk;
    ProfScope prof(ctx, K_SCAN_CHUNKS, 12.0 * n, stream);
    hipLaunchKernelGGL(k_scan1d_reduce, dim3((unsigned)nb), dim3(kScan1dThreads), 0, stream, a, n, scratch);
    DPG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan1d_blocks, dim3(1), dim3(kScan1dThreads), 0, stream, scratch, nb, total);
    DPG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan1d_apply, dim3((unsigned)nb), dim3(kScan1dThreads), 0, stream, a, n, scratch);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

// The whole column scan in one workgroup, for count matrices of at most
// kScanSmallMax entries (lists of a few million rids or fewer), where the
// four-kernel form costs more in launches than in work: the matrix is read
// into LDS in column-major order (rows are read whole, so the loads stay
// coalesced), scanned there as one array, and written back.
constexpr int64_t kScanSmallMax = 15360;  // 60 KiB of LDS

__global__ __launch_bounds__(kScan1dThreads) void k_scan_small(int32_t *__restrict__ cnt, int nT, int B,
                                                               int32_t *__restrict__ bucket_off,
                                                               int32_t *__restrict__ item_off, int chunk,
                                                               const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    extern __shared__ int32_t s_col[];  // nT * B entries, s_col[b * nT + t] = cnt[t][b]
    __shared__ int32_t s_w[kScan1dThreads / 64];
    __shared__ int32_t s_total, s_part, s_carry;
    const int n = nT * B;
    for (int k = threadIdx.x; k < n; k += kScan1dThreads) {
        const int t = k / B, b = k - t * B;
        s_col[b * nT + t] = cnt[k];
    }
    __syncthreads();
    // every thread scans one contiguous segment of the column-major array
    const int per = (n + kScan1dThreads - 1) / kScan1dThreads;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    int32_t sum = 0;
    for (int k = lo; k < hi; ++k) sum += s_col[k];
    int32_t run = block_exclusive_scan(sum, s_w, &s_total);
    for (int k = lo; k < hi; ++k) {
        const int32_t v = s_col[k];
        s_col[k] = run;
        run += v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += kScan1dThreads) {
        const int t = k / B, b = k - t * B;
        cnt[k] = s_col[b * nT + t];
    }
    const int32_t total = s_total;
    if (threadIdx.x == 0) {
        bucket_off[B] = total;
        s_carry = 0;
    }
    for (int b = threadIdx.x; b < B; b += kScan1dThreads) bucket_off[b] = s_col[b * nT];
    if (!item_off) return;
    // item_off[b] = sum over b' < b of ceil(elements of bucket b' / chunk)
    __syncthreads();
    for (int b0 = 0; b0 < B; b0 += kScan1dThreads) {
        const int b = b0 + threadIdx.x;
        int32_t u = 0;
        if (b < B) {
            const int32_t len = (b + 1 < B ? s_col[(b + 1) * nT] : total) - s_col[b * nT];
            u = (len + chunk - 1) / chunk;
        }
        const int32_t ex = block_exclusive_scan(u, s_w, &s_part);
        const int32_t carry = s_carry;
        if (b < B) item_off[b] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + s_part;
        __syncthreads();
    }
    if (threadIdx.x == 0) item_off[B] = s_carry;
}

dpg_status launch_column_scan(dpg_ctx *ctx, int32_t *cnt, int64_t nT, int B, int32_t *csum, int64_t nC,
                              int32_t *total, int32_t *bucket_off, int32_t *item_off, int item_chunk,
                              hipStream_t stream, const int32_t *gate) {
    if (nT * (int64_t)B <= kScanSmallMax) {
        // one workgroup; chunk sums and column totals are not needed
        ProfScope prof(ctx, K_SCAN_SMALL, 8.0 * nT * B + 4.0 * B, stream);
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScan1dThreads), (size_t)nT * B * sizeof(int32_t), stream, cnt,
                           (int)nT, B, bucket_off, item_off, item_chunk > 0 ? item_chunk : 1, gate);
        DPG_HIP(hipGetLastError());
        return DPG_OK;
    }
    const unsigned gy = (unsigned)((B + 255) / 256);
    {
        ProfScope prof(ctx, K_SCAN_CHUNKS, 4.0 * nT * B + 4.0 * nC * B, stream);
        hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nC, gy), dim3(256), 0, stream, cnt, nT, B, csum, nC, gate);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_COLS, 8.0 * nC * B, stream);
        hipLaunchKernelGGL(k_scan_cols, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, stream, csum, nC, B, total, gate);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_BASE, 12.0 * B, stream);
        hipLaunchKernelGGL(k_scan_base, dim3(1), dim3(1024), 0, stream, total, B, bucket_off, item_off, item_chunk,
                           gate);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_SCAN_APPLY, 8.0 * nT * B + 4.0 * nC * B, stream);
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nC, gy), dim3(256), 0, stream, cnt, nT, B, csum, nC,
                           bucket_off, gate);
        DPG_HIP(hipGetLastError());
    }
    return DPG_OK;
}

}  // namespace dpg
