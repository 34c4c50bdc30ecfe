// Sort-merge join with DPG sort (Section 4.1): both relations are sorted on
// the join key by the key-pointer sort of Section 3 (dpg_sort_records, whose
// copy phase is DPG or the direct gather), then merged.
//
// Merge: every sorted R row a finds the range [lo_a, lo_a + cnt_a) of sorted S
// rows with its key by binary search over the S keys (packed big-endian into
// uint64, so integer order is memcmp order); an exclusive scan of cnt gives
// each R row its first output row; each output row o then finds its R row a
// (binary search over the scanned offsets) and its S row lo_a + o - off_a.
// Output rows are written in order, so the writes are coalesced, and the
// sorted rows are read nearly in order.  The result order is (key, R index,
// S index) because both sorts are stable.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

constexpr int kSmjMaxKeyBytes = 8;

// keys[i] = big-endian value of the kb key bytes at koff of row i.
__global__ __launch_bounds__(256) void k_smj_keys(const uint8_t *__restrict__ rows, int64_t n, int rec, int koff,
                                                  int kb, uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint8_t *p = rows + i * rec + koff;
    uint64_t x = 0;
    for (int t = 0; t < kb; ++t) x = (x << 8) | p[t];
    keys[i] = x;
}

// Rows per workgroup of k_smj_ranges, and the S keys it can stage in LDS.
constexpr int kSmjRangeRows = 1024;
constexpr int kSmjRangeCap = 4096;

// First index in [l, h) whose key is > k (upper) or >= k (lower), keys sorted.
template <typename K, bool UPPER>
__device__ __forceinline__ int64_t smj_bound(const K *keys, int64_t l, int64_t h, K k) {
    while (l < h) {
        const int64_t m = (l + h) >> 1;
        const K v = keys[m];
        if (UPPER ? v <= k : v < k) l = m + 1;
        else h = m;
    }
    return l;
}

// lo[a], cnt[a]: the S rows whose key equals R row a's; total += sum of cnt.
// R rows [a0, a1) of one workgroup have keys in [kr[a0], kr[a1-1]], so their
// S ranges lie inside [lower(kr[a0]), upper(kr[a1-1])): two global searches
// per workgroup bound them, and when that span is short it is staged in LDS
// and every row searches there.
template <typename K>
__global__ __launch_bounds__(256) void k_smj_ranges(const K *__restrict__ kr, int64_t nr, const K *__restrict__ ks,
                                                    int64_t ns, int32_t *__restrict__ lo, int32_t *__restrict__ cnt,
                                                    unsigned long long *__restrict__ total) {
    __shared__ K s_key[kSmjRangeCap];
    __shared__ int64_t s_lim[2];
    __shared__ unsigned long long s_sum[4];
    const int64_t a0 = (int64_t)blockIdx.x * kSmjRangeRows;
    const int64_t a1 = min(a0 + (int64_t)kSmjRangeRows, nr);
    if (threadIdx.x == 0) s_lim[0] = smj_bound<K, false>(ks, 0, ns, kr[a0]);
    if (threadIdx.x == 64) s_lim[1] = smj_bound<K, true>(ks, 0, ns, kr[a1 - 1]);
    __syncthreads();
    const int64_t s0 = s_lim[0], s1 = s_lim[1];
    const bool staged = s1 - s0 <= kSmjRangeCap;
    if (staged)
        for (int i = threadIdx.x; i < (int)(s1 - s0); i += 256) s_key[i] = ks[s0 + i];
    __syncthreads();
    unsigned long long sum = 0;
    for (int r = 0; r < kSmjRangeRows / 256; ++r) {
        const int64_t a = a0 + threadIdx.x + r * 256;
        if (a >= a1) break;
        const K k = kr[a];
        int64_t l, u;
        if (staged) {
            l = s0 + smj_bound<K, false>(s_key, 0, s1 - s0, k);
            u = s0 + smj_bound<K, true>(s_key, l - s0, s1 - s0, k);
        } else {
            l = smj_bound<K, false>(ks, s0, s1, k);
            u = smj_bound<K, true>(ks, l, s1, k);
        }
        lo[a] = (int32_t)l;
        cnt[a] = (int32_t)(u - l);
        sum += (unsigned long long)(u - l);
    }
    // block sum, one atomic per block
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long b = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        if (b) atomicAdd(total, b);
    }
}

// Last index in [l, h) with off[i] <= o (off nondecreasing, off[l] <= o).
__device__ __forceinline__ int64_t smj_row_of(const int32_t *off, int64_t l, int64_t h, int64_t o) {
    while (h - l > 1) {
        const int64_t m = (l + h) >> 1;
        if ((int64_t)off[m] <= o) l = m;
        else h = m;
    }
    return l;
}

// Output rows [t*tile, ...): row o = R[a] || S[lo[a] + o - off[a]], a the last R
// row with off[a] <= o (it has cnt[a] > 0).  The R rows of one tile lie
// between those of its first and last output rows; when that span is short,
// its offsets and range starts are staged in LDS.  Rows are copied as dwords
// flattened over the workgroup, every load issued before the stores.
constexpr int kSmjPer = 32;
constexpr int kSmjEmitCap = 2048;

// Result rows [0, n_out) in tiles of `tile` rows, grid-stride over the
// tiles.  n_dev (may be null): the row count is min(*n_dev, n_out), read on
// the device (the caller then sizes n_out by the output's capacity).
__global__ __launch_bounds__(256) void k_smj_emit(const uint32_t *__restrict__ R, int wr, int64_t nr,
                                                  const uint32_t *__restrict__ S, int ws, int64_t ns,
                                                  const int32_t *__restrict__ off, const int32_t *__restrict__ lo,
                                                  uint32_t *__restrict__ out, int64_t n_out, int tile,
                                                  uint32_t magic, const unsigned long long *__restrict__ n_dev) {
    extern __shared__ int32_t s_ab[];
    __shared__ int32_t s_off[kSmjEmitCap], s_lo[kSmjEmitCap];
    __shared__ int64_t s_span[2];
    int32_t *s_a = s_ab, *s_b = s_ab + tile;
    if (n_dev) n_out = min(n_out, (int64_t)*n_dev);
    for (int64_t t = blockIdx.x; t * tile < n_out; t += gridDim.x) {
        const int64_t base = t * tile;
        const int cnt = (int)min((int64_t)tile, n_out - base);
        if (threadIdx.x == 0) s_span[0] = smj_row_of(off, 0, nr, base);
        if (threadIdx.x == 64) s_span[1] = smj_row_of(off, 0, nr, base + cnt - 1);
        __syncthreads();
        const int64_t af = s_span[0], span = s_span[1] - af + 1;
        const bool staged = span <= kSmjEmitCap;
        if (staged)
            for (int i = threadIdx.x; i < (int)span; i += 256) {
                s_off[i] = off[af + i];
                s_lo[i] = lo[af + i];
            }
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += 256) {
            const int64_t o = base + j;
            int64_t a, first, start;
            if (staged) {
                const int i = (int)smj_row_of(s_off, 0, span, o);
                a = af + i;
                first = s_off[i];
                start = s_lo[i];
            } else {
                a = smj_row_of(off, af, af + span, o);
                first = off[a];
                start = lo[a];
            }
            int64_t b = start + (o - first);
            b = (b >= 0 && b < ns) ? b : 0;
            s_a[j] = (int32_t)a;
            s_b[j] = (int32_t)b;
        }
        __syncthreads();
        const int W = wr + ws;
        const int total = cnt * W;
        int64_t src[kSmjPer];
        bool from_r[kSmjPer];
    #pragma unroll
        for (int k = 0; k < kSmjPer; ++k) {
            const int e = min((int)threadIdx.x + k * 256, total - 1);
            const int j = (int)__umulhi((uint32_t)e, magic);
            const int w = e - j * W;
            from_r[k] = w < wr;
            src[k] = from_r[k] ? (int64_t)s_a[j] * wr + w : (int64_t)s_b[j] * ws + (w - wr);
        }
        uint32_t v[kSmjPer];
    #pragma unroll
        for (int k = 0; k < kSmjPer; ++k) v[k] = from_r[k] ? R[src[k]] : S[src[k]];
        uint32_t *o = out + base * W;
    #pragma unroll
        for (int k = 0; k < kSmjPer; ++k) {
            const int e = threadIdx.x + k * 256;
            if (e < total) __builtin_nontemporal_store(v[k], o + e);
        }
        __syncthreads();  // the tile's LDS tables are reused by the next tile
    }
}

struct SmjPlan {
    int64_t nr = 0, ns = 0;
    int rec_r = 0, rec_s = 0, koff_r = 0, koff_s = 0, kb = 0, algo = 0;
    size_t sort_ws = 0;
    size_t off_r = 0, off_s = 0, off_sort = 0, off_kr = 0, off_ks = 0, off_lo = 0, off_cnt = 0, off_scan = 0,
           off_total = 0, workspace = 0;
};

static dpg_status make_smj_plan(const dpg_ctx *ctx, int64_t nr, int32_t rec_r, int32_t koff_r, int64_t ns,
                                int32_t rec_s, int32_t koff_s, int32_t kb, int algo, SmjPlan *p) {
    if (nr < 0 || nr > INT32_MAX - 1 || ns < 0 || ns > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    if (rec_r < 4 || rec_r > kMaxRecBytes || rec_r % 4 || rec_s < 4 || rec_s > kMaxRecBytes || rec_s % 4)
        return DPG_ERR_INVALID_ARG;
    if (kb < 1 || kb > kSmjMaxKeyBytes || koff_r < 0 || koff_s < 0 || koff_r + kb > rec_r || koff_s + kb > rec_s)
        return DPG_ERR_INVALID_ARG;
    if (algo < DPG_ALGO_AUTO || algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    *p = SmjPlan();
    p->nr = nr;
    p->ns = ns;
    p->rec_r = rec_r;
    p->rec_s = rec_s;
    p->koff_r = koff_r;
    p->koff_s = koff_s;
    p->kb = kb;
    p->algo = algo;
    const size_t wr = nr > 0 ? dpg_sort_workspace_bytes(ctx, nr, rec_r, koff_r, kb, (dpg_algo)algo) : 0;
    const size_t wsz = ns > 0 ? dpg_sort_workspace_bytes(ctx, ns, rec_s, koff_s, kb, (dpg_algo)algo) : 0;
    if ((nr > 0 && wr == 0) || (ns > 0 && wsz == 0)) return DPG_ERR_INVALID_ARG;
    p->sort_ws = wr > wsz ? wr : wsz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + (bytes > 0 ? bytes : 1));
        return at;
    };
    p->off_r = take((size_t)nr * rec_r);
    p->off_s = take((size_t)ns * rec_s);
    p->off_sort = take(p->sort_ws);
    p->off_kr = take((size_t)nr * 8);
    p->off_ks = take((size_t)ns * 8);
    p->off_lo = take((size_t)nr * 4);
    p->off_cnt = take((size_t)nr * 4);
    p->off_scan = take(scan_1d_scratch_bytes(nr));
    p->off_total = take(8);
    p->workspace = off;
    return DPG_OK;
}

}  // namespace dpg

using namespace dpg;

extern "C" {

size_t dpg_sort_merge_join_workspace_bytes(const dpg_ctx *ctx, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                                           int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes,
                                           dpg_algo sort_copy_algo) {
    SmjPlan p;
    if (make_smj_plan(ctx, n_r, rec_r, key_off_r, n_s, rec_s, key_off_s, key_bytes, sort_copy_algo, &p) != DPG_OK)
        return 0;
    return p.workspace;
}

}  // extern "C"

namespace dpg {

// dst = *src (one int64 on the device).
__global__ void k_smj_count_out(const unsigned long long *__restrict__ src, int64_t *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = (int64_t)*src;
}

// The join; rows_dev null: the host learns the row count (one stream
// synchronization) and rejects an output that is too small before writing any
// row; rows_dev non-null: never synchronizes, the count goes to *rows_dev and
// at most out_capacity rows are written.
static dpg_status smj_run(dpg_ctx *ctx, const void *r, int64_t n_r, int32_t rec_r, int32_t key_off_r, const void *s,
                          int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes, void *out,
                          int64_t out_capacity, int64_t *out_rows, int64_t *rows_dev, void *workspace,
                          size_t workspace_bytes, dpg_algo sort_copy_algo, hipStream_t stream) {
    SmjPlan p;
    dpg_status st = make_smj_plan(ctx, n_r, rec_r, key_off_r, n_s, rec_s, key_off_s, key_bytes, sort_copy_algo, &p);
    if (st != DPG_OK) return st;
    if ((!out_rows && !rows_dev) || out_capacity < 0) return DPG_ERR_INVALID_ARG;
    if (rows_dev && (((uintptr_t)rows_dev) % 8 || out_capacity >= INT32_MAX)) return DPG_ERR_INVALID_ARG;
    if ((n_r > 0 && (!r || ((uintptr_t)r) % 4)) || (n_s > 0 && (!s || ((uintptr_t)s) % 4))) return DPG_ERR_INVALID_ARG;
    if (out_capacity > 0 && (!out || ((uintptr_t)out) % 4)) return DPG_ERR_INVALID_ARG;
    if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    const size_t rb = (size_t)n_r * rec_r, sb = (size_t)n_s * rec_s;
    const size_t ob = (size_t)out_capacity * (size_t)(rec_r + rec_s);
    if (ranges_overlap(out, ob, r, rb) || ranges_overlap(out, ob, s, sb) ||
        ranges_overlap(out, ob, workspace, p.workspace) || ranges_overlap(workspace, p.workspace, r, rb) ||
        ranges_overlap(workspace, p.workspace, s, sb))
        return DPG_ERR_INVALID_ARG;
    if (rows_dev && (ranges_overlap(rows_dev, 8, out, ob) || ranges_overlap(rows_dev, 8, workspace, p.workspace)))
        return DPG_ERR_INVALID_ARG;
    if (!ctx) return DPG_ERR_INVALID_ARG;
    char *w = (char *)workspace;
    unsigned long long *total = (unsigned long long *)(w + p.off_total);
    if (out_rows) *out_rows = 0;
    if (n_r == 0 || n_s == 0) {
        if (!rows_dev) return DPG_OK;
        dpg_status st0 = launch_fill_i32(ctx, (int32_t *)total, 2, 0, stream);
        if (st0 != DPG_OK) return st0;
        hipLaunchKernelGGL(k_smj_count_out, dim3(1), dim3(64), 0, stream, total, rows_dev);
        DPG_HIP(hipGetLastError());
        return DPG_OK;
    }
    // 1. sort both relations on the join key (Section 3, DPG copy phase); a
    //    key of at most 4 bytes comes out of the sort as sorted uint32 values
    const bool key32 = key_bytes <= 4;
    void *kr = w + p.off_kr, *ks = w + p.off_ks;
    const uint32_t *sorted_keys = nullptr;
    st = sort_records(ctx, r, n_r, rec_r, key_off_r, key_bytes, w + p.off_r, nullptr, w + p.off_sort, p.sort_ws,
                      sort_copy_algo, stream, &sorted_keys);
    if (st != DPG_OK) return st;
    if (key32) {  // the S sort reuses the workspace: keep R's keys
        if (!sorted_keys) return DPG_ERR_UNSUPPORTED;
        DPG_HIP(hipMemcpyAsync(kr, sorted_keys, (size_t)n_r * 4, hipMemcpyDeviceToDevice, stream));
    }
    st = sort_records(ctx, s, n_s, rec_s, key_off_s, key_bytes, w + p.off_s, nullptr, w + p.off_sort, p.sort_ws,
                      sort_copy_algo, stream, &sorted_keys);
    if (st != DPG_OK) return st;
    if (key32) {
        if (!sorted_keys) return DPG_ERR_UNSUPPORTED;
        ks = (void *)sorted_keys;
    } else {
        ProfScope prof(ctx, K_SMJ_KEYS, (double)n_r * (64 + 8) + (double)n_s * (64 + 8), stream);
        hipLaunchKernelGGL(k_smj_keys, dim3((unsigned)((n_r + 255) / 256)), dim3(256), 0, stream,
                           (const uint8_t *)(w + p.off_r), n_r, rec_r, key_off_r, key_bytes, (uint64_t *)kr);
        DPG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_smj_keys, dim3((unsigned)((n_s + 255) / 256)), dim3(256), 0, stream,
                           (const uint8_t *)(w + p.off_s), n_s, rec_s, key_off_s, key_bytes, (uint64_t *)ks);
        DPG_HIP(hipGetLastError());
    }
    // 2. merge: key ranges and the number of result rows
    int32_t *lo = (int32_t *)(w + p.off_lo), *cnt = (int32_t *)(w + p.off_cnt);
    st = launch_fill_i32(ctx, (int32_t *)total, 2, 0, stream);
    if (st != DPG_OK) return st;
    {
        const unsigned grid = (unsigned)((n_r + kSmjRangeRows - 1) / kSmjRangeRows);
        const double kbytes = key32 ? 4.0 : 8.0;
        ProfScope prof(ctx, K_SMJ_RANGES, kbytes * (n_r + n_s) + 8.0 * n_r, stream);
        if (key32)
            hipLaunchKernelGGL(k_smj_ranges<uint32_t>, dim3(grid), dim3(256), 0, stream, (const uint32_t *)kr, n_r,
                               (const uint32_t *)ks, n_s, lo, cnt, total);
        else
            hipLaunchKernelGGL(k_smj_ranges<uint64_t>, dim3(grid), dim3(256), 0, stream, (const uint64_t *)kr, n_r,
                               (const uint64_t *)ks, n_s, lo, cnt, total);
        DPG_HIP(hipGetLastError());
    }
    unsigned long long n_out = 0;
    if (rows_dev) {
        hipLaunchKernelGGL(k_smj_count_out, dim3(1), dim3(64), 0, stream, total, rows_dev);
        DPG_HIP(hipGetLastError());
        n_out = (unsigned long long)out_capacity;  // the emit reads the count on the device
        if (n_out == 0) return DPG_OK;
    } else {
        DPG_HIP(hipMemcpyAsync(&n_out, total, sizeof(n_out), hipMemcpyDeviceToHost, stream));
        DPG_HIP(hipStreamSynchronize(stream));
        *out_rows = (int64_t)n_out;
        if ((int64_t)n_out > out_capacity) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (n_out >= (unsigned long long)INT32_MAX) return DPG_ERR_UNSUPPORTED;
        if (n_out == 0) return DPG_OK;
    }
    // 3. first result row of every R row, then the rows themselves
    st = launch_scan_1d(ctx, cnt, n_r, (int32_t *)(w + p.off_scan), (int32_t *)total, stream);
    if (st != DPG_OK) return st;
    const int wr = rec_r / 4, wsd = rec_s / 4, W = wr + wsd;
    // a multiple of 256 / gcd(row bytes, 256) rows per tile: every tile's
    // output starts on a 256-byte boundary (whole-line streaming stores)
    int g = 4 * W, b = 256;
    while (b) {
        const int t = g % b;
        g = b;
        b = t;
    }
    const int step = 256 / g;
    int tile = (256 * kSmjPer) / W;
    if (tile >= step) tile = tile / step * step;
    if (tile < 1) return DPG_ERR_UNSUPPORTED;
    const uint32_t magic = (uint32_t)((0x100000000ull + (uint64_t)W - 1) / (uint64_t)W);
    int64_t grid = ((int64_t)n_out + tile - 1) / tile;
    if (rows_dev && grid > (int64_t)ctx->n_cu * 16) grid = (int64_t)ctx->n_cu * 16;  // tiles grid-stride
    ProfScope prof(ctx, K_SMJ_EMIT, (double)n_out * (2.0 * (rec_r + rec_s) + 8.0), stream);
    hipLaunchKernelGGL(k_smj_emit, dim3((unsigned)grid), dim3(256), 2 * (size_t)tile * sizeof(int32_t), stream,
                       (const uint32_t *)(w + p.off_r), wr, n_r, (const uint32_t *)(w + p.off_s), wsd, n_s, cnt, lo,
                       (uint32_t *)out, (int64_t)n_out, tile, magic, rows_dev ? total : nullptr);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

}  // namespace dpg

extern "C" {

dpg_status dpg_sort_merge_join(dpg_ctx *ctx, const void *r, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                               const void *s, int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes,
                               void *out, int64_t out_capacity, int64_t *out_rows, void *workspace,
                               size_t workspace_bytes, dpg_algo sort_copy_algo, hipStream_t stream) {
    if (!out_rows) return DPG_ERR_INVALID_ARG;
    return smj_run(ctx, r, n_r, rec_r, key_off_r, s, n_s, rec_s, key_off_s, key_bytes, out, out_capacity, out_rows,
                   nullptr, workspace, workspace_bytes, sort_copy_algo, stream);
}

dpg_status dpg_sort_merge_join_async(dpg_ctx *ctx, const void *r, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                                     const void *s, int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes,
                                     void *out, int64_t out_capacity, int64_t *out_rows_dev, void *workspace,
                                     size_t workspace_bytes, dpg_algo sort_copy_algo, hipStream_t stream) {
    if (!out_rows_dev) return DPG_ERR_INVALID_ARG;
    return smj_run(ctx, r, n_r, rec_r, key_off_r, s, n_s, rec_s, key_off_s, key_bytes, out, out_capacity, nullptr,
                   out_rows_dev, workspace, workspace_bytes, sort_copy_algo, stream);
}

}  // extern "C"
