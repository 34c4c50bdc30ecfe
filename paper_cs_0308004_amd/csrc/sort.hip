// Three-phase key-pointer sort (Section 3) with DPG as the copy phase:
//   1. extraction of key-pointer pairs: k_sort_extract packs the first four
//      key bytes big-endian into a uint32 (so integer order is byte-
//      lexicographic order) next to the record index;
//   2. sorting of the pairs: LSD radix sort, one stable 8-bit partition pass
//      per key byte (the count bucket sort of Section 5.3, once per digit),
//      then k_tie_fix puts every group of equal 4-byte prefixes in final
//      order by the remaining key bytes and the record index;
//   3. copying of the records in the sorted order: dpg_retrieve with the
//      sorted indices as rids (Section 2).
// Uniform 10-byte keys give groups of two or three at most, so the fix-up is
// cheap.  If some group is longer than kMaxTieGroup (low-entropy keys), the
// pairs are instead sorted over the whole key, 8 bytes at a time from the
// last chunk to the first, each chunk by stable passes.  Either way equal
// keys keep record-index order, so the result is unique: lexicographic by key
// bytes, then by index.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

// keys[j] = big-endian packing of nbytes (1..sizeof(K)) key bytes starting at
// byte koff of record r = order ? order[j] : j (zero-padded low bytes);
// idx[j] = r.
template <typename K>
__global__ __launch_bounds__(256) void k_sort_extract(const uint8_t *__restrict__ src, int rec_bytes, int64_t n,
                                                      const uint32_t *__restrict__ order, int koff, int nbytes,
                                                      K *__restrict__ keys, uint32_t *__restrict__ idx,
                                                      const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    const int a = koff & ~3, s = koff - a;
    const int need = (s + nbytes + 3) / 4;  // dwords overlapping the key bytes (1..3), all inside the record
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        const uint32_t r = order ? order[j] : (uint32_t)j;
        const uint32_t *w = (const uint32_t *)(src + (int64_t)r * rec_bytes + a);
        const uint32_t d0 = w[0];
        const uint32_t d1 = need > 1 ? w[1] : 0u;
        const uint32_t d2 = need > 2 ? w[2] : 0u;
        const uint64_t lo = (uint64_t)d0 | ((uint64_t)d1 << 32);
        uint64_t x = s ? ((lo >> (8 * s)) | ((uint64_t)d2 << (64 - 8 * s))) : lo;  // little-endian key bytes
        if (nbytes < 8) x &= (uint64_t(1) << (8 * nbytes)) - 1;
        if constexpr (sizeof(K) == 8) keys[j] = __builtin_bswap64(x);
        else keys[j] = __builtin_bswap32((uint32_t)x);
        idx[j] = r;
    }
}

// Grid of the extraction: a grid-stride loop over at most 64 workgroups per CU
// (a gated-off launch then costs few empty workgroups).
static unsigned extract_grid(const dpg_ctx *ctx, int64_t n) {
    const int64_t want = (n + 255) / 256, cap = (int64_t)ctx->n_cu * 64;
    return (unsigned)(want < cap ? (want > 0 ? want : 1) : cap);
}

// dst[j] = src[j] when *gate is non-zero.
__global__ __launch_bounds__(256) void k_gated_copy(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                                    int64_t n, const int32_t *__restrict__ gate) {
    if (*gate == 0) return;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) dst[j] = src[j];
}

constexpr int kMaxTieGroup = 64;

// Memcmp order of kbytes key bytes at koff of records x and y, then index.
// Bytes are compared eight at a time, all sixteen loads issued together.
__device__ __forceinline__ bool key_less(const uint8_t *__restrict__ src, int rec_bytes, int koff, int kbytes,
                                         uint32_t x, uint32_t y) {
    const uint8_t *a = src + (int64_t)x * rec_bytes + koff;
    const uint8_t *b = src + (int64_t)y * rec_bytes + koff;
    for (int t0 = 0; t0 < kbytes; t0 += 8) {
        uint8_t ca[8], cb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = min(t0 + u, kbytes - 1);
            ca[u] = a[t];
            cb[u] = b[t];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t0 + u < kbytes && ca[u] != cb[u]) return ca[u] < cb[u];
    }
    return x < y;
}

// Final order inside every group of equal prefixes of the sorted pairs: by
// the key bytes after the prefix (koff, kbytes), then by index.  The thread at
// a group's first element sorts it by insertion; a group longer than
// kMaxTieGroup sets *overflow instead and is left alone.
__global__ __launch_bounds__(256) void k_tie_fix(const uint32_t *__restrict__ keys, uint32_t *__restrict__ idx,
                                                 int64_t n, const uint8_t *__restrict__ src, int rec_bytes,
                                                 int koff, int kbytes, int32_t *overflow) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j + 1 >= n) return;
    const uint32_t k = keys[j];
    if (keys[j + 1] != k || (j > 0 && keys[j - 1] == k)) return;
    int64_t e = j + 2;
    while (e < n && e - j <= kMaxTieGroup && keys[e] == k) ++e;
    if (e - j > kMaxTieGroup) {
        atomicOr(overflow, 1);
        return;
    }
    for (int64_t a = j + 1; a < e; ++a) {
        const uint32_t x = idx[a];
        int64_t b = a - 1;
        while (b >= j && key_less(src, rec_bytes, koff, kbytes, x, idx[b])) {
            idx[b + 1] = idx[b];
            --b;
        }
        idx[b + 1] = x;
    }
}

struct SortPlan {
    int64_t n = 0;
    int rec_bytes = 0, key_offset = 0, key_bytes = 0;
    PartPlan part32, part64;  // passes over uint32 prefixes / over uint64 key chunks
    RetrievePlan ret;
    size_t off_keys[2] = {0, 0}, off_idx[2] = {0, 0}, off_part = 0, off_ret = 0, off_flag = 0;
    size_t workspace = 0;
};

static dpg_status make_sort_plan(const dpg_ctx *ctx, int64_t n, int32_t rec_bytes, int32_t key_offset,
                                 int32_t key_bytes, int algo, SortPlan *p) {
    if (n < 0 || n > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    if (rec_bytes < 4 || rec_bytes > kMaxRecBytes || rec_bytes % 4 != 0) return DPG_ERR_INVALID_ARG;
    if (key_offset < 0 || key_bytes < 1 || key_bytes > 64 || key_offset + key_bytes > rec_bytes)
        return DPG_ERR_INVALID_ARG;
    *p = SortPlan();
    p->n = n;
    p->rec_bytes = rec_bytes;
    p->key_offset = key_offset;
    p->key_bytes = key_bytes;
    const dpg_status st = make_retrieve_plan(ctx, n, rec_bytes, n, algo, &p->ret);
    if (st != DPG_OK) return st;
    p->part32 = plan_partition(n, 8, 4, true);
    p->part64 = plan_partition(n, 8, 8, true);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    p->off_flag = take(sizeof(int32_t));
    p->off_keys[0] = take((size_t)n * 8);
    p->off_keys[1] = take((size_t)n * 8);
    p->off_idx[0] = take((size_t)n * 4);
    p->off_idx[1] = take((size_t)n * 4);
    p->off_part = take(p->part32.workspace > p->part64.workspace ? p->part32.workspace : p->part64.workspace);
    p->off_ret = take(p->ret.workspace);
    p->workspace = off;
    return DPG_OK;
}

// Extract 8-byte chunk c of the key (in the order given by `order`, or record
// order) into buffer `cur`, then LSD-sort it by its bytes; returns the buffer
// holding the result.
static dpg_status sort_chunk(dpg_ctx *ctx, const SortPlan &p, const void *src, char *w, int c,
                             const uint32_t *order, int *cur, const int32_t *gate, hipStream_t stream) {
    const int nbytes = p.key_bytes - 8 * c < 8 ? p.key_bytes - 8 * c : 8;
    const int dst_buf = order && (const char *)order == w + p.off_idx[*cur] ? 1 - *cur : *cur;
    {
        ProfScope prof(ctx, K_SORT_EXTRACT, (double)p.n * (64.0 + 12.0 + (order ? 4.0 : 0.0)), stream);
        hipLaunchKernelGGL(k_sort_extract<uint64_t>, dim3(extract_grid(ctx, p.n)), dim3(256), 0, stream,
                           (const uint8_t *)src, p.rec_bytes, p.n, order, p.key_offset + 8 * c, nbytes,
                           (uint64_t *)(w + p.off_keys[dst_buf]), (uint32_t *)(w + p.off_idx[dst_buf]), gate);
        DPG_HIP(hipGetLastError());
    }
    *cur = dst_buf;
    for (int byte = nbytes - 1; byte >= 0; --byte) {
        const int other = 1 - *cur;
        const dpg_status st = launch_partition(ctx, p.part64, w + p.off_keys[*cur], (const uint32_t *)(w + p.off_idx[*cur]),
                                               w + p.off_keys[other], (uint32_t *)(w + p.off_idx[other]), nullptr,
                                               56 - 8 * byte, 0, w + p.off_part, stream, nullptr, nullptr, 0, true,
                                               false, 1, nullptr, 0, nullptr, gate);
        if (st != DPG_OK) return st;
        *cur = other;
    }
    return DPG_OK;
}

// Sort the pairs on the first four key bytes (stable passes, so equal
// prefixes stay in index order); returns the buffer holding the result.
static dpg_status sort_prefix(dpg_ctx *ctx, const SortPlan &p, const void *src, char *w, int *cur,
                              hipStream_t stream) {
    const int nbytes = p.key_bytes < 4 ? p.key_bytes : 4;
    {
        ProfScope prof(ctx, K_SORT_EXTRACT, (double)p.n * (64.0 + 8.0), stream);
        hipLaunchKernelGGL(k_sort_extract<uint32_t>, dim3(extract_grid(ctx, p.n)), dim3(256), 0, stream,
                           (const uint8_t *)src, p.rec_bytes, p.n, nullptr, p.key_offset, nbytes,
                           (uint32_t *)(w + p.off_keys[0]), (uint32_t *)(w + p.off_idx[0]), nullptr);
        DPG_HIP(hipGetLastError());
    }
    *cur = 0;
    // key byte b (0 = most significant) sits at bits 24 - 8b; padding bytes
    // past the key are zero and need no pass
    for (int byte = nbytes - 1; byte >= 0; --byte) {
        const int other = 1 - *cur;
        const dpg_status st = launch_partition(ctx, p.part32, w + p.off_keys[*cur], (const uint32_t *)(w + p.off_idx[*cur]),
                                               w + p.off_keys[other], (uint32_t *)(w + p.off_idx[other]), nullptr,
                                               24 - 8 * byte, 0, w + p.off_part, stream, nullptr);
        if (st != DPG_OK) return st;
        *cur = other;
    }
    return DPG_OK;
}

static dpg_status run_sort(dpg_ctx *ctx, const SortPlan &p, const void *src, void *dst, uint32_t *perm_out,
                           void *ws, hipStream_t stream, const uint32_t **sorted_keys) {
    if (p.n == 0) return DPG_OK;
    char *w = (char *)ws;
    int cur = 0;
    dpg_status st = sort_prefix(ctx, p, src, w, &cur, stream);
    if (st != DPG_OK) return st;
    // a key of at most 4 bytes is its whole prefix: the sorted prefixes are the sorted keys
    if (sorted_keys) *sorted_keys = p.key_bytes <= 4 ? (const uint32_t *)(w + p.off_keys[cur]) : nullptr;
    if (p.key_bytes > 4 && p.n > 1) {
        int32_t *flag = (int32_t *)(w + p.off_flag);
        st = launch_fill_i32(ctx, flag, 1, 0, stream);
        if (st != DPG_OK) return st;
        {
            ProfScope prof(ctx, K_TIE_FIX, 8.0 * p.n, stream);
            hipLaunchKernelGGL(k_tie_fix, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, stream,
                               (const uint32_t *)(w + p.off_keys[cur]), (uint32_t *)(w + p.off_idx[cur]), p.n,
                               (const uint8_t *)src, p.rec_bytes, p.key_offset + 4, p.key_bytes - 4, flag);
            DPG_HIP(hipGetLastError());
        }
        // Long runs of equal prefixes: full LSD over the key, last 8-byte
        // chunk first.  The passes are always enqueued; the fix-up's flag
        // gates them on the device (they return at once when it is 0), and
        // a gated copy brings their result into the fix-up's buffer, so the
        // call never waits on the host.
        const int fixed = cur;
        const int chunks = (p.key_bytes + 7) / 8;
        int fb = 0;
        for (int c = chunks - 1; c >= 0; --c) {
            const uint32_t *order = c == chunks - 1 ? nullptr : (const uint32_t *)(w + p.off_idx[fb]);
            st = sort_chunk(ctx, p, src, w, c, order, &fb, flag, stream);
            if (st != DPG_OK) return st;
        }
        if (fb != fixed) {
            hipLaunchKernelGGL(k_gated_copy, dim3(extract_grid(ctx, p.n)), dim3(256), 0, stream,
                               (const uint32_t *)(w + p.off_idx[fb]), (uint32_t *)(w + p.off_idx[fixed]), p.n, flag);
            DPG_HIP(hipGetLastError());
        }
    }
    const int32_t *sorted = (const int32_t *)(w + p.off_idx[cur]);
    if (perm_out)
        DPG_HIP(hipMemcpyAsync(perm_out, sorted, (size_t)p.n * 4, hipMemcpyDeviceToDevice, stream));
    return run_retrieve(ctx, p.ret, src, sorted, dst, w + p.off_ret, stream);
}

}  // namespace dpg

using namespace dpg;

extern "C" size_t dpg_sort_workspace_bytes(const dpg_ctx *ctx, int64_t n, int32_t rec_bytes, int32_t key_offset,
                                           int32_t key_bytes, dpg_algo algo) {
    SortPlan p;
    if (make_sort_plan(ctx, n, rec_bytes, key_offset, key_bytes, algo, &p) != DPG_OK) return 0;
    return p.workspace;
}

namespace dpg {

dpg_status sort_records(dpg_ctx *ctx, const void *src, int64_t n, int32_t rec_bytes, int32_t key_offset,
                        int32_t key_bytes, void *dst, uint32_t *perm_out, void *workspace, size_t workspace_bytes,
                        int algo, hipStream_t stream, const uint32_t **sorted_keys) {
    if (sorted_keys) *sorted_keys = nullptr;
    SortPlan p;
    dpg_status st = make_sort_plan(ctx, n, rec_bytes, key_offset, key_bytes, algo, &p);
    if (st != DPG_OK) return st;
    st = validate_records(n, rec_bytes, src, n > 0);
    if (st != DPG_OK) return st;
    if (n > 0 && !dst) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)dst) % 4 != 0 || ((uintptr_t)perm_out) % 4 != 0) return DPG_ERR_INVALID_ARG;
    const size_t rb = (size_t)n * rec_bytes;
    if (ranges_overlap(src, rb, dst, rb) || ranges_overlap(perm_out, (size_t)n * 4, dst, rb) ||
        ranges_overlap(perm_out, (size_t)n * 4, src, rb))
        return DPG_ERR_INVALID_ARG;
    if (n > 0) {
        if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!workspace || ((uintptr_t)workspace) % kAlign != 0) return DPG_ERR_INVALID_ARG;
        if (ranges_overlap(workspace, p.workspace, src, rb) || ranges_overlap(workspace, p.workspace, dst, rb) ||
            ranges_overlap(workspace, p.workspace, perm_out, (size_t)n * 4))
            return DPG_ERR_INVALID_ARG;
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    return run_sort(ctx, p, src, dst, perm_out, workspace, stream, sorted_keys);
}

}  // namespace dpg

extern "C" dpg_status dpg_sort_records(dpg_ctx *ctx, const void *src, int64_t n, int32_t rec_bytes,
                                       int32_t key_offset, int32_t key_bytes, void *dst, uint32_t *perm_out,
                                       void *workspace, size_t workspace_bytes, dpg_algo algo, hipStream_t stream) {
    return sort_records(ctx, src, n, rec_bytes, key_offset, key_bytes, dst, perm_out, workspace, workspace_bytes,
                        algo, stream, nullptr);
}
