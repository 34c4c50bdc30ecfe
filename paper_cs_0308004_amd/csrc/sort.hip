// Three-phase key-pointer sort (Section 3) with DPG as the copy phase:
//   1. extraction of key-pointer pairs: k_sort_extract packs key bytes
//      big-endian into a uint64 (so integer order is byte-lexicographic order)
//      next to the record index;
//   2. sorting of the pairs: LSD radix sort, one stable 8-bit partition pass
//      per key byte (the count bucket sort of Section 5.3, once per digit);
//   3. copying of the records in the sorted order: dpg_retrieve with the
//      sorted indices as rids (Section 2).
// Keys longer than 8 bytes: the pairs are first sorted on bytes 0-7 only; if a
// device check finds two equal 8-byte prefixes (k_tie_check), the pairs are
// sorted again over the whole key, 8 bytes at a time from the last chunk to
// the first.  Either way equal keys keep record-index order, so the result is
// unique: lexicographic by key bytes, then by index.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

// keys[j] = big-endian packing of nbytes (1..8) key bytes starting at byte
// koff of record r = order ? order[j] : j (zero-padded low bytes); idx[j] = r.
__global__ __launch_bounds__(256) void k_sort_extract(const uint8_t *__restrict__ src, int rec_bytes, int64_t n,
                                                      const uint32_t *__restrict__ order, int koff, int nbytes,
                                                      uint64_t *__restrict__ keys, uint32_t *__restrict__ idx) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const uint32_t r = order ? order[j] : (uint32_t)j;
    const uint8_t *rec = src + (int64_t)r * rec_bytes;
    const int a = koff & ~3, s = koff - a;
    const uint32_t *w = (const uint32_t *)(rec + a);
    const int need = (s + nbytes + 3) / 4;  // dwords overlapping the key bytes (1..3), all inside the record
    const uint32_t d0 = w[0];
    const uint32_t d1 = need > 1 ? w[1] : 0u;
    const uint32_t d2 = need > 2 ? w[2] : 0u;
    const uint64_t lo = (uint64_t)d0 | ((uint64_t)d1 << 32);
    uint64_t x = s ? ((lo >> (8 * s)) | ((uint64_t)d2 << (64 - 8 * s))) : lo;  // little-endian key bytes
    if (nbytes < 8) x &= (uint64_t(1) << (8 * nbytes)) - 1;
    keys[j] = __builtin_bswap64(x);
    idx[j] = r;
}

// flag |= 1 if two neighbouring keys are equal.
__global__ __launch_bounds__(256) void k_tie_check(const uint64_t *__restrict__ keys, int64_t n, int32_t *flag) {
    int tie = 0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x + 1; j < n; j += (int64_t)gridDim.x * 256)
        tie |= keys[j] == keys[j - 1];
    if (__any(tie) && __lane_id() == 0) atomicOr(flag, 1);
}

struct SortPlan {
    int64_t n = 0;
    int rec_bytes = 0, key_offset = 0, key_bytes = 0;
    PartPlan part;
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
    p->part = plan_partition(n, 8, 8, true);
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
    p->off_part = take(p->part.workspace);
    p->off_ret = take(p->ret.workspace);
    p->workspace = off;
    return DPG_OK;
}

// Extract 8-byte chunk c of the key (in the order given by `order`, or record
// order) into buffer `cur`, then LSD-sort it by its bytes; returns the buffer
// holding the result.
static dpg_status sort_chunk(dpg_ctx *ctx, const SortPlan &p, const void *src, char *w, int c,
                             const uint32_t *order, int *cur, hipStream_t stream) {
    const int nbytes = p.key_bytes - 8 * c < 8 ? p.key_bytes - 8 * c : 8;
    const int dst_buf = order && (const char *)order == w + p.off_idx[*cur] ? 1 - *cur : *cur;
    {
        ProfScope prof(ctx, K_SORT_EXTRACT, (double)p.n * (64.0 + 12.0 + (order ? 4.0 : 0.0)), stream);
        hipLaunchKernelGGL(k_sort_extract, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, stream,
                           (const uint8_t *)src, p.rec_bytes, p.n, order, p.key_offset + 8 * c, nbytes,
                           (uint64_t *)(w + p.off_keys[dst_buf]), (uint32_t *)(w + p.off_idx[dst_buf]));
        DPG_HIP(hipGetLastError());
    }
    *cur = dst_buf;
    for (int byte = nbytes - 1; byte >= 0; --byte) {
        const int other = 1 - *cur;
        const dpg_status st = launch_partition(ctx, p.part, w + p.off_keys[*cur], (const uint32_t *)(w + p.off_idx[*cur]),
                                               w + p.off_keys[other], (uint32_t *)(w + p.off_idx[other]), nullptr,
                                               56 - 8 * byte, 0, w + p.off_part, stream, nullptr);
        if (st != DPG_OK) return st;
        *cur = other;
    }
    return DPG_OK;
}

static dpg_status run_sort(dpg_ctx *ctx, const SortPlan &p, const void *src, void *dst, uint32_t *perm_out,
                           void *ws, hipStream_t stream) {
    if (p.n == 0) return DPG_OK;
    char *w = (char *)ws;
    int cur = 0;
    dpg_status st = sort_chunk(ctx, p, src, w, 0, nullptr, &cur, stream);
    if (st != DPG_OK) return st;
    const int chunks = (p.key_bytes + 7) / 8;
    if (chunks > 1 && p.n > 1) {
        int32_t *flag = (int32_t *)(w + p.off_flag);
        st = launch_fill_i32(ctx, flag, 1, 0, stream);
        if (st != DPG_OK) return st;
        {
            ProfScope prof(ctx, K_TIE_MARK, 8.0 * p.n, stream);
            int64_t grid = (p.n + 255) / 256;
            if (grid > (int64_t)ctx->n_cu * 16) grid = (int64_t)ctx->n_cu * 16;
            hipLaunchKernelGGL(k_tie_check, dim3((unsigned)grid), dim3(256), 0, stream,
                               (const uint64_t *)(w + p.off_keys[cur]), p.n, flag);
            DPG_HIP(hipGetLastError());
        }
        DPG_HIP(hipMemcpyAsync(ctx->host_flag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        DPG_HIP(hipStreamSynchronize(stream));
        if (*ctx->host_flag) {
            // full LSD over the key, last 8-byte chunk first
            cur = 0;
            for (int c = chunks - 1; c >= 0; --c) {
                const uint32_t *order = c == chunks - 1 ? nullptr : (const uint32_t *)(w + p.off_idx[cur]);
                st = sort_chunk(ctx, p, src, w, c, order, &cur, stream);
                if (st != DPG_OK) return st;
            }
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

extern "C" dpg_status dpg_sort_records(dpg_ctx *ctx, const void *src, int64_t n, int32_t rec_bytes,
                                       int32_t key_offset, int32_t key_bytes, void *dst, uint32_t *perm_out,
                                       void *workspace, size_t workspace_bytes, dpg_algo algo, hipStream_t stream) {
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
    return run_sort(ctx, p, src, dst, perm_out, workspace, stream);
}
