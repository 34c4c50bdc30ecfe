// Batched execution of many retrieval / join requests of uneven size.
//
// Direct-algorithm work of every request in the batch (retrievals planned as
// direct, and fact-order joins planned as direct) runs in ONE launch of the
// persistent kernel k_batch: a fixed grid of workgroups pulls work items from
// a device queue (one atomic counter); an item is a tile of output rows of one
// request.  Each output row is A[ia] || B[ib] (retrieval: src[rid], no B;
// fact-order join: fact[i] || dim[fk_i]), so one kernel serves both kinds and
// every record size.  Every workgroup leaves the loop once the queue is
// exhausted; nothing waits on the host.
//
// Requests planned as DPG, and dimension-order joins, run their own phase
// sequence (the same code as dpg_retrieve / dpg_fk_join) in the same stream,
// so every request's output is bit-identical alone and in any batch.
//
// The batch header (item count, descriptor count) lives in device memory, so a
// captured graph of [reset queue, k_batch] can be replayed with new requests:
// only the descriptor upload changes (dpg_batch_graph_*).
#include <algorithm>
#include <cstring>
#include <vector>

#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

struct BatchDesc {
    const uint32_t *a;      // retrieval source records / fact rows
    const int32_t *idx_a;   // rids (retrieval) or null (row i of A)
    const uint32_t *b;      // dimension rows (join) or null
    uint32_t *out;
    int64_t lim_a, lim_b;   // row counts of A and B (indices outside read row 0)
    int64_t n_rows;         // output rows
    int64_t item_start;     // first work item of this request
    int32_t wa, wb;         // dwords taken from A and from B per output row
    int32_t fk_word;        // word of the A row holding the foreign key (join)
    int32_t tile_rows;      // output rows per work item
    uint32_t magic;         // ceil(2^32 / ((wa + wb) / vec)) for the row division
    int32_t request;        // index in the caller's request array
    int32_t vec;            // dwords per access: 4 when rows and pointers are 16-byte aligned, else 1
    int32_t nt;             // nontemporal output stores
};

struct BatchHeader {
    int64_t total_items;
    int32_t n_desc;
    int32_t pad;
};

constexpr int kBatchThreads = 256;
constexpr int kBatchPer = 16;
constexpr int kBatchMaxTileRows = 2048;
constexpr int kBatchItemWords = 16384;  // ~64 KiB of output per work item

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Descriptor pointers are read from memory, so the compiler sees them as
// generic (flat) addresses; flat loads also wait on the LDS counter and were
// issued one at a time.  All of them point at device memory.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *as_global(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Copy the item's rows: element e of the flattened (row, element) space with
// VEC dwords per element.  Loads carry no branches (lanes past the item repeat
// its last element), so all kBatchPer of a lane are in flight together.
template <typename E, bool NT>
__device__ __forceinline__ void batch_copy(const BatchDesc &d, const int32_t *s_ia, const int32_t *s_ib, int rows,
                                           int64_t row0) {
    constexpr int VEC = sizeof(E) / 4;
    const int wa = d.wa / VEC, wb = d.wb / VEC, W = wa + wb;
    const auto *A = as_global((const E *)d.a);
    const auto *B = as_global((const E *)(d.b ? d.b : d.a));
    auto *o = as_global((E *)d.out + row0 * W);
    const int total = rows * W;
    for (int e0 = 0; e0 < total; e0 += kBatchThreads * kBatchPer) {
        int64_t off[kBatchPer];
        bool in_a[kBatchPer];
#pragma unroll
        for (int k = 0; k < kBatchPer; ++k) {
            const int e = min(e0 + (int)threadIdx.x + k * kBatchThreads, total - 1);
            const int j = W == 1 ? e : (int)__umulhi((uint32_t)e, d.magic);
            const int w = e - j * W;
            in_a[k] = w < wa;
            off[k] = in_a[k] ? (int64_t)s_ia[j] * wa + w : (int64_t)s_ib[j] * wb + (w - wa);
        }
        E v[kBatchPer];
#pragma unroll
        for (int k = 0; k < kBatchPer; ++k) v[k] = (in_a[k] ? A : B)[off[k]];
#pragma unroll
        for (int k = 0; k < kBatchPer; ++k) {
            const int e = e0 + threadIdx.x + k * kBatchThreads;
            if (e < total) {
                if constexpr (NT) __builtin_nontemporal_store(v[k], o + e);
                else o[e] = v[k];
            }
        }
    }
}

__global__ __launch_bounds__(kBatchThreads) void k_batch(const BatchHeader *__restrict__ hdr,
                                                         const BatchDesc *__restrict__ descs,
                                                         uint32_t *__restrict__ queue,
                                                         uint32_t *__restrict__ done) {
    __shared__ int64_t s_item;
    __shared__ int s_req;
    __shared__ int32_t s_ia[kBatchMaxTileRows];
    __shared__ int32_t s_ib[kBatchMaxTileRows];
    const int64_t total_items = hdr->total_items;
    const int n_desc = hdr->n_desc;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t item = (int64_t)atomicAdd(queue, 1u);
            s_item = item;
            int r = -1;
            if (item < total_items) {
                int lo = 0, hi = n_desc - 1;  // last descriptor with item_start <= item
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (descs[mid].item_start <= item) lo = mid;
                    else hi = mid - 1;
                }
                r = lo;
            }
            s_req = r;
        }
        __syncthreads();
        const int64_t item = s_item;
        const int r = s_req;
        if (item >= total_items) break;  // queue exhausted: uniform exit
        const BatchDesc d = descs[r];
        const int64_t row0 = (item - d.item_start) * d.tile_rows;
        const int rows = (int)min((int64_t)d.tile_rows, d.n_rows - row0);
        {
            const auto *ga = as_global(d.a);
            const auto *gi = as_global(d.idx_a);
            const int64_t lim_a = d.lim_a, lim_b = d.lim_b;
            const int wa = d.wa, fk_word = d.fk_word;
            auto clamp_a = [=](int64_t ia) -> int64_t { return (ia >= 0 && ia < lim_a) ? ia : 0; };
            if (d.idx_a) stage_rows(s_ia, rows, [&](int j) { return (int32_t)clamp_a(gi[row0 + j]); });
            else stage_rows(s_ia, rows, [&](int j) { return (int32_t)clamp_a(row0 + j); });
            if (d.wb > 0) {
                auto fk = [=](int64_t ia) -> int32_t {
                    const int64_t ib = ga[ia * wa + fk_word];
                    return ib < lim_b ? (int32_t)ib : 0;
                };
                if (d.idx_a) stage_rows(s_ib, rows, [&](int j) { return fk(clamp_a(gi[row0 + j])); });
                else stage_rows(s_ib, rows, [&](int j) { return fk(clamp_a(row0 + j)); });
            }
        }
        __syncthreads();
        if (d.vec == 4) {
            if (d.nt) batch_copy<u32x4, true>(d, s_ia, s_ib, rows, row0);
            else batch_copy<u32x4, false>(d, s_ia, s_ib, rows, row0);
        } else {
            if (d.nt) batch_copy<uint32_t, true>(d, s_ia, s_ib, rows, row0);
            else batch_copy<uint32_t, false>(d, s_ia, s_ib, rows, row0);
        }
        if (threadIdx.x == 0 && done) atomicAdd(&done[d.request], 1u);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchRequestPlan {
    bool direct = false;    // handled by k_batch
    int64_t items = 0;      // work items (direct) ...
    size_t ws_bytes = 0;    // ... or workspace of its own phase sequence
};

// With `arena` non-null the output is not placed yet: it will live somewhere in
// [arena, arena + arena_bytes), so the inputs are checked against that whole
// range instead of against q.dst.
static dpg_status validate_request(const dpg_request &q, const void *arena = nullptr, size_t arena_bytes = 0) {
    const void *out = arena ? arena : q.dst;
    if (q.kind == DPG_REQ_RETRIEVE) {
        dpg_status st = validate_records(q.n_src, q.rec_bytes, q.src, q.n > 0);
        if (st != DPG_OK) return st;
        if (q.n < 0 || q.n > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
        if (q.n > 0 && (!q.rids || !out)) return DPG_ERR_INVALID_ARG;
        if (((uintptr_t)q.rids | (uintptr_t)out) % 4) return DPG_ERR_INVALID_ARG;
        if (q.n > 0 && q.n_src == 0) return DPG_ERR_RID_OUT_OF_RANGE;
        const size_t ob = arena ? arena_bytes : (size_t)q.n * q.rec_bytes;
        if (ranges_overlap(q.src, (size_t)q.n_src * q.rec_bytes, out, ob) ||
            ranges_overlap(q.rids, (size_t)q.n * 4, out, ob))
            return DPG_ERR_INVALID_ARG;
        return DPG_OK;
    }
    if (q.kind == DPG_REQ_FK_JOIN) {
        if (q.n < 0 || q.n > INT32_MAX - 1 || q.n_src < 0 || q.n_src > INT32_MAX) return DPG_ERR_INVALID_ARG;
        if (q.fact_bytes < 4 || q.fact_bytes > kMaxRecBytes || q.fact_bytes % 4) return DPG_ERR_INVALID_ARG;
        if (q.rec_bytes < 4 || q.rec_bytes > kMaxRecBytes || q.rec_bytes % 4) return DPG_ERR_INVALID_ARG;
        if (q.fk_offset < 0 || q.fk_offset % 4 || q.fk_offset + 4 > q.fact_bytes) return DPG_ERR_INVALID_ARG;
        if (q.order != DPG_JOIN_FACT_ORDER && q.order != DPG_JOIN_DIM_ORDER) return DPG_ERR_INVALID_ARG;
        if (q.n > 0 && (!q.fact || !out)) return DPG_ERR_INVALID_ARG;
        if (q.n_src > 0 && !q.src) return DPG_ERR_INVALID_ARG;
        if (((uintptr_t)q.fact | (uintptr_t)q.src | (uintptr_t)out) % 4) return DPG_ERR_INVALID_ARG;
        if (q.n > 0 && q.n_src == 0) return DPG_ERR_FK_OUT_OF_RANGE;
        const size_t ob = arena ? arena_bytes : (size_t)q.n * (q.fact_bytes + q.rec_bytes);
        if (ranges_overlap(out, ob, q.fact, (size_t)q.n * q.fact_bytes) ||
            ranges_overlap(out, ob, q.src, (size_t)q.n_src * q.rec_bytes))
            return DPG_ERR_INVALID_ARG;
        return DPG_OK;
    }
    return DPG_ERR_INVALID_ARG;
}

// Output rows per work item: about kBatchItemWords dwords, and a multiple of
// 256 / gcd(row bytes, 256) rows so that every item's output starts on a
// 256-byte boundary of the (256-byte aligned) output.
static int tile_rows_for(int words) {
    int rows = kBatchItemWords / words;
    if (rows < 1) rows = 1;
    if (rows > kBatchMaxTileRows) rows = kBatchMaxTileRows;
    int a = words * 4, b = 256;
    while (b) {
        const int t = a % b;
        a = b;
        b = t;
    }
    const int step = 256 / a;
    if (rows >= step) rows = rows / step * step;
    return rows;
}

static dpg_status plan_request(const dpg_ctx *ctx, const dpg_request &q, BatchRequestPlan *bp) {
    *bp = BatchRequestPlan();
    if (q.algo < DPG_ALGO_AUTO || q.algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    if (q.kind == DPG_REQ_RETRIEVE) {
        RetrievePlan rp;
        const dpg_status st = make_retrieve_plan(ctx, q.n_src, q.rec_bytes, q.n, q.algo, &rp);
        if (st != DPG_OK) return st;
        if (rp.algo == DPG_ALGO_DIRECT) {
            bp->direct = true;
            const int tr = tile_rows_for(q.rec_bytes / 4);
            bp->items = (q.n + tr - 1) / tr;
        } else {
            bp->ws_bytes = rp.workspace;
        }
        return DPG_OK;
    }
    const size_t ws = dpg_fk_join_workspace_bytes(ctx, q.n, q.fact_bytes, q.fk_offset, q.n_src, q.rec_bytes,
                                                  (dpg_join_order)q.order, (dpg_algo)q.algo);
    if (ws == 0) return DPG_ERR_INVALID_ARG;
    RetrievePlan rp;
    const dpg_status st = make_retrieve_plan(ctx, q.n_src, q.rec_bytes, q.n, q.algo, &rp);
    if (st != DPG_OK) return st;
    if (q.order == DPG_JOIN_FACT_ORDER && rp.algo == DPG_ALGO_DIRECT) {
        bp->direct = true;
        const int tr = tile_rows_for((q.fact_bytes + q.rec_bytes) / 4);
        bp->items = (q.n + tr - 1) / tr;
    } else {
        bp->ws_bytes = ws;
    }
    return DPG_OK;
}

struct BatchLayout {
    size_t off_hdr = 0, off_desc = 0, off_queue = 0, off_done = 0, off_req = 0;
    std::vector<size_t> req_off;  // per request: workspace of its own phase sequence
    size_t total = 0;
};

static BatchLayout batch_layout(int32_t n_desc_cap, int32_t n, const std::vector<BatchRequestPlan> &plans) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.off_hdr = take(sizeof(BatchHeader));
    L.off_queue = take(sizeof(uint32_t));
    L.off_desc = take((size_t)(n_desc_cap > 0 ? n_desc_cap : 1) * sizeof(BatchDesc));
    L.off_done = take((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    L.req_off.assign(plans.size(), 0);
    for (size_t i = 0; i < plans.size(); ++i)
        if (!plans[i].direct && plans[i].ws_bytes) L.req_off[i] = take(plans[i].ws_bytes);
    L.total = off;
    return L;
}

static dpg_status plan_batch(const dpg_ctx *ctx, const dpg_request *reqs, int32_t n,
                             std::vector<BatchRequestPlan> *plans) {
    if (n < 0 || (n > 0 && !reqs)) return DPG_ERR_INVALID_ARG;
    plans->resize(n);
    for (int32_t i = 0; i < n; ++i) {
        dpg_status st = validate_request(reqs[i]);
        if (st != DPG_OK) return st;
        st = plan_request(ctx, reqs[i], &(*plans)[i]);
        if (st != DPG_OK) return st;
    }
    return DPG_OK;
}

// Descriptors of the direct work, in request order.
static void build_descs(const dpg_request *reqs, int32_t n, const std::vector<BatchRequestPlan> &plans,
                        std::vector<BatchDesc> *descs, BatchHeader *hdr) {
    descs->clear();
    int64_t items = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!plans[i].direct || plans[i].items == 0) continue;
        const dpg_request &q = reqs[i];
        BatchDesc d{};
        if (q.kind == DPG_REQ_RETRIEVE) {
            d.a = (const uint32_t *)q.src;
            d.idx_a = q.rids;
            d.lim_a = q.n_src;
            d.wa = q.rec_bytes / 4;
            d.wb = 0;
        } else {
            d.a = (const uint32_t *)q.fact;
            d.idx_a = nullptr;
            d.lim_a = q.n;
            d.b = (const uint32_t *)q.src;
            d.lim_b = q.n_src;
            d.wa = q.fact_bytes / 4;
            d.wb = q.rec_bytes / 4;
            d.fk_word = q.fk_offset / 4;
        }
        d.out = (uint32_t *)q.dst;
        d.n_rows = q.n;
        d.tile_rows = tile_rows_for(d.wa + d.wb);
        const uintptr_t al = (uintptr_t)d.a | (uintptr_t)d.b | (uintptr_t)d.out;
        d.vec = (d.wa % 4 == 0 && d.wb % 4 == 0 && al % 16 == 0) ? 4 : 1;
        const uint64_t we = (uint64_t)(d.wa + d.wb) / (uint64_t)d.vec;
        d.magic = we > 1 ? (uint32_t)((0x100000000ull + we - 1) / we) : 0u;  // one element per row: j = e
        d.nt = (double)q.n * (d.wa + d.wb) * 4 > 256.0 * 1024 * 1024 ? 1 : 0;
        d.item_start = items;
        d.request = i;
        items += plans[i].items;
        descs->push_back(d);
    }
    hdr->total_items = items;
    hdr->n_desc = (int32_t)descs->size();
    hdr->pad = 0;
}

static double batch_bytes(const dpg_request *reqs, int32_t n, const std::vector<BatchRequestPlan> &plans) {
    double b = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!plans[i].direct) continue;
        const dpg_request &q = reqs[i];
        const double row = q.kind == DPG_REQ_RETRIEVE ? q.rec_bytes : q.fact_bytes + q.rec_bytes;
        b += (double)q.n * (2.0 * row + (q.kind == DPG_REQ_RETRIEVE ? 4.0 : 0.0));
    }
    return b;
}

static int batch_grid(const dpg_ctx *ctx) { return ctx->n_cu * 4; }

static dpg_status launch_batch_kernel(dpg_ctx *ctx, char *w, const BatchLayout &L, double bytes, bool with_done,
                                      hipStream_t stream) {
    dpg_status st = launch_fill_i32(ctx, (int32_t *)(w + L.off_queue), 1, 0, stream);
    if (st != DPG_OK) return st;
    ProfScope prof(ctx, K_BATCH, bytes, stream);
    hipLaunchKernelGGL(k_batch, dim3((unsigned)batch_grid(ctx)), dim3(kBatchThreads), 0, stream,
                       (const BatchHeader *)(w + L.off_hdr), (const BatchDesc *)(w + L.off_desc),
                       (uint32_t *)(w + L.off_queue), with_done ? (uint32_t *)(w + L.off_done) : nullptr);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

// The phase sequences of requests not handled by k_batch.
static dpg_status run_own_sequences(dpg_ctx *ctx, const dpg_request *reqs, int32_t n,
                                    const std::vector<BatchRequestPlan> &plans, char *w, const BatchLayout &L,
                                    hipStream_t stream) {
    for (int32_t i = 0; i < n; ++i) {
        if (plans[i].direct) continue;
        const dpg_request &q = reqs[i];
        dpg_status st;
        if (q.kind == DPG_REQ_RETRIEVE)
            st = dpg_retrieve(ctx, q.src, q.n_src, q.rec_bytes, q.rids, q.n, q.dst, w + L.req_off[i],
                              plans[i].ws_bytes, (dpg_algo)q.algo, 0, stream);
        else
            st = dpg_fk_join(ctx, q.fact, q.n, q.fact_bytes, q.fk_offset, q.src, q.n_src, q.rec_bytes, q.dst,
                             (dpg_join_order)q.order, w + L.req_off[i], plans[i].ws_bytes, (dpg_algo)q.algo, 0,
                             stream);
        if (st != DPG_OK) return st;
    }
    return DPG_OK;
}

dpg_status plan_batch_request(const dpg_ctx *ctx, const dpg_request &q, const void *arena, size_t arena_bytes,
                              bool *direct, size_t *own_ws) {
    dpg_status st = validate_request(q, arena, arena_bytes);
    if (st != DPG_OK) return st;
    BatchRequestPlan bp;
    st = plan_request(ctx, q, &bp);
    if (st != DPG_OK) return st;
    *direct = bp.direct;
    *own_ws = q.kind == DPG_REQ_RETRIEVE
                  ? dpg_retrieve_workspace_bytes(ctx, q.n_src, q.rec_bytes, q.n, (dpg_algo)q.algo)
                  : dpg_fk_join_workspace_bytes(ctx, q.n, q.fact_bytes, q.fk_offset, q.n_src, q.rec_bytes,
                                                (dpg_join_order)q.order, (dpg_algo)q.algo);
    return *own_ws > 0 || q.n == 0 ? DPG_OK : DPG_ERR_INVALID_ARG;
}

}  // namespace dpg

struct dpg_batch_graph {
    dpg_ctx *ctx = nullptr;
    int32_t max_requests = 0;
    char *ws = nullptr;
    dpg::BatchLayout layout;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // pinned staging of header + descriptors, so the upload is asynchronous;
    // `uploaded` marks when the previous upload has been consumed
    char *staging = nullptr;
    hipEvent_t uploaded = nullptr;
    bool upload_pending = false;
};

using namespace dpg;

extern "C" {

size_t dpg_batch_workspace_bytes(const dpg_ctx *ctx, const dpg_request *reqs, int32_t n) {
    std::vector<BatchRequestPlan> plans;
    if (plan_batch(ctx, reqs, n, &plans) != DPG_OK) return 0;
    return batch_layout(n, n, plans).total;
}

dpg_status dpg_batch_run(dpg_ctx *ctx, const dpg_request *reqs, int32_t n, void *workspace, size_t workspace_bytes,
                         hipStream_t stream) {
    std::vector<BatchRequestPlan> plans;
    dpg_status st = plan_batch(ctx, reqs, n, &plans);
    if (st != DPG_OK) return st;
    const BatchLayout L = batch_layout(n, n, plans);
    if (n > 0) {
        if (workspace_bytes < L.total) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    if (n == 0) return DPG_OK;
    char *w = (char *)workspace;
    std::vector<BatchDesc> descs;
    BatchHeader hdr;
    build_descs(reqs, n, plans, &descs, &hdr);
    if (hdr.total_items > 0) {
        // pageable source: the copy is staged before hipMemcpyAsync returns
        DPG_HIP(hipMemcpyAsync(w + L.off_hdr, &hdr, sizeof(hdr), hipMemcpyHostToDevice, stream));
        DPG_HIP(hipMemcpyAsync(w + L.off_desc, descs.data(), descs.size() * sizeof(BatchDesc),
                               hipMemcpyHostToDevice, stream));
        st = launch_batch_kernel(ctx, w, L, batch_bytes(reqs, n, plans), false, stream);
        if (st != DPG_OK) return st;
    }
    return run_own_sequences(ctx, reqs, n, plans, w, L, stream);
}

size_t dpg_batch_graph_workspace_bytes(const dpg_ctx *ctx, int32_t max_requests) {
    (void)ctx;
    if (max_requests < 1) return 0;
    std::vector<BatchRequestPlan> none;
    return batch_layout(max_requests, max_requests, none).total;
}

dpg_status dpg_batch_graph_create(dpg_ctx *ctx, int32_t max_requests, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream, dpg_batch_graph **out) {
    if (!ctx || !out || max_requests < 1) return DPG_ERR_INVALID_ARG;
    *out = nullptr;
    std::vector<BatchRequestPlan> none;
    const BatchLayout L = batch_layout(max_requests, max_requests, none);
    if (workspace_bytes < L.total) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    dpg_batch_graph *g = new dpg_batch_graph();
    g->ctx = ctx;
    g->max_requests = max_requests;
    g->ws = (char *)workspace;
    g->layout = L;
    if (hipHostMalloc((void **)&g->staging, L.off_desc - L.off_hdr + (size_t)max_requests * sizeof(BatchDesc),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&g->uploaded, hipEventDisableTiming) != hipSuccess) {
        if (g->staging) (void)hipHostFree(g->staging);
        delete g;
        return DPG_ERR_HIP;
    }
    // the copied span also covers the queue word between header and
    // descriptors (the graph zeroes it again before k_batch runs)
    std::memset(g->staging, 0, L.off_desc - L.off_hdr);
    // capture [reset queue, k_batch]; profiling events are not captured
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    dpg_status st = DPG_OK;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) st = DPG_ERR_HIP;
    if (st == DPG_OK) {
        st = launch_batch_kernel(ctx, g->ws, L, 0, false, stream);
        hipGraph_t graph = nullptr;
        if (hipStreamEndCapture(stream, &graph) != hipSuccess) st = DPG_ERR_HIP;
        g->graph = graph;
        if (st == DPG_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) st = DPG_ERR_HIP;
    }
    ctx->profiling = prof;
    if (st != DPG_OK) {
        dpg_batch_graph_destroy(g);
        return st;
    }
    *out = g;
    return DPG_OK;
}

dpg_status dpg_batch_graph_launch(dpg_batch_graph *g, const dpg_request *reqs, int32_t n, hipStream_t stream) {
    return dpg::batch_graph_launch(g, reqs, n, stream, true);
}

}  // extern "C"

namespace dpg {

dpg_status batch_graph_launch(dpg_batch_graph *g, const dpg_request *reqs, int32_t n, hipStream_t stream,
                              bool replay) {
    if (!g) return DPG_ERR_INVALID_ARG;
    if (n > g->max_requests) return DPG_ERR_INVALID_ARG;
    std::vector<BatchRequestPlan> plans;
    dpg_status st = plan_batch(g->ctx, reqs, n, &plans);
    if (st != DPG_OK) return st;
    for (int32_t i = 0; i < n; ++i)
        if (!plans[i].direct) return DPG_ERR_UNSUPPORTED;  // graph batches carry direct work only
    if (n == 0) return DPG_OK;
    std::vector<BatchDesc> descs;
    BatchHeader hdr;
    build_descs(reqs, n, plans, &descs, &hdr);
    // the staging buffer may still feed the previous upload
    if (g->upload_pending) DPG_HIP(hipEventSynchronize(g->uploaded));
    // header and descriptors keep their workspace layout: one contiguous copy
    const size_t span = g->layout.off_desc - g->layout.off_hdr + descs.size() * sizeof(BatchDesc);
    std::memcpy(g->staging, &hdr, sizeof(hdr));
    if (!descs.empty())
        std::memcpy(g->staging + (g->layout.off_desc - g->layout.off_hdr), descs.data(),
                    descs.size() * sizeof(BatchDesc));
    DPG_HIP(hipMemcpyAsync(g->ws + g->layout.off_hdr, g->staging, span, hipMemcpyHostToDevice, stream));
    DPG_HIP(hipEventRecord(g->uploaded, stream));
    g->upload_pending = true;
    if (!replay) return launch_batch_kernel(g->ctx, g->ws, g->layout, batch_bytes(reqs, n, plans), false, stream);
    ProfScope prof(g->ctx, K_BATCH, batch_bytes(reqs, n, plans), stream);
    DPG_HIP(hipGraphLaunch(g->exec, stream));
    return DPG_OK;
}

}  // namespace dpg

extern "C" {

void dpg_batch_graph_destroy(dpg_batch_graph *g) {
    if (!g) return;
    if (g->upload_pending) (void)hipEventSynchronize(g->uploaded);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->uploaded) (void)hipEventDestroy(g->uploaded);
    if (g->staging) (void)hipHostFree(g->staging);
    delete g;
}

}  // extern "C"
