// Foreign-key joins with DPG (Section 4.2.1).
//
// The fact relation (the paper's R) references the dimension relation (the
// indexed F) through a little-endian uint32 foreign key at fk_offset of each
// fact row.  Dimension ids are dense, so the index lookup that builds join
// triples (k, rid_R, rid_F) (Section 4.2.2) is the identity: rid_F = fk and
// rid_R = the fact row number.  A joined row is the fact row followed by the
// dimension row.
//
//   DPG-Move join (fact order): the rid pairs arrive in rid_R order, so the
//     dimension rows are moved in the order of the fk column by DPG -- no sort
//     and no hash.  Phase III is fused into k_join_assemble, which writes each
//     output row as fact[i] || INTERNAL[inv[i]].
//   DPG-Sort join (dimension order): the pairs (fk, i) are sorted by fk with a
//     stable count bucket sort, 8 bits per pass from the low bits up (Section
//     5.3 sorts rids on their low log N bits in two such passes); the fact rows
//     are moved into that order by DPG and the dimension rows are streamed in
//     fk order; Phase III is again fused into the assembly.
// The direct variants read dim[fk] (or fact[i]) in output order instead.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

constexpr double kJoinStreamingBytes = 256.0 * 1024 * 1024;

// fk[i] = word fk_word of fact row i; idx[i] = i (when idx is non-null).
__global__ __launch_bounds__(256) void k_join_extract(const uint32_t *__restrict__ fact, int64_t n, int wf,
                                                      int fk_word, uint32_t *__restrict__ fk,
                                                      uint32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    fk[i] = fact[i * wf + fk_word];
    if (idx) idx[i] = (uint32_t)i;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// out row i = A[ia] (wa dwords) || B[ib] (wb dwords), ia = idx_a ? idx_a[i] : i,
// ib = idx_b ? idx_b[i] : word fk_word of A row ia.  Indices outside their
// table are replaced by 0 (undefined result, never an out-of-bounds access).
// E is the access width: 16 bytes when both row sizes and all three base
// addresses are multiples of 16, else 4.  A tile of output rows is staged as
// (ia, ib) pairs in LDS, then its (row, element) pairs are flattened over the
// workgroup's lanes; every lane issues its PER loads without branches (lanes
// past the tile repeat its last element) before storing.
template <typename E, bool NT>
__global__ __launch_bounds__(256) void k_join_assemble(const uint32_t *__restrict__ A, int64_t lim_a,
                                                       const int32_t *__restrict__ idx_a,
                                                       const uint32_t *__restrict__ B, int64_t lim_b,
                                                       const int32_t *__restrict__ idx_b, int fk_word,
                                                       uint32_t *__restrict__ out, int64_t n, int wa_dw, int wb_dw,
                                                       uint32_t magic, int tile, int remap) {
    constexpr int VEC = sizeof(E) / 4;
    constexpr int PER = 32 / VEC;
    extern __shared__ int32_t s_ab[];
    int32_t *s_a = s_ab, *s_b = s_ab + tile;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x, remap);
    const int64_t base = t * tile;
    const int cnt = (int)min((int64_t)tile, n - base);
    // Stage (ia, ib) per row.  The branches on idx_a / idx_b are uniform and
    // sit outside the row loops.
    auto clamp_a = [=](int64_t ia) -> int64_t { return (ia >= 0 && ia < lim_a) ? ia : 0; };
    auto clamp_b = [=](int64_t ib) -> int32_t { return (ib >= 0 && ib < lim_b) ? (int32_t)ib : 0; };
    if (idx_a) stage_rows(s_a, cnt, [&](int j) { return (int32_t)clamp_a(idx_a[base + j]); });
    else stage_rows(s_a, cnt, [&](int j) { return (int32_t)clamp_a(base + j); });
    if (idx_b)
        stage_rows(s_b, cnt, [&](int j) { return clamp_b(idx_b[base + j]); });
    else if (idx_a)
        stage_rows(s_b, cnt, [&](int j) { return clamp_b(A[clamp_a(idx_a[base + j]) * wa_dw + fk_word]); });
    else
        stage_rows(s_b, cnt, [&](int j) { return clamp_b(A[clamp_a(base + j) * wa_dw + fk_word]); });
    __syncthreads();
    const int wa = wa_dw / VEC, wb = wb_dw / VEC, W = wa + wb;
    const int total = cnt * W;
    const E *Ae = (const E *)A, *Be = (const E *)B;
    const E *ptr[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = min(threadIdx.x + k * 256, total - 1);
        const int j = (int)__umulhi((uint32_t)e, magic);
        const int w = e - j * W;
        ptr[k] = w < wa ? Ae + ((int64_t)s_a[j] * wa + w) : Be + ((int64_t)s_b[j] * wb + (w - wa));
    }
    E v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) v[k] = *ptr[k];
    E *o = (E *)out + base * W;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        if (e < total) {
            if constexpr (NT) __builtin_nontemporal_store(v[k], o + e);
            else o[e] = v[k];
        }
    }
}

// Output rows per tile: a multiple of 256 / gcd(row bytes, 256), so that every
// tile's output starts on a 256-byte boundary (whole-line streaming stores).
static int join_tile_rows(int raw, int row_bytes) {
    int a = row_bytes, b = 256;
    while (b) {
        const int t = a % b;
        a = b;
        b = t;
    }
    const int step = 256 / a;
    const int rows = raw / step * step;
    return rows > 0 ? rows : raw;
}

template <typename E>
static dpg_status launch_assemble_t(const uint32_t *A, int64_t lim_a, const int32_t *idx_a, const uint32_t *B,
                                    int64_t lim_b, const int32_t *idx_b, int fk_word, uint32_t *out, int64_t n,
                                    int wa, int wb, int remap, hipStream_t stream) {
    constexpr int VEC = sizeof(E) / 4;
    const int W = (wa + wb) / VEC;  // elements per output row (>= 2)
    const int tile = join_tile_rows((256 * (32 / VEC)) / W, (wa + wb) * 4);
    if (tile < 1 || W < 2) return DPG_ERR_UNSUPPORTED;
    const uint32_t magic = (uint32_t)((0x100000000ull + (uint64_t)W - 1) / (uint64_t)W);
    const int64_t grid = (n + tile - 1) / tile;
    if (grid > 0x7fffffffLL) return DPG_ERR_UNSUPPORTED;
    const size_t lds = 2 * (size_t)tile * sizeof(int32_t);
    const bool nt = (double)n * (wa + wb) * 4 > kJoinStreamingBytes;
    if (nt)
        hipLaunchKernelGGL((k_join_assemble<E, true>), dim3((unsigned)grid), dim3(256), lds, stream, A, lim_a, idx_a,
                           B, lim_b, idx_b, fk_word, out, n, wa, wb, magic, tile, remap);
    else
        hipLaunchKernelGGL((k_join_assemble<E, false>), dim3((unsigned)grid), dim3(256), lds, stream, A, lim_a, idx_a,
                           B, lim_b, idx_b, fk_word, out, n, wa, wb, magic, tile, remap);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

static dpg_status launch_assemble(dpg_ctx *ctx, const void *A, int64_t lim_a, const int32_t *idx_a, const void *B,
                                  int64_t lim_b, const int32_t *idx_b, int fk_word, void *out, int64_t n, int a_bytes,
                                  int b_bytes, hipStream_t stream) {
    if (n <= 0) return DPG_OK;
    const double bytes = (double)n * (2.0 * (a_bytes + b_bytes) + (idx_a ? 4 : 0) + (idx_b ? 4 : 0));
    ProfScope prof(ctx, K_JOIN_ASSEMBLE, bytes, stream);
    const int wa = a_bytes / 4, wb = b_bytes / 4, remap = xcd_remap_flag(ctx);
    const uintptr_t al = (uintptr_t)A | (uintptr_t)B | (uintptr_t)out;
    if (a_bytes % 16 == 0 && b_bytes % 16 == 0 && al % 16 == 0)
        return launch_assemble_t<u32x4>((const uint32_t *)A, lim_a, idx_a, (const uint32_t *)B, lim_b, idx_b, fk_word,
                                        (uint32_t *)out, n, wa, wb, remap, stream);
    return launch_assemble_t<uint32_t>((const uint32_t *)A, lim_a, idx_a, (const uint32_t *)B, lim_b, idx_b, fk_word,
                                       (uint32_t *)out, n, wa, wb, remap, stream);
}

struct JoinPlan {
    int64_t n_fact = 0, n_dim = 0;
    int fact_bytes = 0, dim_bytes = 0, fk_offset = 0, order = 0, algo = 0;
    int fk_bits = 0, fk_passes = 0;
    RetrievePlan ret;
    PartPlan part;
    size_t off_flag = 0, off_fk = 0, off_keys[2] = {0, 0}, off_vals[2] = {0, 0}, off_part = 0, off_ret = 0;
    size_t workspace = 0;
};

static dpg_status make_join_plan(const dpg_ctx *ctx, int64_t n_fact, int32_t fact_bytes, int32_t fk_offset,
                                 int64_t n_dim, int32_t dim_bytes, int order, int algo, JoinPlan *p) {
    if (n_fact < 0 || n_fact > INT32_MAX - 1 || n_dim < 0 || n_dim > INT32_MAX) return DPG_ERR_INVALID_ARG;
    if (fact_bytes < 4 || fact_bytes > kMaxRecBytes || fact_bytes % 4) return DPG_ERR_INVALID_ARG;
    if (dim_bytes < 4 || dim_bytes > kMaxRecBytes || dim_bytes % 4) return DPG_ERR_INVALID_ARG;
    if (fk_offset < 0 || fk_offset % 4 || fk_offset + 4 > fact_bytes) return DPG_ERR_INVALID_ARG;
    if (order != DPG_JOIN_FACT_ORDER && order != DPG_JOIN_DIM_ORDER) return DPG_ERR_INVALID_ARG;
    if (algo < DPG_ALGO_AUTO || algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    *p = JoinPlan();
    p->n_fact = n_fact;
    p->n_dim = n_dim;
    p->fact_bytes = fact_bytes;
    p->dim_bytes = dim_bytes;
    p->fk_offset = fk_offset;
    p->order = order;
    // the moved relation: dimension rows (DPG-Move) or fact rows (DPG-Sort)
    const int64_t n_src = order == DPG_JOIN_FACT_ORDER ? n_dim : n_fact;
    const int rec = order == DPG_JOIN_FACT_ORDER ? dim_bytes : fact_bytes;
    dpg_status st = make_retrieve_plan(ctx, n_src, rec, n_fact, algo, &p->ret, /*allow_scatter=*/false);
    if (st != DPG_OK) return st;
    p->algo = p->ret.algo;
    p->fk_bits = n_dim > 1 ? bit_length((uint64_t)(n_dim - 1)) : 1;
    p->fk_passes = (p->fk_bits + 7) / 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    p->off_flag = take(sizeof(int32_t));
    if (order == DPG_JOIN_FACT_ORDER) {
        p->off_fk = take((size_t)n_fact * 4);
    } else {
        p->part = plan_partition(n_fact, 8, 4, true);
        for (int b = 0; b < 2; ++b) {
            p->off_keys[b] = take((size_t)n_fact * 4);
            p->off_vals[b] = take((size_t)n_fact * 4);
        }
        p->off_part = take(p->part.workspace);
    }
    if (p->algo == DPG_ALGO_DPG) p->off_ret = take(p->ret.workspace);
    p->workspace = off;
    return DPG_OK;
}

static dpg_status extract_fk(dpg_ctx *ctx, const JoinPlan &p, const void *fact, uint32_t *fk, uint32_t *idx,
                             hipStream_t stream) {
    ProfScope prof(ctx, K_JOIN_EXTRACT, (double)p.n_fact * (64.0 + 4.0 + (idx ? 4.0 : 0.0)), stream);
    hipLaunchKernelGGL(k_join_extract, dim3((unsigned)((p.n_fact + 255) / 256)), dim3(256), 0, stream,
                       (const uint32_t *)fact, p.n_fact, p.fact_bytes / 4, p.fk_offset / 4, fk, idx);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

// ids_ready: the dense dimension rows of the fact rows are already in the
// workspace (fact order: the fk array; dimension order: keys[0], with the
// fact row numbers in vals[0]) and are not extracted from the fact rows.
static dpg_status run_join(dpg_ctx *ctx, const JoinPlan &p, const void *fact, const void *dim, void *out,
                           int check_fk, void *ws, hipStream_t stream, bool ids_ready = false) {
    if (p.n_fact == 0) return DPG_OK;
    char *w = (char *)ws;
    int32_t *flag = (int32_t *)(w + p.off_flag);
    dpg_status st;
    if (p.order == DPG_JOIN_FACT_ORDER) {
        uint32_t *fk = (uint32_t *)(w + p.off_fk);
        const bool need_fk = ids_ready || check_fk || p.algo == DPG_ALGO_DPG;
        if (need_fk && !ids_ready) {
            st = extract_fk(ctx, p, fact, fk, nullptr, stream);
            if (st != DPG_OK) return st;
        }
        if (check_fk) {
            bool bad = false;
            st = check_ids(ctx, (const int32_t *)fk, p.n_fact, p.n_dim, flag, stream, &bad);
            if (st != DPG_OK) return st;
            if (bad) return DPG_ERR_FK_OUT_OF_RANGE;
        }
        if (p.algo == DPG_ALGO_DIRECT)
            return launch_assemble(ctx, fact, p.n_fact, nullptr, dim, p.n_dim, need_fk ? (const int32_t *)fk : nullptr,
                                   p.fk_offset / 4, out, p.n_fact, p.fact_bytes, p.dim_bytes, stream);
        char *rw = w + p.off_ret;
        st = run_distribute_probe(ctx, p.ret, dim, (const int32_t *)fk, rw, stream);
        if (st != DPG_OK) return st;
        return launch_assemble(ctx, fact, p.n_fact, nullptr, rw + p.ret.off_internal, p.n_fact,
                               (const int32_t *)(rw + p.ret.off_inv), 0, out, p.n_fact, p.fact_bytes, p.dim_bytes,
                               stream);
    }
    // DPG-Sort: (fk, i) pairs sorted by fk, stable
    int cur = 0;
    if (!ids_ready) {
        st = extract_fk(ctx, p, fact, (uint32_t *)(w + p.off_keys[0]), (uint32_t *)(w + p.off_vals[0]), stream);
        if (st != DPG_OK) return st;
    }
    if (check_fk) {
        bool bad = false;
        st = check_ids(ctx, (const int32_t *)(w + p.off_keys[0]), p.n_fact, p.n_dim, flag, stream, &bad);
        if (st != DPG_OK) return st;
        if (bad) return DPG_ERR_FK_OUT_OF_RANGE;
    }
    for (int pass = 0; pass < p.fk_passes; ++pass) {
        const int other = 1 - cur;
        st = launch_partition(ctx, p.part, w + p.off_keys[cur], (const uint32_t *)(w + p.off_vals[cur]),
                              w + p.off_keys[other], (uint32_t *)(w + p.off_vals[other]), nullptr, 8 * pass, 0,
                              w + p.off_part, stream, nullptr);
        if (st != DPG_OK) return st;
        cur = other;
    }
    const int32_t *sorted_fk = (const int32_t *)(w + p.off_keys[cur]);
    const int32_t *sorted_i = (const int32_t *)(w + p.off_vals[cur]);
    if (p.algo == DPG_ALGO_DIRECT)
        return launch_assemble(ctx, fact, p.n_fact, sorted_i, dim, p.n_dim, sorted_fk, 0, out, p.n_fact,
                               p.fact_bytes, p.dim_bytes, stream);
    char *rw = w + p.off_ret;
    st = run_distribute_probe(ctx, p.ret, fact, sorted_i, rw, stream);
    if (st != DPG_OK) return st;
    return launch_assemble(ctx, rw + p.ret.off_internal, p.n_fact, (const int32_t *)(rw + p.ret.off_inv), dim,
                           p.n_dim, sorted_fk, 0, out, p.n_fact, p.fact_bytes, p.dim_bytes, stream);
}

}  // namespace dpg

using namespace dpg;

extern "C" size_t dpg_fk_join_workspace_bytes(const dpg_ctx *ctx, int64_t n_fact, int32_t fact_bytes,
                                              int32_t fk_offset, int64_t n_dim, int32_t dim_bytes,
                                              dpg_join_order order, dpg_algo algo) {
    JoinPlan p;
    if (make_join_plan(ctx, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes, order, algo, &p) != DPG_OK) return 0;
    return p.workspace;
}

extern "C" dpg_status dpg_fk_join(dpg_ctx *ctx, const void *fact, int64_t n_fact, int32_t fact_bytes,
                                  int32_t fk_offset, const void *dim, int64_t n_dim, int32_t dim_bytes, void *out,
                                  dpg_join_order order, void *workspace, size_t workspace_bytes, dpg_algo algo,
                                  int check_fk, hipStream_t stream) {
    JoinPlan p;
    dpg_status st = make_join_plan(ctx, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes, order, algo, &p);
    if (st != DPG_OK) return st;
    if (check_fk != 0 && check_fk != 1) return DPG_ERR_INVALID_ARG;
    if (n_fact > 0 && (!fact || !out)) return DPG_ERR_INVALID_ARG;
    if (n_dim > 0 && !dim) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)fact | (uintptr_t)dim | (uintptr_t)out) % 4) return DPG_ERR_INVALID_ARG;
    const size_t fb = (size_t)n_fact * fact_bytes, db = (size_t)n_dim * dim_bytes;
    const size_t ob = (size_t)n_fact * (fact_bytes + dim_bytes);
    if (ranges_overlap(out, ob, fact, fb) || ranges_overlap(out, ob, dim, db)) return DPG_ERR_INVALID_ARG;
    if (n_fact > 0 && n_dim == 0) return DPG_ERR_FK_OUT_OF_RANGE;
    if (n_fact > 0) {
        if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!workspace || ((uintptr_t)workspace) % kAlign != 0) return DPG_ERR_INVALID_ARG;
        if (ranges_overlap(workspace, p.workspace, out, ob) || ranges_overlap(workspace, p.workspace, fact, fb) ||
            ranges_overlap(workspace, p.workspace, dim, db))
            return DPG_ERR_INVALID_ARG;
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    return run_join(ctx, p, fact, dim, out, check_fk, workspace, stream);
}

// ---- foreign-key join over non-dense keys (Sections 4.2.2 and 4.2.3) -------
// The join triples (k, rid_R, rid_F) come from a batch lookup of the fk
// column in a hash index over the dimension keys; the dense join above then
// runs on rid_F.
namespace dpg {

__global__ __launch_bounds__(256) void k_join_iota(uint32_t *__restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

struct KeyJoinPlan {
    JoinPlan join;
    size_t off_raw = 0, off_lookup = 0, lookup_bytes = 0, workspace = 0;
};

static dpg_status make_key_join_plan(const dpg_ctx *ctx, int64_t n_fact, int32_t fact_bytes, int32_t fk_offset,
                                     int64_t n_dim, int32_t dim_bytes, int32_t log2_slots, int order, int algo,
                                     KeyJoinPlan *p) {
    *p = KeyJoinPlan();
    if (n_dim > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    dpg_status st = make_join_plan(ctx, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes, order, algo, &p->join);
    if (st != DPG_OK) return st;
    p->lookup_bytes = dpg_hash_lookup_workspace_bytes(ctx, n_dim, log2_slots, n_fact, (dpg_algo)algo);
    if (p->lookup_bytes == 0) return DPG_ERR_INVALID_ARG;
    p->off_raw = align_up(p->join.workspace);
    p->off_lookup = align_up(p->off_raw + (size_t)n_fact * 4 + 1);
    p->workspace = align_up(p->off_lookup + p->lookup_bytes);
    return DPG_OK;
}

}  // namespace dpg

extern "C" size_t dpg_key_join_workspace_bytes(const dpg_ctx *ctx, int64_t n_fact, int32_t fact_bytes,
                                               int32_t fk_offset, int64_t n_dim, int32_t dim_bytes,
                                               int32_t log2_slots, dpg_join_order order, dpg_algo algo) {
    KeyJoinPlan p;
    if (make_key_join_plan(ctx, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes, log2_slots, order, algo, &p) !=
        DPG_OK)
        return 0;
    return p.workspace;
}

extern "C" dpg_status dpg_key_join(dpg_ctx *ctx, const void *fact, int64_t n_fact, int32_t fact_bytes,
                                   int32_t fk_offset, const void *dim, int64_t n_dim, int32_t dim_bytes,
                                   const void *index, int32_t log2_slots, void *out, dpg_join_order order,
                                   void *workspace, size_t workspace_bytes, dpg_algo algo, int check_fk,
                                   hipStream_t stream) {
    KeyJoinPlan p;
    dpg_status st = make_key_join_plan(ctx, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes, log2_slots, order,
                                       algo, &p);
    if (st != DPG_OK) return st;
    const JoinPlan &jp = p.join;
    if (check_fk != 0 && check_fk != 1) return DPG_ERR_INVALID_ARG;
    if (n_fact > 0 && (!fact || !out)) return DPG_ERR_INVALID_ARG;
    if (n_dim > 0 && !dim) return DPG_ERR_INVALID_ARG;
    if (!index || ((uintptr_t)index) % kAlign) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)fact | (uintptr_t)dim | (uintptr_t)out) % 4) return DPG_ERR_INVALID_ARG;
    const size_t fb = (size_t)n_fact * fact_bytes, db = (size_t)n_dim * dim_bytes;
    const size_t ob = (size_t)n_fact * (fact_bytes + dim_bytes);
    const size_t ib = dpg_hash_index_bytes(n_dim, log2_slots);
    if (ranges_overlap(out, ob, fact, fb) || ranges_overlap(out, ob, dim, db) || ranges_overlap(out, ob, index, ib))
        return DPG_ERR_INVALID_ARG;
    if (n_fact > 0 && n_dim == 0) return DPG_ERR_FK_OUT_OF_RANGE;
    if (n_fact > 0) {
        if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!workspace || ((uintptr_t)workspace) % kAlign != 0) return DPG_ERR_INVALID_ARG;
        if (ranges_overlap(workspace, p.workspace, out, ob) || ranges_overlap(workspace, p.workspace, fact, fb) ||
            ranges_overlap(workspace, p.workspace, dim, db) || ranges_overlap(workspace, p.workspace, index, ib))
            return DPG_ERR_INVALID_ARG;
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    if (n_fact == 0) return DPG_OK;
    char *w = (char *)workspace;
    uint32_t *raw = (uint32_t *)(w + p.off_raw);
    const bool fact_order = order == DPG_JOIN_FACT_ORDER;
    int32_t *rid = (int32_t *)(w + (fact_order ? jp.off_fk : jp.off_keys[0]));
    // 1. the fk column, then its batch lookup in the index: rid_F per fact row
    st = extract_fk(ctx, jp, fact, raw, nullptr, stream);
    if (st != DPG_OK) return st;
    st = dpg_hash_lookup(ctx, index, n_dim, log2_slots, raw, n_fact, rid, w + p.off_lookup, p.lookup_bytes, algo,
                         stream);
    if (st != DPG_OK) return st;
    // 2. every key must have a dimension row (checked when asked: one stream
    //    synchronization; otherwise a missing key's rid, -1, is read as row 0)
    if (check_fk) {
        bool bad = false;
        st = check_ids(ctx, rid, n_fact, n_dim, (int32_t *)(w + jp.off_flag), stream, &bad);
        if (st != DPG_OK) return st;
        if (bad) return DPG_ERR_FK_OUT_OF_RANGE;
    }
    if (!fact_order) {
        hipLaunchKernelGGL(k_join_iota, dim3((unsigned)((n_fact + 255) / 256)), dim3(256), 0, stream,
                           (uint32_t *)(w + jp.off_vals[0]), n_fact);
        DPG_HIP(hipGetLastError());
    }
    // 3. the dense join on rid_F
    return run_join(ctx, jp, fact, dim, out, 0, workspace, stream, /*ids_ready=*/true);
}
