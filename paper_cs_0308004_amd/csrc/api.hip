// C-ABI entry points of libdpg: context, options, profiling, retrieval.
#include <cstring>

#include "dpg_internal.h"

namespace dpg {

static const char *const kKernelNames[K_COUNT] = {
    "k_direct_gather", "k_dist_hist",       "k_scan_chunks",   "k_scan_cols",      "k_scan_base",
    "k_scan_apply",    "k_dist_scatter",    "k_probe_cached",  "k_probe_lds",      "k_gather_phase",
    "k_check_ids",     "k_fill_i32",        "k_sort_extract",  "k_tie_fix",        "k_join_extract",
    "k_join_assemble", "k_batch",           "k_part_hist",     "k_part_scatter",   "k_part_hist_wide",
    "k_part_scatter_unstable", "k_gather_lds", "k_hash_home", "k_hash_mark", "k_hash_place",
    "k_hash_ov_off", "k_hash_direct", "k_hash_probe", "k_hash_probe_lds", "k_smj_keys", "k_smj_ranges",
    "k_smj_emit", "k_bt_level", "k_bt_direct", "k_bt_probe", "k_bt_probe_lds", "k_probe_scatter",
    "k_stream_copy", "k_scan_small", "k_run_bounds"};

const char *kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? kKernelNames[id] : "unknown"; }

int xcd_remap_flag(const dpg_ctx *ctx) { return (ctx && ctx->opt_xcd == 2) ? 0 : 1; }

static hipEvent_t take_event(dpg_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(dpg_ctx *c, int k, double b, hipStream_t s) : ctx(c), kernel(k), bytes(b), stream(s) {
    if (!ctx || !ctx->profiling) return;
    ev0 = take_event(ctx);
    ev1 = take_event(ctx);
    if (ev0) (void)hipEventRecord(ev0, stream);
}

ProfScope::~ProfScope() {
    if (!ctx || !ctx->profiling || !ev0 || !ev1) return;
    (void)hipEventRecord(ev1, stream);
    ctx->pending.push_back(ProfRecord{kernel, bytes, ev0, ev1});
}

// Phases I and II; INTERNAL then holds the records in run order.
static dpg_status distribute_and_probe(dpg_ctx *ctx, const RetrievePlan &p, const void *src, const int32_t *rids,
                                       void *ws, hipStream_t stream, bool local_inv) {
    const double R = p.rec_bytes, M = (double)p.n_rids;
    char *w = (char *)ws;
    if (local_inv && !p.gather_lds) return DPG_ERR_UNSUPPORTED;
    dpg_status st = launch_distribute(ctx, p, rids, ws, stream, local_inv);
    if (st != DPG_OK) return st;
    if (p.probe == DPG_PROBE_LDS) return launch_probe_lds(ctx, p, src, ws, stream);
    const double touched = (double)(p.n_src < p.n_rids ? p.n_src : p.n_rids);
    return launch_gather(ctx, K_PROBE_CACHED, src, p.n_src, (const int32_t *)(w + p.off_run), w + p.off_internal,
                         p.n_rids, p.rec_bytes, 4.0 * M + R * touched + R * M, stream);
}

dpg_status run_distribute_probe(dpg_ctx *ctx, const RetrievePlan &p, const void *src, const int32_t *rids,
                                void *ws, hipStream_t stream, bool local_inv) {
    if (p.scatter) return DPG_ERR_UNSUPPORTED;  // no INTERNAL to hand over
    dpg_status st = distribute_and_probe(ctx, p, src, rids, ws, stream, local_inv);
    if (st != DPG_OK || p.dist_mode != DIST_TWO_PASS) return st;
    // callers that fuse Phase III need one slot per rid: inv = inv_c o inv_f
    char *w = (char *)ws;
    return launch_gather(ctx, K_GATHER_PHASE, w + p.off_inv_c, p.n_rids, (const int32_t *)(w + p.off_inv_f),
                         w + p.off_inv, p.n_rids, 4, 12.0 * p.n_rids, stream);
}

dpg_status run_retrieve(dpg_ctx *ctx, const RetrievePlan &p, const void *src, const int32_t *rids, void *dst,
                        void *ws, hipStream_t stream) {
    const double R = p.rec_bytes, M = (double)p.n_rids;
    if (p.n_rids == 0) return DPG_OK;
    if (p.algo == DPG_ALGO_DIRECT)
        return launch_gather(ctx, K_DIRECT_GATHER, src, p.n_src, rids, dst, p.n_rids, p.rec_bytes, 4.0 * M + 2.0 * R * M,
                             stream);
    char *w = (char *)ws;
    if (p.scatter) {
        // two phases: distribute (runs and list positions), then the probe
        // writes each record straight to dst[pos]
        dpg_status st = launch_distribute(ctx, p, rids, ws, stream, false);
        if (st != DPG_OK) return st;
        const int32_t *n_valid = (const int32_t *)(w + p.off_bucket) + (1 << p.part_nbits);
        return launch_probe_scatter(ctx, src, p.n_src, (const int32_t *)(w + p.off_run),
                                    (const int32_t *)(w + p.off_inv), n_valid, dst, p.n_rids, p.rec_bytes, stream);
    }
    if (p.dist_mode == DIST_TWO_PASS && p.probe == DPG_PROBE_LDS) {
        // runs staged in LDS: Phase III through the composed slots, one pass
        const dpg_status st = run_distribute_probe(ctx, p, src, rids, ws, stream, false);
        if (st != DPG_OK) return st;
        return launch_gather(ctx, K_GATHER_PHASE, w + p.off_internal, p.n_rids, (const int32_t *)(w + p.off_inv),
                             dst, p.n_rids, p.rec_bytes, 4.0 * M + 2.0 * R * M, stream);
    }
    if (p.dist_mode == DIST_TWO_PASS) {
        // Phase III in two passes, coarse first: u[j] = INTERNAL[inv_c[j]] in
        // the fine pass's order, then dst[i] = u[inv_f[i]]; each pass reads
        // from at most 2^8 or 2^12 streams
        dpg_status st = distribute_and_probe(ctx, p, src, rids, ws, stream, false);
        if (st != DPG_OK) return st;
        st = launch_gather(ctx, K_GATHER_PHASE, w + p.off_internal, p.n_rids, (const int32_t *)(w + p.off_inv_c),
                           w + p.off_u, p.n_rids, p.rec_bytes, 4.0 * M + 2.0 * R * M, stream);
        if (st != DPG_OK) return st;
        return launch_gather(ctx, K_GATHER_PHASE, w + p.off_u, p.n_rids, (const int32_t *)(w + p.off_inv_f), dst,
                             p.n_rids, p.rec_bytes, 4.0 * M + 2.0 * R * M, stream);
    }
    const dpg_status st = run_distribute_probe(ctx, p, src, rids, ws, stream, p.gather_lds);
    if (st != DPG_OK) return st;
    if (p.gather_lds) return launch_gather_lds(ctx, p, ws, dst, stream);
    return launch_gather(ctx, K_GATHER_PHASE, w + p.off_internal, p.n_rids, (const int32_t *)(w + p.off_inv), dst,
                         p.n_rids, p.rec_bytes, 4.0 * M + 2.0 * R * M, stream);
}

}  // namespace dpg

using namespace dpg;

extern "C" {

const char *dpg_status_string(dpg_status s) {
    switch (s) {
        case DPG_OK: return "ok";
        case DPG_ERR_INVALID_ARG: return "invalid argument";
        case DPG_ERR_RID_OUT_OF_RANGE: return "rid out of range";
        case DPG_ERR_FK_OUT_OF_RANGE: return "foreign key out of range";
        case DPG_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case DPG_ERR_UNSUPPORTED: return "unsupported";
        case DPG_ERR_HIP: return "HIP runtime error";
        case DPG_ERR_BUSY: return "busy";
    }
    return "unknown status";
}

dpg_status dpg_create(int device, dpg_ctx **out) {
    if (!out) return DPG_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DPG_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return DPG_ERR_HIP;
    dpg_ctx *ctx = new dpg_ctx();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->lds_bytes = prop.sharedMemPerBlock;
    ctx->l2_bytes = prop.l2CacheSize;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess ||
        hipHostMalloc((void **)&ctx->host_flag, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return DPG_ERR_HIP;
    }
    scratch_init(ctx);  // with `device` current
    (void)hipSetDevice(prev);
    *ctx->host_flag = 0;
    *out = ctx;
    return DPG_OK;
}

void dpg_destroy(dpg_ctx *ctx) {
    if (!ctx) return;
    for (auto &r : ctx->pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->host_flag) (void)hipHostFree(ctx->host_flag);
    delete ctx;
}

dpg_status dpg_set_option(dpg_ctx *ctx, dpg_option option, int64_t value) {
    if (!ctx || value < 0) return DPG_ERR_INVALID_ARG;
    switch (option) {
        case DPG_OPT_LOG2_RUN:
            if (value > 31) return DPG_ERR_INVALID_ARG;
            ctx->opt_log2_run = value;
            return DPG_OK;
        case DPG_OPT_PROBE:
            if (value > DPG_PROBE_LDS) return DPG_ERR_INVALID_ARG;
            ctx->opt_probe = value;
            return DPG_OK;
        case DPG_OPT_DIST_TILE:
            if (value % 64 != 0 || value > (1 << 24)) return DPG_ERR_INVALID_ARG;
            ctx->opt_dist_tile = value;
            return DPG_OK;
        case DPG_OPT_XCD_REMAP:
            if (value > 2) return DPG_ERR_INVALID_ARG;
            ctx->opt_xcd = value ? value : 1;
            return DPG_OK;
        case DPG_OPT_USE_TUNED:
            if (value > 2) return DPG_ERR_INVALID_ARG;
            ctx->opt_use_tuned = value ? value : 1;
            return DPG_OK;
        case DPG_OPT_DISTRIBUTE:
            if (value > kDistOptionMax) return DPG_ERR_INVALID_ARG;
            ctx->opt_distribute = value;
            return DPG_OK;
        case DPG_OPT_GATHER:
            if (value > 3) return DPG_ERR_INVALID_ARG;
            ctx->opt_gather = value;
            return DPG_OK;
    }
    return DPG_ERR_INVALID_ARG;
}

dpg_status dpg_get_option(const dpg_ctx *ctx, dpg_option option, int64_t *value) {
    if (!ctx || !value) return DPG_ERR_INVALID_ARG;
    switch (option) {
        case DPG_OPT_LOG2_RUN: *value = ctx->opt_log2_run; return DPG_OK;
        case DPG_OPT_PROBE: *value = ctx->opt_probe; return DPG_OK;
        case DPG_OPT_DIST_TILE: *value = ctx->opt_dist_tile; return DPG_OK;
        case DPG_OPT_XCD_REMAP: *value = ctx->opt_xcd; return DPG_OK;
        case DPG_OPT_USE_TUNED: *value = ctx->opt_use_tuned; return DPG_OK;
        case DPG_OPT_DISTRIBUTE: *value = ctx->opt_distribute; return DPG_OK;
        case DPG_OPT_GATHER: *value = ctx->opt_gather; return DPG_OK;
    }
    return DPG_ERR_INVALID_ARG;
}

dpg_status dpg_retrieve(dpg_ctx *ctx, const void *src, int64_t n_src, int32_t rec_bytes, const int32_t *rids,
                        int64_t n_rids, void *dst, void *workspace, size_t workspace_bytes, dpg_algo algo,
                        int check_rids, hipStream_t stream) {
    // argument checks first, so they can be exercised without a device
    dpg_status st = validate_records(n_src, rec_bytes, src, n_rids > 0);
    if (st != DPG_OK) return st;
    if (n_rids < 0 || n_rids > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    if (n_rids > 0 && (!rids || !dst)) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)rids) % 4 != 0 || ((uintptr_t)dst) % 4 != 0) return DPG_ERR_INVALID_ARG;
    if (check_rids != 0 && check_rids != 1) return DPG_ERR_INVALID_ARG;
    if (ranges_overlap(src, (size_t)n_src * rec_bytes, dst, (size_t)n_rids * rec_bytes) ||
        ranges_overlap(rids, (size_t)n_rids * 4, dst, (size_t)n_rids * rec_bytes))
        return DPG_ERR_INVALID_ARG;
    RetrievePlan plan;
    st = make_retrieve_plan(ctx, n_src, rec_bytes, n_rids, algo, &plan);
    if (st != DPG_OK) return st;
    if (n_rids > 0 && n_src == 0) return DPG_ERR_RID_OUT_OF_RANGE;
    if (n_rids > 0) {
        if (workspace_bytes < plan.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!workspace || ((uintptr_t)workspace) % kAlign != 0) return DPG_ERR_INVALID_ARG;
        if (ranges_overlap(workspace, plan.workspace, dst, (size_t)n_rids * rec_bytes) ||
            ranges_overlap(workspace, plan.workspace, rids, (size_t)n_rids * 4) ||
            ranges_overlap(workspace, plan.workspace, src, (size_t)n_src * rec_bytes))
            return DPG_ERR_INVALID_ARG;
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    if (n_rids == 0) return DPG_OK;
    if (check_rids) {
        bool bad = false;
        st = check_ids(ctx, rids, n_rids, n_src, (int32_t *)((char *)workspace + plan.off_flag), stream, &bad);
        if (st != DPG_OK) return st;
        if (bad) return DPG_ERR_RID_OUT_OF_RANGE;
    }
    return run_retrieve(ctx, plan, src, rids, dst, workspace, stream);
}

dpg_status dpg_stream_copy(dpg_ctx *ctx, const void *src, void *dst, size_t bytes, int32_t vectors_per_lane,
                           int32_t nontemporal, hipStream_t stream) {
    if (!ctx || bytes % 16 != 0 || ((uintptr_t)src) % 16 != 0 || ((uintptr_t)dst) % 16 != 0 ||
        (bytes > 0 && (!src || !dst)) || ranges_overlap(src, bytes, dst, bytes) ||
        (nontemporal != 0 && nontemporal != 1))
        return DPG_ERR_INVALID_ARG;
    if (vectors_per_lane != 2 && vectors_per_lane != 4 && vectors_per_lane != 8 && vectors_per_lane != 16)
        return DPG_ERR_INVALID_ARG;
    return launch_stream_copy(ctx, src, dst, bytes, vectors_per_lane, nontemporal != 0, stream);
}

dpg_status dpg_profile_enable(dpg_ctx *ctx, int on) {
    if (!ctx) return DPG_ERR_INVALID_ARG;
    ctx->profiling = on != 0;
    return DPG_OK;
}

dpg_status dpg_profile_reset(dpg_ctx *ctx) {
    if (!ctx) return DPG_ERR_INVALID_ARG;
    for (auto &r : ctx->pending) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return DPG_ERR_HIP;
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    ctx->pending.clear();
    ctx->totals.clear();
    ctx->total_order.clear();
    return DPG_OK;
}

dpg_status dpg_profile_collect(dpg_ctx *ctx, int32_t *n_kernels) {
    if (!ctx) return DPG_ERR_INVALID_ARG;
    for (auto &r : ctx->pending) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return DPG_ERR_HIP;
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return DPG_ERR_HIP;
        if (!ctx->totals.count(r.kernel)) ctx->total_order.push_back(r.kernel);
        ProfTotal &t = ctx->totals[r.kernel];
        t.launches += 1;
        t.ms += ms;
        t.bytes += r.bytes;
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    ctx->pending.clear();
    if (n_kernels) *n_kernels = (int32_t)ctx->total_order.size();
    return DPG_OK;
}

dpg_status dpg_profile_entry(const dpg_ctx *ctx, int32_t index, const char **name, int64_t *launches,
                             double *total_ms, double *total_bytes) {
    if (!ctx || index < 0 || index >= (int32_t)ctx->total_order.size()) return DPG_ERR_INVALID_ARG;
    const int k = ctx->total_order[index];
    const ProfTotal &t = ctx->totals.at(k);
    if (name) *name = kernel_name(k);
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.ms;
    if (total_bytes) *total_bytes = t.bytes;
    return DPG_OK;
}

}  // extern "C"
