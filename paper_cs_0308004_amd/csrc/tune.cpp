// Autotuner for retrieval plans.
//
// For one retrieval shape (record size, source and rid-list sizes) it times
// every candidate plan on the caller's buffers -- direct retrieval, and DPG
// with each run length L whose runs span 256 KiB .. 64 MiB of source (the
// region-size constraint of Section 2.1, "Constraints"), with both probe
// flavours and both Phase I flavours (partition up to 4096 runs, append up
// to 8192) where they apply -- and records the
// fastest in the context's table.  DPG_ALGO_AUTO consults that table for
// shapes in the same power-of-two size class.  The table can be saved to and
// loaded from a text file (one line per shape).
#include <cstdio>
#include <vector>

#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

struct Candidate {
    int algo, probe, log2_run, dist_mode;  // dist_mode as the option value (1 append, 2 partition, ...)
};

static std::vector<Candidate> candidates(int64_t n_src, int32_t rec_bytes) {
    std::vector<Candidate> c;
    c.push_back({DPG_ALGO_DIRECT, 0, 0, 0});
    const int64_t N = n_src > 0 ? n_src : 1;
    const int lg_n = ilog2_ceil(N);
    for (int lg = 0; lg <= lg_n; ++lg) {
        const int64_t region = ((int64_t)rec_bytes) << lg;
        const int64_t runs = (N + ((int64_t)1 << lg) - 1) >> lg;
        if (runs > 8192) continue;
        if (region > (64ll << 20)) break;
        if (region < (256 << 10) && lg < lg_n) continue;
        if (runs <= kMaxWideBuckets) c.push_back({DPG_ALGO_DPG, DPG_PROBE_CACHED, lg, 2});
        if (runs > 16) c.push_back({DPG_ALGO_DPG, DPG_PROBE_CACHED, lg, 1});
    }
    // the LDS probe with its natural run length (64 KiB of source per run)
    int lg_lds = -1;
    for (int64_t v = (64 * 1024) / rec_bytes; v; v >>= 1) ++lg_lds;
    if (lg_lds >= 0) {
        if (lg_lds > lg_n) lg_lds = lg_n;
        const int64_t runs = (N + ((int64_t)1 << lg_lds) - 1) >> lg_lds;
        if (runs <= 8192) {
            if (runs <= kMaxWideBuckets) c.push_back({DPG_ALGO_DPG, DPG_PROBE_LDS, lg_lds, 2});
            if (runs > 16) c.push_back({DPG_ALGO_DPG, DPG_PROBE_LDS, lg_lds, 1});
        }
    }
    return c;
}

static dpg_status plan_of(const Candidate &c, int64_t n_src, int32_t rec_bytes, int64_t n_rids, RetrievePlan *p) {
    return make_retrieve_plan_explicit(n_src, rec_bytes, n_rids, c.algo, c.probe, c.log2_run, 0, c.dist_mode, p);
}

}  // namespace dpg

using namespace dpg;

extern "C" {

size_t dpg_autotune_workspace_bytes(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes, int64_t n_rids) {
    (void)ctx;
    if (n_src < 1 || n_rids < 1 || rec_bytes < 4 || rec_bytes > kMaxRecBytes || rec_bytes % 4) return 0;
    size_t need = 0;
    for (const Candidate &c : candidates(n_src, rec_bytes)) {
        RetrievePlan p;
        if (plan_of(c, n_src, rec_bytes, n_rids, &p) != DPG_OK) return 0;
        if (p.workspace > need) need = p.workspace;
    }
    return need;
}

dpg_status dpg_autotune_retrieve(dpg_ctx *ctx, const void *src, int64_t n_src, int32_t rec_bytes,
                                 const int32_t *rids, int64_t n_rids, void *dst, void *workspace,
                                 size_t workspace_bytes, int32_t reps, int32_t dpg_only, hipStream_t stream,
                                 dpg_plan *best, double *best_ms) {
    if (!ctx || !src || !rids || !dst || !workspace || reps < 1 || n_src < 1 || n_rids < 1) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    const size_t need = dpg_autotune_workspace_bytes(ctx, n_src, rec_bytes, n_rids);
    if (need == 0) return DPG_ERR_INVALID_ARG;
    if (workspace_bytes < need) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (ranges_overlap(src, (size_t)n_src * rec_bytes, dst, (size_t)n_rids * rec_bytes)) return DPG_ERR_INVALID_ARG;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DPG_HIP(hipEventCreate(&e0));
    DPG_HIP(hipEventCreate(&e1));
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    double best_t = 1e300;
    Candidate best_c{};
    RetrievePlan best_p;
    dpg_status st = DPG_OK;
    for (const Candidate &c : candidates(n_src, rec_bytes)) {
        if (dpg_only && c.algo != DPG_ALGO_DPG) continue;
        RetrievePlan p;
        st = plan_of(c, n_src, rec_bytes, n_rids, &p);
        if (st != DPG_OK) break;
        st = run_retrieve(ctx, p, src, rids, dst, workspace, stream);  // warm-up
        if (st != DPG_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) { st = DPG_ERR_HIP; break; }
        for (int r = 0; r < reps && st == DPG_OK; ++r) st = run_retrieve(ctx, p, src, rids, dst, workspace, stream);
        if (st != DPG_OK) break;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = DPG_ERR_HIP;
            break;
        }
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = DPG_ERR_HIP; break; }
        const double t = ms / reps;
        if (t < best_t) {
            best_t = t;
            best_c = c;
            best_p = p;
        }
    }
    ctx->profiling = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DPG_OK) return st;
    if (best_t >= 1e300) return DPG_ERR_UNSUPPORTED;
    TuneEntry e{best_c.algo, best_p.algo == DPG_ALGO_DPG ? best_p.probe : 0, best_p.log2_run, 0,
                best_p.algo == DPG_ALGO_DPG ? dist_option_value(best_p.dist_mode) : 0, best_t};
    ctx->tuned[tune_key(rec_bytes, n_src, n_rids)] = e;
    if (best) plan_to_public(best_p, best);
    if (best_ms) *best_ms = best_t;
    return DPG_OK;
}

int32_t dpg_tune_count(const dpg_ctx *ctx) { return ctx ? (int32_t)ctx->tuned.size() : 0; }

dpg_status dpg_tune_clear(dpg_ctx *ctx) {
    if (!ctx) return DPG_ERR_INVALID_ARG;
    ctx->tuned.clear();
    return DPG_OK;
}

dpg_status dpg_tune_save(const dpg_ctx *ctx, const char *path) {
    if (!ctx || !path) return DPG_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return DPG_ERR_INVALID_ARG;
    std::fprintf(f, "# dpg tuning table: rec_bytes log2_n_src log2_n_rids algo probe log2_run dist_mode ms\n");
    for (const auto &kv : ctx->tuned)
        std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", kv.first.rec_bytes, kv.first.log2_n_src, kv.first.log2_n_rids,
                     kv.second.algo, kv.second.probe, kv.second.log2_run, kv.second.dist_mode, kv.second.ms);
    const bool ok = std::fclose(f) == 0;
    return ok ? DPG_OK : DPG_ERR_INVALID_ARG;
}

dpg_status dpg_tune_load(dpg_ctx *ctx, const char *path) {
    if (!ctx || !path) return DPG_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return DPG_ERR_INVALID_ARG;
    char line[256];
    dpg_status st = DPG_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        TuneKey k{};
        TuneEntry e{};
        if (std::sscanf(line, "%d %d %d %d %d %d %d %lf", &k.rec_bytes, &k.log2_n_src, &k.log2_n_rids, &e.algo,
                        &e.probe, &e.log2_run, &e.dist_mode, &e.ms) != 8 ||
            (e.algo != DPG_ALGO_DIRECT && e.algo != DPG_ALGO_DPG) || e.probe < 0 || e.probe > DPG_PROBE_LDS ||
            e.log2_run < 0 || e.log2_run > 31 || e.dist_mode < 0 || e.dist_mode > kDistOptionMax) {
            st = DPG_ERR_INVALID_ARG;
            break;
        }
        ctx->tuned[k] = e;
    }
    std::fclose(f);
    return st;
}

}  // extern "C"
