// Retrieval planner: chooses between direct retrieval and DPG and, for DPG,
// the run length L, the probe flavour and the distribute tile.  Pure host code.
//
// The two constraints of Section 2.1 ("Constraints") become:
//   * Phase II: one source run must fit the store that absorbs the probe's
//     random reads.  With the LDS probe that store is the workgroup's LDS
//     (L*R <= 64 KiB); with the cached probe it is the XCD's 4 MiB L2 backed
//     by the 256 MiB Infinity Cache, so L*R is kept at 2-4 MiB.  Measured on
//     MI355X at 2^26 rids, runs of 2-8 MiB are within 3% of each other and of
//     the best; the autotuner tries 256 KiB to 64 MiB.
//   * Phases I and III: one buffer per run must fit the cache.  Here that is
//     the LDS table of B counters in the distribute (B <= 8192) and the B
//     INTERNAL streams the gather reads, which the L2 and Infinity Cache hold
//     comfortably at B <= 8192.
// Phase I is one partition pass over B <= 4096 runs (an 8-bit pass up to 256
// runs, a 12-bit one above); the append form (B <= 8192) serves as the
// alternative the autotuner and tests can select.
// L is a power of two so the run of rid r is r >> log2(L) (Section 2.1).
#include <algorithm>
#include <cstring>

#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

constexpr int64_t kMaxRuns = 8192;
constexpr int64_t kMaxTwoPassRuns = (int64_t)1 << 20;  // 12 fine bits x 8 coarse bits
// the partition pass that also records every rid's list position stages the
// tile twice in LDS, which leaves room for 2^11 digits
constexpr int64_t kMaxScatterRuns = 2048;
constexpr size_t kLdsRegionBytes = 64 * 1024;
constexpr size_t kCachedRegionBytes = 4 << 20;
// Outputs up to this size take the two-phase form (the probe scatters).
constexpr double kScatterCacheBytes = 192.0 * 1024 * 1024;

dpg_status validate_records(int64_t n, int32_t rec_bytes, const void *ptr, bool need_ptr) {
    if (n < 0 || n > INT32_MAX) return DPG_ERR_INVALID_ARG;
    if (rec_bytes < 4 || rec_bytes > kMaxRecBytes || rec_bytes % 4 != 0) return DPG_ERR_INVALID_ARG;
    if (need_ptr && n > 0 && ptr == nullptr) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)ptr) % 4 != 0) return DPG_ERR_INVALID_ARG;
    return DPG_OK;
}

bool ranges_overlap(const void *a, size_t an, const void *b, size_t bn) {
    if (an == 0 || bn == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bn && b0 < a0 + an;
}

static int floor_log2(uint64_t x) {
    int k = -1;
    while (x) { ++k; x >>= 1; }
    return k;
}

static void layout_workspace(RetrievePlan *p) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    p->off_flag = take(sizeof(int32_t));
    if (p->algo == DPG_ALGO_DPG) {
        const int64_t B = p->n_runs, M = p->n_rids;
        if (p->dist_mode == DIST_PARTITION || p->dist_mode == DIST_SAMPLED) {
            const PartPlan pp = plan_partition(M, p->part_nbits, 4, false, p->wide_per, p->part_wide);
            p->off_part = take(pp.workspace);
            p->off_bucket = p->off_part + pp.off_bucket;
            p->off_items = take((size_t)((1 << p->part_nbits) + 1) * 4);
            if (p->dist_mode == DIST_SAMPLED) {
                const PartPlan sp = plan_partition(p->n_sample, 8, 4, false);
                p->off_sample = take((size_t)p->n_sample * 4);
                p->off_sample2 = take((size_t)p->n_sample * 4);
                p->off_spart = take(sp.workspace);
                p->off_split = take((size_t)B * 4);
            }
        } else if (p->dist_mode == DIST_TWO_PASS) {
            const PartPlan pf = plan_partition(M, p->lg_fine, 4, false);
            const PartPlan pc = plan_partition(M, p->lg_coarse, 4, false);
            p->off_part = take(pf.workspace);
            p->off_part2 = take(pc.workspace);
            p->off_bucket = p->off_part2 + pc.off_bucket;  // coarse run boundaries
            p->off_run_f = take((size_t)M * 4);
            p->off_inv_f = take((size_t)M * 4);
            p->off_inv_c = take((size_t)M * 4);
            if (p->probe == DPG_PROBE_LDS) {
                // the LDS probe: every run's boundaries and work items, found
                // from the sorted list; Phase III is then one pass through
                // the composed slots
                p->off_bucket = take((size_t)(B + 1) * 4);
                p->off_items = take((size_t)(B + 1) * 4);
                p->off_scan = take(scan_1d_scratch_bytes(B));
            } else {
                p->off_u = take((size_t)M * p->rec_bytes);
            }
        } else {
            p->off_cnt = take((size_t)p->n_tiles * B * 4);
            p->off_csum = take((size_t)p->n_chunks * B * 4);
            p->off_total = take((size_t)B * 4);
            p->off_bucket = take((size_t)(B + 1) * 4);
            p->off_items = take((size_t)(B + 1) * 4);
        }
        p->off_run = take((size_t)M * 4);
        p->off_inv = take((size_t)M * 4);  // slots, or list positions when the probe scatters
        p->off_internal = take(p->scatter ? 0 : (size_t)M * p->rec_bytes);
    }
    p->workspace = off;
}

// Rid lists shorter than this take partition tiles of 8192 rids (8 per
// thread), so that Phase I still spreads over 2 x 256 CUs.
constexpr int64_t kSmallTileRids = (int64_t)1 << 23;

// LDS a workgroup of the LDS-staged gather may use (gather_lds_bytes).
constexpr size_t kGatherLdsBytes = 150 * 1024;

static void plan_dpg(RetrievePlan *p, int probe, int log2_run, int dist_tile, int dist_mode, int gather) {
    const int64_t N = p->n_src > 0 ? p->n_src : 1, M = p->n_rids;
    const int R = p->rec_bytes;
    const int lg_n = ilog2_ceil(N);
    const int lg_lds = floor_log2(kLdsRegionBytes / (size_t)R);
    const bool sampled = dist_mode == DIST_SAMPLED + 1, two_pass = dist_mode == DIST_TWO_PASS + 1;
    // runs of uneven width (sampled) are probed through the caches; so are
    // the two-pass runs unless the LDS probe is asked for (their boundaries
    // are then found from the sorted list)
    if (sampled || (two_pass && probe != DPG_PROBE_LDS)) probe = DPG_PROBE_CACHED;
    // records of one 4-, 8- or 16-byte element: the wide LDS probe (128 KiB
    // regions, a whole run per work item) when the runs fit one partition
    // pass.  Chosen by default for 4-byte records only: at 2^26 rids its probe
    // is 2.2x faster than the cached one, but its 16x more runs cost Phases I
    // and III more -- net 4% faster at 4 bytes, 25% slower at 8 bytes.
    const bool small = R == 4 || R == 8 || R == 16;
    const int lg_wide = floor_log2(kProbeWideRegionBytes / (size_t)R);
    // Phase III form 3: no INTERNAL and no gather; the cached probe writes
    // each record to its place in dst (two-phase DPG).  Chosen by default for
    // records of whole 64-byte sectors, whose scattered writes fill whole
    // sectors: at 2^26 rids 2.84 / 4.00 / 7.29 ms against 3.53 / 6.73 / 12.28
    // for the three-phase form at 64 / 128 / 256 bytes.  Scattered records
    // that end mid-sector are far slower (8.3 ms against 5.7 at 100 bytes).
    // gather = -1: automatic without this form (callers that need INTERNAL).
    // It is also the default for outputs of records of 24 bytes or more that
    // the 256 MiB Infinity Cache holds (up to 192 MiB): their scattered
    // partial lines meet there before reaching HBM.  At 2^20 records of
    // 100 B: 82 us against 111 us for three phases; at 2^21 (200 MiB) 198
    // against 233 us, at 2^22 585 against 392 us; 32-byte records gain up to
    // 128 MiB and lose at 256 MiB.
    const bool sector_rows = R >= 64 && R % 64 == 0;
    const bool cache_out = R >= 24 && (double)M * R <= kScatterCacheBytes;
    const bool want_scatter = (gather == 3 || (gather == 0 && (sector_rows || cache_out))) && !sampled &&
                              !two_pass && dist_mode != DIST_APPEND + 1 && probe != DPG_PROBE_LDS;
    const bool want_wide = !want_scatter && !two_pass && small && dist_mode != DIST_APPEND + 1 && probe != DPG_PROBE_CACHED &&
                           (probe == DPG_PROBE_LDS || R == 4) && (log2_run <= 0 || log2_run <= lg_wide) &&
                           ((N + ((int64_t)1 << lg_wide) - 1) >> lg_wide) <= kMaxWideBuckets;
    if (probe == DPG_PROBE_AUTO) probe = want_wide ? DPG_PROBE_LDS : DPG_PROBE_CACHED;
    if (probe == DPG_PROBE_LDS && lg_lds < 0) probe = DPG_PROBE_CACHED;
    int lg;
    if (log2_run > 0) {
        lg = log2_run;
    } else if (probe == DPG_PROBE_LDS) {
        lg = want_wide ? lg_wide : lg_lds;
    } else {
        // records up to 16 bytes: 2 MiB regions (the probe's random reads then
        // hit L2 most); larger records: 4 MiB (measured at 2^26 rids)
        lg = floor_log2((R <= 16 ? kCachedRegionBytes / 2 : kCachedRegionBytes) / (size_t)R);
        if (lg < 0) lg = 0;
    }
    if (lg > lg_n) lg = lg_n;
    // B <= kMaxRuns, and B <= kMaxWideBuckets for the one-pass partition
    // distribute (its count matrix then stays at a quarter of the rid list):
    // lengthen the runs if needed
    const int64_t max_runs = two_pass ? kMaxTwoPassRuns
                             : want_scatter ? kMaxScatterRuns
                             : sampled ? kMaxWideBuckets
                             : (dist_mode == 1 || log2_run > 0) ? kMaxRuns : kMaxWideBuckets;
    while (((N + ((int64_t)1 << lg) - 1) >> lg) > max_runs) ++lg;
    // The LDS-staged gather of 8- and 16-byte records reads a tile of 8192
    // rids as one segment per run: past 1024 runs the segments fall under 8
    // rids and it slows down (2^28 records of 16 bytes: 6.25 ms with 2048
    // runs, 5.86 ms with 1024), so automatic runs stop at 1024 there.
    if (log2_run <= 0 && probe == DPG_PROBE_CACHED && (R == 8 || R == 16) && !want_scatter && !two_pass &&
        dist_mode != DIST_APPEND + 1 && gather != 1)
        while (((N + ((int64_t)1 << lg) - 1) >> lg) > 1024) ++lg;
    if (probe == DPG_PROBE_LDS && lg > (want_wide ? lg_wide : lg_lds)) probe = DPG_PROBE_CACHED;
    p->probe = probe;
    p->log2_run = lg;
    p->n_runs = (N + ((int64_t)1 << lg) - 1) >> lg;
    if (two_pass) {
        // fine bits first (unstable, up to 12), then the coarse bits (stable,
        // up to 8): runs are ordered by (coarse, fine) = by run index
        const int T = p->n_runs > 1 ? std::max(2, bit_length((uint64_t)(p->n_runs - 1))) : 2;
        p->dist_mode = DIST_TWO_PASS;
        p->lg_coarse = std::max(1, T - kMaxWideBits);
        p->lg_fine = T - p->lg_coarse;
        p->part_nbits = p->lg_fine;
        const PartPlan pf = plan_partition(M, p->lg_fine, 4, false);
        p->dist_tile = pf.tile;
        p->n_tiles = pf.n_tiles;
        p->n_chunks = pf.n_chunks;
    } else if (sampled) {
        p->dist_mode = DIST_SAMPLED;
        p->part_nbits = std::max(1, bit_length((uint64_t)(p->n_runs - 1)));
        p->n_sample = std::max<int64_t>(1, std::min<int64_t>(M, kSampleFactor * p->n_runs));
        p->part_wide = true;
        // (splitter buckets: tiles of at most 16384 rids)
        p->wide_per = M < kSmallTileRids ? 8 : 16;
        const PartPlan pp = plan_partition(M, p->part_nbits, 4, false, p->wide_per, true);
        p->dist_tile = pp.tile;
        p->n_tiles = pp.n_tiles;
        p->n_chunks = pp.n_chunks;
    } else if (p->n_runs <= kMaxWideBuckets && dist_mode != 1) {
        // one coalesced partition pass (its own tile size)
        p->dist_mode = DIST_PARTITION;
        p->part_nbits = bit_length((uint64_t)(p->n_runs - 1));
        if (p->part_nbits < 1) p->part_nbits = 1;
        // the 1024-thread unstable pass at any run count: at 2^26 rids it
        // beats the 256-thread pass even with twice the runs (0.22 ms at 512
        // runs against 0.27 ms at 256)
        p->part_wide = true;
        p->wide_per = M < kSmallTileRids ? 8 : 16;
        // 1025..2048 runs: tiles of 32768 rids, so that a tile's segment per
        // run averages 16 rids rather than 8 (at 2^26 rids of 100 B, 2048
        // runs: 0.235 against 0.254 ms; at 1024 runs the 16384 tile is
        // faster).  Not with the two-phase scatter, whose pass also records
        // positions.
        if (M >= kSmallTileRids && p->part_nbits == 11 && !want_scatter) p->wide_per = 32;
        // a distribute tile asked for explicitly: 8192, 16384 or 32768 rids
        if (dist_tile == 8192 || dist_tile == 16384 || (dist_tile == 32768 && !want_scatter))
            p->wide_per = dist_tile / 1024;
        const PartPlan pp = plan_partition(M, p->part_nbits, 4, false, p->wide_per, true);
        p->dist_tile = pp.tile;
        p->n_tiles = pp.n_tiles;
        p->n_chunks = pp.n_chunks;
    } else {
        // A tile holds at least 4 rids per run on average, so the count
        // matrix (tiles x runs) stays below a quarter of the rid list.
        p->dist_mode = DIST_APPEND;
        int64_t T = dist_tile > 0 ? dist_tile : 4 * p->n_runs;
        if (dist_tile <= 0 && T < 1024) T = 1024;
        T = (T + 63) / 64 * 64;
        p->dist_tile = (int)T;
        p->n_tiles = M > 0 ? (M + T - 1) / T : 0;
        p->n_chunks = (p->n_tiles + 31) / 32;
    }
    // Phase III through LDS when a partition tile's records fit (records of
    // 4, 8 or 16 bytes, one LDS element each): every global access of the
    // gather is then coalesced.  The partition tile is then 16384 rids for
    // 4-byte records and 8192 (8 per thread) otherwise, so that two gather
    // workgroups share a CU up to 8-byte records and 16-byte records fit.
    if ((p->dist_mode == DIST_PARTITION || p->dist_mode == DIST_SAMPLED) && gather != 1 &&
        (R == 4 || R == 8 || R == 16)) {
        int per = R == 4 && M >= kSmallTileRids ? 16 : 8;
        PartPlan pt = plan_partition(M, p->part_nbits, 4, false, per, true);
        if (per == 16 && gather_lds_bytes(pt.tile, R, p->part_nbits) > kGatherLdsBytes) {
            per = 8;
            pt = plan_partition(M, p->part_nbits, 4, false, per, true);
        }
        p->wide_per = per;
        p->dist_tile = pt.tile;
        p->n_tiles = pt.n_tiles;
        p->n_chunks = pt.n_chunks;
        const size_t lds = gather_lds_bytes(pt.tile, R, p->part_nbits);
        p->gather_lds = lds <= kGatherLdsBytes;
        p->part_tile = p->dist_tile;
    }
    p->probe_wide = probe == DPG_PROBE_LDS && want_wide && p->dist_mode == DIST_PARTITION;
    if (want_scatter && p->dist_mode == DIST_PARTITION) {
        p->scatter = true;
        p->gather_lds = false;
    }
    if (probe == DPG_PROBE_LDS && want_wide && !p->probe_wide && lg > lg_lds) {
        probe = DPG_PROBE_CACHED;  // the narrow LDS probe cannot hold this region
        p->probe = probe;
    }
    if (p->probe_wide) {
        p->probe_chunk = kProbeWideChunk;
    } else if (probe == DPG_PROBE_LDS) {
        int64_t P = (int64_t)1 << lg;
        if (P < 256) P = 256;
        if (P > 4096) P = 4096;
        const int64_t cap = ((int64_t)1 << 20) / (R / 4);
        if (P > cap) P = cap;
        p->probe_chunk = (int32_t)P;
    }
}

dpg_status make_hash_lookup_plan(int64_t n_queries, int32_t log2_slots, int log2_run_slots, int gather, int probe,
                                 RetrievePlan *p) {
    if (n_queries < 0 || n_queries > INT32_MAX - 1 || log2_slots < 4 || log2_slots > 30) return DPG_ERR_INVALID_ARG;
    *p = RetrievePlan();
    p->algo = DPG_ALGO_DPG;
    p->n_src = 0;  // partition limit 0: every key is valid
    p->n_rids = n_queries;
    p->rec_bytes = 4;  // INTERNAL holds an int32 rid per query
    p->probe = DPG_PROBE_CACHED;
    if (n_queries > 0) {
        // LDS probe: 2^14 slots (128 KiB) per run unless set otherwise, at
        // most 2^14; the cached probe: 2^18 slots (2 MiB).  Measured at 2^26
        // queries: 2^14-slot runs beat 2^13 (fewer runs for Phases I and III).
        const bool lds = probe != DPG_PROBE_CACHED;
        const int l = log2_run_slots > 0 ? log2_run_slots : (lds ? 14 : 18);
        int bits = log2_slots - l;
        if (bits < 1) bits = 1;
        if (bits > kMaxWideBits) bits = kMaxWideBits;
        if (lds && log2_slots - bits <= 14) {
            p->probe = DPG_PROBE_LDS;
            p->probe_chunk = 16384;
        }
        p->log2_run = 32 - bits;  // run of a query = (key * kHashMul) >> (32 - bits)
        p->n_runs = (int64_t)1 << bits;
        p->dist_mode = DIST_PARTITION;
        p->part_nbits = bits;
        const PartPlan pp = plan_partition(n_queries, bits, 4, false);
        p->dist_tile = pp.tile;
        p->n_tiles = pp.n_tiles;
        p->n_chunks = pp.n_chunks;
        if (gather != 1) {
            const size_t lds = gather_lds_bytes(pp.tile, 4, bits);
            p->gather_lds = lds <= kGatherLdsBytes;
            p->part_tile = pp.tile;
        }
    }
    layout_workspace(p);
    return DPG_OK;
}

dpg_status make_split_lookup_plan(int64_t n_queries, int64_t n_runs, int gather, bool lds_probe, RetrievePlan *p) {
    if (n_queries < 0 || n_queries > INT32_MAX - 1 || n_runs < 1 || n_runs > kMaxWideBuckets)
        return DPG_ERR_INVALID_ARG;
    *p = RetrievePlan();
    p->algo = DPG_ALGO_DPG;
    p->n_src = 0;  // every query is valid
    p->n_rids = n_queries;
    p->rec_bytes = 4;  // INTERNAL holds an int32 rid per query
    p->probe = lds_probe ? DPG_PROBE_LDS : DPG_PROBE_CACHED;
    if (n_queries > 0) {
        int bits = n_runs > 1 ? floor_log2((uint64_t)(n_runs - 1)) + 1 : 1;
        p->n_runs = n_runs;
        p->dist_mode = DIST_PARTITION;
        p->part_nbits = bits;
        if (lds_probe) p->probe_chunk = 16384;
        const PartPlan pp = plan_partition(n_queries, bits, 4, false);
        p->dist_tile = pp.tile;
        p->n_tiles = pp.n_tiles;
        p->n_chunks = pp.n_chunks;
        if (gather != 1) {
            const size_t lds = gather_lds_bytes(pp.tile, 4, bits);
            p->gather_lds = lds <= kGatherLdsBytes;
            p->part_tile = pp.tile;
        }
    }
    layout_workspace(p);
    return DPG_OK;
}

TuneKey tune_key(int32_t rec_bytes, int64_t n_src, int64_t n_rids) {
    return TuneKey{rec_bytes, ilog2_ceil(n_src > 0 ? n_src : 1), ilog2_ceil(n_rids > 0 ? n_rids : 1)};
}

dpg_status make_retrieve_plan_explicit(int64_t n_src, int32_t rec_bytes, int64_t n_rids, int algo, int probe,
                                       int log2_run, int dist_tile, int dist_mode, RetrievePlan *p, int gather) {
    if (n_src < 0 || n_src > INT32_MAX || n_rids < 0 || n_rids > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    if (rec_bytes < 4 || rec_bytes > kMaxRecBytes || rec_bytes % 4 != 0) return DPG_ERR_INVALID_ARG;
    if (algo != DPG_ALGO_DIRECT && algo != DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    *p = RetrievePlan();
    p->n_src = n_src;
    p->n_rids = n_rids;
    p->rec_bytes = rec_bytes;
    p->algo = algo;
    if (algo == DPG_ALGO_DPG && n_rids > 0) plan_dpg(p, probe, log2_run, dist_tile, dist_mode, gather);
    layout_workspace(p);
    return DPG_OK;
}

dpg_status make_retrieve_plan(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes, int64_t n_rids, int algo,
                              RetrievePlan *p, bool allow_scatter) {
    if (algo < DPG_ALGO_AUTO || algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    int probe = ctx ? (int)ctx->opt_probe : 0;
    int log2_run = ctx ? (int)ctx->opt_log2_run : 0;
    int dist_tile = ctx ? (int)ctx->opt_dist_tile : 0;
    int dist_mode = ctx ? (int)ctx->opt_distribute : 0;
    int gather = ctx ? (int)ctx->opt_gather : 0;
    if (!allow_scatter && (gather == 3 || gather == 0)) gather = -1;
    if (algo == DPG_ALGO_AUTO) {
        // Measured on MI355X (2^26 records): direct retrieval is faster at every
        // record size from 8 to 256 bytes, so it is the default unless the
        // autotuner has recorded otherwise for this shape.
        algo = DPG_ALGO_DIRECT;
        if (ctx && ctx->opt_use_tuned != 2) {
            auto it = ctx->tuned.find(tune_key(rec_bytes, n_src, n_rids));
            if (it != ctx->tuned.end()) {
                algo = it->second.algo;
                if (!probe) probe = it->second.probe;
                if (!log2_run) log2_run = it->second.log2_run;
                if (!dist_tile) dist_tile = it->second.dist_tile;
                if (!dist_mode) dist_mode = it->second.dist_mode;
            }
        }
    }
    return make_retrieve_plan_explicit(n_src, rec_bytes, n_rids, algo, probe, log2_run, dist_tile, dist_mode, p,
                                       gather);
}

void plan_to_public(const RetrievePlan &p, dpg_plan *out) {
    std::memset(out, 0, sizeof(*out));
    out->algo = p.algo;
    out->probe = p.algo == DPG_ALGO_DPG ? p.probe : 0;
    out->log2_run = p.log2_run;
    out->dist_tile = p.dist_tile;
    out->distribute = p.algo == DPG_ALGO_DPG ? dist_option_value(p.dist_mode) : 0;
    out->gather = p.algo == DPG_ALGO_DPG ? (p.scatter ? 3 : p.gather_lds ? 2 : 1) : 0;
    out->n_runs = p.n_runs;
    out->n_tiles = p.n_tiles;
    out->workspace_bytes = p.workspace;
    if (p.algo == DPG_ALGO_DPG && p.n_rids > 0) {
        out->ws_run_off = p.dist_mode == DIST_TWO_PASS ? 0 : p.off_bucket;
        out->ws_rid_run = p.off_run;
        out->ws_internal = p.scatter ? 0 : p.off_internal;
    }
}

}  // namespace dpg

extern "C" dpg_status dpg_plan_retrieve(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes, int64_t n_rids,
                                        dpg_algo algo, dpg_plan *out) {
    if (!out) return DPG_ERR_INVALID_ARG;
    dpg::RetrievePlan p;
    const dpg_status st = dpg::make_retrieve_plan(ctx, n_src, rec_bytes, n_rids, algo, &p);
    if (st != DPG_OK) return st;
    dpg::plan_to_public(p, out);
    return DPG_OK;
}

extern "C" size_t dpg_retrieve_workspace_bytes(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes,
                                               int64_t n_rids, dpg_algo algo) {
    dpg::RetrievePlan p;
    if (dpg::make_retrieve_plan(ctx, n_src, rec_bytes, n_rids, algo, &p) != DPG_OK) return 0;
    return p.workspace;
}
