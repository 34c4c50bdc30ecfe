// Internal declarations of libdpg: context, profiling, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/dpg.h"

#define DPG_HIP(expr)                                  \
    do {                                               \
        hipError_t dpg_e_ = (expr);                    \
        if (dpg_e_ != hipSuccess) return DPG_ERR_HIP;  \
    } while (0)

namespace dpg {

constexpr int kMaxRecBytes = 4096;
constexpr size_t kProbeWideRegionBytes = 128 * 1024;  // region of the wide LDS probe
constexpr int kProbeWideChunk = 32768;                // rids per work item of the wide LDS probe
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
inline int ilog2_ceil(int64_t x) {
    int k = 0;
    while ((int64_t(1) << k) < x) ++k;
    return k;
}
inline int bit_length(uint64_t x) {
    int k = 0;
    while (x) { ++k; x >>= 1; }
    return k;
}

// Kernels the library launches; names appear in the profile and must match
// the HIP kernel symbol stems so rocprof summaries can be matched.
enum KernelId {
    K_DIRECT_GATHER = 0, // direct retrieval (Section 1's standard approach)
    K_DIST_HIST,         // Phase I count pass
    K_SCAN_CHUNKS,       // Phase I bucket boundaries (column chunk sums)
    K_SCAN_COLS,
    K_SCAN_BASE,
    K_SCAN_APPLY,
    K_DIST_SCATTER,      // Phase I append pass
    K_PROBE_CACHED,      // Phase II, source run read through the caches
    K_PROBE_LDS,         // Phase II, source run staged in LDS
    K_GATHER_PHASE,      // Phase III
    K_CHECK_IDS,
    K_FILL,
    K_SORT_EXTRACT,
    K_TIE_FIX,
    K_JOIN_EXTRACT,
    K_JOIN_ASSEMBLE,
    K_BATCH,
    K_PART_HIST,
    K_PART_SCATTER,
    K_PART_HIST_WIDE,
    K_PART_SCATTER_UNSTABLE,
    K_GATHER_LDS,        // Phase III, distribute tile staged in LDS
    K_HASH_HOME,         // hash index build
    K_HASH_MARK,
    K_HASH_PLACE,
    K_HASH_OVOFF,
    K_HASH_DIRECT,       // batch lookup, one probe per query in query order
    K_HASH_PROBE,        // batch lookup, DPG Phase II over one index partition at a time
    K_HASH_PROBE_LDS,    // the same with the partition's slots staged in LDS
    K_SMJ_KEYS,          // sort-merge join: packed keys of the sorted relations
    K_SMJ_RANGES,        //   matching S range of every R row
    K_SMJ_EMIT,          //   result rows
    K_BT_LEVEL,          // B+ tree build: one inner level
    K_BT_DIRECT,         // B+ tree batch lookup, one root-to-leaf walk per query
    K_BT_PROBE,          //   DPG Phase II, walks over one run's subtrees through the caches
    K_BT_PROBE_LDS,      //   the same with the run's leaves staged in LDS
    K_PROBE_SCATTER,     // two-phase DPG: Phase II writes each record to its place in dst
    K_STREAM_COPY,       // plain streaming copy (the measured copy ceiling)
    K_SCAN_SMALL,        // Phase I bucket boundaries, whole column scan in one workgroup
    K_RUN_BOUNDS,        // two-pass Phase I for the LDS probe: run boundaries and work items
    K_COUNT
};
const char *kernel_name(int id);

struct ProfRecord {
    int kernel;
    double bytes;
    hipEvent_t start, stop;
};

struct ProfTotal {
    int64_t launches = 0;
    double ms = 0, bytes = 0;
};

struct TuneKey {
    int32_t rec_bytes;
    int32_t log2_n_src;
    int32_t log2_n_rids;
    bool operator<(const TuneKey &o) const {
        if (rec_bytes != o.rec_bytes) return rec_bytes < o.rec_bytes;
        if (log2_n_src != o.log2_n_src) return log2_n_src < o.log2_n_src;
        return log2_n_rids < o.log2_n_rids;
    }
};

struct TuneEntry {
    int32_t algo, probe, log2_run, dist_tile, dist_mode;
    double ms;
};

}  // namespace dpg

struct dpg_ctx {
    int device = 0;
    int n_cu = 256;
    size_t lds_bytes = 160 * 1024;
    size_t l2_bytes = 4u << 20;
    // options
    int64_t opt_log2_run = 0, opt_probe = 0, opt_dist_tile = 0, opt_xcd = 1, opt_use_tuned = 1;
    int64_t opt_distribute = 0, opt_gather = 0;
    // profiling
    bool profiling = false;
    std::vector<dpg::ProfRecord> pending;
    std::vector<hipEvent_t> event_pool;
    std::map<int, dpg::ProfTotal> totals;
    std::vector<int> total_order;
    // autotune table
    std::map<dpg::TuneKey, dpg::TuneEntry> tuned;
    // pinned host word used to read device flags
    int32_t *host_flag = nullptr;
    // device address of the library's static scratch array on this device
    // (dpg_retrieve_noalloc), looked up once per device at creation
    void *scratch = nullptr;
};

namespace dpg {

// Profiling scope: records events around one launch when profiling is on.
struct ProfScope {
    dpg_ctx *ctx;
    int kernel;
    double bytes;
    hipStream_t stream;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    ProfScope(dpg_ctx *c, int k, double b, hipStream_t s);
    ~ProfScope();
};

// Phase I flavours: append into up to 8192 runs; one coalesced partition
// pass into up to 4096 runs; the same pass into up to 4096 runs bounded by
// splitters drawn from a sorted sample of the rids (skew, Section 2.3); two
// partition passes (fine run bits, then coarse bits) into up to 2^20 runs,
// gathered back in two passes (the multi-pass DPG of Section 7).
enum { DIST_APPEND = 0, DIST_PARTITION = 1, DIST_SAMPLED = 2, DIST_TWO_PASS = 3 };
// The DPG_OPT_DISTRIBUTE value of a Phase I flavour (1 append, 2 partition,
// 3 sampled, 4 two-pass) and back (0 for an unknown value).
inline int dist_option_value(int dist_mode) { return dist_mode + 1; }
constexpr int kDistOptionMax = 4;
constexpr int kSampleFactor = 64;  // sampled rids per run

// Retrieval plan (resolved), shared by retrieve, sort, join and batch.
struct RetrievePlan {
    int algo = DPG_ALGO_DIRECT;
    int probe = DPG_PROBE_CACHED;
    int log2_run = 0;
    int dist_tile = 0;
    int64_t n_runs = 0, n_tiles = 0;
    int64_t n_src = 0, n_rids = 0;
    int rec_bytes = 0;
    // workspace layout (byte offsets)
    size_t off_cnt = 0, off_csum = 0, off_total = 0, off_bucket = 0, off_items = 0;
    size_t off_run = 0, off_inv = 0, off_internal = 0, off_flag = 0;
    int64_t n_chunks = 0;      // column-scan chunks of the count matrix
    int dist_mode = 0;         // DIST_APPEND, DIST_PARTITION, DIST_SAMPLED or DIST_TWO_PASS
    int part_nbits = 0;        // digit width of the partition pass
    size_t off_part = 0;       // partition scratch (count matrix, bucket offsets)
    int32_t probe_chunk = 0;   // run entries per LDS-probe work item
    bool gather_lds = false;   // Phase III stages each distribute tile in LDS
    bool probe_wide = false;   // Phase II: the 1024-thread LDS probe for 4/8/16-byte records
    bool scatter = false;      // two phases: the probe writes dst[pos] directly (no INTERNAL, no gather)
    int part_tile = 0;         // rids per partition tile (gather_lds)
    int wide_per = 16;         // rids per thread of a 1024-thread partition pass (8: half-size tiles)
    bool part_wide = false;    // the one-pass distribute takes the 1024-thread pass at any run count
    // DIST_SAMPLED: the sample, its sorted copy, its sort scratch, the splitters
    int64_t n_sample = 0;
    size_t off_sample = 0, off_sample2 = 0, off_spart = 0, off_split = 0;
    // DIST_TWO_PASS: digit widths, the fine pass's runs and slots, the coarse
    // pass's slots and scratch, and the intermediate record array of Phase III
    // (with the LDS probe: the runs' boundaries at off_bucket, their work
    // items at off_items and the scan scratch at off_scan instead)
    int lg_fine = 0, lg_coarse = 0;
    size_t off_run_f = 0, off_inv_f = 0, off_inv_c = 0, off_part2 = 0, off_u = 0, off_scan = 0;
    size_t workspace = 0;
};

dpg_status validate_records(int64_t n, int32_t rec_bytes, const void *ptr, bool need_ptr);
bool ranges_overlap(const void *a, size_t an, const void *b, size_t bn);
// allow_scatter = false (callers that need INTERNAL and the slots, such as
// the joins): DPG_OPT_GATHER = 3 is treated as automatic.
dpg_status make_retrieve_plan(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes,
                              int64_t n_rids, int algo, RetrievePlan *plan, bool allow_scatter = true);
// The same with every choice explicit (0 = automatic), ignoring options and
// the tuning table; algo must be DIRECT or DPG.
dpg_status make_retrieve_plan_explicit(int64_t n_src, int32_t rec_bytes, int64_t n_rids, int algo, int probe,
                                       int log2_run, int dist_tile, int dist_mode, RetrievePlan *plan,
                                       int gather = 0);
TuneKey tune_key(int32_t rec_bytes, int64_t n_src, int64_t n_rids);
// The public description of a plan (dpg_plan_retrieve, dpg_autotune_retrieve).
void plan_to_public(const RetrievePlan &p, dpg_plan *out);
// Plan of a batch lookup whose queries are partitioned into n_runs <= 4096
// runs by splitters (one unstable pass); INTERNAL holds an int32 rid per
// query; lds_probe: work items of at most 16384 queries per run.
dpg_status make_split_lookup_plan(int64_t n_queries, int64_t n_runs, int gather, bool lds_probe, RetrievePlan *p);
// The DPG plan of a hash-index batch lookup: queries distributed into 2^bits
// runs of index slots by the top bits of key * kHashMul (their home slot's
// partition); INTERNAL holds one int32 rid per query.  probe: DPG_PROBE_CACHED
// reads each run's slots through the caches (2^18 slots per run by default),
// otherwise they are staged in LDS when a run's slots fit (2^14 by default).
dpg_status make_hash_lookup_plan(int64_t n_queries, int32_t log2_slots, int log2_run_slots, int gather, int probe,
                                 RetrievePlan *plan);

// Phases I and II of a planned DPG retrieval: afterwards the workspace holds
// INTERNAL (at off_internal) and inv (at off_inv), so a caller can fuse Phase
// III into its own kernel.  With local_inv (only for plans with gather_lds)
// inv holds each rid's slot within its distribute tile's segments instead of
// its INTERNAL index.
dpg_status run_distribute_probe(dpg_ctx *ctx, const RetrievePlan &p, const void *src, const int32_t *rids,
                                void *ws, hipStream_t stream, bool local_inv = false);
// Phase III staged through LDS (plans with gather_lds, after
// run_distribute_probe with local_inv).
dpg_status launch_gather_lds(dpg_ctx *ctx, const RetrievePlan &p, void *ws, void *dst, hipStream_t stream);
// LDS of one workgroup of the LDS-staged gather: a tile of T records of R
// bytes, an int32 and a uint16 table over the 2^nbits runs, and one int32 per
// 64 slots (plus two) for the segment index at each 64-slot boundary.
inline size_t gather_lds_bytes(int64_t T, int R, int nbits) {
    return (size_t)T * R + 6u * ((size_t)1 << nbits) + 4u * (size_t)((T + 63) / 64 + 2);
}
// dpg_sort_records; with key_bytes <= 4, *sorted_keys (when given) receives the
// address inside the workspace of the n sorted keys as big-endian uint32 (key
// bytes first, zero padding), valid until the workspace is used again, else null.
dpg_status sort_records(dpg_ctx *ctx, const void *src, int64_t n, int32_t rec_bytes, int32_t key_offset,
                        int32_t key_bytes, void *dst, uint32_t *perm_out, void *workspace, size_t workspace_bytes,
                        int algo, hipStream_t stream, const uint32_t **sorted_keys);
// Enqueue a planned retrieval (arguments already validated).
dpg_status run_retrieve(dpg_ctx *ctx, const RetrievePlan &p, const void *src, const int32_t *rids,
                        void *dst, void *ws, hipStream_t stream);
// Device check that every id lies in [0, limit); synchronizes; *bad = 1 if not.
dpg_status check_ids(dpg_ctx *ctx, const int32_t *ids, int64_t n, int64_t limit, int32_t *flag_dev,
                     hipStream_t stream, bool *bad);

// ---- kernel launchers (copy.hip) ----
// dst[k] = src[idx[k]] (records of rec_bytes) for k in [0, n).
// An index outside [0, limit) copies record 0 (never an out-of-bounds access).
// dst[pos[k]] = src[run[k]] for k < min(*n_valid, n) (device count).
dpg_status launch_probe_scatter(dpg_ctx *ctx, const void *src, int64_t limit, const int32_t *run, const int32_t *pos,
                                const int32_t *n_valid, void *dst, int64_t n, int rec_bytes, hipStream_t stream);
dpg_status launch_gather(dpg_ctx *ctx, int kernel_id, const void *src, int64_t limit, const int32_t *idx,
                         void *dst, int64_t n, int rec_bytes, double alg_bytes, hipStream_t stream);
dpg_status launch_fill_i32(dpg_ctx *ctx, int32_t *p, int64_t n, int32_t value, hipStream_t stream);
// Plain copy of bytes / 16 16-byte vectors, per (2, 4, 8 or 16) vectors per lane.
dpg_status launch_stream_copy(dpg_ctx *ctx, const void *src, void *dst, size_t bytes, int per, bool nt,
                              hipStream_t stream);

// ---- distribute (distribute.hip) ----
dpg_status launch_distribute(dpg_ctx *ctx, const RetrievePlan &p, const int32_t *rids, void *ws,
                             hipStream_t stream, bool local_inv = false);
// ---- probe (probe.hip) ----
dpg_status launch_probe_lds(dpg_ctx *ctx, const RetrievePlan &p, const void *src, void *ws,
                            hipStream_t stream);

int xcd_remap_flag(const dpg_ctx *ctx);
// Look up the device address of the static scratch array on ctx->device (the
// current device) once per device and store it in ctx->scratch.
void scratch_init(dpg_ctx *ctx);

// Validate and plan one request whose output will be placed later somewhere in
// [arena, arena + arena_bytes) (the serving engine's arena): *own_ws is the
// workspace of its single-request entry point; *batch_ws the scratch its
// steps need inside a graph batch (0 for direct work).  Every valid request
// can run inside the persistent batch launch.
dpg_status plan_batch_request(const dpg_ctx *ctx, const dpg_request &q, const void *arena, size_t arena_bytes,
                              size_t *own_ws, size_t *batch_ws);
// Upload a batch into a bound batch graph's workspace and run it: replay the
// captured graph, or (replay = false) launch k_batch directly.
dpg_status batch_graph_launch(dpg_batch_graph *g, const dpg_request *reqs, int32_t n, hipStream_t stream,
                              bool replay);

}  // namespace dpg
