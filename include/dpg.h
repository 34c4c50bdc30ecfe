/*
 * dpg.h -- C ABI of libdpg, MI355X (gfx950) distribute-probe-gather record
 * retrieval and the operators built on it.
 *
 * Method: Cooperman, Ma and Nguyen, "DPG: A Cache-Efficient Accelerator for
 * Sorting and for Join Operators" (arXiv cs/0308004).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every data pointer is a DEVICE pointer owned by the caller.  The
 *           library never allocates device memory: scratch space comes from
 *           the caller as `workspace`, sized by the matching *_workspace_bytes
 *           query, 256-byte aligned.  Inputs are never written.
 * Streams.  Work is enqueued on the caller's `stream` and is asynchronous
 *           unless a documented check (check_rids / check_fk) needs the host
 *           to read a device flag, in which case the call synchronizes the
 *           stream once.
 * Records.  A record is rec_bytes contiguous bytes, rec_bytes a multiple of 4
 *           in [4, 4096]; record r starts at byte r * rec_bytes.  Record
 *           buffers must be 4-byte aligned (16-byte alignment enables wider
 *           loads).  rids are 0-based int32 in [0, n_src).
 * Errors.   Arguments are validated on the host before anything is enqueued;
 *           on an error the call enqueues nothing and outputs are untouched.
 *           A failing HIP call returns DPG_ERR_HIP (outputs unspecified).
 * Results.  Outputs are bit-exact and deterministic: identical across runs,
 *           algorithms, plans, tuning choices and batch membership.
 * Threads.  A dpg_ctx may be used from one host thread at a time.
 */
#ifndef DPG_H_
#define DPG_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DPG_OK = 0,
    DPG_ERR_INVALID_ARG = 1,         /* bad pointer, size, alignment, overlap or enum */
    DPG_ERR_RID_OUT_OF_RANGE = 2,    /* a rid outside [0, n_src) (only detected when asked) */
    DPG_ERR_FK_OUT_OF_RANGE = 3,     /* a foreign key outside [0, n_dim) (only when asked) */
    DPG_ERR_WORKSPACE_TOO_SMALL = 4, /* workspace_bytes below the *_workspace_bytes query */
    DPG_ERR_UNSUPPORTED = 5,         /* valid request the library cannot serve */
    DPG_ERR_HIP = 6,                 /* a HIP runtime call failed */
    DPG_ERR_BUSY = 7                 /* serving: no capacity for the request right now */
} dpg_status;

typedef enum {
    DPG_ALGO_AUTO = 0,   /* planner / autotuner picks the faster of the two */
    DPG_ALGO_DIRECT = 1, /* direct retrieval: read src[rid] in rid-list order (Section 1) */
    DPG_ALGO_DPG = 2     /* distribute-probe-gather (Section 2.1, Figure 1) */
} dpg_algo;

typedef enum {
    DPG_JOIN_FACT_ORDER = 0, /* DPG-Move join: output in fact (rid_R) order (Section 4.2.1) */
    DPG_JOIN_DIM_ORDER = 1   /* DPG-Sort join: output in foreign-key (rid_F) order */
} dpg_join_order;

typedef enum {
    DPG_PROBE_AUTO = 0,
    DPG_PROBE_CACHED = 1, /* probe reads each source run through L2 / Infinity Cache */
    DPG_PROBE_LDS = 2     /* probe stages each source run in LDS with coalesced loads */
} dpg_probe;

/* Tunables, settable per context.  0 always means "automatic". */
typedef enum {
    DPG_OPT_LOG2_RUN = 1,   /* L = 2^v source records per run (Section 2.1 "Constraints") */
    DPG_OPT_PROBE = 2,      /* a dpg_probe value */
    DPG_OPT_DIST_TILE = 3,  /* rids per distribute tile (multiple of 64) */
    DPG_OPT_XCD_REMAP = 4,  /* 1 (default): tiles of one XCD are contiguous; 2: off */
    DPG_OPT_USE_TUNED = 5,  /* 1 (default): consult the autotune table; 2: ignore it */
    DPG_OPT_DISTRIBUTE = 6, /* Phase I: 1 append (any run count up to 8192),
                               2 coalesced partition pass (used only when runs <= 4096),
                               3 the partition pass into up to 4096 runs of equal
                               rid share, bounded by splitters from a sorted
                               sample of 64 rids per run (data skew, Section 2.3;
                               runs are then probed through the caches),
                               4 two partition passes, fine then coarse run bits,
                               into up to 2^20 runs, and Phase III in two passes
                               (multi-pass DPG, Section 7; probed through the caches) */
    DPG_OPT_GATHER = 7      /* Phase III: 1 INTERNAL read through the caches, 2 a
                               distribute tile's records staged in LDS (used only
                               with the partition distribute when they fit), 3 none:
                               the distribute also records every rid's list position
                               and the (cached) probe writes each record straight to
                               its place in dst -- two-phase DPG, up to 2048 runs,
                               no INTERNAL (used only with the one-pass partition;
                               joins treat 3 as automatic).  Automatic picks 3 for
                               records of whole 64-byte multiples, else 2 or 1 */
} dpg_option;

typedef struct dpg_ctx dpg_ctx;

/* Create a context bound to HIP device `device` (reads its properties once).
 * Allocates host memory only.  Returns DPG_ERR_HIP if the device is absent. */
dpg_status dpg_create(int device, dpg_ctx **out);
void dpg_destroy(dpg_ctx *ctx);
const char *dpg_status_string(dpg_status status);

dpg_status dpg_set_option(dpg_ctx *ctx, dpg_option option, int64_t value);
dpg_status dpg_get_option(const dpg_ctx *ctx, dpg_option option, int64_t *value);

/* ------------------------------------------------------------------------- */
/* Record retrieval (Section 2): dst[i] = src[rids[i]] for i in [0, n_rids).  */
/* ------------------------------------------------------------------------- */

/* The plan the library would run for a retrieval of this shape.  Host only;
 * `ctx` may be NULL (then MI355X defaults are assumed: 256 CUs, 160 KiB LDS). */
typedef struct {
    int32_t algo;          /* DPG_ALGO_DIRECT or DPG_ALGO_DPG */
    int32_t probe;         /* DPG_PROBE_CACHED or DPG_PROBE_LDS (DPG only) */
    int32_t log2_run;      /* L = 2^log2_run source records per run */
    int32_t dist_tile;     /* rids per distribute tile */
    int32_t distribute;    /* Phase I form: 1 append, 2 partition, 3 sampled, 4
                              two-pass (DPG only; the values of DPG_OPT_DISTRIBUTE) */
    int32_t gather;        /* Phase III form: 1 cached, 2 LDS-staged, 3 none (the
                              probe scatters; DPG only; the values of DPG_OPT_GATHER) */
    int64_t n_runs;        /* B = ceil(n_src / L), the paper's NUM_RUNS */
    int64_t n_tiles;       /* ceil(n_rids / dist_tile) */
    size_t workspace_bytes;
    /* After a DPG retrieval the workspace holds the phase products at these
     * byte offsets (0 when algo is direct), for inspection or pipelining:
     *   run_off  int32[n_runs + 1]  start of RID run b in rid_run (Phase I;
     *                               not kept by the two-pass form: offset 0)
     *   rid_run  int32[n_rids]      the RID runs, one after another (Phase
     *                               I); each run in rid-list order with the
     *                               append distribute, in unspecified order
     *                               with the partition distribute
     *   internal n_rids records     the INTERNAL runs (Phase II; none when
     *                               the probe scatters: offset 0)          */
    size_t ws_run_off;
    size_t ws_rid_run;
    size_t ws_internal;
} dpg_plan;

dpg_status dpg_plan_retrieve(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes,
                             int64_t n_rids, dpg_algo algo, dpg_plan *out);

/* Bytes of workspace dpg_retrieve needs for this shape, algorithm and the
 * context's current options (256 for direct retrieval: the flag word used by
 * check_rids).  Returns 0 for arguments dpg_retrieve would reject. */
size_t dpg_retrieve_workspace_bytes(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes,
                                    int64_t n_rids, dpg_algo algo);

/* Copy records of `src` (n_src records) into `dst` (n_rids records) in the
 * order of `rids` (Section 2; Figure 1 gives the DPG algorithm, Section 2.3
 * its skewed case; duplicated rids are allowed).
 *   check_rids = 1: validate every rid on the device first (one extra read of
 *     rids plus one stream synchronization); an out-of-range rid returns
 *     DPG_ERR_RID_OUT_OF_RANGE with dst untouched.
 *   check_rids = 0: an out-of-range rid is undefined behaviour.
 * dst must not overlap src, rids or the workspace, and the workspace must not
 * overlap src or rids.  n_rids == 0 returns DPG_OK, enqueuing nothing. */
dpg_status dpg_retrieve(dpg_ctx *ctx, const void *src, int64_t n_src, int32_t rec_bytes,
                        const int32_t *rids, int64_t n_rids, void *dst,
                        void *workspace, size_t workspace_bytes, dpg_algo algo,
                        int check_rids, hipStream_t stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * retrieval as dpg_retrieve (same arguments, plans, kernels, validation and
 * results), with its workspace taken from a static device array of the
 * library instead of the caller.  The array holds DPG_NOALLOC_SCRATCH_BYTES
 * bytes on every device the library runs on, for the life of the process;
 * its device address is looked up when a context is created on the device.
 * A shape whose workspace (dpg_retrieve_workspace_bytes) exceeds that size
 * returns DPG_ERR_WORKSPACE_TOO_SMALL and enqueues nothing (for DPG at 100 B
 * records, about 600,000 rids fit; direct retrieval needs 256 bytes).  The
 * call allocates no device memory, and with per-kernel profiling off
 * (dpg_profile_enable) makes no allocation at all.  `stream` must belong to
 * ctx's device.  Every call on a device shares that device's array: calls that can
 * overlap on one device (different streams, or several host threads) race
 * and give undefined results; serialize them on one stream. */
#define DPG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dpg_status dpg_retrieve_noalloc(dpg_ctx *ctx, const void *src, int64_t n_src, int32_t rec_bytes,
                                const int32_t *rids, int64_t n_rids, void *dst, dpg_algo algo, int check_rids,
                                hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Autotuning.  dpg_autotune_retrieve times every candidate plan for one     */
/* retrieval shape on the caller's buffers (direct retrieval; DPG with each  */
/* run length whose runs hold 256 KiB to 64 MiB of source -- the region-size */
/* constraint of Section 2.1 -- with both probes and both Phase I flavours)  */
/* and records the fastest in the context's table; DPG_ALGO_AUTO uses that   */
/* entry for shapes in the same power-of-two size class.  dst is overwritten */
/* (with the correct result); the call synchronizes the stream.              */
/* ------------------------------------------------------------------------- */
size_t dpg_autotune_workspace_bytes(const dpg_ctx *ctx, int64_t n_src, int32_t rec_bytes,
                                    int64_t n_rids);
/* dpg_only = 1: consider DPG plans only (to find the best DPG configuration).
 * *best (may be null) receives the fastest plan, described as
 * dpg_plan_retrieve describes a plan; *best_ms (may be null) its time. */
dpg_status dpg_autotune_retrieve(dpg_ctx *ctx, const void *src, int64_t n_src, int32_t rec_bytes,
                                 const int32_t *rids, int64_t n_rids, void *dst, void *workspace,
                                 size_t workspace_bytes, int32_t reps, int32_t dpg_only,
                                 hipStream_t stream, dpg_plan *best, double *best_ms);
int32_t dpg_tune_count(const dpg_ctx *ctx);
dpg_status dpg_tune_clear(dpg_ctx *ctx);
/* Text file, one line per shape; load merges into the table and rejects
 * malformed lines with DPG_ERR_INVALID_ARG. */
dpg_status dpg_tune_save(const dpg_ctx *ctx, const char *path);
dpg_status dpg_tune_load(dpg_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------- */
/* Sorting (Section 3): three-phase key-pointer sort with DPG as the copy      */
/* phase.  Records are ordered by key bytes [key_offset, key_offset+key_bytes) */
/* compared as unsigned bytes, lexicographically; records with equal keys keep */
/* their input order, so the output is unique.                                 */
/* ------------------------------------------------------------------------- */

/* Workspace for dpg_sort_records (0 for arguments it would reject). */
size_t dpg_sort_workspace_bytes(const dpg_ctx *ctx, int64_t n, int32_t rec_bytes, int32_t key_offset,
                                int32_t key_bytes, dpg_algo copy_algo);

/* dst[j] = src[perm[j]] where perm sorts the records by key.  perm_out
 * (nullable, uint32[n]) receives perm.  key_bytes in [1, 64].  copy_algo picks
 * the retrieval used for the copy phase (DPG, direct, or AUTO).  The pairs
 * are sorted on the first 4 key bytes, then every group of equal prefixes is
 * put in order by the remaining bytes and the index.  If some group is longer
 * than 64 records, the pairs are sorted over the whole key instead: the
 * device decides (the passes for that case are always enqueued and return at
 * once when not needed), so the call never synchronizes.  src, dst, perm_out
 * and workspace must not overlap. */
dpg_status dpg_sort_records(dpg_ctx *ctx, const void *src, int64_t n, int32_t rec_bytes,
                            int32_t key_offset, int32_t key_bytes, void *dst, uint32_t *perm_out,
                            void *workspace, size_t workspace_bytes, dpg_algo copy_algo,
                            hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Foreign-key joins (Section 4.2.1).  The fact relation (the paper's R)       */
/* references the dimension relation (the indexed F): the little-endian       */
/* uint32 at byte fk_offset (a multiple of 4) of a fact row is the number of  */
/* the dimension row it joins (dense ids, so rid_F = fk).  Every fact row      */
/* yields one joined row of fact_bytes + dim_bytes bytes: the fact row          */
/* followed by its dimension row.                                             */
/*   DPG_JOIN_FACT_ORDER (DPG-Move): out[i] joins fact row i.                 */
/*   DPG_JOIN_DIM_ORDER  (DPG-Sort): rows ordered by foreign key; rows with   */
/*     equal keys keep fact order.                                            */
/* algo picks how the moved relation is retrieved: DPG, direct, or AUTO.      */
/* ------------------------------------------------------------------------- */
size_t dpg_fk_join_workspace_bytes(const dpg_ctx *ctx, int64_t n_fact, int32_t fact_bytes,
                                   int32_t fk_offset, int64_t n_dim, int32_t dim_bytes,
                                   dpg_join_order order, dpg_algo algo);

/* check_fk = 1: verify every foreign key is < n_dim first (one extra pass and
 * one stream synchronization); otherwise an out-of-range key is undefined
 * behaviour (no out-of-bounds access, unspecified row contents).  out must
 * not overlap fact, dim or workspace. */
dpg_status dpg_fk_join(dpg_ctx *ctx, const void *fact, int64_t n_fact, int32_t fact_bytes,
                       int32_t fk_offset, const void *dim, int64_t n_dim, int32_t dim_bytes,
                       void *out, dpg_join_order order, void *workspace, size_t workspace_bytes,
                       dpg_algo algo, int check_fk, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Sort-merge join with DPG sort (Section 4.1): both relations are sorted on   */
/* the join key with dpg_sort_records (copy phase: DPG, direct or AUTO), then  */
/* merged.  The result holds one row per pair of rows with equal keys -- the  */
/* R row followed by the S row (rec_r + rec_s bytes) -- ordered by key        */
/* (unsigned bytes, memcmp order), then R index, then S index.  The join key  */
/* is key_bytes (1..8) bytes at key_off_r of an R row and key_off_s of an S   */
/* row.                                                                       */
/* ------------------------------------------------------------------------- */
size_t dpg_sort_merge_join_workspace_bytes(const dpg_ctx *ctx, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                                           int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes,
                                           dpg_algo sort_copy_algo);

/* out holds out_capacity rows.  The call synchronizes the stream once to learn
 * the number of result rows, stored in *out_rows (host).  If they do not fit,
 * it returns DPG_ERR_WORKSPACE_TOO_SMALL and writes no row; 2^31 or more
 * result rows return DPG_ERR_UNSUPPORTED.  out must not overlap r, s or the
 * workspace. */
dpg_status dpg_sort_merge_join(dpg_ctx *ctx, const void *r, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                               const void *s, int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes,
                               void *out, int64_t out_capacity, int64_t *out_rows, void *workspace,
                               size_t workspace_bytes, dpg_algo sort_copy_algo, hipStream_t stream);
/* The same join without any host synchronization (it can be captured in a
 * graph): out_rows_dev is a DEVICE int64 (8-byte aligned) that receives the
 * number of result rows; the first min(that number, out_capacity) rows are
 * written, out_capacity below 2^31 - 1.  A count above out_capacity means the
 * output was cut short; a count of 2^31 or more leaves the rows unspecified. */
dpg_status dpg_sort_merge_join_async(dpg_ctx *ctx, const void *r, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                                     const void *s, int64_t n_s, int32_t rec_s, int32_t key_off_s, int32_t key_bytes,
                                     void *out, int64_t out_capacity, int64_t *out_rows_dev, void *workspace,
                                     size_t workspace_bytes, dpg_algo sort_copy_algo, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Hash index and batch lookup (Section 4.2.3, batch lookup in hash indexes): */
/* a hash index over uint32 keys (rid = position in the key array) holds one  */
/* key-rid pair per slot and keeps the pairs that collide with an occupied    */
/* slot in an overflow array.  A batch lookup returns, for each query key,    */
/* the smallest rid holding it, or -1.  With DPG the queries are distributed  */
/* by the index partition of their slot, each partition is probed while it    */
/* is cache resident, and the rids are gathered back into query order.        */
/*                                                                           */
/* Index layout (one buffer of dpg_hash_index_bytes, 256-byte aligned):      */
/*   S = 2^log2_slots slots; the home slot of key k is the top log2_slots     */
/*   bits of the 32-bit product k * 0x9E3779B1 (multiplicative hashing).      */
/*   slots  uint32[2S] at byte 0: key, rid of the smallest rid whose key has  */
/*          this home; an empty slot holds key 0, rid 0xFFFFFFFF              */
/*   ov_off int32[S+1] at dpg_hash_ov_off_offset: overflow pairs whose home   */
/*          is below h; ov_off[S] = all of them                               */
/*   ov     uint32[2n] at dpg_hash_ov_offset: the other key-rid pairs in      */
/*          (home, rid) order                                                 */
/* ------------------------------------------------------------------------- */
#define DPG_HASH_EMPTY 0xFFFFFFFFu

/* Bytes of an index over n_keys keys with 2^log2_slots slots (0 if invalid:
 * log2_slots in [4, 30], n_keys in [0, 2^31 - 2]), and the byte offsets of
 * its ov_off and ov arrays. */
size_t dpg_hash_index_bytes(int64_t n_keys, int32_t log2_slots);
size_t dpg_hash_ov_off_offset(int32_t log2_slots);
size_t dpg_hash_ov_offset(int32_t log2_slots);

/* Build the index of `keys` (device, uint32[n_keys]) into `index`.  The
 * contents of slots, ov_off and ov[0, ov_off[S]) are fully determined by the
 * keys (padding bytes between and after them are left as they were). */
size_t dpg_hash_build_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys, int32_t log2_slots);
dpg_status dpg_hash_build(dpg_ctx *ctx, const uint32_t *keys, int64_t n_keys, int32_t log2_slots,
                          void *index, size_t index_bytes, void *workspace, size_t workspace_bytes,
                          hipStream_t stream);

/* rids[i] = smallest rid whose key equals queries[i], or -1 (device arrays of
 * n_queries).  index must have been built for (n_keys, log2_slots).  algo:
 * DPG_ALGO_DIRECT probes the index once per query in query order; DPG_ALGO_DPG
 * distributes the queries by index partition (2^DPG_OPT_LOG2_RUN slots per
 * partition), probes each partition -- staged in LDS (default and at most
 * 2^14 slots per partition) or through the caches (DPG_OPT_PROBE =
 * DPG_PROBE_CACHED, default 2^18 slots) -- and gathers the rids;
 * DPG_ALGO_AUTO picks DPG.  rids must not overlap queries, index or workspace. */
size_t dpg_hash_lookup_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys, int32_t log2_slots,
                                       int64_t n_queries, dpg_algo algo);
dpg_status dpg_hash_lookup(dpg_ctx *ctx, const void *index, int64_t n_keys, int32_t log2_slots,
                           const uint32_t *queries, int64_t n_queries, int32_t *rids,
                           void *workspace, size_t workspace_bytes, dpg_algo algo, hipStream_t stream);

/* Foreign-key join over non-dense keys (Sections 4.2.2 and 4.2.3): the
 * dimension rows carry arbitrary uint32 keys, and `index` is the hash index of
 * those keys (dpg_hash_build over the dimension's key column, uint32[n_dim],
 * rid = dimension row, with 2^log2_slots slots).  The join triples come from
 * a batch lookup of the fact rows' fk column in the index (with DPG unless
 * algo is DPG_ALGO_DIRECT); fact row i then joins dimension row j_i, the
 * smallest row holding its key, exactly as dpg_fk_join joins row fk_i (same
 * output layout, both orders, same algo meaning for the move).  Every fk must
 * be a key of the index.  check_fk = 1: verified on the device first
 * (DPG_ERR_FK_OUT_OF_RANGE otherwise, with one stream synchronization);
 * check_fk = 0: never synchronizes, and a missing key is undefined
 * behaviour (no out-of-bounds access, unspecified row contents).  out must
 * not overlap fact, dim, index or workspace. */
size_t dpg_key_join_workspace_bytes(const dpg_ctx *ctx, int64_t n_fact, int32_t fact_bytes, int32_t fk_offset,
                                    int64_t n_dim, int32_t dim_bytes, int32_t log2_slots, dpg_join_order order,
                                    dpg_algo algo);
dpg_status dpg_key_join(dpg_ctx *ctx, const void *fact, int64_t n_fact, int32_t fact_bytes, int32_t fk_offset,
                        const void *dim, int64_t n_dim, int32_t dim_bytes, const void *index, int32_t log2_slots,
                        void *out, dpg_join_order order, void *workspace, size_t workspace_bytes, dpg_algo algo,
                        int check_fk, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Enhanced B+ tree and batch lookup (Section 4.2.3, batch lookup in B+ tree  */
/* indexes).  The tree indexes uint32 keys (rid = position in the key array); */
/* "enhanced" means every slot of every node is used, so the tree is fixed by */
/* its keys.  A batch lookup returns, for each query key, the smallest rid    */
/* holding it, or -1 (the same result as the hash lookup).  With DPG the      */
/* queries are distributed into runs of consecutive lower subtrees by a       */
/* search of the tree's top (the first pass of the paper's two-pass lookup),  */
/* each run's subtrees are staged in LDS and its queries finish their walk    */
/* there (the second pass), and the rids are gathered back into query order.  */
/*                                                                           */
/* Tree layout (one buffer of dpg_btree_bytes, 256-byte aligned), fanout 32:  */
/*   level 0 keys uint32[32 B0] at byte 0, rids int32[32 B0] at               */
/*          dpg_btree_rids_offset: the (key, rid) entries sorted by key, then */
/*          rid, in B0 = max(1, ceil(n_keys / 32)) blocks; the tail of the    */
/*          last block is (0xFFFFFFFF, -1)                                    */
/*   level l >= 1 at dpg_btree_level_offset(l): ceil(nodes(l-1) / 32) nodes  */
/*          of 32 uint32; entry i of node j = last key of node 32 j + i of    */
/*          level l-1, or 0xFFFFFFFF past its last node; the top level is one */
/*          node (dpg_btree_levels counts the levels, leaves included)        */
/* ------------------------------------------------------------------------- */
#define DPG_BTREE_FANOUT 32

/* Bytes of a tree over n_keys keys, its level count, and the byte offsets of
 * the keys of one level (0 = the leaf keys) and of the leaf rids.  All return
 * 0 when n_keys is outside [0, 2^31 - 2] or level is not a level of the tree. */
size_t dpg_btree_bytes(int64_t n_keys);
int32_t dpg_btree_levels(int64_t n_keys);
size_t dpg_btree_level_offset(int64_t n_keys, int32_t level);
size_t dpg_btree_rids_offset(int64_t n_keys);

/* Build the tree of `keys` (device, uint32[n_keys]) into `tree` (at least
 * dpg_btree_bytes; padding bytes between the arrays are left as they were). */
size_t dpg_btree_build_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys);
dpg_status dpg_btree_build(dpg_ctx *ctx, const uint32_t *keys, int64_t n_keys, void *tree, size_t tree_bytes,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);

/* rids[i] = smallest rid whose key equals queries[i], or -1 (device arrays of
 * n_queries).  tree must have been built for n_keys.  algo: DPG_ALGO_DIRECT
 * walks from the root once per query in query order; DPG_ALGO_DPG (and AUTO)
 * distributes the queries into runs of consecutive leaf blocks (2^DPG_OPT_LOG2_RUN
 * entries per run, at least 1024; by default the fewest that keep the runs
 * within 4096), finishes each run's walks with its leaves staged in LDS (runs
 * of at most 16384 entries) or, with DPG_OPT_PROBE = DPG_PROBE_CACHED or
 * larger runs, through the caches, and gathers the rids.  rids must not
 * overlap queries, tree or workspace. */
size_t dpg_btree_lookup_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys, int64_t n_queries, dpg_algo algo);
dpg_status dpg_btree_lookup(dpg_ctx *ctx, const void *tree, int64_t n_keys, const uint32_t *queries,
                            int64_t n_queries, int32_t *rids, void *workspace, size_t workspace_bytes,
                            dpg_algo algo, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Batches: many retrieval / join requests of uneven size in one call.  The   */
/* work of every request runs in ONE launch of a persistent, queue-driven     */
/* kernel whose work items are (request, step, tile): a direct retrieval or   */
/* direct fact-order join is one copy step; a request planned as DPG          */
/* (retrieval, or fact-order join moving the dimension rows) is the chain of  */
/* Section 2.1's phases -- run histogram, run boundaries, distribute, probe,  */
/* gather -- each step starting once the step before it (same request) has   */
/* finished.  A dimension-order join (Section 4.2.1) is the chain of its     */
/* stable 8-bit passes over the (fk, row) pairs, then the move of the fact    */
/* rows into fk order (DPG chain or one copy) fused with the read of the      */
/* dimension rows.  Every output equals that of the request run alone.        */
/* ------------------------------------------------------------------------- */
typedef enum { DPG_REQ_RETRIEVE = 0, DPG_REQ_FK_JOIN = 1 } dpg_request_kind;

typedef struct {
    int32_t kind;          /* dpg_request_kind */
    int32_t algo;          /* dpg_algo for the retrieval (or the moved relation) */
    const void *src;       /* retrieve: source records; join: dimension rows */
    int64_t n_src;         /* rows of src */
    int32_t rec_bytes;     /* retrieve: record size; join: dimension row size */
    int32_t fact_bytes;    /* join: fact row size */
    const int32_t *rids;   /* retrieve: n rids */
    const void *fact;      /* join: n fact rows */
    int64_t n;             /* retrieve: number of rids; join: number of fact rows */
    int32_t fk_offset;     /* join: byte offset of the uint32 foreign key */
    int32_t order;         /* join: dpg_join_order */
    void *dst;             /* output rows (n x rec_bytes, or n x (fact_bytes + rec_bytes)) */
    /* graph batches only (dpg_batch_graph_launch), for a request whose steps
     * need scratch (DPG work, dimension-order joins): device scratch of
     * dpg_batch_request_workspace_bytes bytes or more,
     * 256-byte aligned; ignored by dpg_batch_run, which keeps every request's
     * scratch in the batch workspace */
    void *workspace;
    size_t workspace_bytes;
} dpg_request;

/* Scratch the steps of one request need inside a graph batch
 * (dpg_request.workspace): its run histogram and boundaries, RID_RUN, inv and
 * INTERNAL when it is planned as DPG; for a dimension-order join the two
 * (fk, i) buffers and the digit counts of the stable sort passes, plus the
 * DPG arrays of the fact-row move when that is planned as DPG; 0 for direct
 * work or an invalid request. */
size_t dpg_batch_request_workspace_bytes(const dpg_ctx *ctx, const dpg_request *req);
/* Workspace for dpg_batch_run (0 if a request is invalid). */
size_t dpg_batch_workspace_bytes(const dpg_ctx *ctx, const dpg_request *reqs, int32_t n);
/* Validates every request first (same rules as the single calls, no device
 * checks of rids or keys); on any error nothing is enqueued. */
dpg_status dpg_batch_run(dpg_ctx *ctx, const dpg_request *reqs, int32_t n, void *workspace,
                         size_t workspace_bytes, hipStream_t stream);

/* A captured graph of the persistent batch launch, bound to a workspace: each
 * dpg_batch_graph_launch uploads the new requests' steps and replays the
 * graph.  Graph batches carry every kind of request; one whose steps need
 * scratch (DPG work, dimension-order joins) brings it in
 * dpg_request.workspace, dpg_batch_request_workspace_bytes of it
 * (DPG_ERR_WORKSPACE_TOO_SMALL otherwise).  Capture needs a
 * non-default stream.  Launches on one graph must not overlap: launch again
 * once the previous launch has finished. */
typedef struct dpg_batch_graph dpg_batch_graph;
size_t dpg_batch_graph_workspace_bytes(const dpg_ctx *ctx, int32_t max_requests);
dpg_status dpg_batch_graph_create(dpg_ctx *ctx, int32_t max_requests, void *workspace,
                                  size_t workspace_bytes, hipStream_t stream, dpg_batch_graph **out);
dpg_status dpg_batch_graph_launch(dpg_batch_graph *graph, const dpg_request *reqs, int32_t n,
                                  hipStream_t stream);
/* 1 once request `request` (index in the array of the last launch) has
 * finished, while the rest of the batch may still run: the kernel writes a
 * completion word in host memory when the request's last step ends (outputs
 * then readable by any stream or the host); 0 otherwise. */
int32_t dpg_batch_graph_request_done(const dpg_batch_graph *graph, int32_t request);
/* Waits for the last launch to finish, then frees the graph (not its workspace). */
void dpg_batch_graph_destroy(dpg_batch_graph *graph);

/* ------------------------------------------------------------------------- */
/* Device-memory arena: best-fit allocator with coalescing over an address    */
/* range the caller owns (the smallest free block that fits, the lowest among */
/* equals; O(log n) per call).  Host bookkeeping only (never touches memory). */
/* The serving engine carves request outputs and workspaces out of one.       */
/* ------------------------------------------------------------------------- */
typedef struct dpg_arena dpg_arena;
/* align: power of two dividing base. */
dpg_status dpg_arena_create(uintptr_t base, size_t bytes, size_t align, dpg_arena **out);
/* DPG_ERR_BUSY when no free block is large enough. */
dpg_status dpg_arena_alloc(dpg_arena *arena, size_t bytes, uintptr_t *addr);
/* DPG_ERR_INVALID_ARG for an address the arena did not hand out (or freed). */
dpg_status dpg_arena_free(dpg_arena *arena, uintptr_t addr);
dpg_status dpg_arena_stats(const dpg_arena *arena, size_t *in_use, size_t *high_water,
                           size_t *largest_free, size_t *free_blocks);
void dpg_arena_destroy(dpg_arena *arena);

/* ------------------------------------------------------------------------- */
/* Serving: continuous batching under an HBM budget.  A scheduler thread      */
/* admits submitted requests in arrival order while their output (plus their */
/* workspace or DPG scratch) fits the arena, and launches admitted requests   */
/* on the first free stream slot: consecutive small requests together as one */
/* persistent batch launch (a graph replay with use_graph) whose DPG and      */
/* direct work share the kernel, others alone through their dedicated        */
/* kernels.  A batched request completes when its own last step ends (the    */
/* kernel sets its completion word), not when its whole batch does.          */
/* Requests arriving while batches run                                       */
/* are admitted and launched on the next free slot, so their work overlaps on */
/* the device.  With max_batch_requests = 1 every request is launched alone   */
/* through its single-request entry point (the per-request baseline).        */
/* While a server exists its scheduler thread owns the context: do not use   */
/* the context from other threads.                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    void *arena;                 /* device memory the server may use (the budget) */
    size_t arena_bytes;
    int32_t max_inflight;        /* stream slots, 1..16 */
    int32_t max_batch_requests;  /* requests per launch; 1 = per-request launches */
    int32_t use_graph;           /* 1: replay a captured batch graph per launch */
    int32_t batch_max_kib;       /* requests with larger outputs run alone
                                    through their dedicated kernels (0: 4096 KiB) */
    int32_t batch_window_us;     /* a partial batch waits up to this long for more
                                    requests before launching (0: launch at once) */
    int32_t reserved;
} dpg_server_config;

typedef enum {
    DPG_TICKET_QUEUED = 0,   /* waiting for memory */
    DPG_TICKET_ADMITTED = 1, /* memory reserved, waiting for a slot */
    DPG_TICKET_RUNNING = 2,
    DPG_TICKET_DONE = 3,     /* output ready until released */
    DPG_TICKET_FAILED = 4    /* status says why (DPG_ERR_BUSY: larger than the budget) */
} dpg_ticket_state;

typedef struct {
    int64_t submitted, completed, failed, batches;
    double p50_ms, p99_ms, max_ms, mean_ms;  /* submit -> completion, completed requests */
    double bytes_delivered;                  /* output bytes of completed requests */
    double span_s;                           /* first submit -> last completion */
    size_t arena_in_use, arena_high_water;
    double launch_s;                         /* host time the scheduler spent enqueueing work */
} dpg_server_stats;

typedef struct dpg_server dpg_server;
dpg_status dpg_server_create(dpg_ctx *ctx, const dpg_server_config *cfg, dpg_server **out);
/* Queue a request (its dst is ignored: the output is allocated in the arena at
 * admission).  Invalid requests are accepted as FAILED tickets: INVALID_ARG
 * for a malformed request or one whose inputs overlap the arena, BUSY for one
 * whose output and workspace (each rounded up to 256 bytes) exceed what the
 * arena can ever hold for requests: its size less the batch workspaces the
 * server keeps per stream slot. */
dpg_status dpg_server_submit(dpg_server *server, const dpg_request *req, uint64_t *ticket);
/* Queue n requests in order, as n calls of dpg_server_submit would, taking the
 * server lock once (a client handing over a burst); tickets[i] receives
 * request i's ticket.  DPG_ERR_INVALID_ARG, with nothing queued, for a null
 * pointer, n < 0 or a server being destroyed. */
dpg_status dpg_server_submit_many(dpg_server *server, const dpg_request *reqs, int32_t n, uint64_t *tickets);
/* *dst: device address of the output once DONE (valid until released). */
dpg_status dpg_server_poll(dpg_server *server, uint64_t ticket, int32_t *state, dpg_status *status,
                           void **dst, double *latency_ms);
/* Next finished (DONE or FAILED) ticket in completion order; waits up to
 * timeout_ms; DPG_ERR_BUSY if none finished in that time. */
dpg_status dpg_server_next_completed(dpg_server *server, int32_t timeout_ms, uint64_t *ticket);
/* Free a finished ticket and its output memory. */
dpg_status dpg_server_release(dpg_server *server, uint64_t ticket);
dpg_status dpg_server_stats_get(dpg_server *server, dpg_server_stats *out);
dpg_status dpg_server_reset_stats(dpg_server *server);
/* Finishes all submitted work, then frees the server (not the arena).  Queued
 * requests that cannot be admitted once no work is left in flight (their
 * memory is held by outputs not yet released) fail with DPG_ERR_BUSY. */
void dpg_server_destroy(dpg_server *server);

/* ------------------------------------------------------------------------- */
/* Per-kernel timing.  When enabled, every kernel the context launches is     */
/* bracketed by HIP events on its own stream, and its algorithmic bytes (what */
/* the algorithm must read and write, excluding cache effects) are recorded.  */
/* ------------------------------------------------------------------------- */
dpg_status dpg_profile_enable(dpg_ctx *ctx, int on);

/* Measurement ceiling (not part of the method): copy `bytes` (a multiple of
 * 16) from src to dst, both 16-byte aligned and not overlapping, as a plain
 * stream of 16-byte vectors -- each lane loads vectors_per_lane (2, 4, 8 or 16)
 * vectors before storing them, nontemporal = 1 uses streaming stores.  The
 * read + write rate this reaches on large buffers is the practical roof the
 * probe and gather phases (which also read once and write once) are held
 * against.  DPG_ERR_INVALID_ARG for a bad size, alignment, overlap or
 * option. */
dpg_status dpg_stream_copy(dpg_ctx *ctx, const void *src, void *dst, size_t bytes, int32_t vectors_per_lane,
                           int32_t nontemporal, hipStream_t stream);
dpg_status dpg_profile_reset(dpg_ctx *ctx);
/* Synchronizes the recorded events and folds them into per-kernel totals.
 * *n_kernels receives the number of distinct kernels seen. */
dpg_status dpg_profile_collect(dpg_ctx *ctx, int32_t *n_kernels);
dpg_status dpg_profile_entry(const dpg_ctx *ctx, int32_t index, const char **name,
                             int64_t *launches, double *total_ms, double *total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* DPG_H_ */
