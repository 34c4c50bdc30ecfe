// Enhanced B+ tree and batch lookup (Section 4.2.3, batch lookup in B+ tree
// indexes).
//
// The tree is "enhanced": every slot of every node is used, so it is fixed by
// its entries.  Fanout 32: a node is 32 uint32 keys, one 128-byte line.
// Level 0 holds the (key, rid) entries sorted by key, then rid, as a key
// array and a rid array, padded with (0xFFFFFFFF, -1) to whole blocks of 32.
// Level l >= 1 has ceil(nodes(l-1) / 32) nodes; entry i of node j is the
// largest key under child 32 j + i (that child's last entry), or 0xFFFFFFFF
// past the last child.  The top level is one node.
//
// Build: the (key, position) pairs are sorted by four stable 8-bit passes, so
// equal keys stay in rid order, and the last pass writes straight into the
// leaf arrays; then every inner level is formed from the one below it.
//
// Lookup, direct: one root-to-leaf walk per query, in query order.  In a node
// the walk takes the first entry that is not below the query; in the leaf the
// first such key, whose rid is the answer when the key equals the query.
//
// Lookup with DPG: the two-pass lookup of Section 4.2.3 with DPG around it.
// The leaf blocks are cut into runs of G consecutive blocks (G a multiple of
// 32: whole level-1 subtrees).  The largest key of every run is the level-1
// entry of its last block; those keys, in order, are the search structure of
// the top of the tree down to the runs' subtree roots.
//   Phase I   one partition pass puts each query into the first run whose
//             largest key is not below it (a search over those keys staged in
//             LDS): the top-half walk;
//   Phase II  for each run, its leaf keys and rids and its level-1 entries are
//             staged in LDS and the walk continues there for all its queries;
//             the rids are written to INTERNAL in run order;
//   Phase III the rids are gathered back into query order.
// A run whose leaves do not fit LDS (trees above 2^26 entries) is probed by
// walking from the root through the caches instead, one run after another.
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBtFan = 32;
constexpr uint32_t kBtPad = 0xFFFFFFFFu;
constexpr int kBtMaxLevels = 8;
constexpr int kBtMaxRunBlocks = 512;  // LDS probe: 16384 entries, 128 KiB of keys and rids
constexpr int kBtTop = 16;            // level-1 nodes of one run, at most kBtMaxRunBlocks / 32

struct BtShape {
    int levels = 0;
    int64_t nodes[kBtMaxLevels] = {};
    size_t off[kBtMaxLevels] = {};  // byte offset of each level's keys
    size_t rid_off = 0;             // byte offset of the leaf rids
    size_t bytes = 0;
};

static bool bt_shape(int64_t n, BtShape *s) {
    if (n < 0 || n > INT32_MAX - 1) return false;
    *s = BtShape();
    int64_t c = (n + kBtFan - 1) / kBtFan;
    if (c < 1) c = 1;
    for (;;) {
        if (s->levels >= kBtMaxLevels) return false;
        s->nodes[s->levels++] = c;
        if (c == 1) break;
        c = (c + kBtFan - 1) / kBtFan;
    }
    const size_t node_bytes = 4 * kBtFan;
    s->rid_off = align_up((size_t)s->nodes[0] * node_bytes);
    size_t end = s->rid_off + (size_t)s->nodes[0] * node_bytes;
    for (int l = 1; l < s->levels; ++l) {
        s->off[l] = align_up(end);
        end = s->off[l] + (size_t)s->nodes[l] * node_bytes;
    }
    s->bytes = align_up(end);
    return true;
}

struct BtView {
    const uint32_t *lv[kBtMaxLevels];
    int64_t nodes[kBtMaxLevels];
    const int32_t *rids;
    int levels;
};

static BtView bt_view(const void *tree, const BtShape &s) {
    BtView v{};
    const char *b = (const char *)tree;
    for (int l = 0; l < s.levels; ++l) {
        v.lv[l] = (const uint32_t *)(b + s.off[l]);
        v.nodes[l] = s.nodes[l];
    }
    v.rids = (const int32_t *)(b + s.rid_off);
    v.levels = s.levels;
    return v;
}

// Number of the 32 keys of a node (16-byte aligned, global or LDS) below q.
__device__ __forceinline__ int bt_rank(const uint32_t *node, uint32_t q) {
    const u32x4 *p = (const u32x4 *)node;
    u32x4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[k];
    int c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) c += (v[k].x < q) + (v[k].y < q) + (v[k].z < q) + (v[k].w < q);
    return c;
}

// Nodes staged in LDS are stored swizzled: entry i of node c at
// c * 32 + (i ^ (c & 31)).  Lanes walking different nodes read the same entry
// index in the same step; unswizzled, every node starts on bank 0 and those
// reads all fall on one bank.
__device__ __forceinline__ int bt_sw(int c, int i) { return c * kBtFan + (i ^ (c & (kBtFan - 1))); }

// Number of the 32 keys of swizzled node c below q, by a branch-free binary
// search (entries ascending): five halving steps, then one more comparison
// for the count 32.
__device__ __forceinline__ int bt_rank_lds_sw(const uint32_t *base, int c, uint32_t q) {
    int pos = 0;
#pragma unroll
    for (int step = kBtFan / 2; step > 0; step >>= 1) pos += base[bt_sw(c, pos + step - 1)] < q ? step : 0;
    return pos + (base[bt_sw(c, pos)] < q ? 1 : 0);
}

// Element k of v (k in 0..3).
__device__ __forceinline__ uint32_t u4_at(const u32x4 &v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// Store the 4 entries 4m..4m+3 of node c (v, in entry order) to their
// swizzled places: the 16-byte group m ^ (c >> 2 & 7), permuted inside by c & 3.
__device__ __forceinline__ void bt_store4_sw(uint32_t *base, int c, int m, const u32x4 &v) {
    const int x = c & (kBtFan - 1);
    const int lo = x & 3;
    u32x4 w;
    w.x = u4_at(v, 0 ^ lo);
    w.y = u4_at(v, 1 ^ lo);
    w.z = u4_at(v, 2 ^ lo);
    w.w = u4_at(v, 3 ^ lo);
    *(u32x4 *)(base + c * kBtFan + 4 * (m ^ (x >> 2))) = w;
}

// Root-to-leaf walk: the rid of the first entry whose key is q, or -1.  The
// level loop is unrolled so that the view's arrays are indexed by constants.
__device__ __forceinline__ int32_t bt_walk(const BtView &t, uint32_t q) {
    int64_t node = 0;
#pragma unroll
    for (int l = kBtMaxLevels - 1; l >= 1; --l) {
        if (l < t.levels) {
            const int r = bt_rank(t.lv[l] + node * kBtFan, q);
            const int64_t c = node * kBtFan + r;
            if (r == kBtFan || c >= t.nodes[l - 1]) return -1;  // above every key
            node = c;
        }
    }
    const int r = bt_rank(t.lv[0] + node * kBtFan, q);
    if (r == kBtFan) return -1;
    const int64_t e = node * kBtFan + r;
    return t.lv[0][e] == q ? t.rids[e] : -1;
}

// ---- build -------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bt_iota(uint32_t *__restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

// Leaf padding: entries [n, slots) become (0xFFFFFFFF, -1).
__global__ __launch_bounds__(64) void k_bt_pad(uint32_t *__restrict__ keys, int32_t *__restrict__ rids, int64_t n,
                                               int64_t slots) {
    const int64_t e = n + threadIdx.x;
    if (threadIdx.x < kBtFan && e < slots) {
        keys[e] = kBtPad;
        rids[e] = -1;
    }
}

// Inner level: entry c = last key of node c of the level below (or padding).
__global__ __launch_bounds__(256) void k_bt_level(const uint32_t *__restrict__ below, int64_t n_below,
                                                  uint32_t *__restrict__ level, int64_t n_entries) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n_entries) return;
    level[c] = c < n_below ? below[c * kBtFan + kBtFan - 1] : kBtPad;
}

// ---- lookup ------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bt_direct(BtView t, const uint32_t *__restrict__ q, int64_t m,
                                                   int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) out[i] = bt_walk(t, q[i]);
}

// Phase II through the caches: the same walk over the queries in run order.
__global__ __launch_bounds__(256) void k_bt_probe(BtView t, const uint32_t *__restrict__ qrun, int64_t m,
                                                  int32_t *__restrict__ internal) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) internal[i] = bt_walk(t, qrun[i]);
}

// split[r] = largest key of run r (the level-1 entry of its last block).
__global__ __launch_bounds__(256) void k_bt_splitters(const uint32_t *__restrict__ level1, int64_t G, int n_split,
                                                      uint32_t *__restrict__ split) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_split) split[i] = level1[(int64_t)(i + 1) * G - 1];
}

constexpr int kBtProbeThreads = 1024;
constexpr int kBtProbeBatch = 8;

// One workgroup per (run, chunk of at most P queries).  The run's G blocks
// (fewer for the last run) are staged in LDS: keys, rids, the level-1
// entries of its blocks (from the tree's level 1, or the single leaf block's
// last key when the tree has no inner level), and the largest key of each of
// its level-1 nodes.  Each query then walks node -> block -> key in LDS.
__global__ __launch_bounds__(kBtProbeThreads) void k_bt_probe_lds(
    const uint32_t *__restrict__ qrun, const int32_t *__restrict__ run_off, const int32_t *__restrict__ item_off,
    int B, int P, const uint32_t *__restrict__ leaf_keys, const int32_t *__restrict__ leaf_rids,
    const uint32_t *__restrict__ level1, int64_t n0, int G, int32_t *__restrict__ internal) {
    extern __shared__ __align__(16) char smem[];
    uint32_t *s_key = (uint32_t *)smem;
    int32_t *s_rid = (int32_t *)(s_key + (size_t)G * kBtFan);
    uint32_t *s_l1 = (uint32_t *)(s_rid + (size_t)G * kBtFan);
    __shared__ __align__(16) uint32_t s_top[kBtTop];
    __shared__ int s_bucket;
    const int32_t item = (int32_t)blockIdx.x;
    if (item >= item_off[B]) return;
    if (threadIdx.x == 0) {
        int lo = 0, hi = B - 1;  // largest b with item_off[b] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        s_bucket = lo;
    }
    __syncthreads();
    const int b = s_bucket;
    const int64_t k0 = (int64_t)run_off[b] + (int64_t)(item - item_off[b]) * P;
    const int64_t k1 = min(k0 + P, (int64_t)run_off[b + 1]);
    const int cnt = (int)(k1 - k0);
    const int64_t blk0 = (int64_t)b * G;
    const int nbr = (int)min((int64_t)G, n0 - blk0);  // blocks of this run (>= 1: every query has a run)
    const int nt = (nbr + kBtFan - 1) / kBtFan;        // its level-1 nodes
    {
        // swizzled staging (bt_sw): 16-byte groups of a node move whole
        const u32x4 *k4 = (const u32x4 *)(leaf_keys + blk0 * kBtFan);
        const u32x4 *r4 = (const u32x4 *)(leaf_rids + blk0 * kBtFan);
        const int n4 = nbr * (kBtFan / 4);
#pragma unroll 4
        for (int e = threadIdx.x; e < n4; e += kBtProbeThreads) {
            const int c = e / (kBtFan / 4), m = e % (kBtFan / 4);
            bt_store4_sw(s_key, c, m, k4[e]);
            bt_store4_sw((uint32_t *)s_rid, c, m, (u32x4)r4[e]);
        }
        for (int e = threadIdx.x; e < nt * kBtFan; e += kBtProbeThreads)
            s_l1[bt_sw(e / kBtFan, e % kBtFan)] =
                level1 ? level1[blk0 + e] : (e == 0 ? leaf_keys[kBtFan - 1] : kBtPad);
    }
    __syncthreads();
    if (threadIdx.x < kBtTop)
        s_top[threadIdx.x] = (int)threadIdx.x < nt ? s_l1[bt_sw((int)threadIdx.x, kBtFan - 1)] : kBtPad;
    __syncthreads();
    for (int j0 = 0; j0 < cnt; j0 += kBtProbeThreads * kBtProbeBatch) {
        uint32_t qq[kBtProbeBatch];
#pragma unroll
        for (int k = 0; k < kBtProbeBatch; ++k)
            qq[k] = qrun[k0 + min(j0 + (int)threadIdx.x + k * kBtProbeThreads, cnt - 1)];
#pragma unroll
        for (int k = 0; k < kBtProbeBatch; ++k) {
            const int j = j0 + (int)threadIdx.x + k * kBtProbeThreads;
            if (j >= cnt) break;
            const uint32_t q = qq[k];
            int32_t res = -1;
            // the run's level-1 node, then its block, then the key
            const u32x4 *tp = (const u32x4 *)s_top;
            int t = 0;
#pragma unroll
            for (int u = 0; u < kBtTop / 4; ++u) {
                const u32x4 v = tp[u];
                t += (v.x < q) + (v.y < q) + (v.z < q) + (v.w < q);
            }
            if (t < nt) {
                const int r1 = bt_rank_lds_sw(s_l1, t, q);
                const int c = t * kBtFan + r1;
                if (r1 < kBtFan && c < nbr) {
                    const int r0 = bt_rank_lds_sw(s_key, c, q);
                    if (r0 < kBtFan) {
                        const int e = bt_sw(c, r0);
                        if (s_key[e] == q) res = s_rid[e];
                    }
                }
            }
            internal[k0 + j] = res;
        }
    }
}

// ---- plans ---------------------------------------------------------------------
struct BtBuildPlan {
    int64_t n = 0;
    BtShape shape;
    PartPlan part;
    size_t off_ka = 0, off_va = 0, off_kb = 0, off_vb = 0, off_part = 0, workspace = 0;
};

static dpg_status make_build_plan(int64_t n, BtBuildPlan *p) {
    *p = BtBuildPlan();
    if (!bt_shape(n, &p->shape)) return DPG_ERR_INVALID_ARG;
    p->n = n;
    p->part = plan_partition(n, 8, 4, true);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + (bytes > 0 ? bytes : 1));
        return at;
    };
    p->off_ka = take((size_t)n * 4);
    p->off_va = take((size_t)n * 4);
    p->off_kb = take((size_t)n * 4);
    p->off_vb = take((size_t)n * 4);
    p->off_part = take(p->part.workspace);
    p->workspace = off;
    return DPG_OK;
}

struct BtLookupPlan {
    BtShape shape;
    RetrievePlan ret;
    int64_t G = 0, S = 0;  // blocks per run, runs
    bool lds = false;
    size_t off_split = 0, workspace = 0;
};

// Runs of G blocks: by default the smallest power of two >= 256 (8192
// entries, 64 KiB staged) that keeps the run count within one partition pass;
// DPG_OPT_LOG2_RUN sets log2 of the entries per run (at least 1024).  Measured
// at 2^24 keys and 2^26 queries: runs of 8192 entries beat 4096 (1.59 vs
// 1.85 ms: fewer runs for Phases I and III); at 2^26 keys the pass limit
// forces 16384.  Runs above 16384 entries are walked through the caches.
static dpg_status make_lookup_plan(const dpg_ctx *ctx, int64_t n_keys, int64_t n_queries, BtLookupPlan *p) {
    *p = BtLookupPlan();
    if (!bt_shape(n_keys, &p->shape) || n_queries < 0 || n_queries > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    const int64_t n0 = p->shape.nodes[0];
    const int lg_entries = ctx ? (int)ctx->opt_log2_run : 0;
    int64_t G = 256;
    if (lg_entries > 0) {
        G = lg_entries >= 10 ? ((int64_t)1 << (lg_entries - 5)) : kBtFan;
        if (G > ((int64_t)1 << 26)) G = (int64_t)1 << 26;
    }
    while ((n0 + G - 1) / G > kMaxWideBuckets) G *= 2;
    p->G = G;
    p->S = (n0 + G - 1) / G;
    const int probe = ctx ? (int)ctx->opt_probe : 0;
    p->lds = G <= kBtMaxRunBlocks && probe != DPG_PROBE_CACHED;
    const dpg_status st =
        make_split_lookup_plan(n_queries, p->S, ctx ? (int)ctx->opt_gather : 0, p->lds, &p->ret);
    if (st != DPG_OK) return st;
    p->off_split = p->ret.workspace;
    p->workspace = align_up(p->off_split + 4 * (size_t)p->S);
    return DPG_OK;
}

static unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace dpg

using namespace dpg;

extern "C" {

size_t dpg_btree_bytes(int64_t n_keys) {
    BtShape s;
    return bt_shape(n_keys, &s) ? s.bytes : 0;
}

int32_t dpg_btree_levels(int64_t n_keys) {
    BtShape s;
    return bt_shape(n_keys, &s) ? s.levels : 0;
}

size_t dpg_btree_level_offset(int64_t n_keys, int32_t level) {
    BtShape s;
    if (!bt_shape(n_keys, &s) || level < 0 || level >= s.levels) return 0;
    return s.off[level];
}

size_t dpg_btree_rids_offset(int64_t n_keys) {
    BtShape s;
    return bt_shape(n_keys, &s) ? s.rid_off : 0;
}

size_t dpg_btree_build_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys) {
    (void)ctx;
    BtBuildPlan p;
    return make_build_plan(n_keys, &p) == DPG_OK ? p.workspace : 0;
}

dpg_status dpg_btree_build(dpg_ctx *ctx, const uint32_t *keys, int64_t n_keys, void *tree, size_t tree_bytes,
                           void *workspace, size_t workspace_bytes, hipStream_t stream) {
    BtBuildPlan p;
    dpg_status st = make_build_plan(n_keys, &p);
    if (st != DPG_OK) return st;
    const BtShape &s = p.shape;
    if (!tree || ((uintptr_t)tree) % kAlign || tree_bytes < s.bytes) return DPG_ERR_INVALID_ARG;
    if (n_keys > 0 && (!keys || ((uintptr_t)keys) % 4)) return DPG_ERR_INVALID_ARG;
    const size_t kb = (size_t)n_keys * 4;
    if (ranges_overlap(tree, s.bytes, keys, kb)) return DPG_ERR_INVALID_ARG;
    if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    if (ranges_overlap(workspace, p.workspace, tree, s.bytes) || ranges_overlap(workspace, p.workspace, keys, kb))
        return DPG_ERR_INVALID_ARG;
    if (!ctx) return DPG_ERR_INVALID_ARG;
    char *w = (char *)workspace;
    char *tb = (char *)tree;
    uint32_t *leaf_keys = (uint32_t *)tb;
    int32_t *leaf_rids = (int32_t *)(tb + s.rid_off);
    const int64_t n = n_keys;
    if (n > 0) {
        // (key, position) pairs by four stable 8-bit passes; the last into the leaves
        uint32_t *ka = (uint32_t *)(w + p.off_ka), *va = (uint32_t *)(w + p.off_va);
        uint32_t *kbuf = (uint32_t *)(w + p.off_kb), *vb = (uint32_t *)(w + p.off_vb);
        hipLaunchKernelGGL(k_bt_iota, dim3(grid256(n)), dim3(256), 0, stream, vb, n);
        DPG_HIP(hipGetLastError());
        const void *kin = keys;
        const uint32_t *vin = vb;
        for (int pass = 0; pass < 4; ++pass) {
            void *kout = pass == 3 ? (void *)leaf_keys : (pass % 2 == 0 ? (void *)ka : (void *)kbuf);
            uint32_t *vout = pass == 3 ? (uint32_t *)leaf_rids : (pass % 2 == 0 ? va : vb);
            st = launch_partition(ctx, p.part, kin, vin, kout, vout, nullptr, 8 * pass, 0, w + p.off_part, stream,
                                  nullptr);
            if (st != DPG_OK) return st;
            kin = kout;
            vin = vout;
        }
    }
    hipLaunchKernelGGL(k_bt_pad, dim3(1), dim3(64), 0, stream, leaf_keys, leaf_rids, n, s.nodes[0] * kBtFan);
    DPG_HIP(hipGetLastError());
    for (int l = 1; l < s.levels; ++l) {
        const uint32_t *below = (const uint32_t *)(tb + s.off[l - 1]);
        const int64_t entries = s.nodes[l] * kBtFan;
        ProfScope prof(ctx, K_BT_LEVEL, 8.0 * entries, stream);
        hipLaunchKernelGGL(k_bt_level, dim3(grid256(entries)), dim3(256), 0, stream, below, s.nodes[l - 1],
                           (uint32_t *)(tb + s.off[l]), entries);
        DPG_HIP(hipGetLastError());
    }
    return DPG_OK;
}

size_t dpg_btree_lookup_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys, int64_t n_queries, dpg_algo algo) {
    BtShape s;
    if (!bt_shape(n_keys, &s) || n_queries < 0 || n_queries > INT32_MAX - 1) return 0;
    if (algo == DPG_ALGO_DIRECT) return kAlign;
    if (algo != DPG_ALGO_AUTO && algo != DPG_ALGO_DPG) return 0;
    BtLookupPlan p;
    if (make_lookup_plan(ctx, n_keys, n_queries, &p) != DPG_OK) return 0;
    return p.workspace;
}

dpg_status dpg_btree_lookup(dpg_ctx *ctx, const void *tree, int64_t n_keys, const uint32_t *queries,
                            int64_t n_queries, int32_t *rids, void *workspace, size_t workspace_bytes,
                            dpg_algo algo, hipStream_t stream) {
    BtShape s;
    if (!bt_shape(n_keys, &s) || n_queries < 0 || n_queries > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    if (algo < DPG_ALGO_AUTO || algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    if (!tree || ((uintptr_t)tree) % kAlign) return DPG_ERR_INVALID_ARG;
    if (n_queries > 0 && (!queries || !rids)) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)queries | (uintptr_t)rids) % 4) return DPG_ERR_INVALID_ARG;
    const size_t qb = (size_t)n_queries * 4;
    if (ranges_overlap(rids, qb, queries, qb) || ranges_overlap(rids, qb, tree, s.bytes))
        return DPG_ERR_INVALID_ARG;
    const bool dpg_path = algo != DPG_ALGO_DIRECT;
    BtLookupPlan p;
    if (dpg_path) {
        const dpg_status st = make_lookup_plan(ctx, n_keys, n_queries, &p);
        if (st != DPG_OK) return st;
        if (n_queries > 0) {
            if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
            if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
            if (ranges_overlap(workspace, p.workspace, rids, qb) ||
                ranges_overlap(workspace, p.workspace, queries, qb) ||
                ranges_overlap(workspace, p.workspace, tree, s.bytes))
                return DPG_ERR_INVALID_ARG;
        }
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    if (n_queries == 0) return DPG_OK;
    const BtView view = bt_view(tree, s);
    const double M = (double)n_queries;
    if (!dpg_path) {
        ProfScope prof(ctx, K_BT_DIRECT, M * (4.0 + 4.0 + kBtFan * 4.0 + 4.0), stream);
        hipLaunchKernelGGL(k_bt_direct, dim3(grid256(n_queries)), dim3(256), 0, stream, view, queries, n_queries,
                           rids);
        DPG_HIP(hipGetLastError());
        return DPG_OK;
    }
    const RetrievePlan &r = p.ret;
    char *w = (char *)workspace;
    const int n_split = (int)(p.S - 1);
    uint32_t *split = (uint32_t *)(w + p.off_split);
    const uint32_t *level1 = s.levels > 1 ? view.lv[1] : nullptr;
    if (n_split > 0) {
        hipLaunchKernelGGL(k_bt_splitters, dim3(grid256(n_split)), dim3(256), 0, stream, level1, p.G, n_split,
                           split);
        DPG_HIP(hipGetLastError());
    }
    // Phase I: each query into the run of the first subtree whose largest key is not below it
    const PartPlan pp = dist_partition(r);
    int32_t *item_off = p.lds ? (int32_t *)(w + r.off_items) : nullptr;
    int32_t *run_off = nullptr;
    dpg_status st = launch_partition(ctx, pp, queries, nullptr, w + r.off_run, nullptr, (int32_t *)(w + r.off_inv),
                                     0, 0, w + r.off_part, stream, &run_off, item_off, p.lds ? r.probe_chunk : 0,
                                     /*stable=*/false, r.gather_lds, 1u, split, n_split);  // no splitter: one run
    if (st != DPG_OK) return st;
    // Phase II: continue each walk inside its run
    const uint32_t *qrun = (const uint32_t *)(w + r.off_run);
    int32_t *internal = (int32_t *)(w + r.off_internal);
    if (p.lds) {
        const int B = 1 << r.part_nbits, P = r.probe_chunk;
        const int G = (int)p.G;
        const size_t lds = (size_t)G * kBtFan * 8 + (size_t)((G + kBtFan - 1) / kBtFan) * kBtFan * 4;
        const int64_t grid = (int64_t)p.S + (n_queries + P - 1) / P;
        ProfScope prof(ctx, K_BT_PROBE_LDS, 8.0 * M + 8.0 * kBtFan * (double)s.nodes[0], stream);
        if (lds > 64 * 1024)
            DPG_HIP(hipFuncSetAttribute((const void *)k_bt_probe_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds));
        hipLaunchKernelGGL(k_bt_probe_lds, dim3((unsigned)grid), dim3(kBtProbeThreads), lds, stream, qrun, run_off,
                           item_off, B, P, view.lv[0], view.rids, level1, s.nodes[0], G, internal);
        DPG_HIP(hipGetLastError());
    } else {
        ProfScope prof(ctx, K_BT_PROBE, 8.0 * M + 8.0 * kBtFan * (double)s.nodes[0], stream);
        hipLaunchKernelGGL(k_bt_probe, dim3(grid256(n_queries)), dim3(256), 0, stream, view, qrun, n_queries,
                           internal);
        DPG_HIP(hipGetLastError());
    }
    // Phase III: rids back into query order
    if (r.gather_lds) return launch_gather_lds(ctx, r, workspace, rids, stream);
    return launch_gather(ctx, K_GATHER_PHASE, internal, n_queries, (const int32_t *)(w + r.off_inv), rids,
                         n_queries, 4, 12.0 * M, stream);
}

}  // extern "C"
