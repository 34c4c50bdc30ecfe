// Hash index and batch lookup (Section 4.2.3, batch lookup in hash indexes).
//
// The index holds one key-rid pair per hash slot and keeps the pairs that
// collide with an occupied slot in an overflow array grouped by home slot
// (the paper's second array of pointers becomes per-slot offsets).  The home
// slot of key k is the top s bits of k * kHashMul (mod 2^32).
//
// Build: the (home, rid) pairs are sorted by home with stable 8-bit passes, so
// the first pair of every home has its smallest rid; that pair takes the slot
// and the others go to the overflow array in sorted order, at positions given
// by an exclusive scan of "not first of its home" flags.  ov_off[h] is then
// the scan value at the first sorted position whose home is >= h.
//
// Batch lookup with DPG: since kHashMul is odd, z = k * kHashMul is a
// bijection of the key, and the partition of the index a key probes is the top
// bits of z.  Phase I partitions the z values of the queries by those bits;
// Phase II runs over the partitioned z values, recovers each key as
// z * kHashMul^-1, and probes the slot z >> (32 - s) and its overflow range
// while that partition of the index is cache resident; Phase III gathers the
// rids back into query order (the DPG gather with 4-byte records).
#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

constexpr uint32_t kHashMul = 0x9E3779B1u;

// Inverse of an odd a modulo 2^32 by Newton's iteration x <- x (2 - a x): the
// start x = a is correct to 3 bits and every step doubles the correct bits.
constexpr uint32_t mul_inverse(uint32_t a) {
    uint32_t x = a;
    for (int i = 0; i < 5; ++i) x *= 2u - a * x;
    return x;
}
constexpr uint32_t kHashMulInv = mul_inverse(kHashMul);
static_assert(kHashMul * kHashMulInv == 1u, "multiplicative inverse");

constexpr int kHashMinLog2 = 4, kHashMaxLog2 = 30;

static size_t ov_off_offset(int s) { return align_up((size_t)8 << s); }
static size_t ov_offset(int s) { return align_up(ov_off_offset(s) + 4 * (((size_t)1 << s) + 1)); }

__device__ __forceinline__ uint32_t slot_of(uint32_t z, int s) { return z >> (32 - s); }

// Probe one key whose home slot is h: the slot, then its overflow range
// (clamped to the n_keys pairs the overflow array can hold).
__device__ __forceinline__ int32_t probe_key(const uint2 *__restrict__ slots, const int32_t *__restrict__ ov_off,
                                             const uint2 *__restrict__ ov, int64_t n_keys, uint32_t q, uint32_t h) {
    const uint2 sl = slots[h];
    if (sl.y == DPG_HASH_EMPTY) return -1;
    if (sl.x == q) return (int32_t)sl.y;
    const int64_t a = max((int64_t)ov_off[h], (int64_t)0), b = min((int64_t)ov_off[h + 1], n_keys);
    for (int64_t x = a; x < b; ++x) {
        const uint2 e = ov[x];
        if (e.x == q) return (int32_t)e.y;
    }
    return -1;
}

// ---- build ---------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hash_home(const uint32_t *__restrict__ keys, int64_t n, int s,
                                                   uint32_t *__restrict__ home, uint32_t *__restrict__ idx) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    home[j] = slot_of(keys[j] * kHashMul, s);
    idx[j] = (uint32_t)j;
}

// flag[p] = 1 when sorted pair p is not the first of its home; empty slots.
__global__ __launch_bounds__(256) void k_hash_mark(const uint32_t *__restrict__ hs, int64_t n,
                                                   int32_t *__restrict__ flag, uint2 *__restrict__ slots,
                                                   int64_t S) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) flag[p] = (p > 0 && hs[p - 1] == hs[p]) ? 1 : 0;
    if (p < S) slots[p] = make_uint2(0u, DPG_HASH_EMPTY);
}

// Place sorted pair p: the first of its home into the slot, the others into
// the overflow array at their scanned position.
__global__ __launch_bounds__(256) void k_hash_place(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ hs,
                                                    const uint32_t *__restrict__ js, const int32_t *__restrict__ ovpos,
                                                    int64_t n, uint2 *__restrict__ slots, uint2 *__restrict__ ov) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const uint32_t h = hs[p], j = js[p];
    const uint2 pair = make_uint2(keys[j], j);
    if (p > 0 && hs[p - 1] == h) ov[ovpos[p]] = pair;
    else slots[h] = pair;
}

// ov_off[h] for h in [0, S]: overflow pairs before the first sorted pair whose
// home is >= h (binary search in the sorted homes).
__global__ __launch_bounds__(256) void k_hash_ov_off(const uint32_t *__restrict__ hs, int64_t n,
                                                     const int32_t *__restrict__ ovpos,
                                                     const int32_t *__restrict__ n_ov, int64_t S,
                                                     int32_t *__restrict__ ov_off) {
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (h > S) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)hs[mid] < h) lo = mid + 1;
        else hi = mid;
    }
    ov_off[h] = lo < n ? ovpos[lo] : *n_ov;
}

// ---- lookup ----------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hash_direct(const uint32_t *__restrict__ queries, int64_t m,
                                                     const uint2 *__restrict__ slots,
                                                     const int32_t *__restrict__ ov_off,
                                                     const uint2 *__restrict__ ov, int64_t n_keys, int s,
                                                     int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const uint32_t q = queries[i];
    out[i] = probe_key(slots, ov_off, ov, n_keys, q, slot_of(q * kHashMul, s));
}

// Phase II over the partitioned z values: internal[p] = rid of key z * kHashMul^-1.
__global__ __launch_bounds__(256) void k_hash_probe(const uint32_t *__restrict__ zrun, int64_t m,
                                                    const uint2 *__restrict__ slots,
                                                    const int32_t *__restrict__ ov_off, const uint2 *__restrict__ ov,
                                                    int64_t n_keys, int s, int32_t *__restrict__ internal) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= m) return;
    const uint32_t z = zrun[p];
    internal[p] = probe_key(slots, ov_off, ov, n_keys, z * kHashMulInv, slot_of(z, s));
}

// Phase II with the run's slots staged in LDS.  Work item = (run b, chunk of
// at most P queries of run b); the workgroup loads slots [b*L, (b+1)*L) with
// 16-byte loads, then probes its queries there (an overflow range, needed only
// when the slot holds another key, is read through the caches).
constexpr int kHashProbeThreads = 1024;
constexpr int kHashProbeBatch = 16;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kHashProbeThreads) void k_hash_probe_lds(
    const uint32_t *__restrict__ zrun, const int32_t *__restrict__ run_off, const int32_t *__restrict__ item_off,
    int B, int lg_l, int P, const uint2 *__restrict__ slots, const int32_t *__restrict__ ov_off,
    const uint2 *__restrict__ ov, int64_t n_keys, int s, int32_t *__restrict__ internal) {
    extern __shared__ __align__(16) char smem[];
    uint2 *s_slots = (uint2 *)smem;
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
    const int L = 1 << lg_l;
    const int64_t base = (int64_t)b << lg_l;
    const u32x4 *src4 = (const u32x4 *)(slots + base);
    u32x4 *dst4 = (u32x4 *)s_slots;
#pragma unroll 4
    for (int e = threadIdx.x; e < L / 2; e += kHashProbeThreads) dst4[e] = src4[e];
    __syncthreads();
    // the chunk's keys are loaded kHashProbeBatch per thread at a time, all in
    // flight together, before any is probed
    for (int j0 = 0; j0 < cnt; j0 += kHashProbeThreads * kHashProbeBatch) {
        uint32_t zz[kHashProbeBatch];
#pragma unroll
        for (int k = 0; k < kHashProbeBatch; ++k)
            zz[k] = zrun[k0 + min(j0 + (int)threadIdx.x + k * kHashProbeThreads, cnt - 1)];
        // 1. the home slot, from LDS; a query whose slot holds another key
        // needs the overflow range of that slot
        int32_t r[kHashProbeBatch];
        uint32_t qk[kHashProbeBatch], hk[kHashProbeBatch];
        bool need[kHashProbeBatch];
#pragma unroll
        for (int k = 0; k < kHashProbeBatch; ++k) {
            const int j = j0 + (int)threadIdx.x + k * kHashProbeThreads;
            const uint32_t z = zz[k];
            qk[k] = z * kHashMulInv;
            hk[k] = slot_of(z, s);
            const int64_t local = (int64_t)hk[k] - base;
            r[k] = -1;
            need[k] = false;
            if (j < cnt && local >= 0 && local < L) {
                const uint2 sl = s_slots[local];
                if (sl.y != DPG_HASH_EMPTY) {
                    if (sl.x == qk[k]) r[k] = (int32_t)sl.y;
                    else need[k] = true;
                }
            }
        }
        // 2. the overflow ranges, all loads in flight together
        int64_t a[kHashProbeBatch], e[kHashProbeBatch];
#pragma unroll
        for (int k = 0; k < kHashProbeBatch; ++k) {
            a[k] = 0;
            e[k] = 0;
            if (need[k]) {
                a[k] = max((int64_t)ov_off[hk[k]], (int64_t)0);
                e[k] = min((int64_t)ov_off[hk[k] + 1], n_keys);
            }
        }
        // 3. the first key of each range that matches
#pragma unroll
        for (int k = 0; k < kHashProbeBatch; ++k) {
            for (int64_t x = a[k]; x < e[k]; ++x) {
                const uint2 o = ov[x];
                if (o.x == qk[k]) {
                    r[k] = (int32_t)o.y;
                    break;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kHashProbeBatch; ++k) {
            const int j = j0 + (int)threadIdx.x + k * kHashProbeThreads;
            if (j < cnt) internal[k0 + j] = r[k];
        }
    }
}

// ---- workspace layout --------------------------------------------------------
struct HashBuildPlan {
    int64_t n = 0;
    int s = 0;
    PartPlan part;
    size_t off_home[2] = {0, 0}, off_idx[2] = {0, 0}, off_part = 0, off_flag = 0, off_scan = 0, off_total = 0;
    size_t workspace = 0;
};

static bool hash_args_ok(int64_t n_keys, int32_t log2_slots) {
    return n_keys >= 0 && n_keys <= INT32_MAX - 1 && log2_slots >= kHashMinLog2 && log2_slots <= kHashMaxLog2;
}

static HashBuildPlan make_build_plan(int64_t n, int s) {
    HashBuildPlan p;
    p.n = n;
    p.s = s;
    p.part = plan_partition(n, 8, 4, true);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    p.off_home[0] = take(nn * 4);
    p.off_home[1] = take(nn * 4);
    p.off_idx[0] = take(nn * 4);
    p.off_idx[1] = take(nn * 4);
    p.off_part = take(p.part.workspace);
    p.off_flag = take(nn * 4);
    p.off_scan = take(scan_1d_scratch_bytes(n));
    p.off_total = take(4);
    p.workspace = off;
    return p;
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

static dpg_status run_build(dpg_ctx *ctx, const HashBuildPlan &p, const uint32_t *keys, void *index, void *ws,
                            hipStream_t stream) {
    char *w = (char *)ws, *ix = (char *)index;
    const int64_t n = p.n, S = (int64_t)1 << p.s;
    uint2 *slots = (uint2 *)ix;
    int32_t *ov_off = (int32_t *)(ix + ov_off_offset(p.s));
    uint2 *ov = (uint2 *)(ix + ov_offset(p.s));
    int32_t *flag = (int32_t *)(w + p.off_flag);
    int32_t *n_ov = (int32_t *)(w + p.off_total);
    int cur = 0;
    if (n > 0) {
        ProfScope prof(ctx, K_HASH_HOME, 12.0 * n, stream);
        hipLaunchKernelGGL(k_hash_home, dim3(grid_of(n)), dim3(256), 0, stream, keys, n, p.s,
                           (uint32_t *)(w + p.off_home[0]), (uint32_t *)(w + p.off_idx[0]));
        DPG_HIP(hipGetLastError());
    }
    // stable LSD passes over the home bits
    for (int shift = 0; n > 0 && shift < p.s; shift += 8) {
        const int other = 1 - cur;
        const dpg_status st = launch_partition(ctx, p.part, w + p.off_home[cur], (const uint32_t *)(w + p.off_idx[cur]),
                                               w + p.off_home[other], (uint32_t *)(w + p.off_idx[other]), nullptr,
                                               shift, 0, w + p.off_part, stream, nullptr);
        if (st != DPG_OK) return st;
        cur = other;
    }
    const uint32_t *hs = (const uint32_t *)(w + p.off_home[cur]);
    const uint32_t *js = (const uint32_t *)(w + p.off_idx[cur]);
    {
        ProfScope prof(ctx, K_HASH_MARK, 8.0 * n + 8.0 * S, stream);
        hipLaunchKernelGGL(k_hash_mark, dim3(grid_of(n > S ? n : S)), dim3(256), 0, stream, hs, n, flag, slots, S);
        DPG_HIP(hipGetLastError());
    }
    dpg_status st = launch_scan_1d(ctx, flag, n, (int32_t *)(w + p.off_scan), n_ov, stream);
    if (st != DPG_OK) return st;
    if (n > 0) {
        ProfScope prof(ctx, K_HASH_PLACE, 24.0 * n, stream);
        hipLaunchKernelGGL(k_hash_place, dim3(grid_of(n)), dim3(256), 0, stream, keys, hs, js, flag, n, slots, ov);
        DPG_HIP(hipGetLastError());
    }
    {
        ProfScope prof(ctx, K_HASH_OVOFF, 4.0 * (S + 1), stream);
        hipLaunchKernelGGL(k_hash_ov_off, dim3(grid_of(S + 1)), dim3(256), 0, stream, hs, n, flag, n_ov, S, ov_off);
        DPG_HIP(hipGetLastError());
    }
    return DPG_OK;
}

}  // namespace dpg

using namespace dpg;

extern "C" {

size_t dpg_hash_ov_off_offset(int32_t log2_slots) {
    return (log2_slots >= kHashMinLog2 && log2_slots <= kHashMaxLog2) ? ov_off_offset(log2_slots) : 0;
}

size_t dpg_hash_ov_offset(int32_t log2_slots) {
    return (log2_slots >= kHashMinLog2 && log2_slots <= kHashMaxLog2) ? ov_offset(log2_slots) : 0;
}

size_t dpg_hash_index_bytes(int64_t n_keys, int32_t log2_slots) {
    if (!hash_args_ok(n_keys, log2_slots)) return 0;
    return ov_offset(log2_slots) + align_up((size_t)(n_keys > 0 ? n_keys : 1) * 8);
}

size_t dpg_hash_build_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys, int32_t log2_slots) {
    (void)ctx;
    if (!hash_args_ok(n_keys, log2_slots)) return 0;
    return make_build_plan(n_keys, log2_slots).workspace;
}

dpg_status dpg_hash_build(dpg_ctx *ctx, const uint32_t *keys, int64_t n_keys, int32_t log2_slots, void *index,
                          size_t index_bytes, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!hash_args_ok(n_keys, log2_slots)) return DPG_ERR_INVALID_ARG;
    if (n_keys > 0 && (!keys || ((uintptr_t)keys) % 4)) return DPG_ERR_INVALID_ARG;
    const size_t need_index = dpg_hash_index_bytes(n_keys, log2_slots);
    if (!index || ((uintptr_t)index) % kAlign || index_bytes < need_index) return DPG_ERR_INVALID_ARG;
    const HashBuildPlan p = make_build_plan(n_keys, log2_slots);
    if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    if (ranges_overlap(index, need_index, keys, (size_t)n_keys * 4) ||
        ranges_overlap(index, need_index, workspace, p.workspace) ||
        ranges_overlap(workspace, p.workspace, keys, (size_t)n_keys * 4))
        return DPG_ERR_INVALID_ARG;
    if (!ctx) return DPG_ERR_INVALID_ARG;
    return run_build(ctx, p, keys, index, workspace, stream);
}

size_t dpg_hash_lookup_workspace_bytes(const dpg_ctx *ctx, int64_t n_keys, int32_t log2_slots, int64_t n_queries,
                                       dpg_algo algo) {
    if (!hash_args_ok(n_keys, log2_slots) || n_queries < 0 || n_queries > INT32_MAX - 1) return 0;
    if (algo == DPG_ALGO_DIRECT) return kAlign;
    if (algo != DPG_ALGO_AUTO && algo != DPG_ALGO_DPG) return 0;
    RetrievePlan p;
    if (make_hash_lookup_plan(n_queries, log2_slots, ctx ? (int)ctx->opt_log2_run : 0,
                              ctx ? (int)ctx->opt_gather : 0, ctx ? (int)ctx->opt_probe : 0, &p) != DPG_OK)
        return 0;
    return p.workspace;
}

dpg_status dpg_hash_lookup(dpg_ctx *ctx, const void *index, int64_t n_keys, int32_t log2_slots,
                           const uint32_t *queries, int64_t n_queries, int32_t *rids, void *workspace,
                           size_t workspace_bytes, dpg_algo algo, hipStream_t stream) {
    if (!hash_args_ok(n_keys, log2_slots) || n_queries < 0 || n_queries > INT32_MAX - 1) return DPG_ERR_INVALID_ARG;
    if (algo < DPG_ALGO_AUTO || algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    const size_t index_bytes = dpg_hash_index_bytes(n_keys, log2_slots);
    if (!index || ((uintptr_t)index) % kAlign) return DPG_ERR_INVALID_ARG;
    if (n_queries > 0 && (!queries || !rids)) return DPG_ERR_INVALID_ARG;
    if (((uintptr_t)queries | (uintptr_t)rids) % 4) return DPG_ERR_INVALID_ARG;
    const size_t qb = (size_t)n_queries * 4;
    if (ranges_overlap(rids, qb, queries, qb) || ranges_overlap(rids, qb, index, index_bytes))
        return DPG_ERR_INVALID_ARG;
    const int a = algo == DPG_ALGO_DIRECT ? DPG_ALGO_DIRECT : DPG_ALGO_DPG;
    RetrievePlan p;
    if (a == DPG_ALGO_DPG) {
        const dpg_status st = make_hash_lookup_plan(n_queries, log2_slots, ctx ? (int)ctx->opt_log2_run : 0,
                                                    ctx ? (int)ctx->opt_gather : 0, ctx ? (int)ctx->opt_probe : 0,
                                                    &p);
        if (st != DPG_OK) return st;
        if (n_queries > 0) {
            if (workspace_bytes < p.workspace) return DPG_ERR_WORKSPACE_TOO_SMALL;
            if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
            if (ranges_overlap(workspace, p.workspace, rids, qb) ||
                ranges_overlap(workspace, p.workspace, queries, qb) ||
                ranges_overlap(workspace, p.workspace, index, index_bytes))
                return DPG_ERR_INVALID_ARG;
        }
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    if (n_queries == 0) return DPG_OK;
    const char *ix = (const char *)index;
    const uint2 *slots = (const uint2 *)ix;
    const int32_t *ov_off = (const int32_t *)(ix + ov_off_offset(log2_slots));
    const uint2 *ov = (const uint2 *)(ix + ov_offset(log2_slots));
    const double M = (double)n_queries;
    if (a == DPG_ALGO_DIRECT) {
        ProfScope prof(ctx, K_HASH_DIRECT, 16.0 * M, stream);
        hipLaunchKernelGGL(k_hash_direct, dim3(grid_of(n_queries)), dim3(256), 0, stream, queries, n_queries, slots,
                           ov_off, ov, n_keys, log2_slots, rids);
        DPG_HIP(hipGetLastError());
        return DPG_OK;
    }
    // Phase I: distribute z = key * kHashMul by its top bits (the index partition)
    char *w = (char *)workspace;
    const PartPlan pp = dist_partition(p);
    const bool lds_probe = p.probe == DPG_PROBE_LDS;
    int32_t *item_off = lds_probe ? (int32_t *)(w + p.off_items) : nullptr;
    int32_t *run_off = nullptr;
    dpg_status st = launch_partition(ctx, pp, queries, nullptr, w + p.off_run, nullptr, (int32_t *)(w + p.off_inv),
                                     p.log2_run, 0, w + p.off_part, stream, &run_off, item_off,
                                     lds_probe ? p.probe_chunk : 0, /*stable=*/false, p.gather_lds, kHashMul);
    if (st != DPG_OK) return st;
    // Phase II: probe one partition of the index at a time
    if (lds_probe) {
        const int B = (int)p.n_runs, lg_l = log2_slots - p.part_nbits, P = p.probe_chunk;
        const size_t lds = (size_t)8 << lg_l;
        const int64_t grid = (int64_t)B + (n_queries + P - 1) / P;
        ProfScope prof(ctx, K_HASH_PROBE_LDS, 8.0 * M + 8.0 * ((double)((int64_t)1 << log2_slots)), stream);
        if (lds > 64 * 1024)
            DPG_HIP(hipFuncSetAttribute((const void *)k_hash_probe_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds));
        hipLaunchKernelGGL(k_hash_probe_lds, dim3((unsigned)grid), dim3(kHashProbeThreads), lds, stream,
                           (const uint32_t *)(w + p.off_run), run_off, item_off, B, lg_l, P, slots, ov_off, ov,
                           n_keys, log2_slots, (int32_t *)(w + p.off_internal));
        DPG_HIP(hipGetLastError());
    } else {
        ProfScope prof(ctx, K_HASH_PROBE, 8.0 * M + 8.0 * ((double)((int64_t)1 << log2_slots)), stream);
        hipLaunchKernelGGL(k_hash_probe, dim3(grid_of(n_queries)), dim3(256), 0, stream,
                           (const uint32_t *)(w + p.off_run), n_queries, slots, ov_off, ov, n_keys, log2_slots,
                           (int32_t *)(w + p.off_internal));
        DPG_HIP(hipGetLastError());
    }
    // Phase III: rids back into query order
    if (p.gather_lds) return launch_gather_lds(ctx, p, workspace, rids, stream);
    return launch_gather(ctx, K_GATHER_PHASE, w + p.off_internal, n_queries, (const int32_t *)(w + p.off_inv), rids,
                         n_queries, 4, 12.0 * M, stream);
}

}  // extern "C"
