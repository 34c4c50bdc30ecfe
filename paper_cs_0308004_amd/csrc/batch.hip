// Batched execution of many retrieval / join requests of uneven size in ONE
// launch of the persistent kernel k_batch.
//
// A fixed grid of workgroups pulls work items from a device queue.  An item is
// one tile of one step of one request:
//
//   OP_COPY     a tile of output rows A[ia] || B[ib] (retrieval: src[rid], no
//               B; fact-order join: fact[i] || dim[fk_i]); the same step is
//               the DPG probe (INTERNAL[k] = src[run[k]]) and the DPG gather
//               (dst[i] = INTERNAL[inv[i]], or fact[i] || INTERNAL[inv[i]])
//   OP_ZERO     clears a request's run histogram
//   OP_HIST     a tile of rids counted into the run histogram (Phase I)
//   OP_SCAN     the run boundaries: exclusive scan of the histogram
//   OP_SCATTER  a tile of rids placed into their runs (RID_RUN) with each
//               rid's slot recorded (inv)
//   OP_SHIST, OP_SSCAN, OP_SSCATTER
//               one stable 8-bit pass of a dimension-order join's sort
//
// A request planned as direct retrieval is one OP_COPY step; a request
// planned as DPG is the chain ZERO -> HIST -> SCAN -> SCATTER -> COPY (probe)
// -> COPY (gather), the three phases of Section 2.1 (DIST1 -> COPY -> COPY
// when its rids fit one distribute tile).  The queue lists every
// request's first step, then every request's second step, and so on, so a
// step rarely waits.  Atomics on one word are serialized by the device (about
// 20-30 ns each here), so the queue is touched as little as possible: when
// no step depends on another, workgroup b starts with item b and only the
// items after the grid's first round come from the queue, spread over eight
// words (with dependencies, one word hands out every item).  Before an
// item, a workgroup waits until every item of the step this one depends on
// (an earlier step of the same request) has finished: those items were taken
// from the queue earlier, by workgroups that are running, so the wait ends;
// a bounded spin (a timeout flag in the header) keeps a kernel from running
// on if that ever failed, and the writes at positions computed by earlier
// steps are bounds-checked, so such a kernel would still stay inside its
// arrays.
// Each finished item bumps its step's counter; the last item of a request's
// last step also writes the launch's sequence number into the request's
// completion word, which lives in host memory, so a host thread learns that
// the request is done while the batch is still running.
//
// A dimension-order (DPG-Sort) join is the chain of its stable 8-bit passes
// over the (fk, i) pairs (SHIST -> SSCAN -> SSCATTER per pass, low digit
// first, as many passes as the dimension's key bits need), then the move of
// the fact rows into fk order (the DPG chain over the sorted row numbers, or
// one copy when direct pays) fused with the read of the dimension rows in fk
// order: the final COPY writes fact[i_j] || dim[fk_j].
//
// The batch header (item count, step count, sequence number, queue words) and
// the steps (with their counters) live in device memory and are uploaded in
// one copy, so a captured graph of k_batch is replayed with new requests
// (dpg_batch_graph_*).
#include <algorithm>
#include <cstring>
#include <vector>

#include "dev_common.h"
#include "dpg_internal.h"
#include "partition.h"

namespace dpg {

enum BatchOp : int32_t {
    OP_COPY = 0,
    OP_ZERO = 1,
    OP_HIST = 2,
    OP_SCAN = 3,
    OP_SCATTER = 4,
    OP_SHIST = 5,     // stable sort pass: digit counts of a tile -> cnt[t][digit]
    OP_SSCAN = 6,     // stable sort pass: column scan of cnt (run boundaries per tile)
    OP_SSCATTER = 7,  // stable sort pass: (key, val) of a tile to their places, input order kept per digit
    OP_DIST1 = 8      // the whole distribute of a request of at most one tile, in LDS
};

struct BatchDesc {
    // OP_COPY: out row j = A[ia] || B[ib], ia = idx_a ? idx_a[j] : j,
    // ib = idx_b ? idx_b[j] : word fk_word of A row ia (when wb > 0)
    const uint32_t *a;
    const int32_t *idx_a;
    const uint32_t *b;
    const int32_t *idx_b;
    uint32_t *out;
    int64_t lim_a, lim_b;   // row counts of A and B (indices outside read row 0)
    int64_t n_rows;         // rows of the step: output rows, or rids of a distribute step
    int64_t item_start;     // first work item of this step
    int64_t n_items;
    int32_t wa, wb;         // dwords taken from A and from B per output row
    int32_t fk_word;        // word of the A row holding the foreign key (join)
    int32_t tile_rows;      // output rows per work item
    uint32_t magic;         // ceil(2^32 / ((wa + wb) / vec)) for the row division
    int32_t request;        // index in the caller's request array
    int32_t vec;            // dwords per access: 4 when rows and pointers are 16-byte aligned, else 1
    int32_t op;             // BatchOp
    int32_t dep;            // step whose items must all have finished first (-1: none)
    int32_t last;           // 1: the request is done when this step is
    // distribute steps: rid of element i = ids[i * id_stride + id_word], valid
    // in [0, lim_a) (else 0); run of a rid = rid >> lg_run, n_runs runs
    const uint32_t *ids;
    int32_t id_stride, id_word;
    int32_t lg_run, n_runs;
    int32_t *hist, *fill, *run_off, *run, *inv;
    // stable sort passes: key of element i as for the distribute (ids), its
    // value vals_in[i] (or i when null); digit (key >> shift) & 255; cnt the
    // (tiles x 256) count matrix
    const uint32_t *vals_in;
    uint32_t *keys_out, *vals_out;
    int32_t *cnt;
    int32_t shift, n_tiles;
    uint32_t done;          // items of this step finished (uploaded as 0)
    uint32_t pad;
};

// Queue words of a batch without dependencies: workgroup b takes its items
// after the grid's first round from queue b % 8 (item 8p + q is the p-th of
// queue q), so the serialized atomics of one word are spread over eight.
constexpr int kBatchQueues = 8;

struct BatchHeader {
    int64_t total_items;
    int32_t n_desc;
    uint32_t seq;         // launch sequence number, written into the completion words
    int32_t timeout;      // set when a dependency wait gave up (never in a correct run)
    int32_t no_deps;      // 1: no step waits on another (workgroup b then starts with item b)
    int32_t n_work;       // workgroups that take items when steps depend on each other
    uint32_t queue[kBatchQueues];  // work items taken from each queue (uploaded as 0)
};

constexpr int kBatchThreads = 256;
constexpr int kBatchPer = 16;
constexpr int kBatchMaxTileRows = 2048;
constexpr int kBatchItemWords = 8192;    // at least ~32 KiB of output per copy item
constexpr int kBatchDistTile = 4096;     // rids per distribute item (16 per thread)
constexpr int kBatchMaxRuns = 2048;      // runs of a request distributed inside the batch
constexpr int kBatchSteps = 6;           // steps of a DPG request
constexpr int kSortDigits = 256;         // 8-bit digits of the stable passes
constexpr int kBatchMaxSteps = 3 * 4 + kBatchSteps;  // most steps of one request (a dimension-order join)
constexpr uint64_t kBatchWaitTicks = 200000000ull;  // 2 s of the 100 MHz real-time counter

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
    // 16 dwords or 8 16-byte vectors in flight per lane
    constexpr int PER = VEC == 4 ? kBatchPer / 2 : kBatchPer;
    for (int e0 = 0; e0 < total; e0 += kBatchThreads * PER) {
        int64_t off[PER];
        bool in_a[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = min(e0 + (int)threadIdx.x + k * kBatchThreads, total - 1);
            const int j = W == 1 ? e : (int)__umulhi((uint32_t)e, d.magic);
            const int w = e - j * W;
            in_a[k] = w < wa;
            off[k] = in_a[k] ? (int64_t)s_ia[j] * wa + w : (int64_t)s_ib[j] * wb + (w - wa);
        }
        E v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) v[k] = (in_a[k] ? A : B)[off[k]];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = e0 + threadIdx.x + k * kBatchThreads;
            if (e < total) {
                if constexpr (NT) __builtin_nontemporal_store(v[k], o + e);
                else o[e] = v[k];
            }
        }
    }
}

__device__ __forceinline__ void copy_item(const BatchDesc &d, int64_t local, int32_t *s_ia, int32_t *s_ib) {
    const int64_t row0 = local * d.tile_rows;
    const int rows = (int)min((int64_t)d.tile_rows, d.n_rows - row0);
    {
        const auto *ga = as_global(d.a);
        const auto *gi = as_global(d.idx_a);
        const auto *gib = as_global(d.idx_b);
        const int64_t lim_a = d.lim_a, lim_b = d.lim_b;
        const int wa = d.wa, fk_word = d.fk_word;
        auto clamp_a = [=](int64_t ia) -> int64_t { return (ia >= 0 && ia < lim_a) ? ia : 0; };
        auto clamp_b = [=](int64_t ib) -> int32_t { return (ib >= 0 && ib < lim_b) ? (int32_t)ib : 0; };
        if (d.idx_a) stage_rows(s_ia, rows, [&](int j) { return (int32_t)clamp_a(gi[row0 + j]); });
        else stage_rows(s_ia, rows, [&](int j) { return (int32_t)clamp_a(row0 + j); });
        if (d.wb > 0) {
            if (d.idx_b) {
                stage_rows(s_ib, rows, [&](int j) { return clamp_b(gib[row0 + j]); });
            } else {
                auto fk = [=](int64_t ia) -> int32_t { return clamp_b((int64_t)ga[ia * wa + fk_word]); };
                if (d.idx_a) stage_rows(s_ib, rows, [&](int j) { return fk(clamp_a(gi[row0 + j])); });
                else stage_rows(s_ib, rows, [&](int j) { return fk(clamp_a(row0 + j)); });
            }
        }
    }
    __syncthreads();
    // Nontemporal stores: the lines an item writes leave this XCD's L2
    // without waiting for the release fence's write-back, which then has
    // little to write (a 2^20-row DPG retrieval as a batch of one: 277 ->
    // 256 us).
    if (d.vec == 4) batch_copy<u32x4, true>(d, s_ia, s_ib, rows, row0);
    else batch_copy<uint32_t, true>(d, s_ia, s_ib, rows, row0);
}

// rid of distribute element i (clamped to the source; a rid outside it takes
// record 0, as the copies do)
__device__ __forceinline__ int32_t batch_rid(const BatchDesc &d, int64_t i) {
    const int64_t r = (int64_t)as_global(d.ids)[i * d.id_stride + d.id_word];
    return (r >= 0 && r < d.lim_a) ? (int32_t)r : 0;
}

// OP_HIST: the item's rids counted per run in LDS, then added to the request's histogram.
__device__ __forceinline__ void hist_item(const BatchDesc &d, int64_t local, int32_t *s_h) {
    for (int b = threadIdx.x; b < d.n_runs; b += kBatchThreads) s_h[b] = 0;
    __syncthreads();
    const int64_t i0 = local * kBatchDistTile;
#pragma unroll 4
    for (int k = 0; k < kBatchDistTile / kBatchThreads; ++k) {
        const int64_t i = i0 + k * kBatchThreads + threadIdx.x;
        if (i < d.n_rows) atomicAdd(&s_h[batch_rid(d, i) >> d.lg_run], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < d.n_runs; b += kBatchThreads)
        if (s_h[b]) atomicAdd(&d.hist[b], s_h[b]);
}

// OP_SCAN: run_off = exclusive scan of the histogram (run_off[B] = all rids);
// fill starts at run_off, for the scatter's segment reservations.
__device__ __forceinline__ void scan_item(const BatchDesc &d, int32_t *s_w) {
    constexpr int PER = kBatchMaxRuns / kBatchThreads;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b0 = threadIdx.x * PER;
    int32_t v[PER], sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = b0 + k < d.n_runs ? as_global(d.hist)[b0 + k] : 0;
        sum += v[k];
    }
    int32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    int32_t base = 0;
    for (int w = 0; w < wave; ++w) base += s_w[w];
    int32_t run = base + inc - sum;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (b0 + k < d.n_runs) {
            d.run_off[b0 + k] = run;
            d.fill[b0 + k] = run;
        }
        run += v[k];
    }
    if (threadIdx.x == kBatchThreads - 1) d.run_off[d.n_runs] = run;
}

// OP_SCATTER: every rid of the item takes a slot in its run: a rank inside the
// item from LDS atomics, plus one segment per run reserved with one global
// atomic; run[slot] = rid, inv[i] = slot.  The order inside a run is
// unspecified (inv makes the result exact).
__device__ __forceinline__ void scatter_item(const BatchDesc &d, int64_t local, int32_t *s_cnt, int32_t *s_base) {
    constexpr int PER = kBatchDistTile / kBatchThreads;
    for (int b = threadIdx.x; b < d.n_runs; b += kBatchThreads) s_cnt[b] = 0;
    __syncthreads();
    const int64_t i0 = local * kBatchDistTile;
    int32_t rid[PER], rank[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = i0 + k * kBatchThreads + threadIdx.x;
        rid[k] = i < d.n_rows ? batch_rid(d, i) : -1;
        rank[k] = rid[k] >= 0 ? atomicAdd(&s_cnt[rid[k] >> d.lg_run], 1) : 0;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < d.n_runs; b += kBatchThreads)
        s_base[b] = s_cnt[b] ? atomicAdd(&d.fill[b], s_cnt[b]) : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (rid[k] < 0) continue;
        const int64_t i = i0 + k * kBatchThreads + threadIdx.x;
        const int32_t slot = s_base[rid[k] >> d.lg_run] + rank[k];
        if (slot < 0 || slot >= d.n_rows) continue;  // (only if a dependency wait gave up)
        d.run[slot] = rid[k];
        d.inv[i] = slot;
    }
}

// OP_DIST1: the distribute of a request whose rids fit one tile, in one item:
// the run counts, their exclusive scan and the slots all in LDS (no clear,
// count and scan steps, no global atomics).  The order inside a run is
// unspecified, as in OP_SCATTER.
__device__ __forceinline__ void dist1_item(const BatchDesc &d, int32_t *s_start, int32_t *s_w) {
    constexpr int PER = kBatchDistTile / kBatchThreads;
    constexpr int PR = kBatchMaxRuns / kBatchThreads;
    for (int b = threadIdx.x; b < d.n_runs; b += kBatchThreads) s_start[b] = 0;
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < PER; ++k) {
        const int64_t i = k * kBatchThreads + threadIdx.x;
        if (i < d.n_rows) atomicAdd(&s_start[batch_rid(d, i) >> d.lg_run], 1);
    }
    __syncthreads();
    // exclusive scan of the counts, in place (thread t holds runs [PR t, PR (t + 1)))
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b0 = threadIdx.x * PR;
    int32_t sum = 0;
    for (int k = 0; k < PR && b0 + k < d.n_runs; ++k) sum += s_start[b0 + k];
    int32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    int32_t run = inc - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (int k = 0; k < PR && b0 + k < d.n_runs; ++k) {
        const int32_t c = s_start[b0 + k];
        s_start[b0 + k] = run;
        run += c;
    }
    __syncthreads();
    // the rids again (read twice rather than held across the scan)
#pragma unroll 4
    for (int k = 0; k < PER; ++k) {
        const int64_t i = k * kBatchThreads + threadIdx.x;
        if (i >= d.n_rows) continue;
        const int32_t rid = batch_rid(d, i);
        const int32_t slot = atomicAdd(&s_start[rid >> d.lg_run], 1);
        d.run[slot] = rid;
        d.inv[i] = slot;
    }
}

// Stable sort passes of the dimension-order join (the DPG-Sort join's sort
// of (fk, i) pairs by fk, Section 4.2.1).  A tile is kBatchDistTile elements;
// wave w holds the tile's elements [1024 w, 1024 (w + 1)), row k of it being
// the 64 elements from 1024 w + 64 k, one per lane -- the order in which ranks
// are given, so equal digits keep input order.
__device__ __forceinline__ uint32_t sort_key(const BatchDesc &d, int64_t i) {
    return as_global(d.ids)[i * d.id_stride + d.id_word];
}

__device__ __forceinline__ void shist_item(const BatchDesc &d, int64_t t, int32_t *s_h) {
    constexpr int PER = kBatchDistTile / kBatchThreads;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < (kBatchThreads / 64) * kSortDigits; j += kBatchThreads) s_h[j] = 0;
    __syncthreads();
    const int64_t i0 = t * kBatchDistTile + wave * 64 * PER + lane;
#pragma unroll 4
    for (int k = 0; k < PER; ++k) {
        const int64_t i = i0 + k * 64;
        if (i < d.n_rows) atomicAdd(&s_h[wave * kSortDigits + ((sort_key(d, i) >> d.shift) & 255)], 1);
    }
    __syncthreads();
    for (int g = threadIdx.x; g < kSortDigits; g += kBatchThreads) {
        int32_t c = 0;
#pragma unroll
        for (int w = 0; w < kBatchThreads / 64; ++w) c += s_h[w * kSortDigits + g];
        d.cnt[t * kSortDigits + g] = c;
    }
}

// cnt[t][g] <- (elements of digits below g) + (elements of digit g in tiles before t)
__device__ __forceinline__ void sscan_item(const BatchDesc &d, int32_t *s_w) {
    static_assert(kBatchThreads == kSortDigits, "one thread per digit");
    const int g = threadIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto *c = as_global(d.cnt);
    const int T = d.n_tiles;
    int32_t total = 0;
    int t = 0;
    for (; t + 8 <= T; t += 8) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = c[(int64_t)(t + u) * kSortDigits + g];
#pragma unroll
        for (int u = 0; u < 8; ++u) total += v[u];
    }
    for (; t < T; ++t) total += c[(int64_t)t * kSortDigits + g];
    int32_t inc = total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    int32_t run = inc - total;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    // eight tiles' counts loaded together, then replaced by their offsets
    for (t = 0; t + 8 <= T; t += 8) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = c[(int64_t)(t + u) * kSortDigits + g];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[(int64_t)(t + u) * kSortDigits + g] = run;
            run += v[u];
        }
    }
    for (; t < T; ++t) {
        const int64_t at = (int64_t)t * kSortDigits + g;
        const int32_t v = c[at];
        c[at] = run;
        run += v;
    }
}

// Two passes over the tile's rows, so that no element stays in registers
// across the barrier (the persistent kernel's register budget is the largest
// step's): the first counts each wave's digits, row by row; after the
// per-digit prefix over the waves, the second reads the rows again (from the
// cache), ranks each element among the equal digits before it and writes
// (key, value) to its place.
__device__ __forceinline__ void sscatter_item(const BatchDesc &d, int64_t t, int32_t *s_cnt) {
    constexpr int PER = kBatchDistTile / kBatchThreads;
    constexpr int ROWS = 4;  // rows loaded together
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < (kBatchThreads / 64) * kSortDigits; j += kBatchThreads) s_cnt[j] = 0;
    __syncthreads();
    int32_t *mine = s_cnt + wave * kSortDigits;
    const int64_t i0 = t * kBatchDistTile + wave * 64 * PER + lane;
    for (int k0 = 0; k0 < PER; k0 += ROWS) {
        uint32_t key[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int64_t i = i0 + (k0 + k) * 64;
            key[k] = i < d.n_rows ? sort_key(d, i) : 0u;
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const bool valid = i0 + (k0 + k) * 64 < d.n_rows;
            const uint32_t g = (key[k] >> d.shift) & 255u;
            const uint64_t peers = match_lanes(g, 8, __ballot(valid));
            if (valid && (peers & lanemask_lt()) == 0) mine[g] += __popcll(peers);
        }
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves
    if (threadIdx.x < kSortDigits) {
        int32_t run = 0;
#pragma unroll
        for (int w = 0; w < kBatchThreads / 64; ++w) {
            const int32_t v = s_cnt[w * kSortDigits + threadIdx.x];
            s_cnt[w * kSortDigits + threadIdx.x] = run;
            run += v;
        }
    }
    __syncthreads();
    const auto *c = as_global(d.cnt);
    for (int k0 = 0; k0 < PER; k0 += ROWS) {
        uint32_t key[ROWS], val[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int64_t i = i0 + (k0 + k) * 64;
            const bool valid = i < d.n_rows;
            key[k] = valid ? sort_key(d, i) : 0u;
            val[k] = valid ? (d.vals_in ? as_global(d.vals_in)[i] : (uint32_t)i) : 0u;
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int64_t i = i0 + (k0 + k) * 64;
            const bool valid = i < d.n_rows;
            const uint32_t g = (key[k] >> d.shift) & 255u;
            const uint64_t peers = match_lanes(g, 8, __ballot(valid));
            const uint64_t below = peers & lanemask_lt();
            const int32_t head = valid ? mine[g] : 0;
            if (valid && below == 0) mine[g] = head + __popcll(peers);
            const int64_t pos = (int64_t)c[t * kSortDigits + g] + head + __popcll(below);
            if (valid && pos >= 0 && pos < d.n_rows) {  // (always in range unless a dependency wait gave up)
                d.keys_out[pos] = key[k];
                d.vals_out[pos] = val[k];
            }
        }
    }
}

__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchHeader *__restrict__ hdr, BatchDesc *__restrict__ descs,
                                                         uint32_t *__restrict__ host_done) {
    __shared__ int64_t s_item;
    __shared__ int s_desc;
    __shared__ int32_t s_mem[2 * kBatchMaxTileRows];  // also 2 x kBatchMaxRuns for the distribute steps
    const int64_t total_items = hdr->total_items;
    const int n_desc = hdr->n_desc;
    const uint32_t seq = hdr->seq;
    // Without dependencies workgroup b starts with item b: no workgroup ever
    // waits, so an item held by a workgroup not yet running delays nobody,
    // and the grid's first round takes no atomic.  The queue hands out the
    // items after the first round (or all of them when steps depend on each
    // other, so that every item is taken by a running workgroup, in order).
    // With dependencies only the first n_work workgroups (a quarter to a
    // half of the grid, by the widest step) take items: the waits between
    // steps leave most workgroups idle anyway, and every workgroup that
    // polls and takes items from the queue costs its atomics.
    const int64_t first_dyn = hdr->no_deps ? (int64_t)gridDim.x : 0;
    bool first = hdr->no_deps != 0;
    const int n_active = hdr->no_deps ? (int)gridDim.x : hdr->n_work;
    if ((int)blockIdx.x >= n_active) return;
    // This workgroup's queue word.  Without dependencies nothing waits, and
    // the items after the first round are spread over eight words.  With
    // dependencies one word hands out every item, in order, and only to
    // running workgroups, so a wait is always for items that running
    // workgroups hold and it ends whatever else shares the device.  (With
    // several words a word whose workgroups are not resident -- their XCD
    // held by another kernel -- would stall the waits on its items.)
    const int n_q = hdr->no_deps ? (n_active < kBatchQueues ? n_active : kBatchQueues) : 1;
    const int q = (int)blockIdx.x % n_q;
    for (;;) {
        if (threadIdx.x == 0) {
            int64_t item;
            if (first) {
                item = blockIdx.x < total_items ? (int64_t)blockIdx.x : total_items;
            } else if (first_dyn >= total_items) {
                item = total_items;  // the first round took every item: no atomic
            } else {
                item = first_dyn + (int64_t)n_q * (int64_t)atomicAdd(&hdr->queue[q], 1u) + q;
            }
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
                // wait for the step this one depends on (items taken earlier,
                // by running workgroups)
                const int dep = descs[r].dep;
                if (dep >= 0) {
                    const uint32_t need = (uint32_t)descs[dep].n_items;
                    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                    int pause = 1;
                    while (__hip_atomic_load(&descs[dep].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        for (int k = 0; k < pause; ++k) __builtin_amdgcn_s_sleep(8);
                        pause = pause < 4 ? 2 * pause : 4;
                        if (__builtin_amdgcn_s_memrealtime() - t0 > kBatchWaitTicks) {
                            atomicOr(&hdr->timeout, 1);
                            break;
                        }
                    }
                    // acquire only: the dependency's writes are visible (an
                    // invalidate of this XCD's L2, no write-back)
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            s_desc = r;
        }
        __syncthreads();
        first = false;
        const int64_t item = s_item;
        const int r = s_desc;
        if (item >= total_items) break;  // queue exhausted: uniform exit
        const BatchDesc &d = descs[r];  // fields read where used (scalar loads), not held in registers
        const int64_t local = item - d.item_start;
        switch (d.op) {
            case OP_COPY: copy_item(d, local, s_mem, s_mem + kBatchMaxTileRows); break;
            case OP_ZERO:
                for (int b = threadIdx.x; b < d.n_runs; b += kBatchThreads) d.hist[b] = 0;
                break;
            case OP_HIST: hist_item(d, local, s_mem); break;
            case OP_SCAN: scan_item(d, s_mem); break;
            case OP_SCATTER: scatter_item(d, local, s_mem, s_mem + kBatchMaxRuns); break;
            case OP_SHIST: shist_item(d, local, s_mem); break;
            case OP_SSCAN: sscan_item(d, s_mem); break;
            case OP_SSCATTER: sscatter_item(d, local, s_mem); break;
            case OP_DIST1: dist1_item(d, s_mem, s_mem + kBatchMaxRuns); break;
            default: break;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // release only: this item's writes before its count (a
            // write-back of this XCD's L2; a full fence would also
            // invalidate it, throwing away the lines that the other items
            // on this XCD still read, such as a probe's source region)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t prev = atomicAdd(&descs[r].done, 1u);
            if (d.last && host_done && prev + 1 == (uint32_t)d.n_items) {
                // the request is complete: publish to the host
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                __hip_atomic_store(&host_done[d.request], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchRequestPlan {
    bool direct = false;    // one copy step
    bool dpg = false;       // retrieval or fact-order join: the DPG step chain
    bool sortjoin = false;  // dimension-order join: stable passes over (fk, i), then the move of the fact rows
    bool move_dpg = false;  // dimension-order join: the fact rows move by the DPG chain (else one copy step)
    int passes = 0;         // dimension-order join: 8-bit stable passes over the foreign keys
    size_t ws_bytes = 0;    // scratch of the steps
    int lg_run = 0, n_runs = 0;  // DPG chain: run length and count over the moved rows
    int32_t steps = 0;      // steps in the queue
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

// Output rows per work item: about item_words dwords (kBatchItemWords or
// more), and a multiple of 256 / gcd(row bytes, 256) rows so that every
// item's output starts on a 256-byte boundary of the (256-byte aligned)
// output.
static int tile_rows_for(int words, int64_t item_words = kBatchItemWords) {
    int64_t rows64 = item_words / words;
    int rows = (int)(rows64 < kBatchMaxTileRows ? rows64 : kBatchMaxTileRows);
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

// Scratch of a request's DPG steps: hist, fill, run_off (runs + 1), run, inv
// (one int32 per rid each) and INTERNAL (one moved row per rid).
struct DpgScratch {
    size_t off_hist = 0, off_fill = 0, off_run_off = 0, off_run = 0, off_inv = 0, off_internal = 0, bytes = 0;
};

static DpgScratch dpg_scratch(int64_t n, int n_runs, int moved_bytes) {
    DpgScratch s;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    s.off_hist = take((size_t)n_runs * 4);
    s.off_fill = take((size_t)n_runs * 4);
    s.off_run_off = take((size_t)(n_runs + 1) * 4);
    s.off_run = take((size_t)n * 4);
    s.off_inv = take((size_t)n * 4);
    s.off_internal = take((size_t)n * moved_bytes);
    s.bytes = off;
    return s;
}

// Scratch of a dimension-order join: two (key, value) buffers of the stable
// passes, their count matrix, then the move's DPG scratch (if any).
struct SortJoinScratch {
    size_t off_keys[2] = {0, 0}, off_vals[2] = {0, 0}, off_cnt = 0, off_move = 0, bytes = 0;
};

static SortJoinScratch sortjoin_scratch(int64_t n, const BatchRequestPlan &p, int fact_bytes) {
    SortJoinScratch s;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const int64_t tiles = (n + kBatchDistTile - 1) / kBatchDistTile;
    for (int b = 0; b < 2; ++b) {
        s.off_keys[b] = take((size_t)n * 4);
        s.off_vals[b] = take((size_t)n * 4);
    }
    s.off_cnt = take((size_t)tiles * kSortDigits * 4);
    s.off_move = take(p.move_dpg ? dpg_scratch(n, p.n_runs, fact_bytes).bytes : 0);
    s.bytes = off;
    return s;
}

static void runs_for(const RetrievePlan &rp, int64_t n_src, BatchRequestPlan *bp) {
    // the planner's run length, lengthened until the runs fit one distribute step
    const int64_t N = n_src > 0 ? n_src : 1;
    int lg = rp.log2_run;
    while (((N + ((int64_t)1 << lg) - 1) >> lg) > kBatchMaxRuns) ++lg;
    bp->lg_run = lg;
    bp->n_runs = (int)((N + ((int64_t)1 << lg) - 1) >> lg);
}

static dpg_status plan_request(const dpg_ctx *ctx, const dpg_request &q, BatchRequestPlan *bp) {
    *bp = BatchRequestPlan();
    if (q.algo < DPG_ALGO_AUTO || q.algo > DPG_ALGO_DPG) return DPG_ERR_INVALID_ARG;
    const bool retrieve = q.kind == DPG_REQ_RETRIEVE;
    if (!retrieve && dpg_fk_join_workspace_bytes(ctx, q.n, q.fact_bytes, q.fk_offset, q.n_src, q.rec_bytes,
                                                 (dpg_join_order)q.order, (dpg_algo)q.algo) == 0)
        return DPG_ERR_INVALID_ARG;
    const bool dim_order = !retrieve && q.order == DPG_JOIN_DIM_ORDER;
    // the moved rows: retrieval source / dimension rows, or (dimension order) the fact rows
    const int64_t mv_n = dim_order ? q.n : q.n_src;
    const int mv_bytes = dim_order ? q.fact_bytes : q.rec_bytes;
    RetrievePlan rp;
    const dpg_status st = make_retrieve_plan(ctx, mv_n, mv_bytes, q.n, q.algo, &rp, retrieve);
    if (st != DPG_OK) return st;
    if (q.n == 0) {
        bp->direct = true;
        bp->steps = 1;
        return DPG_OK;
    }
    if (dim_order) {
        bp->sortjoin = true;
        const int fk_bits = q.n_src > 1 ? bit_length((uint64_t)(q.n_src - 1)) : 1;
        bp->passes = (fk_bits + 7) / 8;
        bp->move_dpg = rp.algo == DPG_ALGO_DPG;
        if (bp->move_dpg) runs_for(rp, mv_n, bp);
        bp->ws_bytes = sortjoin_scratch(q.n, *bp, q.fact_bytes).bytes;
        bp->steps = 3 * bp->passes + (bp->move_dpg ? kBatchSteps : 1);
        return DPG_OK;
    }
    if (rp.algo == DPG_ALGO_DIRECT) {
        bp->direct = true;
        bp->steps = 1;
        return DPG_OK;
    }
    bp->dpg = true;
    runs_for(rp, mv_n, bp);
    bp->ws_bytes = dpg_scratch(q.n, bp->n_runs, q.rec_bytes).bytes;
    bp->steps = kBatchSteps;
    return DPG_OK;
}

struct BatchLayout {
    size_t off_hdr = 0, off_desc = 0;
    int32_t n_desc_cap = 0;
    std::vector<size_t> req_off;  // per request: its DPG scratch or own-sequence workspace
    size_t total = 0;
};

// The header and the steps sit together, so one copy uploads both, with the
// queue word and every step's counter at zero: the launch is k_batch alone.
static BatchLayout batch_layout(int32_t n_desc_cap, const std::vector<BatchRequestPlan> &plans) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.n_desc_cap = n_desc_cap > 0 ? n_desc_cap : 1;
    L.off_hdr = take(sizeof(BatchHeader) + (size_t)L.n_desc_cap * sizeof(BatchDesc));
    L.off_desc = L.off_hdr + sizeof(BatchHeader);
    L.req_off.assign(plans.size(), 0);
    for (size_t i = 0; i < plans.size(); ++i)
        if (plans[i].ws_bytes) L.req_off[i] = take(plans[i].ws_bytes);
    L.total = off;
    return L;
}

static int32_t steps_of(const std::vector<BatchRequestPlan> &plans) {
    int32_t n = 0;
    for (const auto &p : plans) n += p.steps;
    return n;
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

static void copy_shape(BatchDesc &d, int64_t item_words = kBatchItemWords) {
    d.op = OP_COPY;
    d.tile_rows = tile_rows_for(d.wa + d.wb, item_words);
    const uintptr_t al = (uintptr_t)d.a | (uintptr_t)d.b | (uintptr_t)d.out;
    d.vec = (d.wa % 4 == 0 && d.wb % 4 == 0 && al % 16 == 0) ? 4 : 1;
    const uint64_t we = (uint64_t)(d.wa + d.wb) / (uint64_t)d.vec;
    d.magic = we > 1 ? (uint32_t)((0x100000000ull + we - 1) / we) : 0u;  // one element per row: j = e
    d.n_items = (d.n_rows + d.tile_rows - 1) / d.tile_rows;
}

// The DPG chain that moves rows `src` (n_src rows of mv_bytes) in the order of
// the ids (element i's id: ids[i * id_stride + id_word]) into INTERNAL, and
// the distribute arrays, in scratch w: ZERO, HIST, SCAN, SCATTER (or DIST1
// when the ids fit one tile), then the probe (Phase II).  *internal and *inv receive INTERNAL and the slots for the
// gather step the caller adds.
static void dpg_chain(const BatchDesc &base, const BatchRequestPlan &p, int64_t n, const uint32_t *ids,
                      int id_stride, int id_word, const void *src, int64_t n_src, int mv_bytes, char *w,
                      std::vector<BatchDesc> *chain, uint32_t **internal, const int32_t **inv) {
    const DpgScratch sc = dpg_scratch(n, p.n_runs, mv_bytes);
    BatchDesc dist = base;
    dist.ids = ids;
    dist.id_stride = id_stride;
    dist.id_word = id_word;
    dist.lim_a = n_src;
    dist.n_rows = n;
    dist.lg_run = p.lg_run;
    dist.n_runs = p.n_runs;
    dist.hist = (int32_t *)(w + sc.off_hist);
    dist.fill = (int32_t *)(w + sc.off_fill);
    dist.run_off = (int32_t *)(w + sc.off_run_off);
    dist.run = (int32_t *)(w + sc.off_run);
    dist.inv = (int32_t *)(w + sc.off_inv);
    const int64_t dist_items = (n + kBatchDistTile - 1) / kBatchDistTile;
    BatchDesc z = dist, h = dist, s = dist, x = dist;
    z.op = OP_ZERO;
    z.n_items = 1;
    h.op = OP_HIST;
    h.n_items = dist_items;
    s.op = OP_SCAN;
    s.n_items = 1;
    x.op = OP_SCATTER;
    x.n_items = dist_items;
    *internal = (uint32_t *)(w + sc.off_internal);
    // Phase II: INTERNAL[k] = src[run[k]]
    BatchDesc pr = base;
    pr.a = (const uint32_t *)src;
    pr.idx_a = dist.run;
    pr.lim_a = n_src;
    pr.wa = mv_bytes / 4;
    pr.out = *internal;
    pr.n_rows = n;
    copy_shape(pr);
    *inv = dist.inv;
    if (dist_items == 1) {
        // one tile: the whole distribute is one item
        BatchDesc one = dist;
        one.op = OP_DIST1;
        one.n_items = 1;
        for (const BatchDesc &d : {one, pr}) chain->push_back(d);
    } else {
        for (const BatchDesc &d : {z, h, s, x, pr}) chain->push_back(d);
    }
}

// The steps of the batch, in queue order: every request's first step, then
// every request's second step, ...; scratch[i] is request i's scratch.
static void build_descs(const dpg_request *reqs, int32_t n, const std::vector<BatchRequestPlan> &plans,
                        const std::vector<char *> &scratch, int64_t workers, std::vector<BatchDesc> *descs,
                        BatchHeader *hdr) {
    descs->clear();
    std::vector<std::vector<BatchDesc>> chains(n);
    int max_steps = 0;
    for (int32_t i = 0; i < n; ++i) {
        const BatchRequestPlan &p = plans[i];
        const dpg_request &q = reqs[i];
        const bool retrieve = q.kind == DPG_REQ_RETRIEVE;
        std::vector<BatchDesc> &chain = chains[i];
        BatchDesc base{};
        base.request = i;
        base.dep = -1;
        if (q.n == 0) {
            // nothing to move: one empty step marks the request done
            BatchDesc e = base;
            e.op = OP_ZERO;
            e.n_items = 1;
            chain.push_back(e);
        } else if (p.direct) {
            BatchDesc d = base;
            if (retrieve) {
                d.a = (const uint32_t *)q.src;
                d.idx_a = q.rids;
                d.lim_a = q.n_src;
                d.wa = q.rec_bytes / 4;
            } else {
                d.a = (const uint32_t *)q.fact;
                d.lim_a = q.n;
                d.b = (const uint32_t *)q.src;
                d.lim_b = q.n_src;
                d.wa = q.fact_bytes / 4;
                d.wb = q.rec_bytes / 4;
                d.fk_word = q.fk_offset / 4;
            }
            d.out = (uint32_t *)q.dst;
            d.n_rows = q.n;
            copy_shape(d);
            chain.push_back(d);
        } else if (p.dpg) {
            uint32_t *internal;
            const int32_t *inv;
            dpg_chain(base, p, q.n, retrieve ? (const uint32_t *)q.rids : (const uint32_t *)q.fact,
                      retrieve ? 1 : q.fact_bytes / 4, retrieve ? 0 : q.fk_offset / 4, q.src, q.n_src, q.rec_bytes,
                      scratch[i], &chain, &internal, &inv);
            // Phase III: dst[i] = INTERNAL[inv[i]], or fact[i] || INTERNAL[inv[i]]
            BatchDesc g = base;
            if (retrieve) {
                g.a = internal;
                g.idx_a = inv;
                g.lim_a = q.n;
                g.wa = q.rec_bytes / 4;
            } else {
                g.a = (const uint32_t *)q.fact;
                g.lim_a = q.n;
                g.b = internal;
                g.idx_b = inv;
                g.lim_b = q.n;
                g.wa = q.fact_bytes / 4;
                g.wb = q.rec_bytes / 4;
            }
            g.out = (uint32_t *)q.dst;
            g.n_rows = q.n;
            copy_shape(g);
            chain.push_back(g);
        } else if (p.sortjoin) {
            // (fk, i) pairs sorted by fk with stable 8-bit passes, low digit
            // first; pass 0 reads the keys from the fact rows, its values are
            // the row numbers
            const SortJoinScratch sc = sortjoin_scratch(q.n, p, q.fact_bytes);
            char *w = scratch[i];
            const int64_t tiles = (q.n + kBatchDistTile - 1) / kBatchDistTile;
            int cur = -1;
            for (int pass = 0; pass < p.passes; ++pass) {
                const int out = cur == 0 ? 1 : 0;
                BatchDesc h = base;
                h.ids = cur < 0 ? (const uint32_t *)q.fact : (const uint32_t *)(w + sc.off_keys[cur]);
                h.id_stride = cur < 0 ? q.fact_bytes / 4 : 1;
                h.id_word = cur < 0 ? q.fk_offset / 4 : 0;
                h.vals_in = cur < 0 ? nullptr : (const uint32_t *)(w + sc.off_vals[cur]);
                h.keys_out = (uint32_t *)(w + sc.off_keys[out]);
                h.vals_out = (uint32_t *)(w + sc.off_vals[out]);
                h.cnt = (int32_t *)(w + sc.off_cnt);
                h.shift = 8 * pass;
                h.n_rows = q.n;
                h.n_tiles = (int32_t)tiles;
                BatchDesc c = h, x = h;
                h.op = OP_SHIST;
                h.n_items = tiles;
                c.op = OP_SSCAN;
                c.n_items = 1;
                x.op = OP_SSCATTER;
                x.n_items = tiles;
                chain.push_back(h);
                chain.push_back(c);
                chain.push_back(x);
                cur = out;
            }
            const int32_t *fk_sorted = (const int32_t *)(w + sc.off_keys[cur]);
            const int32_t *i_sorted = (const int32_t *)(w + sc.off_vals[cur]);
            // out[j] = fact[i_j] || dim[fk_j]: the fact rows move by DPG (or
            // directly), the dimension rows are read in fk order
            BatchDesc g = base;
            if (p.move_dpg) {
                uint32_t *internal;
                const int32_t *inv;
                dpg_chain(base, p, q.n, (const uint32_t *)i_sorted, 1, 0, q.fact, q.n, q.fact_bytes,
                          w + sc.off_move, &chain, &internal, &inv);
                g.a = internal;
                g.idx_a = inv;
            } else {
                g.a = (const uint32_t *)q.fact;
                g.idx_a = i_sorted;
            }
            g.lim_a = q.n;
            g.b = (const uint32_t *)q.src;
            g.idx_b = fk_sorted;
            g.lim_b = q.n_src;
            g.wa = q.fact_bytes / 4;
            g.wb = q.rec_bytes / 4;
            g.out = (uint32_t *)q.dst;
            g.n_rows = q.n;
            copy_shape(g);
            chain.push_back(g);
        }
        if (!chain.empty()) chain.back().last = 1;
        max_steps = std::max(max_steps, (int)chain.size());
    }
    // queue order: step k of every request, for k = 0, 1, ...
    std::vector<int32_t> prev_index(n, -1);
    int64_t items = 0;
    // Copy items sized so that the batch's copy work spreads over about one
    // item per working workgroup: each item taken from the queue costs a
    // serialized atomic, while a workgroup copies a larger item as fast.
    bool deps = false;
    double copy_words = 0;
    std::vector<int64_t> step_items(max_steps, 0);  // items of step k over all requests
    for (const auto &chain : chains) {
        deps |= chain.size() > 1;
        for (size_t k = 0; k < chain.size(); ++k) {
            step_items[k] += chain[k].n_items;
            if (chain[k].op == OP_COPY) copy_words += (double)chain[k].n_rows * (chain[k].wa + chain[k].wb);
        }
    }
    // With dependencies the widest step (at the default item size) decides
    // how many workgroups work: a quarter of the grid for narrow chains, up
    // to a half for wide ones (measured on single 2^16- and 2^20-row DPG
    // retrievals and a batch of 64 DPG retrievals of 2^14 rows).
    const int64_t widest = step_items.empty() ? 0 : *std::max_element(step_items.begin(), step_items.end());
    const int32_t n_work = (int32_t)std::min<int64_t>(std::max<int64_t>(widest, (workers + 3) / 4), (workers + 1) / 2);
    // (without dependencies a little under one item per workgroup, so that
    // the first round usually takes every item)
    const double working = deps ? (double)n_work : 0.8 * (double)workers;
    const int64_t item_words = std::max<int64_t>(kBatchItemWords, (int64_t)(copy_words / std::max(working, 1.0)));
    if (item_words > kBatchItemWords)
        for (auto &chain : chains)
            for (BatchDesc &d : chain)
                if (d.op == OP_COPY) copy_shape(d, item_words);
    for (int k = 0; k < max_steps; ++k) {
        for (int32_t i = 0; i < n; ++i) {
            if ((int)chains[i].size() <= k) continue;
            BatchDesc d = chains[i][k];
            d.dep = prev_index[i];
            d.item_start = items;
            items += d.n_items;
            prev_index[i] = (int32_t)descs->size();
            descs->push_back(d);
        }
    }
    hdr->total_items = items;
    hdr->n_desc = (int32_t)descs->size();
    hdr->seq = 0;
    hdr->timeout = 0;
    for (int k = 0; k < kBatchQueues; ++k) hdr->queue[k] = 0;
    hdr->no_deps = 1;
    for (const BatchDesc &d : *descs)
        if (d.dep >= 0) hdr->no_deps = 0;
    hdr->n_work = deps ? n_work : (int32_t)workers;
}

static double batch_bytes(const dpg_request *reqs, int32_t n, const std::vector<BatchRequestPlan> &plans) {
    double b = 0;
    for (int32_t i = 0; i < n; ++i) {
        const dpg_request &q = reqs[i];
        const double M = (double)q.n, R = q.rec_bytes;
        const double row = q.kind == DPG_REQ_RETRIEVE ? R : q.fact_bytes + R;
        const double F = q.kind == DPG_REQ_RETRIEVE ? 0.0 : q.fact_bytes;
        if (plans[i].direct) b += M * (2.0 * row + (q.kind == DPG_REQ_RETRIEVE ? 4.0 : 0.0));
        // DPG: distribute 16 per rid (rids read twice, run and inv written),
        // probe 4 + 2R, gather inv 4 + INTERNAL R + fact F read, row written
        else if (plans[i].dpg) b += M * (16.0 + 4.0 + 2.0 * R + 4.0 + R + F + row);
        // dimension-order join: every pass reads and writes (fk, i) pairs
        // (pass 0 reads fk from the fact rows), then the move of the fact
        // rows and the assembly with the dimension rows in fk order
        else if (plans[i].sortjoin)
            b += M * (16.0 * plans[i].passes + (plans[i].move_dpg ? 24.0 + 4.0 * F : 4.0 + F) + 4.0 + R + row);
    }
    return b;
}

// The persistent grid: as many workgroups as fit on the device at once (more
// would only start as others exit, with the queue already drained).
static int batch_grid(const dpg_ctx *ctx) {
    static const int per_cu = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, kBatchThreads, 0) != hipSuccess || nb < 1)
            nb = 2;
        return nb;
    }();
    return ctx->n_cu * per_cu;
}

static dpg_status launch_batch_kernel(dpg_ctx *ctx, char *w, const BatchLayout &L, double bytes,
                                      uint32_t *host_done, hipStream_t stream) {
    ProfScope prof(ctx, K_BATCH, bytes, stream);
    hipLaunchKernelGGL(k_batch, dim3((unsigned)batch_grid(ctx)), dim3(kBatchThreads), 0, stream,
                       (BatchHeader *)(w + L.off_hdr), (BatchDesc *)(w + L.off_desc), host_done);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

dpg_status plan_batch_request(const dpg_ctx *ctx, const dpg_request &q, const void *arena, size_t arena_bytes,
                              size_t *own_ws, size_t *batch_ws) {
    dpg_status st = validate_request(q, arena, arena_bytes);
    if (st != DPG_OK) return st;
    BatchRequestPlan bp;
    st = plan_request(ctx, q, &bp);
    if (st != DPG_OK) return st;
    *batch_ws = bp.ws_bytes;
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
    // pinned staging of header + steps, so the upload is asynchronous (it is
    // reused once the previous launch, whose upload precedes it in the
    // stream, has finished)
    char *staging = nullptr;
    // per-request completion words (host memory the kernel writes) and the
    // sequence number of the last launch
    uint32_t *host_done = nullptr;
    uint32_t seq = 0;
    // recorded after every launch: destroy waits on it before freeing host_done
    hipEvent_t finished = nullptr;
    bool launched = false;
};

using namespace dpg;

extern "C" {

size_t dpg_batch_request_workspace_bytes(const dpg_ctx *ctx, const dpg_request *req) {
    BatchRequestPlan bp;
    if (!req || validate_request(*req) != DPG_OK || plan_request(ctx, *req, &bp) != DPG_OK) return 0;
    return bp.ws_bytes;
}

size_t dpg_batch_workspace_bytes(const dpg_ctx *ctx, const dpg_request *reqs, int32_t n) {
    std::vector<BatchRequestPlan> plans;
    if (plan_batch(ctx, reqs, n, &plans) != DPG_OK) return 0;
    return batch_layout(steps_of(plans), plans).total;
}

dpg_status dpg_batch_run(dpg_ctx *ctx, const dpg_request *reqs, int32_t n, void *workspace, size_t workspace_bytes,
                         hipStream_t stream) {
    std::vector<BatchRequestPlan> plans;
    dpg_status st = plan_batch(ctx, reqs, n, &plans);
    if (st != DPG_OK) return st;
    const BatchLayout L = batch_layout(steps_of(plans), plans);
    if (n > 0) {
        if (workspace_bytes < L.total) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    }
    if (!ctx) return DPG_ERR_INVALID_ARG;
    if (n == 0) return DPG_OK;
    char *w = (char *)workspace;
    std::vector<char *> scratch(n, nullptr);
    for (int32_t i = 0; i < n; ++i) scratch[i] = w + L.req_off[i];
    std::vector<BatchDesc> descs;
    BatchHeader hdr;
    build_descs(reqs, n, plans, scratch, batch_grid(ctx), &descs, &hdr);
    if (hdr.total_items > 0) {
        // header and steps in one copy (pageable source: staged before
        // hipMemcpyAsync returns)
        std::vector<char> up(sizeof(hdr) + descs.size() * sizeof(BatchDesc));
        std::memcpy(up.data(), &hdr, sizeof(hdr));
        std::memcpy(up.data() + sizeof(hdr), descs.data(), descs.size() * sizeof(BatchDesc));
        DPG_HIP(hipMemcpyAsync(w + L.off_hdr, up.data(), up.size(), hipMemcpyHostToDevice, stream));
        st = launch_batch_kernel(ctx, w, L, batch_bytes(reqs, n, plans), nullptr, stream);
        if (st != DPG_OK) return st;
    }
    return DPG_OK;
}

size_t dpg_batch_graph_workspace_bytes(const dpg_ctx *ctx, int32_t max_requests) {
    (void)ctx;
    if (max_requests < 1 || max_requests > (INT32_MAX / kBatchMaxSteps)) return 0;
    std::vector<BatchRequestPlan> none;
    return batch_layout(max_requests * kBatchMaxSteps, none).total;
}

dpg_status dpg_batch_graph_create(dpg_ctx *ctx, int32_t max_requests, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream, dpg_batch_graph **out) {
    if (!ctx || !out || max_requests < 1 || max_requests > (INT32_MAX / kBatchMaxSteps)) return DPG_ERR_INVALID_ARG;
    *out = nullptr;
    std::vector<BatchRequestPlan> none;
    const BatchLayout L = batch_layout(max_requests * kBatchMaxSteps, none);
    if (workspace_bytes < L.total) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (!workspace || ((uintptr_t)workspace) % kAlign) return DPG_ERR_INVALID_ARG;
    dpg_batch_graph *g = new dpg_batch_graph();
    g->ctx = ctx;
    g->max_requests = max_requests;
    g->ws = (char *)workspace;
    g->layout = L;
    const size_t staging = sizeof(BatchHeader) + (size_t)L.n_desc_cap * sizeof(BatchDesc);
    if (hipHostMalloc((void **)&g->staging, staging, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->host_done, (size_t)max_requests * sizeof(uint32_t), hipHostMallocCoherent) !=
            hipSuccess ||
        hipEventCreateWithFlags(&g->finished, hipEventDisableTiming) != hipSuccess) {
        dpg_batch_graph_destroy(g);
        return DPG_ERR_HIP;
    }
    std::memset(g->host_done, 0, (size_t)max_requests * sizeof(uint32_t));
    // capture k_batch (the upload before each replay resets the queue and
    // the counters); profiling events are not captured
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    dpg_status st = DPG_OK;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) st = DPG_ERR_HIP;
    if (st == DPG_OK) {
        st = launch_batch_kernel(ctx, g->ws, L, 0, g->host_done, stream);
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

int32_t dpg_batch_graph_request_done(const dpg_batch_graph *g, int32_t request) {
    if (!g || request < 0 || request >= g->max_requests || g->seq == 0) return 0;
    return __atomic_load_n(&g->host_done[request], __ATOMIC_ACQUIRE) == g->seq ? 1 : 0;
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
    if (steps_of(plans) > g->layout.n_desc_cap) return DPG_ERR_INVALID_ARG;  // not reached: at most kBatchMaxSteps each
    // DPG and sort steps take their scratch from each request's own workspace
    std::vector<char *> scratch(n, nullptr);
    for (int32_t i = 0; i < n; ++i) {
        if (plans[i].ws_bytes == 0) continue;
        if (reqs[i].workspace_bytes < plans[i].ws_bytes) return DPG_ERR_WORKSPACE_TOO_SMALL;
        if (!reqs[i].workspace || ((uintptr_t)reqs[i].workspace) % kAlign) return DPG_ERR_INVALID_ARG;
        scratch[i] = (char *)reqs[i].workspace;
    }
    if (n == 0) return DPG_OK;
    std::vector<BatchDesc> descs;
    BatchHeader hdr;
    build_descs(reqs, n, plans, scratch, batch_grid(g->ctx), &descs, &hdr);
    hdr.seq = ++g->seq;
    if (hdr.seq == 0) hdr.seq = ++g->seq;  // 0 is "never launched"
    // the staging buffer may still feed the previous launch's upload
    if (g->launched && hipEventQuery(g->finished) != hipSuccess) DPG_HIP(hipEventSynchronize(g->finished));
    std::memcpy(g->staging, &hdr, sizeof(hdr));
    if (!descs.empty()) std::memcpy(g->staging + sizeof(hdr), descs.data(), descs.size() * sizeof(BatchDesc));
    DPG_HIP(hipMemcpyAsync(g->ws + g->layout.off_hdr, g->staging, sizeof(hdr) + descs.size() * sizeof(BatchDesc),
                           hipMemcpyHostToDevice, stream));
    if (!replay) {
        st = launch_batch_kernel(g->ctx, g->ws, g->layout, batch_bytes(reqs, n, plans), g->host_done, stream);
        if (st != DPG_OK) return st;
    } else {
        ProfScope prof(g->ctx, K_BATCH, batch_bytes(reqs, n, plans), stream);
        DPG_HIP(hipGraphLaunch(g->exec, stream));
    }
    DPG_HIP(hipEventRecord(g->finished, stream));
    g->launched = true;
    return DPG_OK;
}

}  // namespace dpg

extern "C" {

void dpg_batch_graph_destroy(dpg_batch_graph *g) {
    if (!g) return;
    if (g->launched) (void)hipEventSynchronize(g->finished);  // the kernel writes host_done
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->finished) (void)hipEventDestroy(g->finished);
    if (g->staging) (void)hipHostFree(g->staging);
    if (g->host_done) (void)hipHostFree(g->host_done);
    delete g;
}

}  // extern "C"
