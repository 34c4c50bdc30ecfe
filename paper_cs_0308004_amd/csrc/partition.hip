// Stable partition pass ("count bucket sort", Section 5.3): elements move to
// the bucket named by one digit of their key, keeping input order inside every
// bucket.  It serves the DPG distribute when the run count fits one digit
// (Section 2.1, Phase I), every pass of the LSD radix sort (Section 3), and the
// foreign-key sort of the DPG-Sort join (Section 4.2.1).
//
//   k_part_hist     per tile of T elements: digit counts -> cnt[t][d]
//                   (LDS atomics into one histogram per wave)
//   column scan     (scan.hip) -> off[t][d], bucket_off[d]
//   k_part_scatter  per tile: stable rank of every element within its digit
//                   (one ballot per digit bit inside a wave; each wave owns a
//                   contiguous slice of the tile, so wave order is input
//                   order), the tile reordered by digit in LDS, then written
//                   out as one contiguous segment per digit -- coalesced,
//                   unlike a per-element scatter.  Optionally inv[i] = output
//                   position of input element i, written in input order.
//
//   k_part_scatter_unstable  the DPG distribute's variant: the same tile
//                   layout and offsets, ranks from LDS atomics, so the order
//                   inside a bucket is unspecified (the gather follows inv).
//
// Keys are uint32 or uint64; an optional uint32 value travels with each key.
// A key >= `limit` is invalid: counted nowhere, not moved, its inv entry 0
// (limit 0: every key is valid).
#include "dev_common.h"
#include "partition.h"

namespace dpg {

constexpr int kPartThreads = 256;
constexpr int kPartWaves = kPartThreads / 64;

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
    return (uint32_t)(key >> shift) & mask;
}

// Splitter buckets.  With ascending splitters s[0..ns), the bucket of a key
// is the number of splitters below it.  A table of kSplitCells cells narrows
// the search: cell h holds the keys k with k >> shift == h, where shift is
// the smallest that fits the largest splitter in kSplitCellBits bits (so
// the cells span the splitters' range, whatever the key width), and
// cell_lo[h] = number of splitters below h << shift.  The splitters below a
// key of cell h are then the first cell_lo[h] plus those of
// [cell_lo[h], cell_lo[h+1]) below it; a key beyond the last cell lies above
// every splitter.  cell_lo[kSplitCells + 1] holds shift.
constexpr int kSplitCellBits = 12;
constexpr int kSplitCells = 1 << kSplitCellBits;
constexpr int kSplitTable = kSplitCells + 2;  // int32 entries of the cell table

struct SplitLds {
    const uint32_t *s = nullptr;  // splitters in LDS (null: digits)
    const int32_t *cell_lo = nullptr;
    int shift = 32 - kSplitCellBits;
};

__device__ __forceinline__ uint32_t split_bucket(const SplitLds &sp, uint32_t key) {
    const uint32_t h = key >> sp.shift;
    if (h >= (uint32_t)kSplitCells) return (uint32_t)sp.cell_lo[kSplitCells];
    int l = sp.cell_lo[h], r = sp.cell_lo[h + 1];
    while (l < r) {
        const int m = (l + r) >> 1;
        if (sp.s[m] < key) l = m + 1;
        else r = m;
    }
    return (uint32_t)l;
}

// The bucket of a uint32 key: its digit, or with splitters its splitter
// bucket (SPLIT is a template flag, so the digit path carries no splitter code).
template <bool SPLIT>
__device__ __forceinline__ uint32_t bucket_of(uint32_t key, int shift, uint32_t mask, const SplitLds &sp) {
    if constexpr (SPLIT) return split_bucket(sp, key);
    else return digit_of(key, shift, mask);
}

// Stage the splitters and their cell table (if any) in LDS at `lds`; the
// shift is read from the table in global memory, written by an earlier launch.
__device__ __forceinline__ SplitLds stage_splitters(uint32_t *lds, const uint32_t *split, const int32_t *cell_lo,
                                                    int ns) {
    SplitLds sp;
    if (!split) return sp;
    for (int i = threadIdx.x; i < ns; i += blockDim.x) lds[i] = split[i];
    int32_t *lo = (int32_t *)(lds + ns);
    for (int i = threadIdx.x; i < kSplitTable; i += blockDim.x) lo[i] = cell_lo[i];
    sp.s = lds;
    sp.cell_lo = lo;
    sp.shift = cell_lo[kSplitCells + 1];
    return sp;
}

static size_t split_lds_bytes(int ns, bool on) { return on ? 4 * ((size_t)ns + kSplitTable) : 0; }

// The cell table: cell_lo[h] for h in [0, kSplitCells] = splitters below
// h << shift, and cell_lo[kSplitCells + 1] = shift.
__global__ __launch_bounds__(256) void k_split_cells(const uint32_t *__restrict__ split, int ns,
                                                     int32_t *__restrict__ cell_lo) {
    const int h = blockIdx.x * 256 + threadIdx.x;
    if (h >= kSplitTable) return;
    const uint32_t top = ns > 0 ? split[ns - 1] : 0u;
    const int width = top ? 32 - __clz(top) : 0;  // bits of the largest splitter
    const int shift = width > kSplitCellBits ? width - kSplitCellBits : 0;
    if (h == kSplitCells + 1) {
        cell_lo[h] = shift;
        return;
    }
    if (h == kSplitCells) {
        cell_lo[h] = ns;
        return;
    }
    const uint64_t bound = (uint64_t)h << shift;
    int l = 0, r = ns;
    while (l < r) {
        const int m = (l + r) >> 1;
        if (split[m] < bound) l = m + 1;
        else r = m;
    }
    cell_lo[h] = l;
}

// Rank of each lane's element among the active lanes of its wave that hold
// the same digit and sit below it, plus the running count of that digit in
// `ctr` (LDS), which is advanced by the number of such lanes.  Order among
// equal digits inside one row is lane order only when the row is uniform
// (one atomic for the whole row); otherwise it is the order in which the LDS
// serves the atomics.  Used where stability is not required.
__device__ __forceinline__ int32_t rank_by_atomic(int32_t *ctr, uint32_t d, bool valid) {
    const uint64_t act = __ballot(valid);
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    const uint64_t same = __ballot(valid && d == d0);
    if (same == act) {  // uniform row (every row when keys are heavily skewed)
        int32_t h = 0;
        if (__lane_id() == 0) h = atomicAdd(&ctr[d0], (int32_t)__popcll(act));
        h = __shfl(h, 0, 64);
        return valid ? h + (int32_t)__popcll(act & lanemask_lt()) : -1;
    }
    return valid ? atomicAdd(&ctr[d], 1) : -1;
}

template <typename K, bool SPLIT>
__global__ __launch_bounds__(kPartThreads) void k_part_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                            int nbits, uint64_t limit, int T, uint32_t key_mul,
                                                            int32_t *__restrict__ cnt,
                                                            const uint32_t *__restrict__ split,
                                                            const int32_t *__restrict__ cell_lo, int n_split,
                                                            const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ int32_t h[kPartWaves][kMaxDigitBuckets];
    extern __shared__ uint32_t s_split_h[];
    const int nb = 1 << nbits;
    const uint32_t mask = (uint32_t)nb - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = lane; d < nb; d += 64) h[wave][d] = 0;
    SplitLds sp;
    if constexpr (SPLIT) sp = stage_splitters(s_split_h, split, cell_lo, n_split);
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * T;
    const int64_t end = min(base + T, n);
    // all loads of a batch in flight before the first is used; counts go to
    // the wave's own LDS histogram with one atomic per element (one per row
    // when the row holds a single digit)
    constexpr int kBatch = 8;
    for (int64_t i0 = base + wave * 64; i0 < end; i0 += kPartThreads * kBatch) {
        K kv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t i = i0 + (int64_t)u * kPartThreads + lane;
            kv[u] = i < end ? (K)(keys[i] * (K)key_mul) : K(0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t i = i0 + (int64_t)u * kPartThreads + lane;
            const bool valid = i < end && (limit == 0 || (uint64_t)kv[u] < limit);
            uint32_t d;
            if constexpr (SPLIT) d = bucket_of<true>((uint32_t)kv[u], shift, mask, sp);
            else d = digit_of(kv[u], shift, mask);
            (void)rank_by_atomic(h[wave], d, valid);
        }
    }
    __syncthreads();
    int32_t *row = cnt + (int64_t)blockIdx.x * nb;
    for (int d = threadIdx.x; d < nb; d += kPartThreads) {
        int32_t s = 0;
#pragma unroll
        for (int w = 0; w < kPartWaves; ++w) s += h[w][d];
        row[d] = s;
    }
}

// The histogram for more than 256 buckets: one table per workgroup.
template <int THREADS, bool SPLIT>
__global__ __launch_bounds__(THREADS) void k_part_hist_wide(const uint32_t *__restrict__ keys, int64_t n,
                                                            int shift, int nbits, uint64_t limit, int T,
                                                            uint32_t key_mul, int32_t *__restrict__ cnt,
                                                            const uint32_t *__restrict__ split,
                                                            const int32_t *__restrict__ cell_lo, int n_split) {
    extern __shared__ int32_t hw[];
    const int nb = 1 << nbits;
    const uint32_t mask = (uint32_t)nb - 1;
    for (int d = threadIdx.x; d < nb; d += THREADS) hw[d] = 0;
    SplitLds sp;
    if constexpr (SPLIT) sp = stage_splitters((uint32_t *)(hw + nb), split, cell_lo, n_split);
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * T;
    const int64_t end = min(base + T, n);
    constexpr int kBatch = 8;
    for (int64_t i0 = base + threadIdx.x; i0 < end; i0 += (int64_t)THREADS * kBatch) {
        uint32_t kv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t i = i0 + (int64_t)u * THREADS;
            kv[u] = keys[min(i, end - 1)] * key_mul;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t i = i0 + (int64_t)u * THREADS;
            const bool valid = i < end && (limit == 0 || (uint64_t)kv[u] < limit);
            (void)rank_by_atomic(hw, bucket_of<SPLIT>(kv[u], shift, mask, sp), valid);
        }
    }
    __syncthreads();
    int32_t *row = cnt + (int64_t)blockIdx.x * nb;
    for (int d = threadIdx.x; d < nb; d += THREADS) row[d] = hw[d];
}

// PER elements per thread; a tile is kPartThreads * PER elements; wave w owns
// elements [w*64*PER, (w+1)*64*PER) of the tile, its row k being the 64
// consecutive elements starting at w*64*PER + 64*k.
template <typename K, bool HAS_VAL, int PER>
__global__ __launch_bounds__(kPartThreads) void k_part_scatter(
    const K *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t n, int shift, int nbits,
    uint64_t limit, int64_t nT, const int32_t *__restrict__ off, K *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, int32_t *__restrict__ inv, int remap, const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    constexpr int T = kPartThreads * PER;
    extern __shared__ __align__(16) char smem[];
    K *s_key = (K *)smem;
    uint32_t *s_val = (uint32_t *)(smem + sizeof(K) * T);
    __shared__ int32_t s_cnt[kPartWaves][kMaxDigitBuckets];  // per wave: count, then prefix over waves
    __shared__ int32_t s_start[kMaxDigitBuckets];             // tile-local start of each digit
    __shared__ int32_t s_glob[kMaxDigitBuckets];              // output start of each digit for this tile
    __shared__ int32_t s_nvalid;
    const int nb = 1 << nbits;
    const uint32_t mask = (uint32_t)nb - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = xcd_tile(blockIdx.x, nT, remap);
    const int64_t base = t * T;
    const int cnt = (int)min((int64_t)T, n - base);
    for (int d = lane; d < nb; d += 64) s_cnt[wave][d] = 0;
    for (int d = threadIdx.x; d < nb; d += kPartThreads) s_glob[d] = off[t * nb + d];

    K key[PER];
    uint32_t val[PER];
    int32_t rank[PER];
    const int wbase = wave * 64 * PER;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = wbase + k * 64 + lane;
        key[k] = e < cnt ? keys[base + e] : K(0);
        if constexpr (HAS_VAL) val[k] = e < cnt ? vals[base + e] : 0u;
    }
    __syncthreads();
    // rank within (wave, digit), in row order
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = wbase + k * 64 + lane;
        const bool valid = e < cnt && (limit == 0 || (uint64_t)key[k] < limit);
        const uint32_t d = digit_of(key[k], shift, mask);
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_lanes(d, nbits, act);
        const uint64_t below = peers & lanemask_lt();
        const int32_t head = valid ? s_cnt[wave][d] : 0;
        rank[k] = valid ? head + __popcll(below) : -1;
        if (valid && below == 0) s_cnt[wave][d] = head + __popcll(peers);
    }
    __syncthreads();
    // per digit: exclusive prefix over waves (in place) and tile-local start
    if (threadIdx.x < 64) {
        int32_t carry = 0;
        for (int d0 = 0; d0 < nb; d0 += 64) {
            const int d = d0 + lane;
            int32_t tot = 0;
            if (d < nb) {
#pragma unroll
                for (int w = 0; w < kPartWaves; ++w) {
                    const int32_t c = s_cnt[w][d];
                    s_cnt[w][d] = tot;
                    tot += c;
                }
            }
            int32_t inc = tot;
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) {
                const int32_t y = __shfl_up(inc, s, 64);
                if (lane >= s) inc += y;
            }
            if (d < nb) s_start[d] = carry + inc - tot;
            carry += __shfl(inc, 63, 64);
        }
        if (lane == 0) s_nvalid = carry;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = wbase + k * 64 + lane;
        if (rank[k] >= 0) {
            const uint32_t d = digit_of(key[k], shift, mask);
            const int32_t r = s_cnt[wave][d] + rank[k];
            s_key[s_start[d] + r] = key[k];
            if constexpr (HAS_VAL) s_val[s_start[d] + r] = val[k];
            if (inv) inv[base + e] = s_glob[d] + r;
        } else if (inv && e < cnt) {
            inv[base + e] = 0;
        }
    }
    __syncthreads();
    const int nvalid = s_nvalid;
    for (int j = threadIdx.x; j < nvalid; j += kPartThreads) {
        const K k = s_key[j];
        const uint32_t d = digit_of(k, shift, mask);
        const int64_t pos = (int64_t)s_glob[d] + (j - s_start[d]);
        keys_out[pos] = k;
        if constexpr (HAS_VAL) vals_out[pos] = s_val[j];
    }
}

// The same pass for uint32 keys without values when the order inside a bucket
// does not matter (the DPG distribute, whose gather follows inv): ranks come
// from LDS atomics instead of ballot matching, which costs one LDS atomic per
// element rather than a ballot per digit bit, and up to 2^13 buckets fit.
// Counts per (tile, digit) are those of the histogram pass, so the column-scan
// offsets still apply.  LDS: keys of the tile, then the count / start and the
// output start of every digit.
template <int THREADS, int PER, bool SPLIT>
__global__ __launch_bounds__(THREADS) void k_part_scatter_unstable(
    const uint32_t *__restrict__ keys, int64_t n, int shift, int nbits, uint64_t limit, int64_t nT,
    const int32_t *__restrict__ off, uint32_t *__restrict__ keys_out, int32_t *__restrict__ inv, int local_inv,
    uint32_t key_mul, int remap, const uint32_t *__restrict__ split, const int32_t *__restrict__ cell_lo,
    int n_split, uint32_t *__restrict__ idx_out) {
    constexpr int T = THREADS * PER;
    constexpr int W = THREADS / 64;
    extern __shared__ __align__(16) char smem[];
    uint32_t *s_key = (uint32_t *)smem;
    const int nb = 1 << nbits;
    int32_t *s_cnt = (int32_t *)(smem + sizeof(uint32_t) * T);  // count, then tile-local start
    int32_t *s_glob = s_cnt + nb;                               // output start of each digit for this tile
    SplitLds sp;  // splitters, if any, after the digit tables
    if constexpr (SPLIT) sp = stage_splitters((uint32_t *)(s_glob + nb), split, cell_lo, n_split);
    // the input position of every element of the tile, when idx_out is given
    uint32_t *s_idx = (uint32_t *)(s_glob + nb) + (SPLIT ? n_split + kSplitTable : 0);
    __shared__ int32_t s_wsum[W];
    __shared__ int32_t s_nvalid;
    const uint32_t mask = (uint32_t)nb - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = xcd_tile(blockIdx.x, nT, remap);
    const int64_t base = t * T;
    const int cnt = (int)min((int64_t)T, n - base);
    for (int d = threadIdx.x; d < nb; d += THREADS) {
        s_cnt[d] = 0;
        s_glob[d] = off[t * nb + d];
    }
    // Tiles of 32768 (1024 threads x 32): the rank and digit of every
    // element share one register (rank + 1 in the low 16 bits, 0 for an
    // invalid element; the digit above), keys load from the tile's base with
    // 32-bit lane offsets and are tested in 32 bits, so that the keys and
    // ranks fit the registers of the workgroup.  Smaller tiles keep a
    // register per rank and recompute the digit.
    constexpr bool kPacked = THREADS == 1024 && PER == 32;
    static_assert(!kPacked || !SPLIT, "packed ranks: digits only");
    uint32_t key[PER];
    int32_t rank[kPacked ? 1 : PER];
    uint32_t rd[kPacked ? PER : 1];
    uint32_t bkt[SPLIT ? PER : 1];
    if constexpr (kPacked) {
        const uint32_t *__restrict__ kt = keys + base;
        if (cnt == T) {
#pragma unroll
            for (int k = 0; k < PER; ++k) key[k] = kt[k * THREADS + threadIdx.x] * key_mul;
        } else {
#pragma unroll
            for (int k = 0; k < PER; ++k) key[k] = kt[min(k * THREADS + (int)threadIdx.x, cnt - 1)] * key_mul;
        }
        __syncthreads();
        const bool any_key = limit == 0 || limit > 0xffffffffull;
        const uint32_t lim32 = (uint32_t)limit;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = k * THREADS + threadIdx.x;
            const bool valid = e < cnt && (any_key || key[k] < lim32);
            const uint32_t d = digit_of(key[k], shift, mask);
            const uint32_t r1 = (uint32_t)(rank_by_atomic(s_cnt, d, valid) + 1);
            // one opaque instruction, so that the compiler keeps the packed
            // word rather than the digit and the rank apart
            uint32_t x;
            asm("v_lshl_or_b32 %0, %1, 16, %2" : "=v"(x) : "v"(d), "v"(r1));
            rd[k] = x;
        }
    } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = k * THREADS + threadIdx.x;
            key[k] = keys[base + min(e, cnt - 1)] * key_mul;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = k * THREADS + threadIdx.x;
            const bool valid = e < cnt && (limit == 0 || (uint64_t)key[k] < limit);
            const uint32_t d = bucket_of<SPLIT>(key[k], shift, mask, sp);
            if constexpr (SPLIT) bkt[k] = d;  // a splitter search is kept, a digit recomputed
            rank[k] = rank_by_atomic(s_cnt, d, valid);
        }
    }
    __syncthreads();
    // exclusive prefix of the digit counts: wave w scans the w-th slice of
    // the digits, then the slices are offset by the totals of the slices
    // before them
    {
        const int per_w = (nb + W - 1) / W;
        const int d_lo = min(wave * per_w, nb), d_hi = min(d_lo + per_w, nb);
        int32_t carry = 0;
        for (int d0 = d_lo; d0 < d_hi; d0 += 64) {
            const int d = d0 + lane;
            const int32_t c = d < d_hi ? s_cnt[d] : 0;
            int32_t inc = c;
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) {
                const int32_t y = __shfl_up(inc, s, 64);
                if (lane >= s) inc += y;
            }
            if (d < d_hi) s_cnt[d] = carry + inc - c;
            carry += __shfl(inc, 63, 64);
        }
        if (lane == 0) s_wsum[wave] = carry;
        __syncthreads();
        int32_t before = 0, all = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            before += v < wave ? s_wsum[v] : 0;
            all += s_wsum[v];
        }
        for (int d = d_lo + lane; d < d_hi; d += 64) s_cnt[d] += before;
        if (threadIdx.x == 0) s_nvalid = all;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = k * THREADS + threadIdx.x;
        int32_t rk;
        uint32_t d;
        if constexpr (kPacked) {
            rk = (int32_t)(rd[k] & 0xffffu) - 1;
            d = rd[k] >> 16;
        } else {
            rk = rank[k];
            d = SPLIT ? bkt[k] : digit_of(key[k], shift, mask);
        }
        if (rk >= 0) {
            s_key[s_cnt[d] + rk] = key[k];
            if (idx_out) s_idx[s_cnt[d] + rk] = (uint32_t)(base + e);
            if (inv) inv[base + e] = (local_inv ? s_cnt[d] : s_glob[d]) + rk;
        } else if (inv && e < cnt) {
            inv[base + e] = 0;
        }
    }
    __syncthreads();
    const int nvalid = s_nvalid;
    for (int j = threadIdx.x; j < nvalid; j += THREADS) {
        const uint32_t k = s_key[j];
        const uint32_t d = bucket_of<SPLIT>(k, shift, mask, sp);
        const int64_t pos = (int64_t)s_glob[d] + (j - s_cnt[d]);
        keys_out[pos] = k;
        if (idx_out) idx_out[pos] = s_idx[j];
    }
}

static int part_per(int key_bytes, bool has_val) {
    if (key_bytes == 4 && !has_val) return 32;
    return 16;
}

PartPlan plan_partition(int64_t n, int nbits, int key_bytes, bool has_val, int wide_per, bool wide) {
    PartPlan p;
    p.n = n;
    p.nbits = nbits;
    p.key_bytes = key_bytes;
    p.has_val = has_val;
    p.per = part_per(key_bytes, has_val);
    if (nbits > kMaxDigitBits || (wide && key_bytes == 4 && !has_val)) {  // 1024 threads x 8 or 16 keys
        p.threads = 1024;
        p.per = wide_per == 8 ? 8 : wide_per == 32 && nbits <= 11 && !has_val ? 32 : 16;
    }
    p.tile = p.threads * p.per;
    p.n_tiles = n > 0 ? (n + p.tile - 1) / p.tile : 0;
    p.n_chunks = (p.n_tiles + 31) / 32;
    const int64_t nb = (int64_t)1 << nbits;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    p.off_cnt = take((size_t)p.n_tiles * nb * 4);
    p.off_csum = take((size_t)p.n_chunks * nb * 4);
    p.off_total = take((size_t)nb * 4);
    p.off_bucket = take((size_t)(nb + 1) * 4);
    p.off_cells = take((size_t)kSplitTable * 4);
    p.workspace = off;
    return p;
}

template <typename K, bool HAS_VAL, int PER>
static dpg_status launch_scatter_t(const PartPlan &p, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                                   uint32_t *vals_out, int32_t *inv, int shift, uint64_t limit, const int32_t *off,
                                   int remap, const int32_t *gate, hipStream_t stream) {
    constexpr int T = kPartThreads * PER;
    const size_t lds = sizeof(K) * T + (HAS_VAL ? sizeof(uint32_t) * T : 0);
    hipLaunchKernelGGL((k_part_scatter<K, HAS_VAL, PER>), dim3((unsigned)p.n_tiles), dim3(kPartThreads), lds, stream,
                       (const K *)keys_in, vals_in, p.n, shift, p.nbits, limit, p.n_tiles, off, (K *)keys_out,
                       vals_out, inv, remap, gate);
    DPG_HIP(hipGetLastError());
    return DPG_OK;
}

dpg_status launch_partition(dpg_ctx *ctx, const PartPlan &p, const void *keys_in, const uint32_t *vals_in,
                            void *keys_out, uint32_t *vals_out, int32_t *inv, int shift, uint64_t limit,
                            void *scratch, hipStream_t stream, int32_t **bucket_off_dev, int32_t *item_off,
                            int item_chunk, bool stable, bool local_inv, uint32_t key_mul, const uint32_t *split,
                            int n_split, uint32_t *idx_out, const int32_t *gate) {
    char *w = (char *)scratch;
    int32_t *cnt = (int32_t *)(w + p.off_cnt);
    int32_t *csum = (int32_t *)(w + p.off_csum);
    int32_t *total = (int32_t *)(w + p.off_total);
    int32_t *bucket_off = (int32_t *)(w + p.off_bucket);
    if (bucket_off_dev) *bucket_off_dev = bucket_off;
    if (p.n <= 0) return DPG_OK;
    const bool wide = p.threads == 1024;  // the 1024-thread unstable pass
    if (p.nbits < 1 || p.nbits > kMaxWideBits) return DPG_ERR_UNSUPPORTED;
    if (wide && (stable || p.key_bytes != 4 || p.has_val || p.threads != 1024 ||
                 (p.per != 8 && p.per != 16 && p.per != 32) || (p.per == 32 && (split || idx_out))))
        return DPG_ERR_UNSUPPORTED;
    if (local_inv && stable) return DPG_ERR_UNSUPPORTED;
    if (key_mul != 1 && (stable || p.key_bytes != 4 || p.has_val)) return DPG_ERR_UNSUPPORTED;
    const int nb = 1 << p.nbits;
    if (!split) n_split = 0;
    if (split && (stable || p.key_bytes != 4 || p.has_val || n_split < 0 || n_split >= nb)) return DPG_ERR_UNSUPPORTED;
    if (idx_out && (stable || p.key_bytes != 4 || p.has_val)) return DPG_ERR_UNSUPPORTED;
    // a gate (device word: the pass runs only if it is non-zero) is taken by
    // the stable 256-thread pass only
    if (gate && (!stable || wide || split)) return DPG_ERR_UNSUPPORTED;
    const size_t split_lds = split_lds_bytes(n_split, split != nullptr);
    const int32_t *cells = (const int32_t *)(w + p.off_cells);
    if (split) {
        hipLaunchKernelGGL(k_split_cells, dim3((kSplitTable + 255) / 256), dim3(256), 0, stream, split, n_split,
                           (int32_t *)(w + p.off_cells));
        DPG_HIP(hipGetLastError());
    }
    const double elem = p.key_bytes + (p.has_val ? 4.0 : 0.0);
    {
        ProfScope prof(ctx, wide ? K_PART_HIST_WIDE : K_PART_HIST, (double)p.key_bytes * p.n + 4.0 * p.n_tiles * nb,
                       stream);
        if (wide)
            hipLaunchKernelGGL((split ? k_part_hist_wide<1024, true> : k_part_hist_wide<1024, false>),
                               dim3((unsigned)p.n_tiles), dim3(1024), (size_t)nb * sizeof(int32_t) + split_lds, stream,
                               (const uint32_t *)keys_in, p.n, shift, p.nbits, limit, p.tile, key_mul, cnt, split, cells,
                               n_split);
        else if (p.key_bytes == 8)
            hipLaunchKernelGGL((k_part_hist<uint64_t, false>), dim3((unsigned)p.n_tiles), dim3(kPartThreads), 0, stream,
                               (const uint64_t *)keys_in, p.n, shift, p.nbits, limit, p.tile, 1u, cnt, nullptr,
                               nullptr, 0, gate);
        else
            hipLaunchKernelGGL((split ? k_part_hist<uint32_t, true> : k_part_hist<uint32_t, false>),
                               dim3((unsigned)p.n_tiles), dim3(kPartThreads), split_lds,
                               stream, (const uint32_t *)keys_in, p.n, shift, p.nbits, limit, p.tile, key_mul, cnt,
                               split, cells, n_split, gate);
        DPG_HIP(hipGetLastError());
    }
    dpg_status st = launch_column_scan(ctx, cnt, p.n_tiles, nb, csum, p.n_chunks, total, bucket_off, item_off,
                                       item_chunk, stream, gate);
    if (st != DPG_OK) return st;
    ProfScope prof(ctx, stable ? K_PART_SCATTER : K_PART_SCATTER_UNSTABLE,
                   2.0 * elem * p.n + (inv ? 4.0 * p.n : 0.0) + 4.0 * p.n_tiles * nb, stream);
    const int remap = xcd_remap_flag(ctx);
    if (p.key_bytes == 8) {
        if (p.has_val)
            return launch_scatter_t<uint64_t, true, 16>(p, keys_in, vals_in, keys_out, vals_out, inv, shift, limit,
                                                        cnt, remap, gate, stream);
        return launch_scatter_t<uint64_t, false, 16>(p, keys_in, vals_in, keys_out, vals_out, inv, shift, limit, cnt,
                                                     remap, gate, stream);
    }
    if (p.has_val)
        return launch_scatter_t<uint32_t, true, 16>(p, keys_in, vals_in, keys_out, vals_out, inv, shift, limit, cnt,
                                                    remap, gate, stream);
    if (!stable) {
        const size_t lds = sizeof(uint32_t) * p.tile + 2 * sizeof(int32_t) * nb + split_lds +
                           (idx_out ? sizeof(uint32_t) * p.tile : 0);
        if (lds + 1024 > kMaxPartitionLds) return DPG_ERR_UNSUPPORTED;
        if (wide) {
            if (p.threads != 1024 || (p.per != 8 && p.per != 16 && p.per != 32)) return DPG_ERR_UNSUPPORTED;
            // 32 rids per thread (tiles of 32768, no splitters): segments of
            // twice the length per run for the same count matrix
            auto fn = p.per == 32  ? k_part_scatter_unstable<1024, 32, false>
                      : p.per == 8 ? (split ? k_part_scatter_unstable<1024, 8, true> : k_part_scatter_unstable<1024, 8, false>)
                                   : (split ? k_part_scatter_unstable<1024, 16, true>
                                            : k_part_scatter_unstable<1024, 16, false>);
            if (lds > 64 * 1024)
                DPG_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(fn, dim3((unsigned)p.n_tiles), dim3(1024), lds, stream, (const uint32_t *)keys_in, p.n,
                               shift, p.nbits, limit, p.n_tiles, cnt, (uint32_t *)keys_out, inv, local_inv ? 1 : 0,
                               key_mul, remap, split, cells, n_split, idx_out);
        } else {
            if (p.per != 32 || p.threads != kPartThreads) return DPG_ERR_UNSUPPORTED;
            if (lds > 64 * 1024) {
                const void *fn = split ? (const void *)k_part_scatter_unstable<kPartThreads, 32, true>
                                       : (const void *)k_part_scatter_unstable<kPartThreads, 32, false>;
                DPG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            }
            hipLaunchKernelGGL((split ? k_part_scatter_unstable<kPartThreads, 32, true>
                                      : k_part_scatter_unstable<kPartThreads, 32, false>),
                               dim3((unsigned)p.n_tiles), dim3(kPartThreads), lds, stream, (const uint32_t *)keys_in,
                               p.n, shift, p.nbits, limit, p.n_tiles, cnt, (uint32_t *)keys_out, inv,
                               local_inv ? 1 : 0, key_mul, remap, split, cells, n_split, idx_out);
        }
        DPG_HIP(hipGetLastError());
        return DPG_OK;
    }
    return launch_scatter_t<uint32_t, false, 32>(p, keys_in, vals_in, keys_out, vals_out, inv, shift, limit, cnt,
                                                 remap, gate, stream);
}

}  // namespace dpg
