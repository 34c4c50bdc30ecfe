// One-digit partition pass (count bucket sort), shared by the DPG
// distribute, the radix sort and the foreign-key sort of the DPG-Sort join.
#pragma once

#include "dpg_internal.h"

namespace dpg {

constexpr int kMaxDigitBits = 8;                    // stable passes
constexpr int kMaxDigitBuckets = 1 << kMaxDigitBits;
constexpr int kMaxWideBits = 12;                    // unstable uint32 passes (the DPG distribute)
constexpr int kMaxWideBuckets = 1 << kMaxWideBits;
constexpr size_t kMaxPartitionLds = 160 * 1024;  // LDS of one workgroup

struct PartPlan {
    int64_t n = 0;
    int nbits = 0;       // digit width; 2^nbits buckets
    int key_bytes = 4;   // 4 or 8
    bool has_val = false;
    int threads = 256;   // workgroup size
    int per = 0;         // elements per thread
    int tile = 0;        // elements per workgroup
    int64_t n_tiles = 0, n_chunks = 0;
    size_t off_cnt = 0, off_csum = 0, off_total = 0, off_bucket = 0, off_cells = 0;
    size_t workspace = 0;
};

// Layout of the scratch one pass needs (count matrix and bucket offsets).
// nbits up to kMaxDigitBits for any pass; up to kMaxWideBits only for uint32
// keys without values, which are then partitioned without stability, by
// 1024-thread workgroups of wide_per (8, 16, or 32 up to 2^11 digits) keys per thread.  wide: use
// that 1024-thread unstable pass for any digit width (uint32 keys without
// values only).
PartPlan plan_partition(int64_t n, int nbits, int key_bytes, bool has_val, int wide_per = 16, bool wide = false);

// The partition pass of a planned one-pass DPG distribute (DIST_PARTITION or
// DIST_SAMPLED).
inline PartPlan dist_partition(const RetrievePlan &p) {
    return plan_partition(p.n_rids, p.part_nbits, 4, false, p.wide_per, p.part_wide);
}

// One pass: elements whose key is < limit (any key if limit is 0) move to the
// bucket of digit (key >> shift) & (2^nbits - 1), in input order within a
// bucket.  With stable = false (uint32 keys without values only) the order
// inside a bucket is unspecified; inv stays exact.  local_inv (unstable passes
// only): inv[i] is instead the slot of element i within its tile's output
// segments laid end to end (digit order), i.e. relative to the tile.
// split / n_split (unstable uint32 passes only): the bucket of a key is
// instead the number of the n_split ascending splitters below it (device
// array, n_split < 2^nbits), i.e. bucket b holds the keys in
// (split[b-1], split[b]].
// idx_out (unstable passes only; may be null) receives, beside each output
// key, the input position of its element; the tile is then staged in LDS
// twice over, which needs the digit tables small enough (up to 2^11 digits
// for the wide pass).
// key_mul (unstable uint32 passes only): every key is first multiplied by it
// (mod 2^32), and the products are what is partitioned and written out.  inv (may be
// null) receives the output position of every input element (0 if invalid).
// bucket_off (in the scratch, also returned through *bucket_off_dev when
// non-null) holds the 2^nbits + 1 bucket boundaries.
// item_off / item_chunk (optional) as for the column scan: work items of at
// most item_chunk elements per bucket, for the LDS probe.
// gate (stable passes only; may be null): a device word; the pass's kernels
// return at once when it is zero, leaving every output as it was, so a host
// can enqueue passes that the device decides to skip.
dpg_status launch_partition(dpg_ctx *ctx, const PartPlan &p, const void *keys_in, const uint32_t *vals_in,
                            void *keys_out, uint32_t *vals_out, int32_t *inv, int shift, uint64_t limit,
                            void *scratch, hipStream_t stream, int32_t **bucket_off_dev,
                            int32_t *item_off = nullptr, int item_chunk = 0, bool stable = true,
                            bool local_inv = false, uint32_t key_mul = 1, const uint32_t *split = nullptr,
                            int n_split = 0, uint32_t *idx_out = nullptr, const int32_t *gate = nullptr);

// Exclusive scan of a[0..n) in place; *total = the sum (device).  scratch:
// scan_1d_scratch_bytes(n).
size_t scan_1d_scratch_bytes(int64_t n);
dpg_status launch_scan_1d(dpg_ctx *ctx, int32_t *a, int64_t n, int32_t *scratch, int32_t *total,
                          hipStream_t stream);

// gate (may be null): a device word; every kernel of the scan returns at once
// when it is zero (the scan then writes nothing).
dpg_status launch_column_scan(dpg_ctx *ctx, int32_t *cnt, int64_t nT, int B, int32_t *csum, int64_t nC,
                              int32_t *total, int32_t *bucket_off, int32_t *item_off, int item_chunk,
                              hipStream_t stream, const int32_t *gate = nullptr);

}  // namespace dpg
