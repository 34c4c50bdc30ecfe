/*
 * CPU oracle for DPG record retrieval, DPG sorting and the two DPG foreign-key
 * joins (Cooperman, Ma, Nguyen, "DPG: A Cache-Efficient Accelerator for Sorting
 * and for Join Operators", arXiv cs/0308004).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a deliberately plain, slow and
 * obviously correct statement of what the GPU library computes.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header, table or helper with the HIP library, and nothing in
 * the library may call it.
 *
 * It also states the hash index and the enhanced B+ tree of Section 4.2.3
 * (batch lookup in indexes), the result of a batch lookup in either, and the
 * sort-merge join of Section 4.1.
 *
 * Conventions (readings of the paper, listed again in the design notes):
 *   - rids are 0-based and must lie in [0, n_src) (Section 2.1 says rid values
 *     lie between 0 and N; Figure 1 is written 1-based, the text and the worked
 *     example of Section 2.2 are 0-based).  An rid outside that range is an
 *     error, never clamped.
 *   - a record is rec_bytes contiguous bytes; record r starts at byte r*rec_bytes.
 *   - sort keys compare as unsigned bytes, lexicographically (memcmp order); equal
 *     keys keep the original record index order, which makes the result unique.
 *   - join rows: the fact (referencing) row bytes followed by the dimension
 *     (referenced, indexed) row bytes.  Dimension ids are dense, so the index
 *     lookup of Section 4.2.2 maps a foreign key k to rid_F = k.
 *
 * Return codes: 0 success, 1 invalid argument, 2 rid / foreign key out of range.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifndef INT32_MAX
#define INT32_MAX 2147483647
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ERANGE 2

/* ------------------------------------------------------------------------- */
/* Record retrieval: the problem statement of Section 2, D[i] = R[S_rid[i]].   */
/* ------------------------------------------------------------------------- */
int oracle_retrieve(const uint8_t *src, int64_t n_src, int32_t rec_bytes,
                    const int32_t *rids, int64_t n_rids, uint8_t *dst)
{
    if (rec_bytes <= 0 || n_src < 0 || n_rids < 0)
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < n_rids; ++i) {
        int64_t r = rids[i];
        if (r < 0 || r >= n_src)
            return ORACLE_ERANGE;
    }
    for (int64_t i = 0; i < n_rids; ++i) {
        int64_t r = rids[i];
#ifdef ORACLE_MUTANT_SHORT_COPY
        memcpy(dst + i * (int64_t)rec_bytes, src + r * (int64_t)rec_bytes, (size_t)rec_bytes - 4);
#elif defined(ORACLE_MUTANT_NEIGHBOUR)
        int64_t q = (r + 1 < n_src) ? r + 1 : r;
        memcpy(dst + i * (int64_t)rec_bytes, src + q * (int64_t)rec_bytes, (size_t)rec_bytes);
#else
        memcpy(dst + i * (int64_t)rec_bytes, src + r * (int64_t)rec_bytes, (size_t)rec_bytes);
#endif
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Figure 1 of Section 2.1 carried out phase by phase, 0-based.  Used only to   */
/* check the phase invariants and the worked example of Section 2.2; parity   */
/* of the library is always checked against oracle_retrieve.                   */
/*                                                                             */
/* run_len  : L, records per run (region) of the input file                    */
/* rid_run  : out, n_rids entries: the RID runs stored one after another        */
/* run_off  : out, n_runs+1 entries: run i occupies rid_run[run_off[i] ..       */
/*            run_off[i+1])                                                   */
/* record_run: out, n_rids*rec_bytes bytes: the INTERNAL runs, same layout     */
/* dst      : out, the gathered output                                        */
/* ------------------------------------------------------------------------- */
int oracle_dpg_phases(const uint8_t *src, int64_t n_src, int32_t rec_bytes,
                      const int32_t *rids, int64_t n_rids, int64_t run_len,
                      int32_t *rid_run, int64_t *run_off, uint8_t *record_run,
                      uint8_t *dst)
{
    if (rec_bytes <= 0 || n_src < 0 || n_rids < 0 || run_len <= 0)
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < n_rids; ++i)
        if (rids[i] < 0 || rids[i] >= n_src)
            return ORACLE_ERANGE;
    int64_t n_runs = (n_src + run_len - 1) / run_len;
    int64_t *count = calloc((size_t)(n_runs + 1), sizeof(int64_t));
    int64_t *cursor = calloc((size_t)(n_runs + 1), sizeof(int64_t));
    uint8_t *cache = malloc((size_t)(run_len * rec_bytes) + 1);
    if (!count || !cursor || !cache) {
        free(count); free(cursor); free(cache);
        return ORACLE_EINVAL;
    }

    /* Phase I, Distribute: every rid is appended, in RID order, to the run that
     * holds it; the run of rid r is floor(r / L).  Runs are sized by a count
     * first so that duplicated rids and skew fit (Section 2.3). */
    for (int64_t i = 0; i < n_rids; ++i)
        count[rids[i] / run_len]++;
    run_off[0] = 0;
    for (int64_t b = 0; b < n_runs; ++b)
        run_off[b + 1] = run_off[b] + count[b];
    for (int64_t b = 0; b < n_runs; ++b)
        cursor[b] = run_off[b];
    for (int64_t i = 0; i < n_rids; ++i) {
        int64_t b = rids[i] / run_len;
        rid_run[cursor[b]++] = rids[i];
    }

    /* Phase II, Probe: load input run b into the "cache", then append, in the
     * order of RID run b, the records it names to INTERNAL run b. */
    for (int64_t b = 0; b < n_runs; ++b) {
        int64_t first = b * run_len;
        int64_t len = n_src - first < run_len ? n_src - first : run_len;
        memcpy(cache, src + first * (int64_t)rec_bytes, (size_t)(len * rec_bytes));
        for (int64_t k = run_off[b]; k < run_off[b + 1]; ++k) {
            int64_t local = rid_run[k] - first;
            memcpy(record_run + k * (int64_t)rec_bytes, cache + local * (int64_t)rec_bytes,
                   (size_t)rec_bytes);
        }
    }

    /* Phase III, Gather: walk RID again; for rid r take the next unread record
     * of INTERNAL run floor(r / L) and append it to the output. */
    for (int64_t b = 0; b < n_runs; ++b)
        cursor[b] = run_off[b];
    for (int64_t i = 0; i < n_rids; ++i) {
        int64_t b = rids[i] / run_len;
        memcpy(dst + i * (int64_t)rec_bytes, record_run + cursor[b] * (int64_t)rec_bytes,
               (size_t)rec_bytes);
        cursor[b]++;
    }
    free(count); free(cursor); free(cache);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Three-phase key-pointer sort of Section 3: (1) extract key-pointer pairs,   */
/* (2) sort the pairs, (3) copy the records in the sorted order.               */
/* ------------------------------------------------------------------------- */
#define ORACLE_MAX_KEY 64
typedef struct {
    uint8_t key[ORACLE_MAX_KEY];
    int64_t index;
} key_pointer;

static int32_t g_key_bytes;

static int compare_key_pointer(const void *pa, const void *pb)
{
    const key_pointer *a = (const key_pointer *)pa;
    const key_pointer *b = (const key_pointer *)pb;
    int c = memcmp(a->key, b->key, (size_t)g_key_bytes);
    if (c != 0)
        return c;
#ifdef ORACLE_MUTANT_TIES_DESCENDING
    return (a->index < b->index) ? 1 : (a->index > b->index ? -1 : 0);
#else
    return (a->index < b->index) ? -1 : (a->index > b->index ? 1 : 0);
#endif
}

int oracle_sort_records(const uint8_t *src, int64_t n, int32_t rec_bytes,
                        int32_t key_offset, int32_t key_bytes,
                        uint8_t *dst, int64_t *perm)
{
    if (n < 0 || rec_bytes <= 0 || key_offset < 0 || key_bytes <= 0 ||
        key_bytes > ORACLE_MAX_KEY || key_offset + key_bytes > rec_bytes)
        return ORACLE_EINVAL;
    if (n == 0)
        return ORACLE_OK;
    key_pointer *pairs = malloc((size_t)n * sizeof(key_pointer));
    if (!pairs)
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        memcpy(pairs[i].key, src + i * (int64_t)rec_bytes + key_offset, (size_t)key_bytes);
        pairs[i].index = i;
    }
    g_key_bytes = key_bytes;
    qsort(pairs, (size_t)n, sizeof(key_pointer), compare_key_pointer);
    for (int64_t j = 0; j < n; ++j) {
        int64_t r = pairs[j].index;
        memcpy(dst + j * (int64_t)rec_bytes, src + r * (int64_t)rec_bytes, (size_t)rec_bytes);
        if (perm)
            perm[j] = r;
    }
    free(pairs);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Foreign-key joins of Section 4.2.1.  The fact relation references the       */
/* dimension relation; the little-endian uint32 at fk_offset of a fact row is  */
/* the dimension row id.                                                       */
/* ------------------------------------------------------------------------- */
static uint32_t read_le_u32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

static void emit_joined_row(uint8_t *out_row, const uint8_t *fact_row, int32_t fact_bytes,
                            const uint8_t *dim_row, int32_t dim_bytes)
{
    memcpy(out_row, fact_row, (size_t)fact_bytes);
    memcpy(out_row + fact_bytes, dim_row, (size_t)dim_bytes);
}

static int check_join_args(int64_t n_fact, int32_t fact_bytes, int32_t fk_offset,
                           int64_t n_dim, int32_t dim_bytes)
{
    if (n_fact < 0 || n_dim < 0 || fact_bytes <= 0 || dim_bytes <= 0 || fk_offset < 0 ||
        fk_offset + 4 > fact_bytes)
        return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* DPG-Move goal: dimension rows brought into fact (rid_R) order. */
int oracle_fk_join_fact_order(const uint8_t *fact, int64_t n_fact, int32_t fact_bytes,
                              int32_t fk_offset, const uint8_t *dim, int64_t n_dim,
                              int32_t dim_bytes, uint8_t *out)
{
    int rc = check_join_args(n_fact, fact_bytes, fk_offset, n_dim, dim_bytes);
    if (rc)
        return rc;
    int64_t out_bytes = (int64_t)fact_bytes + dim_bytes;
    for (int64_t i = 0; i < n_fact; ++i)
        if ((int64_t)read_le_u32(fact + i * (int64_t)fact_bytes + fk_offset) >= n_dim)
            return ORACLE_ERANGE;
    for (int64_t i = 0; i < n_fact; ++i) {
        const uint8_t *f = fact + i * (int64_t)fact_bytes;
        int64_t k = read_le_u32(f + fk_offset);
        emit_joined_row(out + i * out_bytes, f, fact_bytes, dim + k * (int64_t)dim_bytes, dim_bytes);
    }
    return ORACLE_OK;
}

typedef struct {
    uint32_t fk;
    int64_t rid;
} rid_pair;

static int compare_rid_pair(const void *pa, const void *pb)
{
    const rid_pair *a = (const rid_pair *)pa;
    const rid_pair *b = (const rid_pair *)pb;
    if (a->fk != b->fk)
        return a->fk < b->fk ? -1 : 1;
#ifdef ORACLE_MUTANT_UNSTABLE_JOIN
    return (a->rid < b->rid) ? 1 : (a->rid > b->rid ? -1 : 0);
#else
    return (a->rid < b->rid) ? -1 : (a->rid > b->rid ? 1 : 0);
#endif
}

/* DPG-Sort goal: rid pairs sorted by rid_F (the foreign key), fact rows brought
 * into that order; equal keys keep fact (rid_R) order. */
int oracle_fk_join_dim_order(const uint8_t *fact, int64_t n_fact, int32_t fact_bytes,
                             int32_t fk_offset, const uint8_t *dim, int64_t n_dim,
                             int32_t dim_bytes, uint8_t *out)
{
    int rc = check_join_args(n_fact, fact_bytes, fk_offset, n_dim, dim_bytes);
    if (rc)
        return rc;
    if (n_fact == 0)
        return ORACLE_OK;
    int64_t out_bytes = (int64_t)fact_bytes + dim_bytes;
    rid_pair *pairs = malloc((size_t)n_fact * sizeof(rid_pair));
    if (!pairs)
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < n_fact; ++i) {
        pairs[i].fk = read_le_u32(fact + i * (int64_t)fact_bytes + fk_offset);
        pairs[i].rid = i;
        if ((int64_t)pairs[i].fk >= n_dim) {
            free(pairs);
            return ORACLE_ERANGE;
        }
    }
    qsort(pairs, (size_t)n_fact, sizeof(rid_pair), compare_rid_pair);
    for (int64_t j = 0; j < n_fact; ++j) {
        const uint8_t *f = fact + pairs[j].rid * (int64_t)fact_bytes;
        emit_joined_row(out + j * out_bytes, f, fact_bytes,
                        dim + (int64_t)pairs[j].fk * dim_bytes, dim_bytes);
    }
    free(pairs);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Hash index and batch lookup (Section 4.2.3, batch lookup in hash indexes). */
/*                                                                           */
/* The paper's hash index holds one key-rid pair per hash slot and keeps the */
/* pairs that collide with an occupied slot in a second, overflow array.    */
/* This oracle fixes the layout so that two builds can be compared byte for  */
/* byte:                                                                     */
/*   - S = 2^log2_slots slots; the home slot of key k is the top log2_slots  */
/*     bits of the 32-bit product k * 0x9E3779B1 (Knuth's multiplicative     */
/*     hashing with the golden-ratio constant);                              */
/*   - slots[2h], slots[2h+1] = key, rid of the smallest rid whose key has   */
/*     home h; an empty slot holds key 0, rid 0xFFFFFFFF;                    */
/*   - every other key-rid pair sits in ov (pairs of uint32), ordered by     */
/*     (home slot, rid); ov_off[h] = number of overflow pairs whose home is  */
/*     below h, ov_off[S] = all of them.                                     */
/* The lookup result is defined without the index: for each query, the      */
/* smallest rid whose key equals it, or -1.                                  */
/* ------------------------------------------------------------------------- */
#define ORACLE_HASH_MUL 0x9E3779B1u
#define ORACLE_HASH_EMPTY 0xFFFFFFFFu

static uint32_t hash_home(uint32_t key, int32_t log2_slots)
{
    return (uint32_t)(key * ORACLE_HASH_MUL) >> (32 - log2_slots);
}

int oracle_hash_build(const uint32_t *keys, int64_t n, int32_t log2_slots,
                      uint32_t *slots, int64_t *ov_off, uint32_t *ov, int64_t *n_ov)
{
    if (n < 0 || n > INT32_MAX - 1 || log2_slots < 1 || log2_slots > 30)
        return ORACLE_EINVAL;
    int64_t S = (int64_t)1 << log2_slots;
    int64_t *count = calloc((size_t)S, sizeof(int64_t));
    int64_t *cursor = malloc((size_t)S * sizeof(int64_t));
    if (!count || !cursor) {
        free(count);
        free(cursor);
        return ORACLE_EINVAL;
    }
    for (int64_t h = 0; h < S; ++h) {
        slots[2 * h] = 0;
        slots[2 * h + 1] = ORACLE_HASH_EMPTY;
    }
    /* the first key of each slot (in rid order) takes the slot */
    for (int64_t j = 0; j < n; ++j) {
        uint32_t h = hash_home(keys[j], log2_slots);
#ifdef ORACLE_MUTANT_HASH_LAST
        if (count[h] >= 0) {
#else
        if (count[h] == 0) {
#endif
            slots[2 * h] = keys[j];
            slots[2 * h + 1] = (uint32_t)j;
        }
        count[h] += 1;
    }
    /* overflow offsets: one fewer pair per occupied slot */
    int64_t total = 0;
    for (int64_t h = 0; h < S; ++h) {
        ov_off[h] = total;
        cursor[h] = total;
        if (count[h] > 1)
            total += count[h] - 1;
    }
    ov_off[S] = total;
    /* the other keys, in (home, rid) order */
    for (int64_t j = 0; j < n; ++j) {
        uint32_t h = hash_home(keys[j], log2_slots);
        if (slots[2 * h + 1] == (uint32_t)j)
            continue;
        ov[2 * cursor[h]] = keys[j];
        ov[2 * cursor[h] + 1] = (uint32_t)j;
        cursor[h] += 1;
    }
    *n_ov = total;
    free(count);
    free(cursor);
    return ORACLE_OK;
}

typedef struct {
    uint32_t key;
    int64_t rid;
} key_rid;

static int compare_key_rid(const void *pa, const void *pb)
{
    const key_rid *a = pa, *b = pb;
    if (a->key != b->key)
        return a->key < b->key ? -1 : 1;
    return (a->rid > b->rid) - (a->rid < b->rid);
}

int oracle_hash_lookup(const uint32_t *keys, int64_t n, const uint32_t *queries, int64_t m,
                       int32_t *out)
{
    if (n < 0 || n > INT32_MAX - 1 || m < 0)
        return ORACLE_EINVAL;
    key_rid *pairs = malloc((size_t)(n > 0 ? n : 1) * sizeof(key_rid));
    if (!pairs)
        return ORACLE_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        pairs[j].key = keys[j];
        pairs[j].rid = j;
    }
    qsort(pairs, (size_t)n, sizeof(key_rid), compare_key_rid);
    for (int64_t i = 0; i < m; ++i) {
        /* first pair whose key is >= the query */
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (pairs[mid].key < queries[i])
                lo = mid + 1;
            else
                hi = mid;
        }
#ifdef ORACLE_MUTANT_LOOKUP_LAST
        while (lo + 1 < n && pairs[lo + 1].key == queries[i])
            ++lo;
#endif
        out[i] = (lo < n && pairs[lo].key == queries[i]) ? (int32_t)pairs[lo].rid : -1;
    }
    free(pairs);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Sort-merge join (Section 4.1): both relations sorted on the join key, then */
/* merged.  The result is every pair (i, j) whose join keys are equal (the    */
/* key_bytes bytes at key_off_r of R row i and at key_off_s of S row j), each */
/* written as R row i followed by S row j, ordered by key (unsigned bytes,    */
/* memcmp order), then i, then j.                                            */
/* Returns ERANGE with *n_out = the number of result rows when out_capacity  */
/* rows do not hold them (nothing is written then).                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    const uint8_t *key;
    int64_t idx;
} keyed_row;

static int32_t g_smj_key_bytes;

static int compare_keyed_row(const void *pa, const void *pb)
{
    const keyed_row *a = pa, *b = pb;
    int c = memcmp(a->key, b->key, (size_t)g_smj_key_bytes);
    if (c)
        return c;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static keyed_row *sorted_rows(const uint8_t *rows, int64_t n, int32_t rec_bytes, int32_t key_off)
{
    keyed_row *k = malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed_row));
    if (!k)
        return NULL;
    for (int64_t i = 0; i < n; ++i) {
        k[i].key = rows + i * (int64_t)rec_bytes + key_off;
        k[i].idx = i;
    }
    qsort(k, (size_t)n, sizeof(keyed_row), compare_keyed_row);
    return k;
}

int oracle_sort_merge_join(const uint8_t *r, int64_t n_r, int32_t rec_r, int32_t key_off_r,
                           const uint8_t *s, int64_t n_s, int32_t rec_s, int32_t key_off_s,
                           int32_t key_bytes, uint8_t *out, int64_t out_capacity, int64_t *n_out)
{
    if (n_r < 0 || n_s < 0 || rec_r < 1 || rec_s < 1 || key_bytes < 1 || key_off_r < 0 || key_off_s < 0 ||
        key_off_r + key_bytes > rec_r || key_off_s + key_bytes > rec_s)
        return ORACLE_EINVAL;
    g_smj_key_bytes = key_bytes;
    keyed_row *kr = sorted_rows(r, n_r, rec_r, key_off_r);
    keyed_row *ks = sorted_rows(s, n_s, rec_s, key_off_s);
    if (!kr || !ks) {
        free(kr);
        free(ks);
        return ORACLE_EINVAL;
    }
    int64_t out_bytes = (int64_t)rec_r + rec_s;
    for (int pass = 0; pass < 2; ++pass) {  /* count, then write */
        int64_t a = 0, b = 0, n = 0;
        while (a < n_r && b < n_s) {
            int c = memcmp(kr[a].key, ks[b].key, (size_t)key_bytes);
            if (c < 0) {
                ++a;
            } else if (c > 0) {
                ++b;
            } else {
                int64_t a2 = a, b2 = b;
                while (a2 < n_r && memcmp(kr[a2].key, kr[a].key, (size_t)key_bytes) == 0)
                    ++a2;
                while (b2 < n_s && memcmp(ks[b2].key, ks[b].key, (size_t)key_bytes) == 0)
                    ++b2;
                /* the pairs of one key, R index major */
                for (int64_t u = 0; u < (a2 - a) * (b2 - b); ++u) {
#ifdef ORACLE_MUTANT_SMJ_J_MAJOR
                    int64_t x = a + u % (a2 - a), y = b + u / (a2 - a);
#else
                    int64_t x = a + u / (b2 - b), y = b + u % (b2 - b);
#endif
                    if (pass == 1) {
                        uint8_t *row = out + n * out_bytes;
                        memcpy(row, r + kr[x].idx * (int64_t)rec_r, (size_t)rec_r);
                        memcpy(row + rec_r, s + ks[y].idx * (int64_t)rec_s, (size_t)rec_s);
                    }
                    ++n;
                }
                a = a2;
                b = b2;
            }
        }
        if (pass == 0) {
            *n_out = n;
            if (n > out_capacity) {
                free(kr);
                free(ks);
                return ORACLE_ERANGE;
            }
        }
    }
    free(kr);
    free(ks);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Enhanced B+ tree and batch lookup in it (Section 4.2.3, batch lookup in
 * B+ tree indexes).
 *
 * "Enhanced" means every slot of every node is used, so the tree is fixed by
 * its entries and the fanout (32 here).  Level 0 holds the (key, rid) entries
 * sorted by key, then rid, in blocks of 32; the last block is padded with key
 * 0xFFFFFFFF and rid -1, and there is always at least one block.  Level l >= 1
 * has ceil(nodes of level l-1 / 32) nodes of 32 keys: entry i of node j is the
 * largest key under child c = 32 j + i of level l-1 (the child's last entry),
 * or 0xFFFFFFFF when there is no such child.  The top level has one node.
 *
 * A lookup walks down from the root: in each node it takes the first entry not
 * less than the query (the children before it hold only smaller keys), and in
 * the leaf block the first key not less than the query; the result is that
 * entry's rid when its key equals the query, else -1.  So a key held by
 * several entries returns its smallest rid, as the hash lookup does.
 * ------------------------------------------------------------------------- */
#define ORACLE_BTREE_FANOUT 32
#define ORACLE_BTREE_PAD 0xFFFFFFFFu

/* Number of levels (leaf level included); nodes[l] = nodes of level l. */
int oracle_btree_shape(int64_t n, int64_t *nodes, int32_t max_levels)
{
    if (n < 0 || n > INT32_MAX - 1)
        return -1;
    int64_t c = (n + ORACLE_BTREE_FANOUT - 1) / ORACLE_BTREE_FANOUT;
    if (c < 1)
        c = 1;
    int32_t levels = 0;
    for (;;) {
        if (levels >= max_levels)
            return -1;
        nodes[levels++] = c;
        if (c == 1)
            break;
        c = (c + ORACLE_BTREE_FANOUT - 1) / ORACLE_BTREE_FANOUT;
    }
    return levels;
}

/* leaf_keys, leaf_rids: nodes[0] * 32 entries; inner: the levels 1, 2, ...
 * laid end to end, nodes[l] * 32 keys each. */
int oracle_btree_build(const uint32_t *keys, int64_t n, uint32_t *leaf_keys, int32_t *leaf_rids,
                       uint32_t *inner)
{
    int64_t nodes[16];
    int32_t levels = oracle_btree_shape(n, nodes, 16);
    if (levels < 1)
        return ORACLE_EINVAL;
    key_rid *pairs = malloc((size_t)(n > 0 ? n : 1) * sizeof(key_rid));
    if (!pairs)
        return ORACLE_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        pairs[j].key = keys[j];
        pairs[j].rid = j;
    }
    qsort(pairs, (size_t)n, sizeof(key_rid), compare_key_rid);
    int64_t slots = nodes[0] * ORACLE_BTREE_FANOUT;
    for (int64_t e = 0; e < slots; ++e) {
        leaf_keys[e] = e < n ? pairs[e].key : ORACLE_BTREE_PAD;
        leaf_rids[e] = e < n ? (int32_t)pairs[e].rid : -1;
    }
    free(pairs);
    const uint32_t *below = leaf_keys;
    uint32_t *level = inner;
    for (int32_t l = 1; l < levels; ++l) {
        for (int64_t j = 0; j < nodes[l]; ++j) {
            for (int i = 0; i < ORACLE_BTREE_FANOUT; ++i) {
                int64_t c = j * ORACLE_BTREE_FANOUT + i;
#ifdef ORACLE_MUTANT_BTREE_FIRST_ENTRY
                uint32_t v = c < nodes[l - 1] ? below[c * ORACLE_BTREE_FANOUT] : ORACLE_BTREE_PAD;
#else
                uint32_t v = c < nodes[l - 1] ? below[c * ORACLE_BTREE_FANOUT + ORACLE_BTREE_FANOUT - 1]
                                              : ORACLE_BTREE_PAD;
#endif
                level[j * ORACLE_BTREE_FANOUT + i] = v;
            }
        }
        below = level;
        level += nodes[l] * ORACLE_BTREE_FANOUT;
    }
    return ORACLE_OK;
}

/* Position of the first of the 32 keys of a node that is not less than q
 * (32 when every key is less). */
static int btree_first_not_less(const uint32_t *node, uint32_t q)
{
    int i = 0;
#ifdef ORACLE_MUTANT_BTREE_STRICT
    while (i < ORACLE_BTREE_FANOUT && node[i] <= q)
#else
    while (i < ORACLE_BTREE_FANOUT && node[i] < q)
#endif
        ++i;
    return i;
}

int oracle_btree_lookup(const uint32_t *leaf_keys, const int32_t *leaf_rids, const uint32_t *inner,
                        int64_t n, const uint32_t *queries, int64_t m, int32_t *out)
{
    int64_t nodes[16];
    int32_t levels = oracle_btree_shape(n, nodes, 16);
    if (levels < 1 || m < 0)
        return ORACLE_EINVAL;
    const uint32_t *level_at[16];
    level_at[0] = leaf_keys;
    const uint32_t *p = inner;
    for (int32_t l = 1; l < levels; ++l) {
        level_at[l] = p;
        p += nodes[l] * ORACLE_BTREE_FANOUT;
    }
    for (int64_t k = 0; k < m; ++k) {
        uint32_t q = queries[k];
        int64_t node = 0;
        int32_t result = -1;
        int found_path = 1;
        for (int32_t l = levels - 1; l >= 1; --l) {
            int i = btree_first_not_less(level_at[l] + node * ORACLE_BTREE_FANOUT, q);
            int64_t c = node * ORACLE_BTREE_FANOUT + i;
            if (i == ORACLE_BTREE_FANOUT || c >= nodes[l - 1]) {
                found_path = 0; /* larger than every key */
                break;
            }
            node = c;
        }
        if (found_path) {
            int i = btree_first_not_less(leaf_keys + node * ORACLE_BTREE_FANOUT, q);
            if (i < ORACLE_BTREE_FANOUT) {
                int64_t e = node * ORACLE_BTREE_FANOUT + i;
                if (leaf_keys[e] == q && leaf_rids[e] >= 0)
                    result = leaf_rids[e];
            }
        }
        out[k] = result;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Foreign-key join over non-dense keys (Sections 4.2.2 and 4.2.3): the      */
/* dimension rows carry a uint32 key at key_offset, and the join triple of   */
/* fact row i is (fk_i, i, j) with j the first dimension row whose key is    */
/* fk_i -- the rid an index lookup of fk_i returns.  Every fk must have a    */
/* dimension row (ORACLE_ERANGE otherwise).  order 0: out[i] = fact[i] ||    */
/* dim[j_i] (fact order); order 1: the same rows ordered by j, ties in fact  */
/* order (dimension order).                                                  */
/* ------------------------------------------------------------------------- */
int oracle_key_join(const uint8_t *fact, int64_t n_fact, int32_t fact_bytes, int32_t fk_offset,
                    const uint8_t *dim, int64_t n_dim, int32_t dim_bytes, int32_t key_offset, int32_t order,
                    uint8_t *out)
{
    if (n_fact < 0 || n_dim < 0 || n_dim > INT32_MAX - 1 || fact_bytes < 1 || dim_bytes < 1 || fk_offset < 0 ||
        fk_offset + 4 > fact_bytes || key_offset < 0 || key_offset + 4 > dim_bytes || (order != 0 && order != 1))
        return ORACLE_EINVAL;
    if (n_fact == 0)
        return ORACLE_OK;
    key_rid *keys = malloc((size_t)(n_dim > 0 ? n_dim : 1) * sizeof(key_rid));
    rid_pair *pairs = malloc((size_t)n_fact * sizeof(rid_pair));
    if (!keys || !pairs) {
        free(keys);
        free(pairs);
        return ORACLE_EINVAL;
    }
    for (int64_t j = 0; j < n_dim; ++j) {
        keys[j].key = read_le_u32(dim + j * (int64_t)dim_bytes + key_offset);
        keys[j].rid = j;
    }
    qsort(keys, (size_t)n_dim, sizeof(key_rid), compare_key_rid);
    for (int64_t i = 0; i < n_fact; ++i) {
        uint32_t fk = read_le_u32(fact + i * (int64_t)fact_bytes + fk_offset);
        int64_t lo = 0, hi = n_dim; /* first (key, rid) with key >= fk */
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (keys[mid].key < fk)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo == n_dim || keys[lo].key != fk) {
            free(keys);
            free(pairs);
            return ORACLE_ERANGE;
        }
#ifdef ORACLE_MUTANT_KEYJOIN_LAST_MATCH
        while (lo + 1 < n_dim && keys[lo + 1].key == fk)
            ++lo;
#endif
        pairs[i].fk = (uint32_t)keys[lo].rid;
        pairs[i].rid = i;
    }
    if (order == 1)
        qsort(pairs, (size_t)n_fact, sizeof(rid_pair), compare_rid_pair);
    int64_t out_bytes = (int64_t)fact_bytes + dim_bytes;
    for (int64_t k = 0; k < n_fact; ++k)
        emit_joined_row(out + k * out_bytes, fact + pairs[k].rid * (int64_t)fact_bytes, fact_bytes,
                        dim + (int64_t)pairs[k].fk * dim_bytes, dim_bytes);
    free(keys);
    free(pairs);
    return ORACLE_OK;
}
