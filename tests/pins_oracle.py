"""Pins for the CPU oracle: checks against what the paper and plain mathematics
fix, never against the oracle's own formula.

Each ``pin_*`` function takes a loaded oracle library and raises
AssertionError on a mismatch, so the same pins also run against deliberately
broken builds of the oracle (see test_oracle_mutants.py).
"""
from __future__ import annotations

import itertools
import os

import numpy as np

import oracle
from paper_cs_0308004_amd import synth

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def distinct_records(n: int, rec_bytes: int, seed: int = 7) -> np.ndarray:
    """n records whose contents are pairwise distinct in every 4-byte word.

    Word w of record r holds the little-endian uint32 r * 4099 + w * 65537 + seed,
    so a copied record identifies its source even if only part was copied."""
    r = np.arange(n, dtype=np.uint64)[:, None]
    w = np.arange(rec_bytes // 4, dtype=np.uint64)[None, :]
    words = ((r * np.uint64(4099) + w * np.uint64(65537) + np.uint64(seed)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return words.view(np.uint8).reshape(n, rec_bytes)


def identify(dst: np.ndarray, src: np.ndarray) -> np.ndarray:
    """For each row of dst, the index of the equal row of src (-1 if none)."""
    table = {src[r].tobytes(): r for r in range(src.shape[0])}
    return np.array([table.get(dst[i].tobytes(), -1) for i in range(dst.shape[0])], dtype=np.int64)


# ---------------------------------------------------------------------------
# retrieval (problem statement of Section 2)
# ---------------------------------------------------------------------------
def pin_retrieve_brute_force(lib):
    """Every rid sequence for N <= 4, M <= 4: output record i is exactly source record rids[i]."""
    for rec_bytes in (4, 8, 12, 100):
        for n in range(1, 5):
            src = distinct_records(n, rec_bytes)
            for m in range(0, 5):
                for seq in itertools.product(range(n), repeat=m):
                    rids = np.array(seq, dtype=np.int32)
                    dst = oracle.retrieve(src, rids, lib=lib)
                    assert dst.shape == (m, rec_bytes)
                    got = identify(dst, src)
                    assert np.array_equal(got, rids.astype(np.int64)), (rec_bytes, n, seq, got)


def pin_retrieve_closed_forms(lib):
    """Identity, reversal, an affine permutation and a blocked permutation."""
    for rec_bytes in (8, 100, 256):
        n = 1 << 10
        src = synth.record_bytes(n, rec_bytes, seed=11)
        ident = np.arange(n, dtype=np.int32)
        assert np.array_equal(oracle.retrieve(src, ident, lib=lib), src)
        assert np.array_equal(oracle.retrieve(src, ident[::-1].copy(), lib=lib), src[::-1])
        a, c = 389, 77  # i -> (a*i + c) mod 2^10 is a bijection because a is odd
        aff = ((a * ident.astype(np.int64) + c) % n).astype(np.int32)
        dst = oracle.retrieve(src, aff, lib=lib)
        for i in (0, 1, 2, 500, n - 1):
            assert np.array_equal(dst[i], src[(a * i + c) % n])
        blocked = synth.rids_blocked(n, rec_bytes, seed=3)
        run = 4096 // rec_bytes
        dst = oracle.retrieve(src, blocked, lib=lib)
        pieces, pos = [], 0
        while pos < n:  # each run is a contiguous ascending slice of the source
            start = int(blocked[pos])
            length = min(run - start % run, n - start)
            pieces.append(src[start:start + length])
            pos += length
        assert np.array_equal(dst, np.concatenate(pieces))


def pin_retrieve_multiset(lib):
    """A permutation moves every record exactly once; with replacement the
    number of copies of each record equals the number of times its rid occurs."""
    n, rec_bytes = 3000, 12
    src = distinct_records(n, rec_bytes)
    perm = synth.rids_permutation(n, seed=5)
    got = identify(oracle.retrieve(src, perm, lib=lib), src)
    assert np.array_equal(np.sort(got), np.arange(n))
    rids = synth.rids_uniform(n, 2 * n, seed=9)
    got = identify(oracle.retrieve(src, rids, lib=lib), src)
    assert np.array_equal(np.bincount(got, minlength=n), np.bincount(rids, minlength=n))


def pin_retrieve_errors(lib):
    src = distinct_records(4, 8)
    for bad in (4, -1, 1 << 30):
        try:
            oracle.retrieve(src, np.array([0, bad], dtype=np.int32), lib=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.ERANGE
        else:
            raise AssertionError(f"rid {bad} accepted")
    assert oracle.retrieve(src, np.zeros(0, np.int32), lib=lib).shape == (0, 8)


# ---------------------------------------------------------------------------
# Figure 1 / Section 2.2
# ---------------------------------------------------------------------------
def load_fig2():
    keys, rids, facts = [], [], {}
    with open(os.path.join(GOLDEN_DIR, "fig2_example.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if len(parts) == 2 and len(parts[0]) == 1:
                keys.append(parts[0])
                rids.append(int(parts[1]))
            else:
                facts[parts[0]] = parts[1:]
    return keys, rids, facts


def pin_fig2_example(lib):
    keys, rids, facts = load_fig2()
    n = len(keys)
    run_len = int(facts["run_len"][0])
    # record r carries the key whose rid is r, as one byte, padded to 4 bytes
    src = np.zeros((n, 4), dtype=np.uint8)
    for k, r in zip(keys, rids):
        src[r, 0] = ord(k)
    input_run0 = [chr(src[r, 0]) for r in range(run_len)]
    assert input_run0 == facts["input_run0_keys"]
    rid_arr = np.array(rids, dtype=np.int32)
    rid_run, run_off, record_run, dst = oracle.dpg_phases(src, rid_arr, run_len, lib=lib)
    assert [r // run_len for r in rids[:4]] == [int(x) for x in facts["first_four_runs"]]
    assert list(rid_run[run_off[0]:run_off[1]]) == [int(x) for x in facts["rid_run0"]]
    internal0 = [chr(record_run[k, 0]) for k in range(run_off[0], run_off[1])]
    assert internal0 == facts["internal_run0_keys"]
    out_keys = [chr(dst[i, 0]) for i in range(n)]
    assert out_keys == sorted(keys)  # the output is the records in key order
    assert np.array_equal(dst, oracle.retrieve(src, rid_arr, lib=lib))


def pin_phase_invariants(lib):
    """Section 2.1: RID run b of a permutation is a permutation of [bL, (b+1)L);
    INTERNAL run b holds the records of input run b; runs keep RID order; the
    gathered output equals the definition."""
    rec_bytes = 8
    for n, run_len in ((1000, 64), (1 << 12, 256), (777, 1000)):
        src = distinct_records(n, rec_bytes)
        rids = synth.rids_permutation(n, seed=n)
        rid_run, run_off, record_run, dst = oracle.dpg_phases(src, rids, run_len, lib=lib)
        n_runs = -(-n // run_len)
        assert run_off[0] == 0 and run_off[-1] == n and len(run_off) == n_runs + 1
        position = np.empty(n, dtype=np.int64)
        position[rids] = np.arange(n)
        for b in range(n_runs):
            run = rid_run[run_off[b]:run_off[b + 1]]
            lo, hi = b * run_len, min(n, (b + 1) * run_len)
            assert np.array_equal(np.sort(run), np.arange(lo, hi))
            assert np.all(np.diff(position[run]) > 0)  # stable: RID order kept
            got = identify(record_run[run_off[b]:run_off[b + 1]], src)
            assert np.array_equal(got, run)
        assert np.array_equal(identify(dst, src), rids.astype(np.int64))
    # duplicates (Section 2's non-permutation case): runs are sized by counts
    n, run_len = 500, 32
    src = distinct_records(n, rec_bytes)
    rids = synth.rids_uniform(n, 3 * n, seed=1)
    rid_run, run_off, record_run, dst = oracle.dpg_phases(src, rids, run_len, lib=lib)
    counts = np.bincount(rids // run_len, minlength=-(-n // run_len))
    assert np.array_equal(np.diff(run_off), counts)
    assert np.array_equal(identify(dst, src), rids.astype(np.int64))


# ---------------------------------------------------------------------------
# Section 3: key-pointer sort
# ---------------------------------------------------------------------------
def _check_sorted(src, dst, perm, key_offset, key_bytes):
    n = src.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n)), "perm is not a permutation"
    assert np.array_equal(dst, src[perm])
    keys = dst[:, key_offset:key_offset + key_bytes]
    for j in range(1, n):
        a, b = keys[j - 1].tobytes(), keys[j].tobytes()
        assert a <= b, f"keys out of order at {j}"
        if a == b:
            assert perm[j - 1] < perm[j], f"equal keys not in index order at {j}"


def pin_sort_random(lib):
    for n, rec_bytes in ((1000, 100), (513, 12), (1, 16)):
        src = synth.record_bytes(n, rec_bytes, seed=n + rec_bytes)
        dst, perm = oracle.sort_records(src, 0, 10, lib=lib)
        _check_sorted(src, dst, perm, 0, 10)
        # numpy's stable lexsort on the key columns gives the same unique order
        order = np.lexsort(tuple(src[:, j] for j in range(9, -1, -1)))
        assert np.array_equal(perm, order)


def pin_sort_ties(lib):
    rng = np.random.default_rng(0)
    n, rec_bytes = 600, 16
    src = rng.integers(0, 256, size=(n, rec_bytes), dtype=np.uint8)
    src[:, 0:8] = rng.integers(0, 3, size=(n, 1), dtype=np.uint8)  # 3 distinct 8-byte prefixes
    src[:, 8:10] = rng.integers(0, 2, size=(n, 2), dtype=np.uint8)  # bytes 8, 9 decide within
    dst, perm = oracle.sort_records(src, 0, 10, lib=lib)
    _check_sorted(src, dst, perm, 0, 10)
    same = np.zeros((50, rec_bytes), dtype=np.uint8)
    same[:, 10:] = np.arange(50, dtype=np.uint8)[:, None]
    dst, perm = oracle.sort_records(same, 0, 10, lib=lib)
    assert np.array_equal(perm, np.arange(50))
    desc = np.zeros((40, 12), dtype=np.uint8)
    desc[:, 9] = np.arange(40, 0, -1, dtype=np.uint8)  # strictly decreasing keys
    dst, perm = oracle.sort_records(desc, 0, 10, lib=lib)
    assert np.array_equal(perm, np.arange(39, -1, -1))
    # key at a non-zero offset
    dst, perm = oracle.sort_records(src, 6, 4, lib=lib)
    _check_sorted(src, dst, perm, 6, 4)


# ---------------------------------------------------------------------------
# Section 4.2.1: foreign-key joins
# ---------------------------------------------------------------------------
def _join_inputs(n_fact, n_dim, s, seed):
    fact = synth.fact_table(n_fact, n_dim, s, seed)
    dim = synth.dim_table(n_dim, seed)
    fk = fact[:, 0:4].copy().view(np.uint32).reshape(-1).astype(np.int64)
    return fact, dim, fk


def pin_join_fact_order(lib):
    for n_fact, n_dim, s in ((5000, 300, 0.0), (4000, 1 << 10, 1.2), (1, 1, 0.0)):
        fact, dim, fk = _join_inputs(n_fact, n_dim, s, seed=n_fact)
        out = oracle.fk_join_fact_order(fact, dim, 0, lib=lib)
        assert out.shape == (n_fact, 80)
        assert np.array_equal(out[:, :16], fact)
        assert np.array_equal(out[:, 16:20], out[:, 0:4])  # dimension id == foreign key
        assert np.array_equal(out[:, 16:], dim[fk])


def pin_join_dim_order(lib):
    for n_fact, n_dim, s in ((5000, 300, 0.8), (3000, 64, 1.2), (2, 5, 0.0)):
        fact, dim, fk = _join_inputs(n_fact, n_dim, s, seed=n_fact + 1)
        out = oracle.fk_join_dim_order(fact, dim, 0, lib=lib)
        ofk = out[:, 0:4].copy().view(np.uint32).reshape(-1)
        assert np.all(np.diff(ofk.astype(np.int64)) >= 0)
        assert np.array_equal(np.bincount(ofk, minlength=n_dim), np.bincount(fk, minlength=n_dim))
        assert np.array_equal(out[:, 16:20], out[:, 0:4])
        # fact rows carry distinct payloads; recover each row's fact index
        rid_r = identify(out[:, :16], fact)
        assert np.array_equal(rid_r, np.argsort(fk, kind="stable"))
        assert np.array_equal(out[:, 16:], dim[ofk])


def pin_join_errors(lib):
    fact, dim, fk = _join_inputs(100, 50, 0.0, seed=3)
    fact = fact.copy()
    fact[17, 0:4] = np.array([50], dtype=np.uint32).view(np.uint8)
    for fn in (oracle.fk_join_fact_order, oracle.fk_join_dim_order):
        try:
            fn(fact, dim, 0, lib=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.ERANGE
        else:
            raise AssertionError("foreign key out of range accepted")


# ---------------------------------------------------------------------------
# hash index and batch lookup (Section 4.2.3)
# ---------------------------------------------------------------------------
def stated_home(keys: np.ndarray, log2_slots: int) -> np.ndarray:
    """The index's stated slot function: top log2_slots bits of k * 0x9E3779B1 (mod 2^32)."""
    prod = (keys.astype(np.uint64) * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    return (prod >> np.uint64(32 - log2_slots)).astype(np.int64)


def pin_hash_lookup_brute_force(lib):
    """Every key list of length <= 4 over a 3-letter alphabet, every query of
    the alphabet plus one absent value: the answer is the first position
    holding the query (linear scan), or -1."""
    alphabet = [0, 7, 0xFFFFFFFF]
    queries = np.array(alphabet + [12345], dtype=np.uint32)
    for n in range(0, 5):
        for seq in itertools.product(alphabet, repeat=n):
            keys = np.array(seq, dtype=np.uint32)
            got = oracle.hash_lookup(keys, queries, lib=lib)
            want = [next((j for j in range(n) if seq[j] == q), -1) for q in queries.tolist()]
            assert got.tolist() == want, (seq, got, want)


def pin_hash_lookup_closed_forms(lib):
    """Distinct keys: looking up the keys themselves returns 0..n-1, a shuffled
    subset returns its positions, and values never stored return -1."""
    n = 5000
    keys = (2 * synth.rids_permutation(1 << 16, seed=5)[:n].astype(np.uint32) + 1)  # odd, distinct
    assert np.array_equal(oracle.hash_lookup(keys, keys, lib=lib), np.arange(n, dtype=np.int32))
    pick = synth.rids_permutation(n, seed=6)[:700]
    assert np.array_equal(oracle.hash_lookup(keys, keys[pick], lib=lib), pick.astype(np.int32))
    even = np.arange(0, 4000, 2, dtype=np.uint32)
    assert np.all(oracle.hash_lookup(keys, even, lib=lib) == -1)
    assert oracle.hash_lookup(keys, np.zeros(0, dtype=np.uint32), lib=lib).size == 0


def pin_hash_build_invariants(lib):
    """The stated layout: every rid stored exactly once; a slot holds the
    smallest rid of its home; the overflow pairs of home h sit in
    [ov_off[h], ov_off[h+1]) in rid order; and a lookup through the index
    (slot, then its overflow range) gives the batch-lookup result."""
    rng = np.random.default_rng(8)
    for n, log2_slots, span in ((5000, 10, 1 << 32), (5000, 12, 3000), (3000, 14, 1 << 32), (1, 3, 10), (0, 4, 10)):
        keys = rng.integers(0, span, n, dtype=np.uint64).astype(np.uint32)
        slots, ov_off, ov = oracle.hash_build(keys, log2_slots, lib=lib)
        S = 1 << log2_slots
        home = stated_home(keys, log2_slots)
        occupied = slots[:, 1] != oracle.HASH_EMPTY
        # every rid once
        rids = np.concatenate([slots[occupied, 1], ov[:, 1]]).astype(np.int64)
        assert np.array_equal(np.sort(rids), np.arange(n))
        # slots: the smallest rid of each home
        first = np.full(S, -1, dtype=np.int64)
        for j in range(n - 1, -1, -1):
            first[home[j]] = j
        assert np.array_equal(occupied, first >= 0)
        assert np.array_equal(slots[occupied, 1].astype(np.int64), first[occupied])
        assert np.array_equal(slots[occupied, 0], keys[first[occupied]])
        assert np.all(slots[~occupied, 0] == 0)
        # overflow: grouped by home in slot order, rids ascending within a home
        assert ov_off[0] == 0 and ov_off[S] == len(ov) == n - occupied.sum()
        assert np.all(np.diff(ov_off) >= 0)
        ov_home = np.repeat(np.arange(S), np.diff(ov_off))
        assert np.array_equal(home[ov[:, 1].astype(np.int64)], ov_home)
        assert np.array_equal(keys[ov[:, 1].astype(np.int64)], ov[:, 0])
        order = np.lexsort((ov[:, 1].astype(np.int64), ov_home))
        assert np.array_equal(order, np.arange(len(ov)))
        # a lookup through the index
        queries = np.concatenate([keys[: min(n, 500)], rng.integers(0, 1 << 32, 300, dtype=np.uint64).astype(np.uint32)])
        want = oracle.hash_lookup(keys, queries, lib=lib)
        qh = stated_home(queries, log2_slots)
        for i, q in enumerate(queries.tolist()):
            h = int(qh[i])
            got = -1
            if slots[h, 1] != oracle.HASH_EMPTY and int(slots[h, 0]) == q:
                got = int(slots[h, 1])
            else:
                for a in range(int(ov_off[h]), int(ov_off[h + 1])):
                    if int(ov[a, 0]) == q:
                        got = int(ov[a, 1])
                        break
            assert got == want[i], (i, q, got, want[i])


def pin_hash_errors(lib):
    for log2_slots in (0, 31):
        try:
            oracle.hash_build(np.zeros(4, dtype=np.uint32), log2_slots, lib=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.EINVAL
        else:
            raise AssertionError("bad slot count accepted")


# ---------------------------------------------------------------------------
# sort-merge join (Section 4.1)
# ---------------------------------------------------------------------------
def _smj_brute(r, s, kr, ks, kb):
    """Every pair of equal keys by nested loops, ordered by (key bytes, i, j)."""
    pairs = [(bytes(r[i, kr:kr + kb]), i, j) for i in range(r.shape[0]) for j in range(s.shape[0])
             if bytes(r[i, kr:kr + kb]) == bytes(s[j, ks:ks + kb])]
    pairs.sort()
    w = r.shape[1] + s.shape[1]
    if not pairs:
        return np.zeros((0, w), dtype=np.uint8)
    return np.stack([np.concatenate([r[i], s[j]]) for _, i, j in pairs])


def pin_smj_brute_force(lib):
    """Small relations over a tiny key alphabet (many duplicates on both
    sides): the join equals the nested-loop pairs in (key, i, j) order."""
    rng = np.random.default_rng(12)
    for trial in range(60):
        kb = int(rng.integers(1, 4))
        nr, ns = int(rng.integers(0, 13)), int(rng.integers(0, 13))
        wr, ws = kb + int(rng.integers(0, 6)), kb + int(rng.integers(0, 6))
        kr, ks = int(rng.integers(0, wr - kb + 1)), int(rng.integers(0, ws - kb + 1))
        r = rng.integers(0, 256, (nr, wr), dtype=np.uint8)
        s = rng.integers(0, 256, (ns, ws), dtype=np.uint8)
        alphabet = rng.integers(0, 256, (3, kb), dtype=np.uint8)
        if nr:
            r[:, kr:kr + kb] = alphabet[rng.integers(0, 3, nr)]
        if ns:
            s[:, ks:ks + kb] = alphabet[rng.integers(0, 3, ns)]
        got = oracle.sort_merge_join(r, s, kr, ks, kb, lib=lib)
        want = _smj_brute(r, s, kr, ks, kb)
        assert got.shape == want.shape and np.array_equal(got, want), (trial, got.shape, want.shape)


def pin_smj_closed_forms(lib):
    """Distinct keys: the join is the matching rows in key order; disjoint key
    sets give nothing; one shared key gives the full cross product, R major."""
    n = 300
    r = distinct_records(n, 8, seed=1)
    s = distinct_records(2 * n, 12, seed=2)
    keys = synth.rids_permutation(2 * n, seed=9).astype(">u4")  # big-endian: memcmp order = integer order
    s[:, 4:8] = keys.view(np.uint8).reshape(-1, 4)
    r[:, 0:4] = (np.arange(n, dtype=np.uint32) * 2).astype(">u4").view(np.uint8).reshape(-1, 4)  # even keys
    out = oracle.sort_merge_join(r, s, 0, 4, 4, lib=lib)
    ks = keys.astype(np.int64)
    match = [(k, i, int(np.nonzero(ks == k)[0][0])) for i, k in enumerate(range(0, 2 * n, 2)) if k < 2 * n]
    assert out.shape[0] == len(match)
    for row, (k, i, j) in zip(out, match):
        assert np.array_equal(row[:8], r[i]) and np.array_equal(row[8:], s[j])
    s2 = s.copy()
    s2[:, 4:8] = np.frombuffer((np.arange(2 * n, dtype=np.uint32) * 2 + 1).astype(">u4").tobytes(),
                               dtype=np.uint8).reshape(-1, 4)  # odd keys
    assert oracle.sort_merge_join(r, s2, 0, 4, 4, lib=lib).shape == (0, 20)
    r3, s3 = r[:7].copy(), s[:5].copy()
    r3[:, 0:4] = 77
    s3[:, 4:8] = 77
    out3 = oracle.sort_merge_join(r3, s3, 0, 4, 4, lib=lib)
    want = np.stack([np.concatenate([r3[i], s3[j]]) for i in range(7) for j in range(5)])
    assert np.array_equal(out3, want)


def pin_smj_errors(lib):
    r = np.zeros((4, 8), dtype=np.uint8)
    for kr, kb in ((5, 4), (0, 0), (-1, 2)):
        try:
            oracle.sort_merge_join(r, r, kr, 0, kb, lib=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.EINVAL
        else:
            raise AssertionError("bad key accepted")


# ---------------------------------------------------------------------------
# enhanced B+ tree and batch lookup in it (Section 4.2.3)
# ---------------------------------------------------------------------------
BT_PAD = 0xFFFFFFFF


def _first_position(keys, q):
    """The batch-lookup answer by linear scan: first position holding q, or -1."""
    hit = np.nonzero(keys == np.uint32(q))[0]
    return int(hit[0]) if hit.size else -1


def pin_btree_lookup_brute_force(lib):
    """Walking the tree gives the first position holding the query (linear
    scan), or -1: every key list of length <= 5 on a 3-letter alphabet (with
    0xFFFFFFFF, the padding key, as a real key), then trees of 1 to 4 levels
    whose queries include every separator of the inner levels and its
    neighbours."""
    alphabet = [0, 7, BT_PAD]
    queries = np.array(alphabet + [3, 8, 12345], dtype=np.uint32)
    for n in range(0, 6):
        for seq in itertools.product(alphabet, repeat=n):
            keys = np.array(seq, dtype=np.uint32)
            got = oracle.btree_lookup(oracle.btree_build(keys, lib=lib), n, queries, lib=lib)
            want = [_first_position(keys, q) for q in queries.tolist()]
            assert got.tolist() == want, (seq, got, want)
    rng = np.random.default_rng(21)
    for n, span in ((33, 1 << 32), (1024, 50), (1025, 1 << 32), (2000, 700), (32 * 32 * 32 + 5, 1 << 32),
                    (33000, 20000)):
        keys = rng.integers(0, span, n, dtype=np.uint64).astype(np.uint32)
        tree = oracle.btree_build(keys, lib=lib)
        seps = np.concatenate([lv.reshape(-1) for lv in tree[2]]) if tree[2] else np.zeros(0, np.uint32)
        seps = seps[seps != BT_PAD].astype(np.int64)
        near = np.concatenate([seps - 1, seps, seps + 1]) % (1 << 32)
        q = np.concatenate([keys[rng.integers(0, n, 400)], rng.integers(0, 1 << 32, 200, dtype=np.uint64),
                            rng.choice(near, min(near.size, 600), replace=False) if near.size else [],
                            [0, BT_PAD, int(keys.max()), int(keys.max()) + 1, int(keys.min())]])
        q = (np.asarray(q, dtype=np.int64) % (1 << 32)).astype(np.uint32)
        got = oracle.btree_lookup(tree, n, q, lib=lib)
        want = np.array([_first_position(keys, x) for x in q.tolist()], dtype=np.int32)
        assert np.array_equal(got, want), (n, span)


def pin_btree_structure(lib):
    """The stated layout: leaf entries are the (key, rid) pairs sorted by key
    then rid, padded with (0xFFFFFFFF, -1) to whole blocks of 32; each level
    has ceil(nodes below / 32) nodes; an inner entry is the last entry of its
    child, or 0xFFFFFFFF past the last child; the top level is one node."""
    rng = np.random.default_rng(22)
    for n, span in ((0, 10), (1, 10), (31, 5), (32, 1 << 32), (33, 1 << 32), (1025, 300), (40000, 1 << 32)):
        keys = rng.integers(0, span, n, dtype=np.uint64).astype(np.uint32)
        leaf_keys, leaf_rids, levels = oracle.btree_build(keys, lib=lib)
        shape = oracle.btree_shape(n, lib=lib)
        blocks = max(1, -(-n // 32))
        assert shape[0] == blocks and leaf_keys.size == 32 * blocks
        for a, b in zip(shape, shape[1:]):
            assert b == -(-a // 32)
        assert shape[-1] == 1 and len(levels) == len(shape) - 1
        order = np.lexsort((np.arange(n), keys))
        assert np.array_equal(leaf_rids[:n], order.astype(np.int32))
        assert np.array_equal(leaf_keys[:n], keys[order])
        assert np.all(leaf_keys[n:] == BT_PAD) and np.all(leaf_rids[n:] == -1)
        below = leaf_keys.reshape(-1, 32)
        for lv, c in zip(levels, shape[1:]):
            assert lv.shape == (c, 32)
            flat = lv.reshape(-1)
            kids = below.shape[0]
            assert np.array_equal(flat[:kids], below[:, 31])
            assert np.all(flat[kids:] == BT_PAD)
            below = lv


def pin_btree_closed_forms(lib):
    """Distinct keys 3e in shuffled order: the leaves hold 3e in order with the
    position of 3e as rid; the level-1 entry of block c is 3 (32 c + 31); the
    lookup of 3e returns that position and of 3e + 1 returns -1."""
    n = 32 * 32 * 3 + 17
    perm = synth.rids_permutation(n, seed=23)
    keys = (3 * perm).astype(np.uint32)
    leaf_keys, leaf_rids, levels = oracle.btree_build(keys, lib=lib)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    assert np.array_equal(leaf_keys[:n], 3 * np.arange(n, dtype=np.uint32))
    assert np.array_equal(leaf_rids[:n], inv.astype(np.int32))
    full = n // 32
    assert np.array_equal(levels[0].reshape(-1)[:full], 3 * (32 * np.arange(full) + 31).astype(np.uint32))
    tree = (leaf_keys, leaf_rids, levels)
    e = np.arange(n, dtype=np.uint32)
    assert np.array_equal(oracle.btree_lookup(tree, n, 3 * e, lib=lib), inv.astype(np.int32))
    assert np.all(oracle.btree_lookup(tree, n, 3 * e + 1, lib=lib) == -1)


def pin_btree_errors(lib):
    for n in (-1, 1 << 31):
        try:
            oracle.btree_shape(n, lib=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.EINVAL
        else:
            raise AssertionError("bad entry count accepted")


# ---------------------------------------------------------------------------
# foreign-key join over non-dense keys (Sections 4.2.2-4.2.3)
# ---------------------------------------------------------------------------
def _key_join_brute(fact, dim, fk_off, key_off, order):
    fk = fact[:, fk_off:fk_off + 4].copy().view("<u4").reshape(-1)
    dk = dim[:, key_off:key_off + 4].copy().view("<u4").reshape(-1)
    j = [next(r for r in range(dim.shape[0]) if dk[r] == k) for k in fk.tolist()]
    rows = list(range(fact.shape[0]))
    if order == 1:
        rows.sort(key=lambda i: (j[i], i))
    return np.array([np.concatenate([fact[i], dim[j[i]]]) for i in rows], dtype=np.uint8).reshape(
        fact.shape[0], fact.shape[1] + dim.shape[1])


def pin_key_join_brute_force(lib):
    """Each fact row joins the first dimension row holding its key: every
    dimension key list of length <= 4 on a 3-letter alphabet (duplicates
    included) and every fact key list of length <= 3 drawn from it, in both
    orders, against nested loops."""
    alphabet = [3, 9, 0xFFFFFFFF]
    rng = np.random.default_rng(31)
    for nd in range(1, 5):
        for dkeys in itertools.product(alphabet, repeat=nd):
            dim = rng.integers(0, 256, (nd, 12), dtype=np.uint8)
            dim[:, 4:8] = np.array(dkeys, dtype="<u4").view(np.uint8).reshape(nd, 4)
            present = sorted(set(dkeys))
            for nf in range(0, 4):
                for fkeys in itertools.product(present, repeat=nf):
                    fact = rng.integers(0, 256, (nf, 8), dtype=np.uint8)
                    if nf:
                        fact[:, 0:4] = np.array(fkeys, dtype="<u4").view(np.uint8).reshape(nf, 4)
                    for order in (0, 1):
                        got = oracle.key_join(fact, dim, 0, 4, order, lib=lib)
                        assert np.array_equal(got, _key_join_brute(fact, dim, 0, 4, order)), (dkeys, fkeys, order)


def pin_key_join_dense_keys(lib):
    """With dimension keys equal to the row numbers the join is the dense
    foreign-key join of Section 4.2.1, in either order."""
    n_fact, n_dim = 3000, 257
    fact = synth.fact_table(n_fact, n_dim, 0.8, seed=32)
    dim = synth.dim_table(n_dim, seed=33)  # key = row number at byte 0
    assert np.array_equal(oracle.key_join(fact, dim, 0, 0, 0, lib=lib), oracle.fk_join_fact_order(fact, dim, 0))
    assert np.array_equal(oracle.key_join(fact, dim, 0, 0, 1, lib=lib), oracle.fk_join_dim_order(fact, dim, 0))


def pin_key_join_errors(lib):
    fact = np.zeros((2, 8), dtype=np.uint8)
    fact[1, 0] = 5
    dim = np.zeros((3, 8), dtype=np.uint8)  # keys 0, 0, 0: key 5 is missing
    for args, code in (((0, 0, 0), oracle.ERANGE), ((5, 0, 0), oracle.EINVAL), ((0, 6, 0), oracle.EINVAL),
                       ((0, 0, 2), oracle.EINVAL)):
        try:
            oracle.key_join(fact, dim, *args, lib=lib)
        except oracle.OracleError as e:
            assert e.code == code
        else:
            raise AssertionError(f"accepted {args}")


ALL_PINS = [
    pin_retrieve_brute_force, pin_retrieve_closed_forms, pin_retrieve_multiset, pin_retrieve_errors,
    pin_fig2_example, pin_phase_invariants, pin_sort_random, pin_sort_ties,
    pin_join_fact_order, pin_join_dim_order, pin_join_errors,
    pin_hash_lookup_brute_force, pin_hash_lookup_closed_forms, pin_hash_build_invariants, pin_hash_errors,
    pin_smj_brute_force, pin_smj_closed_forms, pin_smj_errors,
    pin_btree_lookup_brute_force, pin_btree_structure, pin_btree_closed_forms, pin_btree_errors,
    pin_key_join_brute_force, pin_key_join_dense_keys, pin_key_join_errors,
]
