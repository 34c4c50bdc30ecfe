"""Every byte of the full-size results against the CPU oracle.

The workloads are the benchmark's, in the launch configurations it times:
retrieval of 2^23 and 2^26 records of 100 B by a permutation (the shapes that
take the nontemporal-store copy kernels and the partition tiles of 16 rids
per thread), the key-pointer sort of 10^6, 10^7 and 10^8 records of 100 B
(Section 3), a sort whose key prefixes repeat in long groups (the full-key
passes), and both foreign-key joins of 2^28 fact rows with 2^24 dimension rows
under Zipf(1.2) keys (Section 4.2.1).  Results above a few GB are compared in
chunks (tests/fullsize.py); the expected bytes of every chunk come from the
oracle run on that chunk's inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_cs_0308004_amd import dpg, synth
from tests.fullsize import compare_chunks, groups_by_small_key, note

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = dpg.Context(0)
    yield c
    c.close()


def free_device():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Retrieval (Section 2)
# ---------------------------------------------------------------------------
# (algorithm, Phase I flavour, expected distribute tile): the default
# partition pass, splitter runs from a sample, the two-pass distribute and its
# LDS probe, and direct retrieval
# (2048 runs: log2 of the run length forced to 12)
P23_VARIANTS = {
    "dpg": (dpg.ALGO_DPG, 0, 0, 0, 16384),
    "dpg-2048-runs": (dpg.ALGO_DPG, 0, 0, 12, 32768),
    "dpg-sampled": (dpg.ALGO_DPG, dpg.DIST_SAMPLED, 0, 0, 16384),
    "dpg-sampled-2048-runs": (dpg.ALGO_DPG, dpg.DIST_SAMPLED, 0, 12, 16384),
    "dpg-two-pass": (dpg.ALGO_DPG, dpg.DIST_TWO_PASS, 0, 0, None),
    "dpg-two-pass-lds": (dpg.ALGO_DPG, dpg.DIST_TWO_PASS, dpg.PROBE_LDS, 0, None),
    "direct": (dpg.ALGO_DIRECT, 0, 0, 0, None),
}


@pytest.mark.parametrize("variant", list(P23_VARIANTS))
def test_retrieve_2p23x100B_full_oracle(ctx, variant):
    """2^23 records of 100 B, a permutation: 839 MB of output (nontemporal
    stores) and, for the one-pass DPG distribute, partition tiles of 16384
    rids (16 per thread); every Phase I flavour at this size."""
    algo, dist, probe, log2_run, tile = P23_VARIANTS[variant]
    n, rec = 1 << 23, 100
    seed = synth.SEED_BASE + 23
    src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
    rids = synth.rids_permutation(n, seed, backend="torch", device=DEV)
    ctx.set_option(dpg.OPT_DISTRIBUTE, dist)
    ctx.set_option(dpg.OPT_PROBE, probe)
    ctx.set_option(dpg.OPT_LOG2_RUN, log2_run)
    try:
        plan = ctx.plan_retrieve(n, rec, n, algo)
        if tile is not None:
            assert plan.dist_tile == tile
        if dist:
            assert plan.distribute == dist
        if log2_run:
            assert plan.n_runs == 2048
        out = ctx.retrieve(src, rids, algo=algo)
        torch.cuda.synchronize()
    finally:
        for opt in (dpg.OPT_DISTRIBUTE, dpg.OPT_PROBE, dpg.OPT_LOG2_RUN):
            ctx.set_option(opt, 0)
    src_h, rids_h = src.cpu().numpy(), rids.cpu().numpy()
    assert np.array_equal(rids_h[:1000], synth.rids_permutation(n, seed, count=1000))
    got = out.cpu().numpy()
    want = oracle.retrieve(src_h, rids_h)
    assert np.array_equal(got, want)
    del src, rids, out
    free_device()


@pytest.mark.parametrize("algo", [dpg.ALGO_DPG, dpg.ALGO_DIRECT], ids=["dpg", "direct"])
def test_retrieve_2p26x100B_headline_full_oracle(ctx, algo):
    """The headline workload: 2^26 records of 100 B, a permutation of 2^26
    rids, the default plan (for DPG: 2048 runs, partition tiles of 32768
    rids).  All 6.7 GB of output against the oracle, in chunks of 2^22
    rids."""
    n, rec = 1 << 26, 100
    seed = synth.SEED_BASE + 1
    if algo == dpg.ALGO_DPG:
        plan = ctx.plan_retrieve(n, rec, n, algo)
        assert (plan.n_runs, plan.dist_tile, plan.distribute) == (2048, 32768, dpg.DIST_PARTITION)
    src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
    rids = synth.rids_permutation(n, seed, backend="torch", device=DEV)
    rids_h = rids.cpu().numpy()
    assert np.array_equal(rids_h[:1000], synth.rids_permutation(n, seed, count=1000))
    out = ctx.retrieve(src, rids, algo=algo)
    src_h = src.cpu().numpy()
    del src
    step = 1 << 22
    chunks = [(a, min(n, a + step)) for a in range(0, n, step)]
    compare_chunks(f"retrieve 2^26 x 100 B algo {algo}", chunks,
                   fetch=lambda c: out[c[0]:c[1]].cpu().numpy(),
                   expect=lambda c: oracle.retrieve(src_h, rids_h[c[0]:c[1]]))
    del rids, out
    free_device()


def test_retrieve_2p26x100B_two_pass_lds_probe_full_oracle(ctx):
    """The headline workload with every source run staged in LDS for the
    probe (Section 2.1's Phase II as stated): 2^17 runs of 512 records from
    two partition passes.  All 6.7 GB of output against the oracle."""
    n, rec = 1 << 26, 100
    seed = synth.SEED_BASE + 1
    for opt, v in ((dpg.OPT_DISTRIBUTE, dpg.DIST_TWO_PASS), (dpg.OPT_PROBE, dpg.PROBE_LDS)):
        ctx.set_option(opt, v)
    try:
        plan = ctx.plan_retrieve(n, rec, n, dpg.ALGO_DPG)
        assert (plan.probe, plan.n_runs) == (dpg.PROBE_LDS, 1 << 17)
        src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
        rids = synth.rids_permutation(n, seed, backend="torch", device=DEV)
        out = ctx.retrieve(src, rids, algo=dpg.ALGO_DPG)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(dpg.OPT_DISTRIBUTE, 0)
        ctx.set_option(dpg.OPT_PROBE, 0)
    rids_h = rids.cpu().numpy()
    src_h = src.cpu().numpy()
    del src
    step = 1 << 22
    chunks = [(a, min(n, a + step)) for a in range(0, n, step)]
    compare_chunks("retrieve 2^26 x 100 B, two-pass LDS probe", chunks,
                   fetch=lambda c: out[c[0]:c[1]].cpu().numpy(),
                   expect=lambda c: oracle.retrieve(src_h, rids_h[c[0]:c[1]]))
    del rids, out
    free_device()


# ---------------------------------------------------------------------------
# Key-pointer sort (Section 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1_000_000, 10_000_000], ids=["1e6", "1e7"])
def test_sort_full_oracle(ctx, n):
    """10^6 and 10^7 records of 100 B with 10-byte uniform keys, both copy
    phases: records and permutation against the oracle."""
    rec = 100
    seed = synth.SEED_BASE + 2
    src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
    src_h = src.cpu().numpy()
    want_dst, want_perm = oracle.sort_records(src_h, 0, 10)
    for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
        dst, perm = ctx.sort_records(src, 0, 10, algo=algo)
        assert np.array_equal(perm.cpu().numpy().astype(np.int64), want_perm), f"perm, algo {algo}"
        assert np.array_equal(dst.cpu().numpy(), want_dst), f"records, algo {algo}"
        del dst, perm
    del src
    free_device()


def test_sort_full_key_passes(ctx):
    """Keys whose first four bytes take only 1500 values: groups of equal
    prefixes hold about 1300 records, beyond the fix-up's limit of 64, so the
    pairs are sorted over the whole 10-byte key instead -- decided on the
    device, without a host synchronization.  2 * 10^6 records of 100 B
    against the oracle; the fix-up's flag (the first word of the workspace)
    shows that the full-key passes ran, and that uniform keys skip them."""
    n, rec = 2_000_000, 100
    seed = synth.SEED_BASE + 92
    src_h = synth.record_bytes(n, rec, seed)
    pool = synth.record_bytes(1500, 4, seed, stream=synth.STREAM_MIX)
    src_h[:, 0:4] = pool[synth.uniform_at(1500, np.arange(n, dtype=np.uint64), seed, synth.STREAM_FK)]
    want_dst, want_perm = oracle.sort_records(src_h, 0, 10)
    src = torch.from_numpy(src_h).to(DEV)
    uniform = torch.from_numpy(synth.record_bytes(n, rec, seed)).to(DEV)
    for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
        ws = torch.empty(ctx.sort_workspace_bytes(n, rec, 0, 10, algo), dtype=torch.uint8, device=DEV)
        dst, perm = ctx.sort_records(src, 0, 10, algo=algo, workspace=ws)
        assert int(ws[:4].view(torch.int32).item()) == 1
        assert np.array_equal(perm.cpu().numpy().astype(np.int64), want_perm), f"perm, algo {algo}"
        assert np.array_equal(dst.cpu().numpy(), want_dst), f"records, algo {algo}"
        ctx.sort_records(uniform, 0, 10, algo=algo, workspace=ws)
        assert int(ws[:4].view(torch.int32).item()) == 0
        del dst, perm, ws
    del src, uniform
    free_device()


def test_sort_1e8x100B_full_oracle(ctx):
    """The benchmark's sort: 10^8 records of 100 B, 10-byte uniform keys, with
    the DPG and the direct copy phase.  The records are cut by their first key
    byte into 64 groups of 4 values; a group's records occupy one contiguous
    range of the sorted output, and the oracle sorts each group on its own
    (equal keys share their first byte, and a group lists its records in
    index order, so its tie order is the global one)."""
    n, rec = 100_000_000, 100
    seed = synth.SEED_BASE + 2
    src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
    outs = []
    for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
        dst, perm = ctx.sort_records(src, 0, 10, algo=algo)
        outs.append((dst, perm))
    src_h = src.cpu().numpy()
    del src
    order, starts = groups_by_small_key(src_h[:, 0] >> 2, 64)

    def fetch(g):
        a, b = int(starts[g]), int(starts[g + 1])
        parts = []
        for dst, perm in outs:
            parts += [dst[a:b].cpu().numpy(), perm[a:b].cpu().numpy().astype(np.int64)]
        return tuple(parts)

    def expect(g):
        sel = order[starts[g]:starts[g + 1]]
        d, p = oracle.sort_records(src_h[sel], 0, 10)
        return (d, sel[p]) * len(outs)

    compare_chunks("sort 10^8 x 100 B (dpg, direct)", range(64), fetch, expect)
    del outs
    free_device()


def test_sort_1e8x100B_full_key_passes_full_oracle(ctx):
    """The benchmark's tied-prefix sort: the same 10^8 records of 100 B with
    key bytes 0-3 drawn from 4096 values, so that groups of about 24,000
    equal prefixes send the pairs through the full-key passes (the flag in
    the workspace's first word shows it).  Both copy phases, every byte,
    compared with the oracle group by group as above."""
    n, rec = 100_000_000, 100
    seed = synth.SEED_BASE + 2
    src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
    pool = synth.record_bytes(4096, 4, seed, stream=synth.STREAM_MIX, backend="torch", device=DEV)
    pick = synth.uniform_at(4096, torch.arange(n, device=DEV), seed, synth.STREAM_FK, backend="torch", device=DEV)
    src[:, 0:4] = pool[pick]
    del pool, pick
    outs = []
    for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
        ws = torch.empty(ctx.sort_workspace_bytes(n, rec, 0, 10, algo), dtype=torch.uint8, device=DEV)
        dst, perm = ctx.sort_records(src, 0, 10, algo=algo, workspace=ws)
        assert int(ws[:4].view(torch.int32).item()) == 1, "the full-key passes did not run"
        outs.append((dst, perm))
        del ws
    src_h = src.cpu().numpy()
    del src
    order, starts = groups_by_small_key(src_h[:, 0] >> 2, 64)

    def fetch(g):
        a, b = int(starts[g]), int(starts[g + 1])
        parts = []
        for dst, perm in outs:
            parts += [dst[a:b].cpu().numpy(), perm[a:b].cpu().numpy().astype(np.int64)]
        return tuple(parts)

    def expect(g):
        sel = order[starts[g]:starts[g + 1]]
        d, p = oracle.sort_records(src_h[sel], 0, 10)
        return (d, sel[p]) * len(outs)

    compare_chunks("sort 10^8 x 100 B, tied prefixes (dpg, direct)", range(64), fetch, expect)
    del outs
    free_device()


# ---------------------------------------------------------------------------
# Foreign-key joins (Section 4.2.1)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def join_tables():
    """The benchmark's join inputs: dimension 2^24 x 64 B, fact 2^28 x 16 B
    with Zipf(1.2) foreign keys, on the device and on the host."""
    n_dim, n_fact, s = 1 << 24, 1 << 28, 1.2
    seed = synth.SEED_BASE + 3
    fact = synth.fact_table(n_fact, n_dim, s, seed, backend="torch", device=DEV)
    dim = synth.dim_table(n_dim, seed, backend="torch", device=DEV)
    fact_h, dim_h = fact.cpu().numpy(), dim.cpu().numpy()
    idx = np.arange(0, n_fact, 999_983, dtype=np.uint64)
    assert np.array_equal(fact_h[idx.astype(np.int64), 0:4].view(np.uint32).reshape(-1),
                          synth.zipf_fk_at(n_dim, s, idx, seed).astype(np.uint32))
    yield fact, dim, fact_h, dim_h
    del fact, dim
    free_device()


def test_join_fact_order_2p28_full_oracle(ctx, join_tables):
    """DPG-Move join (fact order), moved rows retrieved by DPG and directly:
    all 2^28 joined rows of 80 B against the oracle, in chunks of 2^24 fact
    rows."""
    fact, dim, fact_h, dim_h = join_tables
    n_fact = fact.shape[0]
    outs = [ctx.fk_join(fact, dim, 0, dpg.JOIN_FACT_ORDER, algo=a) for a in (dpg.ALGO_DPG, dpg.ALGO_DIRECT)]
    step = 1 << 24
    chunks = [(a, min(n_fact, a + step)) for a in range(0, n_fact, step)]
    compare_chunks("fact-order join 2^28", chunks,
                   fetch=lambda c: tuple(o[c[0]:c[1]].cpu().numpy() for o in outs),
                   expect=lambda c: (oracle.fk_join_fact_order(fact_h[c[0]:c[1]], dim_h, 0),) * len(outs))
    del outs
    free_device()


def test_join_dim_order_2p28_full_oracle(ctx, join_tables):
    """DPG-Sort join (foreign-key order, equal keys in fact order), fact rows
    moved by DPG and directly: all 2^28 joined rows against the oracle.  The
    fact rows are cut into 256 groups by the top 8 bits of their 24-bit key;
    a group's rows occupy one contiguous range of the output, and the oracle
    joins each group on its own (its rows listed in fact order)."""
    fact, dim, fact_h, dim_h = join_tables
    outs = [ctx.fk_join(fact, dim, 0, dpg.JOIN_DIM_ORDER, algo=a) for a in (dpg.ALGO_DPG, dpg.ALGO_DIRECT)]
    fk = fact_h[:, 0:4].copy().view(np.uint32).reshape(-1)
    order, starts = groups_by_small_key((fk >> 16).astype(np.uint8), 256)
    del fk
    note(f"dim-order join: largest key group {int(np.diff(starts).max())} rows")
    compare_chunks("dim-order join 2^28", range(256),
                   fetch=lambda g: tuple(o[int(starts[g]):int(starts[g + 1])].cpu().numpy() for o in outs),
                   expect=lambda g: (oracle.fk_join_dim_order(fact_h[order[starts[g]:starts[g + 1]]], dim_h, 0),)
                   * len(outs))
    del outs
    free_device()


# ---------------------------------------------------------------------------
# The record-size and rid-pattern sweep at its full size (2^26 records)
# ---------------------------------------------------------------------------
SWEEP = [(r, "perm") for r in (4, 8, 16, 32, 64, 128, 256)] + \
        [(r, p) for r in (16, 100, 256) for p in ("uniform", "blocked")]


@pytest.mark.parametrize("rec,pattern", SWEEP, ids=[f"{r}B-{p}" for r, p in SWEEP])
def test_retrieve_2p26_sweep_full_oracle(ctx, rec, pattern):
    """2^26 source records of R bytes, 2^26 rids (a permutation, uniform draws
    with repeats, or shuffled 4 KB runs), the default DPG plan for that shape:
    every output byte against the oracle, in chunks of 2^22 rids."""
    n = 1 << 26
    seed = synth.SEED_BASE + 5 + rec
    src = synth.record_bytes(n, rec, seed, backend="torch", device=DEV)
    if pattern == "perm":
        rids = synth.rids_permutation(n, seed, backend="torch", device=DEV)
    elif pattern == "uniform":
        rids = synth.rids_uniform(n, n, seed, backend="torch", device=DEV)
    else:
        rids = synth.rids_blocked(n, rec, seed, backend="torch", device=DEV)
    out = ctx.retrieve(src, rids, algo=dpg.ALGO_DPG)
    rids_h = rids.cpu().numpy()
    src_h = src.cpu().numpy()
    del src
    step = 1 << 22
    chunks = [(a, min(n, a + step)) for a in range(0, n, step)]
    compare_chunks(f"retrieve 2^26 x {rec} B {pattern}", chunks,
                   fetch=lambda c: out[c[0]:c[1]].cpu().numpy(),
                   expect=lambda c: oracle.retrieve(src_h, rids_h[c[0]:c[1]]))
    del rids, out
    free_device()
