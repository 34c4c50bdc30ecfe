"""Hash index and batch lookup (Section 4.2.3) on the GPU through the C ABI:
the built index equals the oracle's build byte for byte, and every lookup
(direct, and DPG with either gather form and several partition sizes)
equals the oracle's batch lookup."""
import numpy as np
import pytest
import torch

import oracle
from paper_cs_0308004_amd import dpg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = dpg.Context(0)
    yield c
    c.close()


def make_keys(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "distinct":  # odd, pairwise distinct
        return (2 * synth.rids_permutation(max(n, 1) * 2, seed)[:n].astype(np.uint64) + 1).astype(np.uint32)
    if kind == "random":
        return rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    if kind == "dups":  # few distinct values, many duplicates
        return rng.integers(0, max(1, n // 8), n, dtype=np.uint64).astype(np.uint32)
    if kind == "same":
        return np.full(n, 12345, dtype=np.uint32)
    raise ValueError(kind)


def make_queries(keys, m, seed, hit=0.8):
    rng = np.random.default_rng(seed)
    if keys.size == 0:
        return rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
    q = keys[rng.integers(0, keys.size, m)]
    miss = rng.random(m) >= hit
    q[miss] = rng.integers(0, 1 << 32, int(miss.sum()), dtype=np.uint64).astype(np.uint32)
    return q


def dev(a: np.ndarray):
    """A uint32 numpy array on the device (as int32: the library reads the bits)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def index_parts(index, n, s):
    """(slots (S, 2), ov_off (S + 1), ov (n_ov, 2)) of a GPU-built index."""
    b = index.cpu().numpy()
    S = 1 << s
    slots = b[: 8 * S].view(np.uint32).reshape(S, 2)
    o = dpg.lib().dpg_hash_ov_off_offset(s)
    ov_off = b[o: o + 4 * (S + 1)].view(np.int32).astype(np.int64)
    v = dpg.lib().dpg_hash_ov_offset(s)
    ov = b[v: v + 8 * int(ov_off[S])].view(np.uint32).reshape(-1, 2)
    return slots, ov_off, ov


BUILD_CASES = [
    # (n_keys, log2_slots, key kind)
    (0, 4, "random"),
    (1, 4, "random"),
    (1000, 10, "random"),
    (5000, 10, "random"),      # load 4.9: most pairs overflow
    (20000, 16, "distinct"),
    (65537, 17, "dups"),
    (3000, 12, "same"),        # every key in one home
    (100003, 18, "random"),
]


@pytest.mark.parametrize("case", BUILD_CASES, ids=lambda c: f"n{c[0]}-s{c[1]}-{c[2]}")
def test_build_matches_oracle(ctx, case):
    n, s, kind = case
    keys = make_keys(kind, n, seed=n + s)
    index = ctx.hash_build(dev(keys), s)
    torch.cuda.synchronize()
    want_slots, want_off, want_ov = oracle.hash_build(keys, s)
    slots, ov_off, ov = index_parts(index, n, s)
    assert np.array_equal(slots, want_slots)
    assert np.array_equal(ov_off, want_off)
    assert np.array_equal(ov, want_ov)
    # a second build holds the same index
    again = index_parts(ctx.hash_build(dev(keys), s), n, s)
    for a, b in zip((slots, ov_off, ov), again):
        assert np.array_equal(a, b)


LOOKUP_VARIANTS = {
    "direct": (dpg.ALGO_DIRECT, {}),
    "dpg": (dpg.ALGO_DPG, {}),
    "dpg-cached-gather": (dpg.ALGO_DPG, dict(gather=dpg.GATHER_CACHED)),
    "dpg-cached-probe": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED)),
    "dpg-cached-probe-and-gather": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, gather=dpg.GATHER_CACHED)),
    "dpg-small-partitions": (dpg.ALGO_DPG, dict(log2_run=6)),     # many (wide-partition) runs
    "dpg-one-partition": (dpg.ALGO_DPG, dict(log2_run=30)),        # the minimum of two runs
    "auto": (dpg.ALGO_AUTO, {}),
}

LOOKUP_CASES = [
    # (n_keys, log2_slots, key kind, n_queries)
    (0, 4, "random", 1000),
    (1000, 10, "random", 1),
    (5000, 10, "random", 70001),
    (20000, 16, "distinct", 100000),
    (65537, 17, "dups", 50000),
    (3000, 12, "same", 9000),
    (100003, 18, "random", 300007),
    (4096, 12, "distinct", 0),
]


@pytest.mark.parametrize("variant", sorted(LOOKUP_VARIANTS))
@pytest.mark.parametrize("case", LOOKUP_CASES, ids=lambda c: f"n{c[0]}-s{c[1]}-{c[2]}-m{c[3]}")
def test_lookup_matches_oracle(ctx, case, variant):
    n, s, kind, m = case
    algo, opts = LOOKUP_VARIANTS[variant]
    keys = make_keys(kind, n, seed=n + s)
    queries = make_queries(keys, m, seed=m + 1)
    index = ctx.hash_build(dev(keys), s)
    ctx.set_option(dpg.OPT_LOG2_RUN, opts.get("log2_run", 0))
    ctx.set_option(dpg.OPT_GATHER, opts.get("gather", 0))
    ctx.set_option(dpg.OPT_PROBE, opts.get("probe", 0))
    try:
        got = ctx.hash_lookup(index, n, s, dev(queries), algo=algo)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(dpg.OPT_LOG2_RUN, 0)
        ctx.set_option(dpg.OPT_GATHER, 0)
        ctx.set_option(dpg.OPT_PROBE, 0)
    want = oracle.hash_lookup(keys, queries)
    assert np.array_equal(got.cpu().numpy(), want)


def test_lookup_full_size_sampled(ctx):
    """2^24 distinct keys in 2^25 slots, 2^26 queries (80 % hits) in the
    benchmark's configuration: every hit returns the rid holding its key,
    misses return -1, and a sample equals the oracle."""
    n, s, m = 1 << 24, 25, 1 << 26
    # odd, pairwise distinct keys (bit patterns of int32)
    keys_d = (2 * synth.rids_permutation(1 << 25, 77, backend="torch", device=DEV)[:n].to(torch.int64) + 1)
    keys_d = (keys_d - (keys_d >= (1 << 31)).to(torch.int64) * (1 << 32)).to(torch.int32)
    index = ctx.hash_build(keys_d, s)
    g = torch.Generator(device=DEV).manual_seed(5)
    pick = torch.randint(0, n, (m,), device=DEV, generator=g)
    queries = keys_d[pick].clone()
    miss = torch.rand(m, device=DEV, generator=g) >= 0.8
    queries[miss] = 2 * torch.randint(0, 1 << 30, (int(miss.sum()),), device=DEV, generator=g).to(torch.int32)
    for algo, probe in ((dpg.ALGO_DIRECT, 0), (dpg.ALGO_DPG, dpg.PROBE_CACHED), (dpg.ALGO_DPG, 0)):
        ctx.set_option(dpg.OPT_PROBE, probe)
        try:
            got = ctx.hash_lookup(index, n, s, queries, algo=algo)
            torch.cuda.synchronize()
        finally:
            ctx.set_option(dpg.OPT_PROBE, 0)
        assert torch.equal(got[miss], torch.full_like(got[miss], -1))
        hit = ~miss
        assert torch.equal(got[hit].to(torch.int64), pick[hit])
    sample = np.random.default_rng(1).integers(0, m, 4096)
    want = oracle.hash_lookup(keys_d.cpu().numpy().view(np.uint32), queries.cpu().numpy().view(np.uint32)[sample])
    assert np.array_equal(got.cpu().numpy()[sample], want)
