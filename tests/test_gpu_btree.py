"""Enhanced B+ tree and batch lookup (Section 4.2.3) on the GPU through the C
ABI: the built tree equals the oracle's tree byte for byte, and every lookup
(direct, and DPG with the LDS and cached probes, several run sizes and both
gathers) equals the oracle's walk of that tree."""
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
    if kind == "top":  # many keys at the padding value 0xFFFFFFFF and just below it
        return (0xFFFFFFFF - rng.integers(0, 3, n, dtype=np.uint64)).astype(np.uint32)
    raise ValueError(kind)


def make_queries(keys, m, seed, hit=0.8):
    rng = np.random.default_rng(seed)
    q = rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
    if keys.size:
        take = rng.random(m) < hit
        q[take] = keys[rng.integers(0, keys.size, int(take.sum()))]
    if m >= 4:  # the extremes
        q[:4] = [0, 0xFFFFFFFF, 0xFFFFFFFE, 1]
    return q


def dev(a: np.ndarray):
    """A uint32 numpy array on the device (as int32: the library reads the bits)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def tree_parts(tree, n):
    """(leaf_keys, leaf_rids, [inner levels]) of a GPU-built tree."""
    lib = dpg.lib()
    b = tree.cpu().numpy()
    levels = lib.dpg_btree_levels(n)
    blocks = max(1, -(-n // 32))
    leaf_keys = b[: 128 * blocks].view(np.uint32)
    r = lib.dpg_btree_rids_offset(n)
    leaf_rids = b[r: r + 128 * blocks].view(np.int32)
    inner, nodes = [], blocks
    for lv in range(1, levels):
        nodes = -(-nodes // 32)
        o = lib.dpg_btree_level_offset(n, lv)
        inner.append(b[o: o + 128 * nodes].view(np.uint32).reshape(nodes, 32))
    return leaf_keys, leaf_rids, inner


BUILD_CASES = [
    # (n_keys, key kind)
    (0, "random"),
    (1, "random"),
    (31, "dups"),
    (32, "random"),
    (33, "random"),
    (1025, "random"),
    (20000, "distinct"),
    (65537, "dups"),
    (3000, "same"),
    (5000, "top"),
    ((1 << 15) + 1, "random"),   # four levels
    (100003, "random"),
]


@pytest.mark.parametrize("case", BUILD_CASES, ids=lambda c: f"n{c[0]}-{c[1]}")
def test_build_matches_oracle(ctx, case):
    n, kind = case
    keys = make_keys(kind, n, seed=n + 3)
    tree = ctx.btree_build(dev(keys))
    torch.cuda.synchronize()
    want_k, want_r, want_inner = oracle.btree_build(keys)
    got_k, got_r, got_inner = tree_parts(tree, n)
    assert np.array_equal(got_k, want_k)
    assert np.array_equal(got_r, want_r)
    assert len(got_inner) == len(want_inner)
    for a, b in zip(got_inner, want_inner):
        assert np.array_equal(a, b)


LOOKUP_VARIANTS = {
    "direct": (dpg.ALGO_DIRECT, {}),
    "dpg": (dpg.ALGO_DPG, {}),
    "dpg-cached-probe": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED)),
    "dpg-cached-gather": (dpg.ALGO_DPG, dict(gather=dpg.GATHER_CACHED)),
    "dpg-small-runs": (dpg.ALGO_DPG, dict(log2_run=10)),      # runs of one level-1 subtree
    "dpg-large-runs": (dpg.ALGO_DPG, dict(log2_run=14)),      # 512 blocks staged per run
    "dpg-huge-runs": (dpg.ALGO_DPG, dict(log2_run=16)),       # beyond LDS: walked through the caches
    "auto": (dpg.ALGO_AUTO, {}),
}

LOOKUP_CASES = [
    # (n_keys, key kind, n_queries)
    (0, "random", 1000),
    (1, "random", 50),
    (1000, "random", 1),
    (5000, "random", 70001),
    (20000, "distinct", 100000),
    (65537, "dups", 50000),
    (3000, "same", 9000),
    (5000, "top", 20000),
    ((1 << 15) + 1, "random", 40000),
    (300007, "random", 300007),
    (4096, "distinct", 0),
]


@pytest.mark.parametrize("variant", sorted(LOOKUP_VARIANTS))
@pytest.mark.parametrize("case", LOOKUP_CASES, ids=lambda c: f"n{c[0]}-{c[1]}-m{c[2]}")
def test_lookup_matches_oracle(ctx, case, variant):
    n, kind, m = case
    algo, opts = LOOKUP_VARIANTS[variant]
    keys = make_keys(kind, n, seed=n + 3)
    queries = make_queries(keys, m, seed=m + 1)
    tree = ctx.btree_build(dev(keys))
    ctx.set_option(dpg.OPT_LOG2_RUN, opts.get("log2_run", 0))
    ctx.set_option(dpg.OPT_GATHER, opts.get("gather", 0))
    ctx.set_option(dpg.OPT_PROBE, opts.get("probe", 0))
    try:
        got = ctx.btree_lookup(tree, n, dev(queries), algo=algo)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(dpg.OPT_LOG2_RUN, 0)
        ctx.set_option(dpg.OPT_GATHER, 0)
        ctx.set_option(dpg.OPT_PROBE, 0)
    want = oracle.btree_lookup(oracle.btree_build(keys), n, queries)
    assert np.array_equal(got.cpu().numpy(), want)


def test_lookup_full_size(ctx):
    """2^26 distinct keys and 2^26 queries (80 % stored) in the benchmark's
    configuration: every stored query returns the rid holding it and every
    other query returns -1, which fixes each answer."""
    n, m = 1 << 26, 1 << 26
    keys_d = 2 * synth.rids_permutation(1 << 27, 91, backend="torch", device=DEV)[:n].to(torch.int64) + 1
    keys_d = (keys_d - (keys_d >= (1 << 31)).to(torch.int64) * (1 << 32)).to(torch.int32)  # odd, distinct
    tree = ctx.btree_build(keys_d)
    g = torch.Generator(device=DEV).manual_seed(9)
    pick = torch.randint(0, n, (m,), device=DEV, generator=g)
    queries = keys_d[pick].clone()
    miss = torch.rand(m, device=DEV, generator=g) >= 0.8
    queries[miss] = 2 * torch.randint(0, 1 << 30, (int(miss.sum()),), device=DEV, generator=g).to(torch.int32)
    for algo, probe in ((dpg.ALGO_DIRECT, 0), (dpg.ALGO_DPG, 0), (dpg.ALGO_DPG, dpg.PROBE_CACHED)):
        ctx.set_option(dpg.OPT_PROBE, probe)
        try:
            got = ctx.btree_lookup(tree, n, queries, algo=algo)
            torch.cuda.synchronize()
        finally:
            ctx.set_option(dpg.OPT_PROBE, 0)
        assert torch.equal(got[miss], torch.full_like(got[miss], -1))
        assert torch.equal(got[~miss].to(torch.int64), pick[~miss])
    del tree, keys_d, queries, pick, miss
    torch.cuda.empty_cache()
