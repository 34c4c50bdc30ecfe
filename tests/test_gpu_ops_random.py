"""Seeded random joins and batch lookups against the oracle: table sizes,
row widths, key positions, key distributions (distinct, duplicated, narrow,
full 32-bit), index sizes and forced plan options drawn at random."""
import random

import numpy as np
import pytest
import torch

import oracle
from paper_cs_0308004_amd import dpg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

OPTS = [{}, {dpg.OPT_PROBE: dpg.PROBE_CACHED}, {dpg.OPT_PROBE: dpg.PROBE_LDS}, {dpg.OPT_GATHER: dpg.GATHER_CACHED},
        {dpg.OPT_GATHER: dpg.GATHER_LDS}, {dpg.OPT_LOG2_RUN: 4}, {dpg.OPT_LOG2_RUN: 10},
        {dpg.OPT_DISTRIBUTE: dpg.DIST_SAMPLED}, {dpg.OPT_DISTRIBUTE: dpg.DIST_TWO_PASS}]


@pytest.fixture(scope="module")
def ctx():
    c = dpg.Context(0)
    yield c
    c.close()


def configure(ctx, opts):
    for k in (dpg.OPT_PROBE, dpg.OPT_GATHER, dpg.OPT_LOG2_RUN, dpg.OPT_DISTRIBUTE):
        ctx.set_option(k, opts.get(k, 0))


def dev_u32(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def random_keys(rng: random.Random, np_rng, n: int) -> np.ndarray:
    kind = rng.choice(["full", "narrow", "dups", "distinct", "top"])
    if kind == "full":
        return np_rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    if kind == "narrow":  # keys of few bits: the splitters span a small range
        return np_rng.integers(0, max(2, n // 3), n, dtype=np.uint64).astype(np.uint32)
    if kind == "dups":
        return (np_rng.integers(0, max(1, n // 16), n, dtype=np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32)
    if kind == "distinct":
        return (2 * np_rng.permutation(2 * max(n, 1))[:n].astype(np.uint64) + 1).astype(np.uint32)
    return (0xFFFFFFFF - np_rng.integers(0, 5, n, dtype=np.uint64)).astype(np.uint32)


def random_queries(rng, np_rng, keys: np.ndarray, m: int) -> np.ndarray:
    q = np_rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
    if keys.size:
        take = np_rng.random(m) < rng.choice([0.0, 0.5, 0.9])
        q[take] = keys[np_rng.integers(0, keys.size, int(take.sum()))]
    return q


@pytest.mark.parametrize("case", range(40))
def test_random_join_matches_oracle(ctx, case):
    rng = random.Random(0x51 + case)
    np_rng = np.random.default_rng(0x51 + case)
    n_fact = rng.choice([1, 97, 5000, 40001, 120000])
    n_dim = rng.choice([1, 13, 4096, 70001])
    fb = rng.choice([4, 8, 16, 20, 32])
    db = rng.choice([4, 16, 36, 64, 100])
    fk_off = 4 * rng.randrange(fb // 4)
    fact = np_rng.integers(0, 256, (n_fact, fb), dtype=np.uint8)
    s = rng.choice([0.0, 0.8, 1.2])
    fk = synth.zipf_fk_at(n_dim, s, np.arange(n_fact, dtype=np.uint64), 0x51 + case) if s else \
        np_rng.integers(0, n_dim, n_fact)
    fact[:, fk_off:fk_off + 4] = np.asarray(fk, dtype=np.uint32).view(np.uint8).reshape(-1, 4)
    dim = np_rng.integers(0, 256, (n_dim, db), dtype=np.uint8)
    order = rng.choice([dpg.JOIN_FACT_ORDER, dpg.JOIN_DIM_ORDER])
    fn = oracle.fk_join_fact_order if order == dpg.JOIN_FACT_ORDER else oracle.fk_join_dim_order
    want = fn(fact, dim, fk_off)
    opts = rng.choice(OPTS)
    configure(ctx, opts)
    try:
        for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
            got = ctx.fk_join(torch.from_numpy(fact).to(DEV), torch.from_numpy(dim).to(DEV), fk_off, order, algo=algo)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (case, n_fact, n_dim, fb, db, fk_off, order, opts, algo)
    finally:
        configure(ctx, {})


@pytest.mark.parametrize("case", range(40))
def test_random_hash_lookup_matches_oracle(ctx, case):
    rng = random.Random(0x61 + case)
    np_rng = np.random.default_rng(0x61 + case)
    n = rng.choice([1, 50, 3000, 65536, 200003])
    keys = random_keys(rng, np_rng, n)
    s = max(4, int(np.ceil(np.log2(max(n, 1)))) + rng.choice([-1, 0, 1, 2]))
    queries = random_queries(rng, np_rng, keys, rng.choice([1, 777, 50000, 300001]))
    want = oracle.hash_lookup(keys, queries)
    index = ctx.hash_build(dev_u32(keys), s)
    opts = rng.choice([{}, {dpg.OPT_PROBE: dpg.PROBE_CACHED}, {dpg.OPT_GATHER: dpg.GATHER_CACHED},
                       {dpg.OPT_LOG2_RUN: rng.choice([4, 8, 12])}])
    configure(ctx, opts)
    try:
        for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
            got = ctx.hash_lookup(index, n, s, dev_u32(queries), algo=algo)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (case, n, s, opts, algo)
    finally:
        configure(ctx, {})


@pytest.mark.parametrize("case", range(40))
def test_random_btree_lookup_matches_oracle(ctx, case):
    rng = random.Random(0x71 + case)
    np_rng = np.random.default_rng(0x71 + case)
    n = rng.choice([1, 31, 33, 1025, 40000, 300007])
    keys = random_keys(rng, np_rng, n)
    queries = random_queries(rng, np_rng, keys, rng.choice([1, 999, 60000, 250001]))
    want = oracle.btree_lookup(oracle.btree_build(keys), n, queries)
    tree = ctx.btree_build(dev_u32(keys))
    opts = rng.choice([{}, {dpg.OPT_PROBE: dpg.PROBE_CACHED}, {dpg.OPT_GATHER: dpg.GATHER_CACHED},
                       {dpg.OPT_LOG2_RUN: rng.choice([10, 12, 14, 16])}])
    configure(ctx, opts)
    try:
        for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
            got = ctx.btree_lookup(tree, n, dev_u32(queries), algo=algo)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (case, n, opts, algo)
    finally:
        configure(ctx, {})
