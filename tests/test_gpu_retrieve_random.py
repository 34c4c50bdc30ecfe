"""Seeded random retrievals against the oracle (200 cases): record sizes, source and list
lengths, rid patterns, source alignment and forced plan options drawn at
random, so that combinations no hand-written case names are covered too
(every Phase I / II / III form, tile counts around the partition tile,
runs of a few records, sources 4 bytes past an aligned address)."""
import random

import numpy as np
import pytest
import torch

import oracle
from paper_cs_0308004_amd import dpg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

OPTS = [
    {}, {"probe": dpg.PROBE_CACHED}, {"probe": dpg.PROBE_LDS}, {"gather": dpg.GATHER_LDS},
    {"gather": dpg.GATHER_CACHED}, {"gather": dpg.GATHER_NONE}, {"dist": dpg.DIST_SAMPLED},
    {"dist": dpg.DIST_TWO_PASS}, {"dist": dpg.DIST_APPEND}, {"log2_run": 3},
    {"log2_run": 6, "gather": dpg.GATHER_LDS}, {"log2_run": 9}, {"dist": dpg.DIST_SAMPLED, "log2_run": 4},
    {"probe": dpg.PROBE_LDS, "log2_run": 5},
]
OPT_IDS = {"probe": dpg.OPT_PROBE, "gather": dpg.OPT_GATHER, "dist": dpg.OPT_DISTRIBUTE, "log2_run": dpg.OPT_LOG2_RUN}


def draw(case):
    """One case's shape, rids and options, from its own seed."""
    rng = random.Random(0x0308004 + case)
    R = rng.choice([4, 8, 12, 16, 20, 32, 64, 100, 128, 256])
    n_src = rng.choice([1, 2, 7, 100, 1000, 4099, 65537, 300001])
    n_rids = rng.choice([1, 5, 64, 1000, 8191, 8192, 8193, 16385, 100003])
    kind = rng.choice(["perm", "uniform", "same", "skewed", "sorted"])
    seed = synth.SEED_BASE + 1000 + case
    np_rng = np.random.default_rng(seed)
    if kind == "perm" and n_rids <= n_src:
        rids = synth.rids_permutation(n_src, seed)[:n_rids]
    elif kind == "same":
        rids = np.full(n_rids, rng.randrange(n_src), dtype=np.int32)
    elif kind == "skewed":  # most rids among the first records
        rids = np.minimum((n_src * np_rng.random(n_rids) ** 4).astype(np.int64), n_src - 1).astype(np.int32)
    elif kind == "sorted":
        rids = np.sort(synth.rids_uniform(n_src, n_rids, seed))
    else:
        rids = synth.rids_uniform(n_src, n_rids, seed)
    src = synth.record_bytes(n_src, R, seed)
    return R, src, np.ascontiguousarray(rids, dtype=np.int32), rng.choice(OPTS), rng.choice([0, 0, 0, 4])


@pytest.fixture(scope="module")
def ctx():
    c = dpg.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", range(200))
def test_random_retrieval_matches_oracle(ctx, case):
    R, src_np, rids_np, opts, offset = draw(case)
    want = oracle.retrieve(src_np, rids_np)
    n_src = src_np.shape[0]
    if offset:  # the source 4 bytes past an aligned address
        base = torch.empty(n_src * R + 16, dtype=torch.uint8, device=DEV)
        src = base[offset: offset + n_src * R].view(n_src, R)
        src.copy_(torch.from_numpy(src_np))
    else:
        src = torch.from_numpy(src_np).to(DEV)
    rids = torch.from_numpy(rids_np).to(DEV)
    for k, v in opts.items():
        ctx.set_option(OPT_IDS[k], v)
    try:
        for algo in (dpg.ALGO_DPG, dpg.ALGO_AUTO):
            got = ctx.retrieve(src, rids, algo=algo)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (case, R, n_src, rids_np.size, opts, offset, algo)
    finally:
        for k in opts:
            ctx.set_option(OPT_IDS[k], 0)
