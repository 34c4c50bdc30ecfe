"""Sort-merge join with DPG sort (Section 4.1) on the GPU through the C ABI,
against the oracle (rows, order and count, byte for byte)."""
import ctypes

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


def relation(n, rec, koff, kb, pool, seed):
    """n rows of random bytes whose key field holds a random entry of pool."""
    rows = synth.record_bytes(n, rec, seed=seed) if n else np.zeros((0, rec), dtype=np.uint8)
    if n:
        rows[:, koff:koff + kb] = pool[np.random.default_rng(seed).integers(0, len(pool), n)]
    return rows


def key_pool(n_keys, kb, seed=7):
    return np.random.default_rng(seed).integers(0, 256, (n_keys, kb), dtype=np.uint8)


CASES = [
    # (n_r, rec_r, koff_r, n_s, rec_s, koff_s, key_bytes, distinct keys per side)
    (1000, 16, 0, 1200, 32, 4, 4, 700),          # about one match per row, duplicates
    (5000, 64, 3, 3000, 16, 8, 8, 100000),       # mostly distinct: few matches
    (2000, 8, 1, 2500, 12, 0, 2, 300),           # many pairs per key
    (1, 4, 0, 1, 4, 0, 4, 1),                    # one row each, same key
    (0, 16, 0, 100, 16, 0, 4, 10),               # empty R
    (300, 100, 90, 400, 20, 13, 7, 3),           # three keys: large cross products
    (70001, 32, 0, 65537, 16, 4, 4, 50000),      # many tiles, ragged
    (70001, 4, 0, 65537, 4, 0, 4, 50000),        # 4-byte rows: a tile spans more R rows than LDS holds
    (40000, 4, 0, 3000, 4, 0, 4, 1 << 20),       # mostly unmatched R rows
    (3000, 8, 0, 9000, 8, 4, 2, 5),              # an R block's S span exceeds LDS: global search
    (2000, 12, 4, 2500, 8, 0, 8, 40),            # 8-byte keys (packed keys path), heavy duplicates
]


@pytest.mark.parametrize("algo", [dpg.ALGO_DPG, dpg.ALGO_DIRECT])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"r{c[0]}x{c[1]}-s{c[3]}x{c[4]}-k{c[6]}-d{c[7]}")
def test_smj_matches_oracle(ctx, case, algo):
    nr, rr, kr, ns, rs, ks, kb, nk = case
    pool = key_pool(nk, kb)  # both sides draw from one pool
    r = relation(nr, rr, kr, kb, pool, seed=nr + 11)
    s = relation(ns, rs, ks, kb, pool, seed=ns + 12)
    want = oracle.sort_merge_join(r, s, kr, ks, kb)
    got = ctx.sort_merge_join(torch.from_numpy(r).to(DEV), torch.from_numpy(s).to(DEV), kr, ks, kb, algo=algo)
    torch.cuda.synchronize()
    assert got.shape == want.shape
    assert np.array_equal(got.cpu().numpy(), want)


def test_smj_capacity_and_errors(ctx):
    pool = key_pool(50, 4)
    r = relation(500, 16, 0, 4, pool, seed=3)
    s = relation(400, 16, 0, 4, pool, seed=4)
    want = oracle.sort_merge_join(r, s, 0, 0, 4)
    lib = dpg.lib()
    rd, sd = torch.from_numpy(r).to(DEV), torch.from_numpy(s).to(DEV)
    need = lib.dpg_sort_merge_join_workspace_bytes(ctx.handle, 500, 16, 0, 400, 16, 0, 4, dpg.ALGO_DPG)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    out = torch.empty((1, 32), dtype=torch.uint8, device=DEV)
    n = ctypes.c_int64()
    st = lib.dpg_sort_merge_join(ctx.handle, rd.data_ptr(), 500, 16, 0, sd.data_ptr(), 400, 16, 0, 4,
                                 out.data_ptr(), 1, ctypes.byref(n), ws.data_ptr(), ws.numel(), dpg.ALGO_DPG, None)
    assert st == dpg.ERR_WORKSPACE_TOO_SMALL and n.value == want.shape[0] > 1
    for bad in ((0, 0), (0, 9), (13, 4)):  # key_bytes 0, 9; key past the row
        assert lib.dpg_sort_merge_join_workspace_bytes(ctx.handle, 500, 16, bad[0], 400, 16, 0, bad[1],
                                                       dpg.ALGO_DPG) == 0
    # through the binding: an output of one row is replaced by one of the exact size
    got = ctx.sort_merge_join(rd, sd, 0, 0, 4, out=torch.empty((1, 32), dtype=torch.uint8, device=DEV))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)


def test_smj_full_size(ctx):
    """The benchmark's configuration: R and S of 2^24 x 100 B rows, a 4-byte
    key uniform over 2^24 values.  The result is fixed by its definition:
    for every key, a block of cR * cS rows, R index major, at the position the
    counts of the smaller keys give.  Checked: the row count, that both halves
    of every row hold the same key, that keys never decrease, and for 64
    sampled keys the exact block."""
    n, R = 1 << 24, 100
    rel, keys, counts = [], [], []
    for side in range(2):
        rows = synth.record_bytes(n, R, 300 + side, backend="torch", device=DEV)
        k = synth.uniform_at(n, torch.arange(n, device=DEV), 300 + side, synth.STREAM_FK, backend="torch",
                             device=DEV).to(torch.int32)
        rows[:, 0:4] = k.view(torch.uint8).reshape(-1, 4)
        rel.append(rows)
        keys.append(k.to(torch.int64))
        counts.append(torch.bincount(k.to(torch.int64), minlength=n))
    # the key compares as big-endian bytes: order the blocks by that value
    be = lambda k: ((k & 0xFF) << 24) | (((k >> 8) & 0xFF) << 16) | (((k >> 16) & 0xFF) << 8) | ((k >> 24) & 0xFF)
    per_key = counts[0] * counts[1]
    total = int(per_key.sum())
    ids = torch.arange(n, device=DEV)
    order = torch.argsort(be(ids))
    start = torch.zeros(n, dtype=torch.int64, device=DEV)
    start[order] = torch.cumsum(per_key[order], 0) - per_key[order]
    for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
        out = ctx.sort_merge_join(rel[0], rel[1], 0, 0, 4, algo=algo,
                                  out=torch.empty((total + 16, 2 * R), dtype=torch.uint8, device=DEV))
        torch.cuda.synchronize()
        assert out.shape[0] == total
        assert torch.equal(out[:, 0:4], out[:, R:R + 4])
        kk = be(out[:, 0:4].contiguous().view(torch.int32).view(-1).to(torch.int64) & 0xFFFFFFFF)
        assert bool((kk[1:] >= kk[:-1]).all())
        hot = torch.nonzero(per_key > 0).view(-1)
        pick = hot[torch.randperm(hot.numel(), device=DEV, generator=torch.Generator(device=DEV).manual_seed(3))[:64]]
        for key in pick.tolist():
            ri = torch.nonzero(keys[0] == key).view(-1)
            si = torch.nonzero(keys[1] == key).view(-1)
            want = torch.cat([rel[0][ri].repeat_interleave(si.numel(), 0), rel[1][si].repeat(ri.numel(), 1)], 1)
            s0 = int(start[key])
            assert torch.equal(out[s0:s0 + want.shape[0]], want), key
        del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[4], CASES[6], CASES[10]],
                         ids=lambda c: f"r{c[0]}x{c[1]}-s{c[3]}x{c[4]}-k{c[6]}")
def test_smj_async_matches_oracle_and_cuts_at_capacity(ctx, case):
    """dpg_sort_merge_join_async: no host synchronization, the row count in
    device memory; with room for every row the output equals the oracle's,
    with room for half of them it holds the first half and the count is still
    the full one."""
    nr, rr, kr, ns, rs, ks, kb, nk = case
    pool = key_pool(nk, kb)
    r = relation(nr, rr, kr, kb, pool, seed=nr + 11)
    s = relation(ns, rs, ks, kb, pool, seed=ns + 12)
    want = oracle.sort_merge_join(r, s, kr, ks, kb)
    rt, st = torch.from_numpy(r).to(DEV), torch.from_numpy(s).to(DEV)
    for cap in (want.shape[0] + 5, want.shape[0] // 2):
        out = torch.full((max(cap, 1), rr + rs), 7, dtype=torch.uint8, device=DEV)[:cap]
        rows = torch.full((1,), -1, dtype=torch.int64, device=DEV)
        ctx.sort_merge_join_async(rt, st, kr, ks, kb, out, rows, algo=dpg.ALGO_DPG)
        torch.cuda.synchronize()
        assert int(rows.item()) == want.shape[0]
        k = min(cap, want.shape[0])
        assert np.array_equal(out[:k].cpu().numpy(), want[:k])
        assert bool((out[k:] == 7).all())


def test_smj_async_in_a_captured_graph(ctx):
    """The asynchronous join (both sorts, the merge, the emit) captured into a
    HIP graph and replayed three times, with eager work between replays;
    every replay against the oracle."""
    nr, rr, kr, ns, rs, ks, kb, nk = CASES[0]
    pool = key_pool(nk, kb)
    r = relation(nr, rr, kr, kb, pool, seed=nr + 11)
    s = relation(ns, rs, ks, kb, pool, seed=ns + 12)
    want = oracle.sort_merge_join(r, s, kr, ks, kb)
    rt, st = torch.from_numpy(r).to(DEV), torch.from_numpy(s).to(DEV)
    out = torch.empty((want.shape[0] + 16, rr + rs), dtype=torch.uint8, device=DEV)
    rows = torch.zeros(1, dtype=torch.int64, device=DEV)
    need = ctx.sort_merge_join_workspace_bytes(nr, rr, kr, ns, rs, ks, kb, dpg.ALGO_DPG)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        ctx.sort_merge_join_async(rt, st, kr, ks, kb, out, rows, algo=dpg.ALGO_DPG, workspace=ws,
                                  stream=torch.cuda.current_stream())
    for rep in range(3):
        out.fill_(0)
        rows.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(rows.item()) == want.shape[0], rep
        assert np.array_equal(out[:want.shape[0]].cpu().numpy(), want), rep
        x = torch.randn(1 << 16, device=DEV)
        assert float(x.abs().sum()) > 0
