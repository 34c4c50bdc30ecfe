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
