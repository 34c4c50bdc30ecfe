"""Foreign-key join over non-dense keys (Sections 4.2.2 and 4.2.3) on the GPU
through the C ABI: the fk column is looked up in a hash index of the
dimension keys, then joined as the dense join does; compared byte for byte
with the oracle in both orders."""
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


def tables(n_fact, n_dim, kind, fact_bytes, dim_bytes, seed):
    """Dimension rows with uint32 keys at byte 4; fact rows whose fk (byte 0)
    is a key of some dimension row (Zipf-skewed choice of row)."""
    rng = np.random.default_rng(seed)
    dim = synth.record_bytes(n_dim, dim_bytes, seed)
    if kind == "distinct":
        keys = (synth.rids_permutation(1 << 20, seed)[:n_dim].astype(np.uint64) * 4093 + 7).astype(np.uint32)
    elif kind == "dups":  # few distinct keys: a key's first row is the join partner
        keys = rng.integers(0, max(1, n_dim // 5), n_dim, dtype=np.uint64).astype(np.uint32) * 977
    else:
        raise ValueError(kind)
    dim[:, 4:8] = keys.view(np.uint8).reshape(-1, 4)
    pick = synth.zipf_fk_at(n_dim, 0.8, np.arange(n_fact), seed)
    fact = synth.record_bytes(n_fact, fact_bytes, seed + 1)
    fact[:, 0:4] = keys[pick].view(np.uint8).reshape(-1, 4)
    return fact, dim, keys


CASES = [
    # (n_fact, n_dim, key kind, fact bytes, dim bytes, log2 slots)
    (1, 1, "distinct", 8, 8, 4),
    (5000, 300, "distinct", 16, 64, 9),
    (70001, 4096, "distinct", 16, 64, 12),
    (30000, 20000, "dups", 24, 36, 14),
    (100000, 65537, "distinct", 16, 100, 16),
]


@pytest.mark.parametrize("algo", [dpg.ALGO_DPG, dpg.ALGO_DIRECT])
@pytest.mark.parametrize("order", [dpg.JOIN_FACT_ORDER, dpg.JOIN_DIM_ORDER], ids=["fact-order", "dim-order"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"F{c[0]}-D{c[1]}-{c[2]}-f{c[3]}-d{c[4]}-s{c[5]}")
def test_key_join_matches_oracle(ctx, case, order, algo):
    n_fact, n_dim, kind, fb, db, s = case
    fact, dim, keys = tables(n_fact, n_dim, kind, fb, db, seed=n_fact + n_dim)
    want = oracle.key_join(fact, dim, 0, 4, 0 if order == dpg.JOIN_FACT_ORDER else 1)
    index = ctx.hash_build(torch.from_numpy(keys.view(np.int32)).to(DEV), s)
    got = ctx.key_join(torch.from_numpy(fact).to(DEV), torch.from_numpy(dim).to(DEV), 0, index, s, order,
                       algo=algo)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)


def test_key_join_missing_key(ctx):
    fact, dim, keys = tables(1000, 200, "distinct", 16, 16, seed=5)
    fact[777, 0:4] = np.array([1], dtype="<u4").view(np.uint8)  # keys are 7 mod 4093: 1 is absent
    index = ctx.hash_build(torch.from_numpy(keys.view(np.int32)).to(DEV), 8)
    for order in (dpg.JOIN_FACT_ORDER, dpg.JOIN_DIM_ORDER):
        with pytest.raises(dpg.DPGError) as e:
            ctx.key_join(torch.from_numpy(fact).to(DEV), torch.from_numpy(dim).to(DEV), 0, index, 8, order)
        assert e.value.status == dpg.ERR_FK_OUT_OF_RANGE
        # unchecked: no synchronization and no error; every row whose key
        # exists is still the oracle's (fact order: all rows but row 777)
        got = ctx.key_join(torch.from_numpy(fact).to(DEV), torch.from_numpy(dim).to(DEV), 0, index, 8, order,
                           check_fk=False)
        torch.cuda.synchronize()
        if order == dpg.JOIN_FACT_ORDER:
            good = np.ones(len(fact), dtype=bool)
            good[777] = False
            want = oracle.key_join(fact[good], dim, 0, 4, 0)
            assert np.array_equal(got.cpu().numpy()[good], want)
