"""Key-pointer sort with DPG as the copy phase (Section 3), on the GPU through
the C ABI, against the CPU oracle (records and permutation, byte for byte)."""
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


def tied_records(n, rec_bytes, n_prefixes, seed):
    """Records whose first 8 key bytes take only n_prefixes values (bytes 8-9
    then decide), the tie case the paper's 10-byte key allows."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, 256, size=(n, rec_bytes), dtype=np.uint8)
    pref = rng.integers(0, 256, size=(n_prefixes, 8), dtype=np.uint8)
    src[:, 0:8] = pref[rng.integers(0, n_prefixes, n)]
    src[:, 8:10] = rng.integers(0, 3, size=(n, 2), dtype=np.uint8)
    return src


CASES = [
    # (n, rec_bytes, key_offset, key_bytes, kind)
    (1, 100, 0, 10, "random"),
    (2, 100, 0, 10, "random"),
    (1000, 100, 0, 10, "random"),
    (4099, 100, 0, 10, "tied"),
    (100003, 100, 0, 10, "random"),
    (30000, 100, 0, 10, "tied"),
    (5000, 12, 0, 10, "random"),
    (5000, 16, 6, 4, "few"),
    (7000, 36, 3, 13, "random"),
    (7000, 36, 1, 20, "tied"),
    (3000, 64, 0, 8, "few"),
    (3000, 8, 0, 8, "equal"),
    (2000, 100, 90, 10, "random"),
    (20000, 100, 0, 10, "pairs"),
    (9000, 36, 3, 13, "pairs"),
    (5000, 20, 2, 5, "pairs"),
]


@pytest.mark.parametrize("algo", [dpg.ALGO_DPG, dpg.ALGO_DIRECT])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}-R{c[1]}-off{c[2]}-k{c[3]}-{c[4]}")
def test_sort_matches_oracle(ctx, case, algo):
    n, rec, koff, kbytes, kind = case
    if kind == "random":
        src = synth.record_bytes(n, rec, seed=n + rec)
    elif kind == "tied":
        src = tied_records(n, rec, max(1, n // 50), seed=n)
    elif kind == "pairs":
        # the first four key bytes repeat in small groups (about four records
        # each), so the prefix sort leaves short tie groups for the fix-up
        src = synth.record_bytes(n, rec, seed=n + 7)
        pool = np.random.default_rng(n).integers(0, 256, size=(max(1, n // 4), 4), dtype=np.uint8)
        src[:, koff:koff + 4] = pool[np.random.default_rng(n + 1).integers(0, len(pool), n)]
    elif kind == "few":
        src = synth.record_bytes(n, rec, seed=n)
        src[:, koff:koff + kbytes] = np.random.default_rng(1).integers(0, 3, size=(n, kbytes), dtype=np.uint8)
    else:
        src = np.zeros((n, rec), dtype=np.uint8)
        src[:, -1] = np.arange(n) % 251
    want_dst, want_perm = oracle.sort_records(src, koff, kbytes)
    dst, perm = ctx.sort_records(torch.from_numpy(src).to(DEV), koff, kbytes, algo=algo)
    torch.cuda.synchronize()
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), want_perm)
    assert np.array_equal(dst.cpu().numpy(), want_dst)


def test_sort_without_perm_and_errors(ctx):
    src = torch.from_numpy(synth.record_bytes(1000, 100, seed=2)).to(DEV)
    dst, perm = ctx.sort_records(src, 0, 10, want_perm=False)
    assert perm is None
    want, _ = oracle.sort_records(src.cpu().numpy(), 0, 10)
    assert np.array_equal(dst.cpu().numpy(), want)
    for koff, kb in ((95, 10), (0, 0), (0, 65), (-1, 4)):
        with pytest.raises(dpg.DPGError) as e:
            ctx.sort_records(src, koff, kb)
        assert e.value.status == dpg.ERR_INVALID_ARG
