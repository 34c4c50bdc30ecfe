"""The serving engine's device-memory arena: host bookkeeping only, so it is
exercised here without a GPU against a plain Python model of the free list."""
import numpy as np
import pytest

from paper_cs_0308004_amd import dpg

BASE = 1 << 32


def test_alloc_free_coalesce():
    a = dpg.Arena(BASE, 1 << 20, 256)
    x = a.alloc(100)
    y = a.alloc(1000)
    z = a.alloc(256)
    assert x == BASE and y == BASE + 256 and z == BASE + 256 + 1024
    assert a.stats()["in_use"] == 256 + 1024 + 256
    a.free(y)
    assert a.stats()["free_blocks"] == 2
    w = a.alloc(900)  # the hole is the smallest block that fits
    assert w == y
    a.free(w)
    a.free(x)
    a.free(z)
    st = a.stats()
    assert st["in_use"] == 0 and st["free_blocks"] == 1 and st["largest_free"] == 1 << 20
    assert st["high_water"] == 256 + 1024 + 256


def test_exhaustion_and_bad_free():
    a = dpg.Arena(BASE, 4096, 256)
    blocks = [a.alloc(1000) for _ in range(4)]
    assert all(b is not None for b in blocks)
    assert a.alloc(1) is None
    with pytest.raises(dpg.DPGError):
        a.free(BASE + 17)
    a.free(blocks[1])
    with pytest.raises(dpg.DPGError):
        a.free(blocks[1])  # double free
    assert a.alloc(1024) == blocks[1]
    with pytest.raises(dpg.DPGError):
        dpg.Arena(BASE + 3, 4096, 256)  # misaligned base


def test_random_against_model():
    """Random alloc/free sequences: the arena never hands out overlapping
    blocks, stays within its range, and its byte count matches the model."""
    rng = np.random.default_rng(0)
    size = 1 << 22
    a = dpg.Arena(BASE, size, 256)
    live = {}
    for step in range(5000):
        if live and rng.random() < 0.45:
            addr = list(live)[rng.integers(0, len(live))]
            a.free(addr)
            del live[addr]
        else:
            n = int(rng.integers(1, 200000))
            addr = a.alloc(n)
            need = -(-n // 256) * 256
            if addr is None:
                assert a.stats()["largest_free"] < need
                continue
            assert addr % 256 == 0 and BASE <= addr and addr + need <= BASE + size
            for b, m in live.items():
                assert addr + need <= b or b + m <= addr
            live[addr] = need
        assert a.stats()["in_use"] == sum(live.values())
    for addr in list(live):
        a.free(addr)
    assert a.stats()["free_blocks"] == 1


def test_best_fit_takes_the_smallest_hole():
    """Of the free blocks that hold a request, the smallest is taken (the
    lowest address among equals), so small requests do not split the large
    holes."""
    a = dpg.Arena(BASE, 1 << 20, 256)
    blocks = [a.alloc(n) for n in (4096, 256, 1024, 256, 1024, 256, 2048, 256)]
    for k in (0, 2, 4, 6):
        a.free(blocks[k])  # holes of 4096, 1024, 1024 and 2048 bytes, then the rest
    assert a.alloc(1000) == blocks[2]
    assert a.alloc(1024) == blocks[4]
    assert a.alloc(1500) == blocks[6]
    assert a.alloc(3000) == blocks[0]
    assert a.alloc(4096) == blocks[7] + 256  # only the tail is left


def test_best_fit_ties_take_the_lowest_address():
    """Among free blocks of the same length the lowest address is taken, and
    freeing everything coalesces back to one block."""
    a = dpg.Arena(BASE, 1 << 16, 256)
    blocks = [a.alloc(512) for _ in range(8)]
    for k in (5, 1, 3):  # three holes of 512 bytes, freed out of order
        a.free(blocks[k])
    assert a.alloc(300) == blocks[1]
    assert a.alloc(512) == blocks[3]
    assert a.alloc(1) == blocks[5]
    for b in blocks:
        a.free(b)
    st = a.stats()
    assert st["free_blocks"] == 1 and st["largest_free"] == 1 << 16 and st["in_use"] == 0
