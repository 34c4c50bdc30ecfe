"""The C-ABI library without a GPU: it loads, exports what include/dpg.h
declares, plans sensibly and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_cs_0308004_amd import dpg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(dpg_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(dpg.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    # every declared function has a ctypes signature in the binding
    assert set(declared_functions()) <= set(dpg.SIGNATURES)


def test_status_strings():
    lib = dpg.lib()
    for code in range(8):
        assert lib.dpg_status_string(code)
    assert lib.dpg_status_string(99) == b"unknown status"


@pytest.mark.parametrize("rec_bytes", [4, 8, 16, 32, 64, 100, 128, 256, 4096])
def test_plan_constraints(rec_bytes):
    for n in (1, 1000, 1 << 20, 1 << 26):
        p = dpg.plan_retrieve(n, rec_bytes, n, dpg.ALGO_DPG)
        L = 1 << p.log2_run
        assert p.algo == dpg.ALGO_DPG
        assert p.n_runs == -(-n // L) and 1 <= p.n_runs <= 8192
        assert p.dist_tile % 64 == 0 and p.n_tiles == -(-n // p.dist_tile)
        assert p.n_tiles * p.n_runs <= max(n, 1024 * 8192) // 4 + 8192
        if p.probe == dpg.PROBE_LDS:  # 128 KiB regions for 4..16-byte records, else 64 KiB
            assert L * rec_bytes <= (128 if rec_bytes in (4, 8, 16) else 64) * 1024
        # workspace holds the runs, the slots (or list positions) and INTERNAL,
        # which the two-phase form (Phase III "none") does without: taken for
        # whole 64-byte sectors, and for records of 24 bytes or more whose
        # output fits 192 MiB (the Infinity Cache combines the partial lines)
        two_phase = rec_bytes % 64 == 0 or (rec_bytes >= 24 and n * rec_bytes <= 192 << 20)
        assert p.gather in (1, 2, 3) and (p.gather == 3) == two_phase
        assert p.workspace_bytes >= n * (8 + (0 if p.gather == 3 else rec_bytes))
        if p.gather == 3:
            assert p.ws_internal == 0
        else:
            assert p.ws_internal + n * rec_bytes <= p.workspace_bytes
        assert p.ws_rid_run + 4 * n <= p.workspace_bytes
        d = dpg.plan_retrieve(n, rec_bytes, n, dpg.ALGO_DIRECT)
        assert d.algo == dpg.ALGO_DIRECT and d.workspace_bytes == 256


def test_plan_lds_probe_fits():
    lib = dpg.lib()
    # with a NULL context the default options apply: cached probe, except the
    # wide LDS probe for 4-byte records
    p = dpg.plan_retrieve(1 << 20, 100, 1 << 20, dpg.ALGO_DPG)
    assert p.probe == dpg.PROBE_CACHED
    p4 = dpg.plan_retrieve(1 << 26, 4, 1 << 26, dpg.ALGO_DPG)
    assert p4.probe == dpg.PROBE_LDS and p4.log2_run == 15 and p4.distribute == dpg.DIST_PARTITION
    assert lib.dpg_retrieve_workspace_bytes(None, 100, 6, 10, 0) == 0  # rejected shape


# fake, aligned device addresses: validation never dereferences them
SRC, DST, RIDS, WS = 0x10000000, 0x20000000, 0x30000000, 0x40000000


def call(n_src=100, rec=8, rids=RIDS, n=10, dst=DST, ws=WS, ws_bytes=1 << 24, algo=0, check=0, src=SRC, ctx=None):
    return dpg.lib().dpg_retrieve(ctx, src, n_src, rec, rids, n, dst, ws, ws_bytes, algo, check, None)


def test_retrieve_argument_validation():
    E = dpg
    assert call() == E.ERR_INVALID_ARG  # valid arguments, but no context
    assert call(rec=6) == E.ERR_INVALID_ARG
    assert call(rec=0) == E.ERR_INVALID_ARG
    assert call(rec=4100) == E.ERR_INVALID_ARG
    assert call(n_src=-1) == E.ERR_INVALID_ARG
    assert call(n=-1) == E.ERR_INVALID_ARG
    assert call(n_src=1 << 31) == E.ERR_INVALID_ARG
    assert call(rids=0) == E.ERR_INVALID_ARG
    assert call(dst=0) == E.ERR_INVALID_ARG
    assert call(src=0) == E.ERR_INVALID_ARG
    assert call(src=SRC + 2) == E.ERR_INVALID_ARG
    assert call(algo=7) == E.ERR_INVALID_ARG
    assert call(check=2) == E.ERR_INVALID_ARG
    # overlapping src and dst, rids and dst, rids and workspace
    assert call(dst=SRC + 400) == E.ERR_INVALID_ARG
    assert call(dst=RIDS + 8) == E.ERR_INVALID_ARG
    # no source records but rids to retrieve: every rid is out of range
    assert call(n_src=0, src=0) == E.ERR_RID_OUT_OF_RANGE
    # workspace: too small, missing, misaligned, overlapping
    need = dpg.lib().dpg_retrieve_workspace_bytes(None, 100, 8, 10, dpg.ALGO_DPG)
    assert call(algo=dpg.ALGO_DPG, ws_bytes=need - 1) == E.ERR_WORKSPACE_TOO_SMALL
    assert call(algo=dpg.ALGO_DPG, ws=0, ws_bytes=need) == E.ERR_INVALID_ARG
    assert call(algo=dpg.ALGO_DPG, ws=WS + 16, ws_bytes=need) == E.ERR_INVALID_ARG
    assert call(algo=dpg.ALGO_DPG, ws=DST, ws_bytes=need) == E.ERR_INVALID_ARG
    assert call(algo=dpg.ALGO_DPG, ws=RIDS - 256, ws_bytes=need) == E.ERR_INVALID_ARG
    # empty rid list with valid arguments passes validation (then needs a context)
    assert call(n=0, rids=0, dst=0, ws=0, ws_bytes=0) == E.ERR_INVALID_ARG


def test_options_need_context():
    lib = dpg.lib()
    assert lib.dpg_set_option(None, dpg.OPT_LOG2_RUN, 3) == dpg.ERR_INVALID_ARG
    v = ctypes.c_int64()
    assert lib.dpg_get_option(None, dpg.OPT_LOG2_RUN, ctypes.byref(v)) == dpg.ERR_INVALID_ARG


def test_batch_validation_without_device():
    lib = dpg.lib()
    good = dpg.Request(dpg.REQ_RETRIEVE, dpg.ALGO_DIRECT, SRC, 100, 16, 0, RIDS, None, 10, 0, 0, DST)
    join = dpg.Request(dpg.REQ_FK_JOIN, dpg.ALGO_DIRECT, SRC, 100, 64, 16, None, RIDS, 10, 0, 0, DST)
    arr = (dpg.Request * 2)(good, join)
    need = lib.dpg_batch_workspace_bytes(None, arr, 2)
    assert need > 0
    assert lib.dpg_batch_run(None, arr, 2, WS, need, None) == dpg.ERR_INVALID_ARG  # no context
    assert lib.dpg_batch_run(None, arr, 2, WS, need - 1, None) == dpg.ERR_WORKSPACE_TOO_SMALL
    bad = dpg.Request.from_buffer_copy(good)
    bad.rec_bytes = 6
    arr2 = (dpg.Request * 2)(good, bad)
    assert lib.dpg_batch_workspace_bytes(None, arr2, 2) == 0
    assert lib.dpg_batch_run(None, arr2, 2, WS, 1 << 30, None) == dpg.ERR_INVALID_ARG
    bad = dpg.Request.from_buffer_copy(join)
    bad.fk_offset = 14
    arr3 = (dpg.Request * 1)(bad)
    assert lib.dpg_batch_run(None, arr3, 1, WS, 1 << 30, None) == dpg.ERR_INVALID_ARG
    bad = dpg.Request.from_buffer_copy(good)
    bad.kind = 5
    arr4 = (dpg.Request * 1)(bad)
    assert lib.dpg_batch_run(None, arr4, 1, WS, 1 << 30, None) == dpg.ERR_INVALID_ARG
    bad = dpg.Request.from_buffer_copy(good)
    bad.dst = RIDS + 4  # output over the rid list
    arr5 = (dpg.Request * 1)(bad)
    assert lib.dpg_batch_run(None, arr5, 1, WS, 1 << 30, None) == dpg.ERR_INVALID_ARG
    assert lib.dpg_batch_graph_workspace_bytes(None, 0) == 0
    assert lib.dpg_batch_graph_workspace_bytes(None, 16) > 0
    # scratch of a request's steps in a graph batch: none for direct work; for
    # DPG the run arrays, RID_RUN, inv (4 bytes per rid each) and INTERNAL
    assert lib.dpg_batch_request_workspace_bytes(None, ctypes.byref(good)) == 0
    q = dpg.Request.from_buffer_copy(good)
    q.algo = dpg.ALGO_DPG
    assert lib.dpg_batch_request_workspace_bytes(None, ctypes.byref(q)) >= 10 * (4 + 4 + 16)
    q.n = 1 << 20
    q.n_src = 1 << 20
    assert lib.dpg_batch_request_workspace_bytes(None, ctypes.byref(q)) >= (1 << 20) * (8 + 16)
    q.rec_bytes = 6
    assert lib.dpg_batch_request_workspace_bytes(None, ctypes.byref(q)) == 0


def test_plan_phase_forms():
    """The planner's Phase I / Phase III forms: one partition pass for up to
    4096 runs; Phase III staged in LDS for 4-, 8- and 16-byte records; no
    Phase III (the probe scatters, at most 2048 runs) for whole 64-byte
    sectors; the cached gather otherwise."""
    for rec in (4, 8, 16):
        p = dpg.plan_retrieve(1 << 26, rec, 1 << 26, dpg.ALGO_DPG)
        assert p.distribute == dpg.DIST_PARTITION and p.gather == dpg.GATHER_LDS, rec
    for rec in (12, 32, 100, 96):
        p = dpg.plan_retrieve(1 << 26, rec, 1 << 26, dpg.ALGO_DPG)
        assert p.distribute == dpg.DIST_PARTITION and p.gather == dpg.GATHER_CACHED, rec
        assert p.n_runs <= 4096
    for rec in (64, 128, 256, 4096):
        p = dpg.plan_retrieve(1 << 26, rec, 1 << 26, dpg.ALGO_DPG)
        assert p.distribute == dpg.DIST_PARTITION and p.gather == dpg.GATHER_NONE, rec
        assert p.n_runs <= 2048 and p.ws_internal == 0
    p = dpg.plan_retrieve(1 << 26, 8, 1 << 26, dpg.ALGO_DIRECT)
    assert p.distribute == 0 and p.gather == 0
    # the one-pass distribute takes the 1024-thread partition pass at any run
    # count; with the LDS-staged gather its tiles are 16384 rids for 4-byte
    # records and 8192 otherwise, and automatic runs of 8- and 16-byte records
    # stop at 1024 (2 MiB regions below that)
    for n, rec, runs, tile in ((1 << 26, 4, 2048, 16384), (1 << 26, 8, 256, 8192), (1 << 26, 16, 512, 8192),
                               (1 << 28, 8, 1024, 8192), (1 << 28, 16, 1024, 8192)):
        p = dpg.plan_retrieve(n, rec, n, dpg.ALGO_DPG)
        assert (p.n_runs, p.gather, p.dist_tile) == (runs, dpg.GATHER_LDS, tile), (n, rec)
        assert p.n_tiles == n // tile
    # short rid lists take tiles of 8192 rids so that Phase I fills the chip
    p = dpg.plan_retrieve(1 << 20, 100, 1 << 20, dpg.ALGO_DPG)
    assert p.dist_tile == 8192 and p.n_tiles == 128
    # 1025..2048 runs of a long rid list: tiles of 32768 rids
    p = dpg.plan_retrieve(1 << 26, 100, 1 << 26, dpg.ALGO_DPG)
    assert p.dist_tile == 32768 and p.n_runs == 2048 and p.n_tiles == 2048
    p = dpg.plan_retrieve(1 << 25, 100, 1 << 25, dpg.ALGO_DPG)
    assert p.dist_tile == 16384 and p.n_runs == 1024


def test_hash_index_layout_and_validation():
    lib = dpg.lib()
    s = 10
    assert lib.dpg_hash_ov_off_offset(s) == 8 << s
    assert lib.dpg_hash_ov_offset(s) == (8 << s) + (((4 * ((1 << s) + 1)) + 255) // 256) * 256
    assert lib.dpg_hash_index_bytes(1000, s) == lib.dpg_hash_ov_offset(s) + 8192
    for bad in ((1000, 3), (1000, 31), (-1, 10), (1 << 31, 10)):
        assert lib.dpg_hash_index_bytes(*bad) == 0
    assert lib.dpg_hash_build_workspace_bytes(None, 1000, 3) == 0
    need_ix = lib.dpg_hash_index_bytes(1000, s)
    need_ws = lib.dpg_hash_build_workspace_bytes(None, 1000, s)
    assert need_ws > 0
    IX = 0x50000000
    E = dpg
    # valid arguments, but no context
    assert lib.dpg_hash_build(None, SRC, 1000, s, IX, need_ix, WS, need_ws, None) == E.ERR_INVALID_ARG
    assert lib.dpg_hash_build(None, SRC, 1000, s, IX, need_ix - 1, WS, need_ws, None) == E.ERR_INVALID_ARG
    assert lib.dpg_hash_build(None, SRC, 1000, s, IX + 16, need_ix, WS, need_ws, None) == E.ERR_INVALID_ARG
    assert lib.dpg_hash_build(None, SRC, 1000, s, IX, need_ix, WS, need_ws - 1, None) == E.ERR_WORKSPACE_TOO_SMALL
    assert lib.dpg_hash_build(None, SRC, 1000, s, IX, need_ix, IX + 256, need_ws, None) == E.ERR_INVALID_ARG
    need_q = lib.dpg_hash_lookup_workspace_bytes(None, 1000, s, 5000, dpg.ALGO_DPG)
    assert need_q > 0
    assert lib.dpg_hash_lookup_workspace_bytes(None, 1000, s, 5000, dpg.ALGO_DIRECT) == 256
    assert lib.dpg_hash_lookup_workspace_bytes(None, 1000, s, 5000, 7) == 0
    assert lib.dpg_hash_lookup(None, IX, 1000, s, RIDS, 5000, DST, WS, need_q, dpg.ALGO_DPG, None) == E.ERR_INVALID_ARG
    assert lib.dpg_hash_lookup(None, IX, 1000, s, RIDS, 5000, DST, WS, need_q - 1, dpg.ALGO_DPG,
                               None) == E.ERR_WORKSPACE_TOO_SMALL
    assert lib.dpg_hash_lookup(None, IX, 1000, s, RIDS, 5000, RIDS + 4, WS, need_q, dpg.ALGO_DPG,
                               None) == E.ERR_INVALID_ARG  # output over the queries
    assert lib.dpg_hash_lookup(None, IX, 1000, s, RIDS, 5000, DST, WS, need_q, 9, None) == E.ERR_INVALID_ARG


def test_sort_merge_join_validation():
    lib = dpg.lib()
    E = dpg
    args = (1000, 16, 0, 2000, 32, 4, 4)
    need = lib.dpg_sort_merge_join_workspace_bytes(None, *args, dpg.ALGO_DPG)
    assert need >= 1000 * 16 + 2000 * 32 + 8 * 3000
    for bad in ((1000, 16, 0, 2000, 32, 4, 0), (1000, 16, 0, 2000, 32, 4, 9), (1000, 16, 13, 2000, 32, 4, 4),
                (1000, 18, 0, 2000, 32, 4, 4), (-1, 16, 0, 2000, 32, 4, 4), (1000, 16, 0, 2000, 32, 29, 4)):
        assert lib.dpg_sort_merge_join_workspace_bytes(None, *bad, dpg.ALGO_DPG) == 0
    assert lib.dpg_sort_merge_join_workspace_bytes(None, *args, 7) == 0
    n = ctypes.c_int64(-5)
    OUT = 0x50000000
    call = lambda out, cap, ws, wsb, rows=ctypes.byref(n): lib.dpg_sort_merge_join(
        None, SRC, 1000, 16, 0, DST, 2000, 32, 4, 4, out, cap, rows, ws, wsb, dpg.ALGO_DPG, None)
    assert call(OUT, 100, WS, need) == E.ERR_INVALID_ARG                 # valid, but no context
    assert call(OUT, 100, WS, need - 1) == E.ERR_WORKSPACE_TOO_SMALL
    assert call(OUT, 100, WS, need, None) == E.ERR_INVALID_ARG          # no row count
    assert call(OUT, -1, WS, need) == E.ERR_INVALID_ARG
    assert call(OUT + 2, 100, WS, need) == E.ERR_INVALID_ARG            # misaligned output
    assert call(SRC + 64, 100, WS, need) == E.ERR_INVALID_ARG           # output over R
    assert call(OUT, 100, WS + 16, need) == E.ERR_INVALID_ARG           # misaligned workspace
    assert call(OUT, 100, DST, need) == E.ERR_INVALID_ARG               # workspace over S
    assert n.value == -5                                                # nothing written on a rejected call


def test_btree_layout_and_validation():
    lib = dpg.lib()
    E = dpg
    # 1000 keys: 32 leaf blocks, one inner node
    assert lib.dpg_btree_levels(1000) == 2
    assert lib.dpg_btree_rids_offset(1000) == 4096
    assert lib.dpg_btree_level_offset(1000, 0) == 0
    assert lib.dpg_btree_level_offset(1000, 1) == 8192
    assert lib.dpg_btree_bytes(1000) == 8192 + 256
    # 0 keys: one (padding) leaf block; 2^15 + 1 keys: 1025 blocks -> 33 -> 2 -> 1
    assert lib.dpg_btree_levels(0) == 1 and lib.dpg_btree_bytes(0) == 512  # keys, then rids at 256
    assert lib.dpg_btree_levels((1 << 15) + 1) == 4
    for bad in ((-1, 0), (1 << 31, 0), (1000, 2), (1000, -1)):
        assert lib.dpg_btree_level_offset(*bad) == 0
    assert lib.dpg_btree_bytes(-1) == 0 and lib.dpg_btree_levels(-1) == 0
    n = 5000
    tb = lib.dpg_btree_bytes(n)
    need = lib.dpg_btree_build_workspace_bytes(None, n)
    assert need >= 16 * n
    T = 0x50000000
    assert lib.dpg_btree_build(None, SRC, n, T, tb, WS, need, None) == E.ERR_INVALID_ARG  # no context
    assert lib.dpg_btree_build(None, SRC, n, T, tb - 1, WS, need, None) == E.ERR_INVALID_ARG
    assert lib.dpg_btree_build(None, SRC, n, T + 16, tb, WS, need, None) == E.ERR_INVALID_ARG
    assert lib.dpg_btree_build(None, SRC, n, T, tb, WS, need - 1, None) == E.ERR_WORKSPACE_TOO_SMALL
    assert lib.dpg_btree_build(None, SRC, n, T, tb, T + 256, need, None) == E.ERR_INVALID_ARG
    assert lib.dpg_btree_build(None, SRC, n, SRC + 256, tb, WS, need, None) == E.ERR_INVALID_ARG  # tree over keys
    need_q = lib.dpg_btree_lookup_workspace_bytes(None, n, 7000, dpg.ALGO_DPG)
    assert need_q > 7000 * 12
    assert lib.dpg_btree_lookup_workspace_bytes(None, n, 7000, dpg.ALGO_DIRECT) == 256
    assert lib.dpg_btree_lookup_workspace_bytes(None, n, 7000, 7) == 0
    assert lib.dpg_btree_lookup_workspace_bytes(None, -1, 7000, dpg.ALGO_DPG) == 0
    assert lib.dpg_btree_lookup(None, T, n, RIDS, 7000, DST, WS, need_q, dpg.ALGO_DPG, None) == E.ERR_INVALID_ARG
    assert lib.dpg_btree_lookup(None, T, n, RIDS, 7000, DST, WS, need_q - 1, dpg.ALGO_DPG,
                                None) == E.ERR_WORKSPACE_TOO_SMALL
    assert lib.dpg_btree_lookup(None, T, n, RIDS, 7000, RIDS + 4, WS, need_q, dpg.ALGO_DPG,
                                None) == E.ERR_INVALID_ARG  # output over the queries
    assert lib.dpg_btree_lookup(None, T, n, RIDS, 7000, DST, WS, need_q, 9, None) == E.ERR_INVALID_ARG
    assert lib.dpg_btree_lookup(None, T + 64, n, RIDS, 7000, DST, WS, need_q, dpg.ALGO_DPG,
                                None) == E.ERR_INVALID_ARG  # misaligned tree


def test_key_join_validation():
    lib = dpg.lib()
    E = dpg
    need = lib.dpg_key_join_workspace_bytes(None, 5000, 16, 0, 300, 64, 9, dpg.JOIN_FACT_ORDER, dpg.ALGO_DPG)
    assert need > 5000 * 8
    assert lib.dpg_key_join_workspace_bytes(None, 5000, 16, 0, 300, 64, 3, 0, dpg.ALGO_DPG) == 0  # slots
    assert lib.dpg_key_join_workspace_bytes(None, 5000, 16, 2, 300, 64, 9, 0, dpg.ALGO_DPG) == 0  # fk offset
    assert lib.dpg_key_join_workspace_bytes(None, 5000, 16, 0, 300, 64, 9, 5, dpg.ALGO_DPG) == 0  # order
    IX, OUT = 0x50000000, 0x60000000
    call = lambda ix, out, ws, wsb: lib.dpg_key_join(None, SRC, 5000, 16, 0, DST, 300, 64, ix, 9, out,
                                                      dpg.JOIN_FACT_ORDER, ws, wsb, dpg.ALGO_DPG, 1, None)
    assert call(IX, OUT, WS, need) == E.ERR_INVALID_ARG            # valid, but no context
    assert call(IX, OUT, WS, need - 1) == E.ERR_WORKSPACE_TOO_SMALL
    assert call(IX + 16, OUT, WS, need) == E.ERR_INVALID_ARG       # misaligned index
    assert call(IX, SRC + 64, WS, need) == E.ERR_INVALID_ARG       # output over the fact rows
    assert call(IX, OUT, IX, need) == E.ERR_INVALID_ARG            # workspace over the index
