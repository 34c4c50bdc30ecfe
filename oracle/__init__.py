"""CPU oracle for DPG record retrieval, sorting and foreign-key joins.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the library under
``paper_cs_0308004_amd`` never does.  The arithmetic lives in ``oracle.c``
(plain C, compiled with gcc by :func:`build`); this module only marshals numpy
arrays into it.

Every function follows a passage of Cooperman, Ma and Nguyen, "DPG: A
Cache-Efficient Accelerator for Sorting and for Join Operators":

* :func:`retrieve` -- the record-retrieval problem of Section 2 (D[i] = R[S_rid[i]]).
* :func:`dpg_phases` -- Figure 1 (Section 2.1) run phase by phase, 0-based.
* :func:`sort_records` -- the three-phase key-pointer sort of Section 3.
* :func:`fk_join_fact_order` / :func:`fk_join_dim_order` -- the DPG-Move and
  DPG-Sort goals of Section 4.2.1.
* :func:`sort_merge_join` -- the sort-merge join of Section 4.1 (all pairs of
  equal join keys, ordered by key, then R index, then S index).
* :func:`hash_build` / :func:`hash_lookup` -- the hash index of Section 4.2.3
  (one key-rid pair per slot, collisions in an overflow array) and the result
  of a batch lookup (smallest rid holding each query key, or -1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(defines: tuple[str, ...] = (), out_path: str | None = None) -> str:
    """Compile oracle.c into a shared library with gcc and return its path."""
    out = out_path or _LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-Wextra", "-o", out, _SRC]
    cmd[1:1] = [f"-D{d}" for d in defines]
    subprocess.run(cmd, check=True)
    return out


def _stale() -> bool:
    return (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)


_I64, _I32, _VP = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    lib.oracle_retrieve.argtypes = [_VP, _I64, _I32, _VP, _I64, _VP]
    lib.oracle_dpg_phases.argtypes = [_VP, _I64, _I32, _VP, _I64, _I64, _VP, _VP, _VP, _VP]
    lib.oracle_sort_records.argtypes = [_VP, _I64, _I32, _I32, _I32, _VP, _VP]
    join = [_VP, _I64, _I32, _I32, _VP, _I64, _I32, _VP]
    lib.oracle_fk_join_fact_order.argtypes = join
    lib.oracle_fk_join_dim_order.argtypes = join
    lib.oracle_hash_build.argtypes = [_VP, _I64, _I32, _VP, _VP, _VP, _VP]
    lib.oracle_hash_lookup.argtypes = [_VP, _I64, _VP, _I64, _VP]
    lib.oracle_sort_merge_join.argtypes = [_VP, _I64, _I32, _I32, _VP, _I64, _I32, _I32, _I32, _VP, _I64, _VP]
    lib.oracle_key_join.argtypes = [_VP, _I64, _I32, _I32, _VP, _I64, _I32, _I32, _I32, _VP]
    lib.oracle_btree_shape.argtypes = [_I64, _VP, _I32]
    lib.oracle_btree_build.argtypes = [_VP, _I64, _VP, _VP, _VP]
    lib.oracle_btree_lookup.argtypes = [_VP, _VP, _VP, _I64, _VP, _I64, _VP]
    for f in (lib.oracle_retrieve, lib.oracle_dpg_phases, lib.oracle_sort_records,
              lib.oracle_fk_join_fact_order, lib.oracle_fk_join_dim_order, lib.oracle_hash_build,
              lib.oracle_hash_lookup, lib.oracle_sort_merge_join, lib.oracle_btree_shape,
              lib.oracle_btree_build, lib.oracle_btree_lookup, lib.oracle_key_join):
        f.restype = ctypes.c_int
    return lib


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the oracle library (building it first when the C source is newer)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if _stale():
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _records(a: np.ndarray, rec_bytes: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.size % rec_bytes:
        raise ValueError("byte array is not a whole number of records")
    return a.reshape(-1, rec_bytes)


def retrieve(src: np.ndarray, rids: np.ndarray, rec_bytes: int | None = None, lib=None) -> np.ndarray:
    """dst[i] = src[rids[i]] (Section 2).  ``src`` is (N, R) uint8 or flat with rec_bytes."""
    lib = lib or load()
    if rec_bytes is None:
        rec_bytes = src.shape[1]
    s = _records(src, rec_bytes)
    r = np.ascontiguousarray(rids, dtype=np.int32)
    dst = np.empty((r.size, rec_bytes), dtype=np.uint8)
    rc = lib.oracle_retrieve(_ptr(s), s.shape[0], rec_bytes, _ptr(r), r.size, _ptr(dst))
    if rc:
        raise OracleError(rc, "retrieve")
    return dst


def dpg_phases(src: np.ndarray, rids: np.ndarray, run_len: int, lib=None):
    """Figure 1 phase by phase.  Returns (rid_run, run_off, record_run, dst)."""
    lib = lib or load()
    s = _records(src, src.shape[1])
    rec_bytes = s.shape[1]
    r = np.ascontiguousarray(rids, dtype=np.int32)
    n_runs = -(-s.shape[0] // run_len)
    rid_run = np.empty(r.size, dtype=np.int32)
    run_off = np.empty(n_runs + 1, dtype=np.int64)
    record_run = np.empty((r.size, rec_bytes), dtype=np.uint8)
    dst = np.empty((r.size, rec_bytes), dtype=np.uint8)
    rc = lib.oracle_dpg_phases(_ptr(s), s.shape[0], rec_bytes, _ptr(r), r.size, run_len,
                               _ptr(rid_run), _ptr(run_off), _ptr(record_run), _ptr(dst))
    if rc:
        raise OracleError(rc, "dpg_phases")
    return rid_run, run_off, record_run, dst


def sort_records(src: np.ndarray, key_offset: int = 0, key_bytes: int = 10, lib=None):
    """Three-phase key-pointer sort (Section 3).  Returns (dst, perm)."""
    lib = lib or load()
    s = _records(src, src.shape[1])
    n, rec_bytes = s.shape
    dst = np.empty_like(s)
    perm = np.empty(n, dtype=np.int64)
    rc = lib.oracle_sort_records(_ptr(s), n, rec_bytes, key_offset, key_bytes, _ptr(dst), _ptr(perm))
    if rc:
        raise OracleError(rc, "sort_records")
    return dst, perm


def _join(fn_name: str, fact: np.ndarray, dim: np.ndarray, fk_offset: int, lib=None) -> np.ndarray:
    lib = lib or load()
    f = _records(fact, fact.shape[1])
    d = _records(dim, dim.shape[1])
    out = np.empty((f.shape[0], f.shape[1] + d.shape[1]), dtype=np.uint8)
    rc = getattr(lib, fn_name)(_ptr(f), f.shape[0], f.shape[1], fk_offset,
                               _ptr(d), d.shape[0], d.shape[1], _ptr(out))
    if rc:
        raise OracleError(rc, fn_name)
    return out


def fk_join_fact_order(fact: np.ndarray, dim: np.ndarray, fk_offset: int = 0, lib=None) -> np.ndarray:
    """DPG-Move goal (Section 4.2.1): out[i] = fact[i] || dim[fk_i]."""
    return _join("oracle_fk_join_fact_order", fact, dim, fk_offset, lib)


def fk_join_dim_order(fact: np.ndarray, dim: np.ndarray, fk_offset: int = 0, lib=None) -> np.ndarray:
    """DPG-Sort goal (Section 4.2.1): joined rows in foreign-key order, ties in fact order."""
    return _join("oracle_fk_join_dim_order", fact, dim, fk_offset, lib)


def key_join(fact: np.ndarray, dim: np.ndarray, fk_offset: int, key_offset: int, order: int = 0, lib=None):
    """Join over non-dense keys (Sections 4.2.2-4.2.3): fact row i joins the
    first dimension row whose uint32 key at key_offset equals its fk; order 0
    keeps fact order, order 1 orders by that dimension row (ties in fact order)."""
    lib = lib or load()
    f = _records(fact, fact.shape[1])
    d = _records(dim, dim.shape[1])
    out = np.empty((f.shape[0], f.shape[1] + d.shape[1]), dtype=np.uint8)
    rc = lib.oracle_key_join(_ptr(f), f.shape[0], f.shape[1], fk_offset, _ptr(d), d.shape[0], d.shape[1],
                             key_offset, order, _ptr(out))
    if rc:
        raise OracleError(rc, "key_join")
    return out


HASH_EMPTY = 0xFFFFFFFF


def hash_build(keys: np.ndarray, log2_slots: int, lib=None):
    """The hash index of Section 4.2.3 over uint32 keys (rid = position).

    Returns (slots, ov_off, ov): slots is (S, 2) uint32 of (key, rid) with
    empty slots (0, 0xFFFFFFFF); ov_off is int64[S + 1]; ov is (n_ov, 2) uint32
    of the overflow (key, rid) pairs in (home slot, rid) order."""
    lib = lib or load()
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    S = 1 << log2_slots
    slots = np.empty((S, 2), dtype=np.uint32)
    ov_off = np.empty(S + 1, dtype=np.int64)
    ov = np.empty((max(k.size, 1), 2), dtype=np.uint32)
    n_ov = ctypes.c_int64()
    rc = lib.oracle_hash_build(_ptr(k), k.size, log2_slots, _ptr(slots), _ptr(ov_off), _ptr(ov),
                               ctypes.byref(n_ov))
    if rc:
        raise OracleError(rc, "hash_build")
    return slots, ov_off, ov[:n_ov.value].copy()


def hash_lookup(keys: np.ndarray, queries: np.ndarray, lib=None) -> np.ndarray:
    """Batch lookup (Section 4.2.3): for each query, the smallest rid whose key
    equals it, or -1."""
    lib = lib or load()
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    q = np.ascontiguousarray(queries, dtype=np.uint32)
    out = np.empty(q.size, dtype=np.int32)
    rc = lib.oracle_hash_lookup(_ptr(k), k.size, _ptr(q), q.size, _ptr(out))
    if rc:
        raise OracleError(rc, "hash_lookup")
    return out


def sort_merge_join(r: np.ndarray, s: np.ndarray, key_off_r: int, key_off_s: int, key_bytes: int, lib=None):
    """Sort-merge join (Section 4.1): rows R[i] || S[j] for every pair of equal
    join keys, ordered by key (memcmp), then i, then j."""
    lib = lib or load()
    a = _records(r, r.shape[1])
    b = _records(s, s.shape[1])
    n = ctypes.c_int64()
    rc = lib.oracle_sort_merge_join(_ptr(a), a.shape[0], a.shape[1], key_off_r, _ptr(b), b.shape[0], b.shape[1],
                                    key_off_s, key_bytes, ctypes.c_void_p(0), 0, ctypes.byref(n))
    if rc not in (OK, ERANGE):
        raise OracleError(rc, "sort_merge_join")
    out = np.empty((n.value, a.shape[1] + b.shape[1]), dtype=np.uint8)
    if n.value:
        rc = lib.oracle_sort_merge_join(_ptr(a), a.shape[0], a.shape[1], key_off_r, _ptr(b), b.shape[0],
                                        b.shape[1], key_off_s, key_bytes, _ptr(out), n.value, ctypes.byref(n))
        if rc:
            raise OracleError(rc, "sort_merge_join")
    return out


BTREE_FANOUT = 32


def btree_shape(n: int, lib=None) -> list:
    """Nodes per level of the enhanced B+ tree over n entries, leaf level first."""
    lib = lib or load()
    nodes = np.zeros(16, dtype=np.int64)
    levels = lib.oracle_btree_shape(n, _ptr(nodes), 16)
    if levels < 1:
        raise OracleError(EINVAL, "btree_shape")
    return [int(x) for x in nodes[:levels]]


def btree_build(keys: np.ndarray, lib=None):
    """The enhanced B+ tree of Section 4.2.3 over uint32 keys (rid = position).

    Returns (leaf_keys uint32, leaf_rids int32, [level 1, level 2, ...]) where
    level l is a (nodes, 32) uint32 array of the largest key under each child."""
    lib = lib or load()
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    shape = btree_shape(k.size, lib)
    leaf_keys = np.empty(shape[0] * BTREE_FANOUT, dtype=np.uint32)
    leaf_rids = np.empty(shape[0] * BTREE_FANOUT, dtype=np.int32)
    inner = np.empty(max(1, sum(shape[1:])) * BTREE_FANOUT, dtype=np.uint32)
    rc = lib.oracle_btree_build(_ptr(k), k.size, _ptr(leaf_keys), _ptr(leaf_rids), _ptr(inner))
    if rc:
        raise OracleError(rc, "btree_build")
    levels, at = [], 0
    for c in shape[1:]:
        levels.append(inner[at:at + c * BTREE_FANOUT].reshape(c, BTREE_FANOUT).copy())
        at += c * BTREE_FANOUT
    return leaf_keys, leaf_rids, levels


def btree_lookup(tree, n: int, queries: np.ndarray, lib=None) -> np.ndarray:
    """Batch lookup by walking the tree from the root (Section 4.2.3): the rid
    of the first entry whose key equals the query, or -1."""
    lib = lib or load()
    leaf_keys, leaf_rids, levels = tree
    inner = np.concatenate([lv.reshape(-1) for lv in levels]) if levels else np.zeros(1, dtype=np.uint32)
    inner = np.ascontiguousarray(inner, dtype=np.uint32)
    q = np.ascontiguousarray(queries, dtype=np.uint32)
    out = np.empty(q.size, dtype=np.int32)
    rc = lib.oracle_btree_lookup(_ptr(np.ascontiguousarray(leaf_keys, dtype=np.uint32)),
                                 _ptr(np.ascontiguousarray(leaf_rids, dtype=np.int32)), _ptr(inner), n, _ptr(q),
                                 q.size, _ptr(out))
    if rc:
        raise OracleError(rc, "btree_lookup")
    return out
