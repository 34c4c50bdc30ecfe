"""ctypes binding over libdpg (include/dpg.h).

Argument marshalling only: every step of every operation runs in the HIP
kernels of libdpg.so.  Device buffers are torch tensors (or raw device
addresses); the stream is torch's current stream unless one is given.  If the
library has not been built, :func:`lib` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpg.so")

OK, ERR_INVALID_ARG, ERR_RID_OUT_OF_RANGE, ERR_FK_OUT_OF_RANGE = 0, 1, 2, 3
ERR_WORKSPACE_TOO_SMALL, ERR_UNSUPPORTED, ERR_HIP, ERR_BUSY = 4, 5, 6, 7

ALGO_AUTO, ALGO_DIRECT, ALGO_DPG = 0, 1, 2
JOIN_FACT_ORDER, JOIN_DIM_ORDER = 0, 1
PROBE_AUTO, PROBE_CACHED, PROBE_LDS = 0, 1, 2
OPT_LOG2_RUN, OPT_PROBE, OPT_DIST_TILE, OPT_XCD_REMAP, OPT_USE_TUNED, OPT_DISTRIBUTE, OPT_GATHER = 1, 2, 3, 4, 5, 6, 7
DIST_AUTO, DIST_APPEND, DIST_PARTITION, DIST_SAMPLED, DIST_TWO_PASS = 0, 1, 2, 3, 4
GATHER_AUTO, GATHER_CACHED, GATHER_LDS, GATHER_NONE = 0, 1, 2, 3  # NONE: the probe scatters (two-phase DPG)

_VP, _I32, _I64, _SZ, _DBL = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double


class DPGError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().dpg_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})")


class Plan(ctypes.Structure):
    _fields_ = [("algo", _I32), ("probe", _I32), ("log2_run", _I32), ("dist_tile", _I32),
                ("distribute", _I32), ("gather", _I32), ("n_runs", _I64), ("n_tiles", _I64), ("workspace_bytes", _SZ),
                ("ws_run_off", _SZ), ("ws_rid_run", _SZ), ("ws_internal", _SZ)]


REQ_RETRIEVE, REQ_FK_JOIN = 0, 1


class Request(ctypes.Structure):
    """dpg_request: one retrieval or join of a batch."""
    _fields_ = [("kind", _I32), ("algo", _I32), ("src", _VP), ("n_src", _I64), ("rec_bytes", _I32),
                ("fact_bytes", _I32), ("rids", _VP), ("fact", _VP), ("n", _I64), ("fk_offset", _I32),
                ("order", _I32), ("dst", _VP), ("workspace", _VP), ("workspace_bytes", _SZ)]


def retrieve_request(src, rids, dst, algo: int = ALGO_AUTO) -> Request:
    return Request(REQ_RETRIEVE, algo, _addr(src), src.shape[0], _rec_bytes(src), 0, _addr(rids), None,
                   rids.numel(), 0, 0, _addr(dst))


def join_request(fact, dim, dst, fk_offset: int = 0, order: int = 0, algo: int = ALGO_AUTO) -> Request:
    return Request(REQ_FK_JOIN, algo, _addr(dim), dim.shape[0], _rec_bytes(dim), _rec_bytes(fact), None,
                   _addr(fact), fact.shape[0], fk_offset, order, _addr(dst))


TICKET_QUEUED, TICKET_ADMITTED, TICKET_RUNNING, TICKET_DONE, TICKET_FAILED = 0, 1, 2, 3, 4


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena", _VP), ("arena_bytes", _SZ), ("max_inflight", _I32), ("max_batch_requests", _I32),
                ("use_graph", _I32), ("batch_max_kib", _I32), ("batch_window_us", _I32), ("reserved", _I32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _I64), ("completed", _I64), ("failed", _I64), ("batches", _I64),
                ("p50_ms", _DBL), ("p99_ms", _DBL), ("max_ms", _DBL), ("mean_ms", _DBL),
                ("bytes_delivered", _DBL), ("span_s", _DBL), ("arena_in_use", _SZ), ("arena_high_water", _SZ),
                ("launch_s", _DBL)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/dpg.h
SIGNATURES = {
    "dpg_create": (_I32, [ctypes.c_int, ctypes.POINTER(_VP)]),
    "dpg_destroy": (None, [_VP]),
    "dpg_status_string": (ctypes.c_char_p, [_I32]),
    "dpg_set_option": (_I32, [_VP, _I32, _I64]),
    "dpg_get_option": (_I32, [_VP, _I32, ctypes.POINTER(_I64)]),
    "dpg_plan_retrieve": (_I32, [_VP, _I64, _I32, _I64, _I32, ctypes.POINTER(Plan)]),
    "dpg_retrieve_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I64, _I32]),
    "dpg_retrieve": (_I32, [_VP, _VP, _I64, _I32, _VP, _I64, _VP, _VP, _SZ, _I32, _I32, _VP]),
    "dpg_retrieve_noalloc": (_I32, [_VP, _VP, _I64, _I32, _VP, _I64, _VP, _I32, _I32, _VP]),
    "dpg_sort_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I32, _I32, _I32]),
    "dpg_sort_records": (_I32, [_VP, _VP, _I64, _I32, _I32, _I32, _VP, _VP, _VP, _SZ, _I32, _VP]),
    "dpg_fk_join_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I32, _I64, _I32, _I32, _I32]),
    "dpg_fk_join": (_I32, [_VP, _VP, _I64, _I32, _I32, _VP, _I64, _I32, _VP, _I32, _VP, _SZ, _I32, _I32, _VP]),
    "dpg_sort_merge_join_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I32, _I64, _I32, _I32, _I32, _I32]),
    "dpg_sort_merge_join": (_I32, [_VP, _VP, _I64, _I32, _I32, _VP, _I64, _I32, _I32, _I32, _VP, _I64,
                                   ctypes.POINTER(_I64), _VP, _SZ, _I32, _VP]),
    "dpg_sort_merge_join_async": (_I32, [_VP, _VP, _I64, _I32, _I32, _VP, _I64, _I32, _I32, _I32, _VP, _I64, _VP,
                                         _VP, _SZ, _I32, _VP]),
    "dpg_hash_index_bytes": (_SZ, [_I64, _I32]),
    "dpg_hash_ov_off_offset": (_SZ, [_I32]),
    "dpg_hash_ov_offset": (_SZ, [_I32]),
    "dpg_hash_build_workspace_bytes": (_SZ, [_VP, _I64, _I32]),
    "dpg_hash_build": (_I32, [_VP, _VP, _I64, _I32, _VP, _SZ, _VP, _SZ, _VP]),
    "dpg_hash_lookup_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I64, _I32]),
    "dpg_hash_lookup": (_I32, [_VP, _VP, _I64, _I32, _VP, _I64, _VP, _VP, _SZ, _I32, _VP]),
    "dpg_key_join_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I32, _I64, _I32, _I32, _I32, _I32]),
    "dpg_key_join": (_I32, [_VP, _VP, _I64, _I32, _I32, _VP, _I64, _I32, _VP, _I32, _VP, _I32, _VP, _SZ, _I32,
                            _I32, _VP]),
    "dpg_btree_bytes": (_SZ, [_I64]),
    "dpg_btree_levels": (_I32, [_I64]),
    "dpg_btree_level_offset": (_SZ, [_I64, _I32]),
    "dpg_btree_rids_offset": (_SZ, [_I64]),
    "dpg_btree_build_workspace_bytes": (_SZ, [_VP, _I64]),
    "dpg_btree_build": (_I32, [_VP, _VP, _I64, _VP, _SZ, _VP, _SZ, _VP]),
    "dpg_btree_lookup_workspace_bytes": (_SZ, [_VP, _I64, _I64, _I32]),
    "dpg_btree_lookup": (_I32, [_VP, _VP, _I64, _VP, _I64, _VP, _VP, _SZ, _I32, _VP]),
    "dpg_batch_request_workspace_bytes": (_SZ, [_VP, ctypes.POINTER(Request)]),
    "dpg_batch_workspace_bytes": (_SZ, [_VP, ctypes.POINTER(Request), _I32]),
    "dpg_batch_run": (_I32, [_VP, ctypes.POINTER(Request), _I32, _VP, _SZ, _VP]),
    "dpg_batch_graph_workspace_bytes": (_SZ, [_VP, _I32]),
    "dpg_batch_graph_create": (_I32, [_VP, _I32, _VP, _SZ, _VP, ctypes.POINTER(_VP)]),
    "dpg_batch_graph_launch": (_I32, [_VP, ctypes.POINTER(Request), _I32, _VP]),
    "dpg_batch_graph_request_done": (_I32, [_VP, _I32]),
    "dpg_batch_graph_destroy": (None, [_VP]),
    "dpg_arena_create": (_I32, [ctypes.c_size_t, _SZ, _SZ, ctypes.POINTER(_VP)]),
    "dpg_arena_alloc": (_I32, [_VP, _SZ, ctypes.POINTER(ctypes.c_size_t)]),
    "dpg_arena_free": (_I32, [_VP, ctypes.c_size_t]),
    "dpg_arena_stats": (_I32, [_VP, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ), ctypes.POINTER(_SZ),
                               ctypes.POINTER(_SZ)]),
    "dpg_arena_destroy": (None, [_VP]),
    "dpg_server_create": (_I32, [_VP, ctypes.POINTER(ServerConfig), ctypes.POINTER(_VP)]),
    "dpg_server_submit": (_I32, [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "dpg_server_submit_many": (_I32, [_VP, ctypes.POINTER(Request), _I32, ctypes.POINTER(ctypes.c_uint64)]),
    "dpg_server_poll": (_I32, [_VP, ctypes.c_uint64, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                               ctypes.POINTER(_VP), ctypes.POINTER(_DBL)]),
    "dpg_server_next_completed": (_I32, [_VP, _I32, ctypes.POINTER(ctypes.c_uint64)]),
    "dpg_server_release": (_I32, [_VP, ctypes.c_uint64]),
    "dpg_server_stats_get": (_I32, [_VP, ctypes.POINTER(ServerStats)]),
    "dpg_server_reset_stats": (_I32, [_VP]),
    "dpg_server_destroy": (None, [_VP]),
    "dpg_autotune_workspace_bytes": (_SZ, [_VP, _I64, _I32, _I64]),
    "dpg_autotune_retrieve": (_I32, [_VP, _VP, _I64, _I32, _VP, _I64, _VP, _VP, _SZ, _I32, _I32, _VP,
                                     ctypes.POINTER(Plan), ctypes.POINTER(_DBL)]),
    "dpg_tune_count": (_I32, [_VP]),
    "dpg_tune_clear": (_I32, [_VP]),
    "dpg_tune_save": (_I32, [_VP, ctypes.c_char_p]),
    "dpg_tune_load": (_I32, [_VP, ctypes.c_char_p]),
    "dpg_profile_enable": (_I32, [_VP, ctypes.c_int]),
    "dpg_stream_copy": (_I32, [_VP, _VP, _VP, _SZ, _I32, _I32, _VP]),
    "dpg_profile_reset": (_I32, [_VP]),
    "dpg_profile_collect": (_I32, [_VP, ctypes.POINTER(_I32)]),
    "dpg_profile_entry": (_I32, [_VP, _I32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_I64),
                                 ctypes.POINTER(_DBL), ctypes.POINTER(_DBL)]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libdpg.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_cs_0308004_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(status: int, what: str):
    if status != OK:
        raise DPGError(status, what)


def _addr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("tensors passed to libdpg must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _rec_bytes(t) -> int:
    if t.dim() != 2:
        raise ValueError("record tensors are (n, rec_bytes) uint8")
    return t.shape[1] * t.element_size()


class Context:
    """Owns a dpg_ctx bound to one HIP device."""

    def __init__(self, device: int = 0):
        h = _VP()
        _check(lib().dpg_create(device, ctypes.byref(h)), "dpg_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().dpg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- options -------------------------------------------------------
    def set_option(self, option: int, value: int):
        _check(lib().dpg_set_option(self.handle, option, value), "dpg_set_option")

    def get_option(self, option: int) -> int:
        v = _I64()
        _check(lib().dpg_get_option(self.handle, option, ctypes.byref(v)), "dpg_get_option")
        return v.value

    # ---- retrieval -----------------------------------------------------
    def plan_retrieve(self, n_src: int, rec_bytes: int, n_rids: int, algo: int = ALGO_AUTO) -> Plan:
        return plan_retrieve(n_src, rec_bytes, n_rids, algo, self)

    def retrieve_workspace_bytes(self, n_src: int, rec_bytes: int, n_rids: int, algo: int = ALGO_AUTO) -> int:
        return lib().dpg_retrieve_workspace_bytes(self.handle, n_src, rec_bytes, n_rids, algo)

    def retrieve(self, src, rids, dst=None, algo: int = ALGO_AUTO, check_rids: bool = False, workspace=None,
                 stream=None):
        """dst[i] = src[rids[i]]; src is an (N, R) uint8 device tensor, rids int32."""
        import torch

        n_src, rec_bytes = src.shape[0], _rec_bytes(src)
        n_rids = rids.numel()
        if dst is None:
            dst = torch.empty((n_rids, src.shape[1]), dtype=src.dtype, device=src.device)
        need = self.retrieve_workspace_bytes(n_src, rec_bytes, n_rids, algo)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=src.device)
        st = lib().dpg_retrieve(self.handle, _addr(src), n_src, rec_bytes, _addr(rids), n_rids, _addr(dst),
                                _addr(workspace), workspace.numel(), algo, int(check_rids), _stream(stream))
        _check(st, "dpg_retrieve")
        return dst

    # ---- autotuning ----------------------------------------------------
    def autotune_retrieve(self, src, rids, dst=None, reps: int = 3, dpg_only: bool = False, stream=None):
        """Time the candidate plans; returns (best Plan, ms per retrieval)."""
        import torch

        n_src, rec_bytes = src.shape[0], _rec_bytes(src)
        n = rids.numel()
        if dst is None:
            dst = torch.empty((n, src.shape[1]), dtype=src.dtype, device=src.device)
        need = lib().dpg_autotune_workspace_bytes(self.handle, n_src, rec_bytes, n)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=src.device)
        best, ms = Plan(), _DBL()
        _check(lib().dpg_autotune_retrieve(self.handle, _addr(src), n_src, rec_bytes, _addr(rids), n, _addr(dst),
                                           _addr(ws), ws.numel(), reps, int(dpg_only), _stream(stream),
                                           ctypes.byref(best), ctypes.byref(ms)), "dpg_autotune_retrieve")
        return best, ms.value

    def tune_count(self) -> int:
        return lib().dpg_tune_count(self.handle)

    def tune_clear(self):
        _check(lib().dpg_tune_clear(self.handle), "dpg_tune_clear")

    def tune_save(self, path: str):
        _check(lib().dpg_tune_save(self.handle, path.encode()), "dpg_tune_save")

    def tune_load(self, path: str):
        _check(lib().dpg_tune_load(self.handle, path.encode()), "dpg_tune_load")

    # ---- sorting -------------------------------------------------------
    def sort_workspace_bytes(self, n: int, rec_bytes: int, key_offset: int = 0, key_bytes: int = 10,
                             algo: int = ALGO_AUTO) -> int:
        return lib().dpg_sort_workspace_bytes(self.handle, n, rec_bytes, key_offset, key_bytes, algo)

    def sort_records(self, src, key_offset: int = 0, key_bytes: int = 10, dst=None, perm=None,
                     algo: int = ALGO_AUTO, workspace=None, stream=None, want_perm: bool = True):
        """Sort (N, R) uint8 records by key bytes; returns (dst, perm or None)."""
        import torch

        n, rec_bytes = src.shape[0], _rec_bytes(src)
        if dst is None:
            dst = torch.empty_like(src)
        if perm is None and want_perm:
            perm = torch.empty(n, dtype=torch.int32, device=src.device)
        if workspace is None:
            need = self.sort_workspace_bytes(n, rec_bytes, key_offset, key_bytes, algo)
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=src.device)
        st = lib().dpg_sort_records(self.handle, _addr(src), n, rec_bytes, key_offset, key_bytes, _addr(dst),
                                    _addr(perm), _addr(workspace), workspace.numel(), algo, _stream(stream))
        _check(st, "dpg_sort_records")
        return dst, perm

    # ---- joins ---------------------------------------------------------
    def fk_join_workspace_bytes(self, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes, order, algo=ALGO_AUTO):
        return lib().dpg_fk_join_workspace_bytes(self.handle, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes,
                                                 order, algo)

    def fk_join(self, fact, dim, fk_offset: int = 0, order: int = JOIN_FACT_ORDER, out=None, algo: int = ALGO_AUTO,
                check_fk: bool = False, workspace=None, stream=None):
        """Joined rows fact || dim[fk]; fact is (F, fact_bytes) uint8, dim (D, dim_bytes) uint8."""
        import torch

        n_fact, fb = fact.shape[0], _rec_bytes(fact)
        n_dim, db = dim.shape[0], _rec_bytes(dim)
        if out is None:
            out = torch.empty((n_fact, fb + db), dtype=torch.uint8, device=fact.device)
        if workspace is None:
            need = self.fk_join_workspace_bytes(n_fact, fb, fk_offset, n_dim, db, order, algo)
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=fact.device)
        st = lib().dpg_fk_join(self.handle, _addr(fact), n_fact, fb, fk_offset, _addr(dim), n_dim, db, _addr(out),
                               order, _addr(workspace), workspace.numel(), algo, int(check_fk), _stream(stream))
        _check(st, "dpg_fk_join")
        return out

    # ---- sort-merge join (Section 4.1) ------------------------------------
    def sort_merge_join_workspace_bytes(self, n_r: int, rec_r: int, key_off_r: int, n_s: int, rec_s: int,
                                        key_off_s: int, key_bytes: int, algo: int = ALGO_AUTO) -> int:
        return lib().dpg_sort_merge_join_workspace_bytes(self.handle, n_r, rec_r, key_off_r, n_s, rec_s, key_off_s,
                                                         key_bytes, algo)

    def sort_merge_join(self, r, s, key_off_r: int, key_off_s: int, key_bytes: int, algo: int = ALGO_AUTO,
                        out=None, workspace=None, stream=None):
        """Rows R[i] || S[j] for every pair of equal join keys, ordered by key,
        then i, then j.  r, s: (n, rec) uint8 device tensors.  Returns a view
        of the first result rows of `out` ((capacity, rec_r + rec_s) uint8;
        default: as many rows as the larger relation).  When the result does
        not fit, a new output of the exact size is allocated and the call
        repeated."""
        import torch

        nr, ns = r.shape[0], s.shape[0]
        rec_r, rec_s = _rec_bytes(r), _rec_bytes(s)
        need = self.sort_merge_join_workspace_bytes(nr, rec_r, key_off_r, ns, rec_s, key_off_s, key_bytes, algo)
        if need == 0:
            raise DPGError(ERR_INVALID_ARG, "dpg_sort_merge_join_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=r.device)
        if out is None:
            out = torch.empty((max(nr, ns, 1), rec_r + rec_s), dtype=torch.uint8, device=r.device)
        for _ in range(2):
            n_out = _I64()
            st = lib().dpg_sort_merge_join(self.handle, _addr(r), nr, rec_r, key_off_r, _addr(s), ns, rec_s,
                                           key_off_s, key_bytes, _addr(out), out.shape[0], ctypes.byref(n_out),
                                           _addr(workspace), workspace.numel(), algo, _stream(stream))
            if st == ERR_WORKSPACE_TOO_SMALL and n_out.value > out.shape[0]:
                out = torch.empty((n_out.value, rec_r + rec_s), dtype=torch.uint8, device=r.device)
                continue
            _check(st, "dpg_sort_merge_join")
            return out[: n_out.value]
        raise DPGError(ERR_WORKSPACE_TOO_SMALL, "dpg_sort_merge_join")

    def sort_merge_join_async(self, r, s, key_off_r: int, key_off_s: int, key_bytes: int, out, rows,
                              algo: int = ALGO_AUTO, workspace=None, stream=None):
        """The same join without a host synchronization: `out` is a
        (capacity, rec_r + rec_s) uint8 device tensor, `rows` a one-element
        int64 device tensor that receives the number of result rows (at most
        `capacity` of them are written)."""
        import torch

        nr, ns = r.shape[0], s.shape[0]
        rec_r, rec_s = _rec_bytes(r), _rec_bytes(s)
        if workspace is None:
            need = self.sort_merge_join_workspace_bytes(nr, rec_r, key_off_r, ns, rec_s, key_off_s, key_bytes, algo)
            if need == 0:
                raise DPGError(ERR_INVALID_ARG, "dpg_sort_merge_join_workspace_bytes")
            workspace = torch.empty(need, dtype=torch.uint8, device=r.device)
        _check(lib().dpg_sort_merge_join_async(self.handle, _addr(r), nr, rec_r, key_off_r, _addr(s), ns, rec_s,
                                               key_off_s, key_bytes, _addr(out), out.shape[0], _addr(rows),
                                               _addr(workspace), workspace.numel(), algo, _stream(stream)),
               "dpg_sort_merge_join_async")
        return workspace

    # ---- hash index and batch lookup (Section 4.2.3) --------------------
    def hash_build(self, keys, log2_slots: int, stream=None):
        """Build the hash index of a uint32 key tensor (rid = position); returns
        the index as a uint8 device tensor."""
        import torch

        n = keys.numel()
        nbytes = lib().dpg_hash_index_bytes(n, log2_slots)
        if nbytes == 0:
            raise DPGError(ERR_INVALID_ARG, "dpg_hash_index_bytes")
        index = torch.empty(nbytes, dtype=torch.uint8, device=keys.device)
        need = lib().dpg_hash_build_workspace_bytes(self.handle, n, log2_slots)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
        _check(lib().dpg_hash_build(self.handle, _addr(keys), n, log2_slots, _addr(index), index.numel(), _addr(ws),
                                    ws.numel(), _stream(stream)), "dpg_hash_build")
        return index

    def hash_lookup_workspace_bytes(self, n_keys: int, log2_slots: int, n_queries: int, algo: int = ALGO_AUTO) -> int:
        return lib().dpg_hash_lookup_workspace_bytes(self.handle, n_keys, log2_slots, n_queries, algo)

    def hash_lookup(self, index, n_keys: int, log2_slots: int, queries, rids=None, algo: int = ALGO_AUTO,
                    workspace=None, stream=None):
        """rids[i] = smallest rid whose key equals queries[i], or -1."""
        import torch

        m = queries.numel()
        if rids is None:
            rids = torch.empty(m, dtype=torch.int32, device=queries.device)
        if workspace is None:
            need = self.hash_lookup_workspace_bytes(n_keys, log2_slots, m, algo)
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=queries.device)
        _check(lib().dpg_hash_lookup(self.handle, _addr(index), n_keys, log2_slots, _addr(queries), m, _addr(rids),
                                     _addr(workspace), workspace.numel(), algo, _stream(stream)), "dpg_hash_lookup")
        return rids

    def key_join_workspace_bytes(self, n_fact: int, fact_bytes: int, fk_offset: int, n_dim: int, dim_bytes: int,
                                 log2_slots: int, order: int = 0, algo: int = ALGO_AUTO) -> int:
        return lib().dpg_key_join_workspace_bytes(self.handle, n_fact, fact_bytes, fk_offset, n_dim, dim_bytes,
                                                  log2_slots, order, algo)

    def key_join(self, fact, dim, fk_offset: int, index, log2_slots: int, order: int = 0, out=None,
                 algo: int = ALGO_AUTO, workspace=None, stream=None, check_fk: bool = True):
        """Join fact rows to the dimension row holding their fk as a key
        (index: the hash index of the dimension keys, rid = dimension row)."""
        import torch

        nf, nd = fact.shape[0], dim.shape[0]
        fb, db = _rec_bytes(fact), _rec_bytes(dim)
        if out is None:
            out = torch.empty((nf, fb + db), dtype=torch.uint8, device=fact.device)
        if workspace is None:
            need = self.key_join_workspace_bytes(nf, fb, fk_offset, nd, db, log2_slots, order, algo)
            if need == 0:
                raise DPGError(ERR_INVALID_ARG, "dpg_key_join_workspace_bytes")
            workspace = torch.empty(need, dtype=torch.uint8, device=fact.device)
        _check(lib().dpg_key_join(self.handle, _addr(fact), nf, fb, fk_offset, _addr(dim), nd, db, _addr(index),
                                  log2_slots, _addr(out), order, _addr(workspace), workspace.numel(), algo,
                                  int(check_fk), _stream(stream)), "dpg_key_join")
        return out

    # ---- enhanced B+ tree and batch lookup (Section 4.2.3) -------------
    def btree_build(self, keys, stream=None):
        """Build the enhanced B+ tree of a uint32 key tensor (rid = position);
        returns the tree as a uint8 device tensor."""
        import torch

        n = keys.numel()
        nbytes = lib().dpg_btree_bytes(n)
        if nbytes == 0:
            raise DPGError(ERR_INVALID_ARG, "dpg_btree_bytes")
        tree = torch.empty(nbytes, dtype=torch.uint8, device=keys.device)
        need = lib().dpg_btree_build_workspace_bytes(self.handle, n)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
        _check(lib().dpg_btree_build(self.handle, _addr(keys), n, _addr(tree), tree.numel(), _addr(ws), ws.numel(),
                                     _stream(stream)), "dpg_btree_build")
        return tree

    def btree_lookup_workspace_bytes(self, n_keys: int, n_queries: int, algo: int = ALGO_AUTO) -> int:
        return lib().dpg_btree_lookup_workspace_bytes(self.handle, n_keys, n_queries, algo)

    def btree_lookup(self, tree, n_keys: int, queries, rids=None, algo: int = ALGO_AUTO, workspace=None,
                     stream=None):
        """rids[i] = smallest rid whose key equals queries[i], or -1."""
        import torch

        m = queries.numel()
        if rids is None:
            rids = torch.empty(m, dtype=torch.int32, device=queries.device)
        if workspace is None:
            need = self.btree_lookup_workspace_bytes(n_keys, m, algo)
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=queries.device)
        _check(lib().dpg_btree_lookup(self.handle, _addr(tree), n_keys, _addr(queries), m, _addr(rids),
                                      _addr(workspace), workspace.numel(), algo, _stream(stream)), "dpg_btree_lookup")
        return rids

    # ---- batches -------------------------------------------------------
    def batch_workspace_bytes(self, reqs) -> int:
        arr = (Request * len(reqs))(*reqs)
        return lib().dpg_batch_workspace_bytes(self.handle, arr, len(reqs))

    def batch_request_workspace_bytes(self, req) -> int:
        """Scratch of one request's steps inside a graph batch (0: direct work)."""
        return lib().dpg_batch_request_workspace_bytes(self.handle, ctypes.byref(req))

    def batch_run(self, reqs, workspace=None, stream=None):
        import torch

        arr = (Request * len(reqs))(*reqs)
        if workspace is None:
            need = lib().dpg_batch_workspace_bytes(self.handle, arr, len(reqs))
            if need == 0 and len(reqs):
                raise DPGError(ERR_INVALID_ARG, "dpg_batch_workspace_bytes")
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        _check(lib().dpg_batch_run(self.handle, arr, len(reqs), _addr(workspace), workspace.numel(),
                                   _stream(stream)), "dpg_batch_run")
        return workspace

    # ---- profiling -----------------------------------------------------
    def stream_copy(self, src, dst, vectors_per_lane: int = 8, nontemporal: bool = True, stream=None):
        """Plain device copy of src into dst (same byte size; the copy-ceiling kernel)."""
        nbytes = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nbytes:
            raise ValueError("src and dst differ in size")
        _check(lib().dpg_stream_copy(self.handle, _addr(src), _addr(dst), nbytes, vectors_per_lane,
                                     int(nontemporal), _stream(stream)), "dpg_stream_copy")

    def profile_enable(self, on: bool = True):
        _check(lib().dpg_profile_enable(self.handle, int(on)), "dpg_profile_enable")

    def profile_reset(self):
        _check(lib().dpg_profile_reset(self.handle), "dpg_profile_reset")

    def profile_collect(self) -> dict:
        """{kernel name: {"launches", "ms", "bytes"}} accumulated since the last reset."""
        n = _I32()
        _check(lib().dpg_profile_collect(self.handle, ctypes.byref(n)), "dpg_profile_collect")
        out = {}
        for i in range(n.value):
            name, launches, ms, by = ctypes.c_char_p(), _I64(), _DBL(), _DBL()
            _check(lib().dpg_profile_entry(self.handle, i, ctypes.byref(name), ctypes.byref(launches),
                                           ctypes.byref(ms), ctypes.byref(by)), "dpg_profile_entry")
            out[name.value.decode()] = {"launches": launches.value, "ms": ms.value, "bytes": by.value}
        return out


def plan_retrieve(n_src: int, rec_bytes: int, n_rids: int, algo: int = ALGO_AUTO, ctx: Context | None = None) -> Plan:
    p = Plan()
    _check(lib().dpg_plan_retrieve(ctx.handle if ctx else None, n_src, rec_bytes, n_rids, algo, ctypes.byref(p)),
           "dpg_plan_retrieve")
    return p


class BatchGraph:
    """A captured persistent-batch launch bound to its own workspace."""

    def __init__(self, ctx: Context, max_requests: int, stream):
        import torch

        need = lib().dpg_batch_graph_workspace_bytes(ctx.handle, max_requests)
        self.workspace = torch.empty(need, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        h = _VP()
        _check(lib().dpg_batch_graph_create(ctx.handle, max_requests, _addr(self.workspace), need, _stream(stream),
                                            ctypes.byref(h)), "dpg_batch_graph_create")
        self.handle = h

    def launch(self, reqs, stream):
        arr = (Request * len(reqs))(*reqs)
        _check(lib().dpg_batch_graph_launch(self.handle, arr, len(reqs), _stream(stream)), "dpg_batch_graph_launch")

    def request_done(self, index: int) -> bool:
        """Whether request `index` of the last launch has finished."""
        return bool(lib().dpg_batch_graph_request_done(self.handle, index))

    def close(self):
        if self.handle:
            lib().dpg_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Arena:
    """Host bookkeeping of a device address range (no device access)."""

    def __init__(self, base: int, size: int, align: int = 256):
        h = _VP()
        _check(lib().dpg_arena_create(base, size, align, ctypes.byref(h)), "dpg_arena_create")
        self.handle = h

    def alloc(self, nbytes: int):
        a = ctypes.c_size_t()
        st = lib().dpg_arena_alloc(self.handle, nbytes, ctypes.byref(a))
        if st == ERR_BUSY:
            return None
        _check(st, "dpg_arena_alloc")
        return a.value

    def free(self, addr: int):
        _check(lib().dpg_arena_free(self.handle, addr), "dpg_arena_free")

    def stats(self):
        v = [_SZ() for _ in range(4)]
        _check(lib().dpg_arena_stats(self.handle, *[ctypes.byref(x) for x in v]), "dpg_arena_stats")
        return dict(zip(("in_use", "high_water", "largest_free", "free_blocks"), (x.value for x in v)))

    def close(self):
        if self.handle:
            lib().dpg_arena_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a device arena of `arena_bytes`."""

    def __init__(self, ctx: Context, arena_bytes: int, max_inflight: int = 4, max_batch_requests: int = 64,
                 use_graph: bool = True, batch_max_kib: int = 0, batch_window_us: int = 0):
        import torch

        self.ctx = ctx
        self.arena_mem = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        torch.cuda.synchronize()
        cfg = ServerConfig(self.arena_mem.data_ptr(), arena_bytes, max_inflight, max_batch_requests,
                           int(use_graph), batch_max_kib, batch_window_us, 0)
        h = _VP()
        _check(lib().dpg_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "dpg_server_create")
        self.handle = h

    def submit(self, req: Request) -> int:
        t = ctypes.c_uint64()
        _check(lib().dpg_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "dpg_server_submit")
        return t.value

    def submit_many(self, reqs) -> list:
        n = len(reqs)
        arr = (Request * max(n, 1))(*reqs)
        t = (ctypes.c_uint64 * max(n, 1))()
        _check(lib().dpg_server_submit_many(self.handle, arr, n, t), "dpg_server_submit_many")
        return list(t[:n])

    def poll(self, ticket: int):
        state, status, dst, lat = _I32(), _I32(), _VP(), _DBL()
        _check(lib().dpg_server_poll(self.handle, ticket, ctypes.byref(state), ctypes.byref(status),
                                     ctypes.byref(dst), ctypes.byref(lat)), "dpg_server_poll")
        return state.value, status.value, dst.value, lat.value

    def next_completed(self, timeout_ms: int = 1000):
        t = ctypes.c_uint64()
        st = lib().dpg_server_next_completed(self.handle, timeout_ms, ctypes.byref(t))
        if st == ERR_BUSY:
            return None
        _check(st, "dpg_server_next_completed")
        return t.value

    def release(self, ticket: int):
        _check(lib().dpg_server_release(self.handle, ticket), "dpg_server_release")

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().dpg_server_stats_get(self.handle, ctypes.byref(s)), "dpg_server_stats_get")
        return s.as_dict()

    def reset_stats(self):
        _check(lib().dpg_server_reset_stats(self.handle), "dpg_server_reset_stats")

    def close(self):
        if self.handle:
            lib().dpg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def copy_device_bytes(addr: int, nbytes: int, device: int = 0):
    """A new uint8 device tensor holding nbytes copied from device address addr
    (hipMemcpy, device to device)."""
    global _hip
    import torch

    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [_VP, _VP, _SZ, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    out = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
    if nbytes:
        torch.cuda.synchronize()
        rc = _hip.hipMemcpy(out.data_ptr(), addr, nbytes, 3)  # hipMemcpyDeviceToDevice
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed: {rc}")
    return out
