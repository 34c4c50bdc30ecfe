"""Seeded synthetic inputs for record retrieval, sorting and joins.

This module holds no part of the retrieval method: it only makes inputs.  Both
the CPU oracle side (numpy, ``backend="numpy"``) and the GPU side (torch on a
device, ``backend="torch"``) draw from the same counter-based definitions, so a
value can be recomputed at any index without generating the rest:

* ``word(seed, stream, i)`` is the i-th output (0-based) of the splitmix64
  generator (Steele, Lea and Flood, OOPSLA 2014) whose state starts at
  ``stream_key(seed, stream)``.  Byte streams are the little-endian bytes of
  successive words.
* Random permutations use a 4-round balanced Feistel network on the smallest
  even number of bits covering n, with splitmix64 round functions, and cycle
  walking for n that is not a power of four (Black and Rogaway, CT-RSA 2002).
  It stands in for a uniform random permutation.
* Uniform draws in [0, n) take the top 53 bits of a word modulo n.
* Zipf ranks are drawn by inverse CDF against an integer threshold table that is
  built once on the host in float64, so CPU and GPU draws agree bit for bit.

Streams: 0 record bytes, 1 rids, 2 foreign keys, 3 request mix, 4 arrivals,
5 Zipf id permutation, 6 fact payload, 7 dimension payload.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 0x0308004

STREAM_RECORDS, STREAM_RIDS, STREAM_FK, STREAM_MIX, STREAM_ARRIVALS = 0, 1, 2, 3, 4
STREAM_ZIPF_PERM, STREAM_FACT, STREAM_DIM = 5, 6, 7

_MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB
_STREAM_MUL = 0xD1B54A32D192ED03


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _MIX1) & _MASK64
    z = ((z ^ (z >> 27)) * _MIX2) & _MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """Starting state of the splitmix64 generator for (seed, stream)."""
    return _mix64_int(seed * _GOLDEN + stream * _STREAM_MUL + 1)


# --------------------------------------------------------------------------
# Array backends: numpy works in uint64, torch in int64 with the same bits.
# --------------------------------------------------------------------------
class _Numpy:
    name = "numpy"

    def __init__(self):
        self.device = None

    def arange(self, start, stop):
        return np.arange(start, stop, dtype=np.uint64)

    def asarray(self, a):
        return np.asarray(a).astype(np.uint64)

    def const(self, c):
        return np.uint64(c & _MASK64)

    def shr(self, x, k):
        return x >> np.uint64(k)

    def shl(self, x, k):
        return x << np.uint64(k)

    def to_i64(self, x):
        return x.astype(np.int64)


class _Torch:
    name = "torch"

    def __init__(self, device):
        import torch

        self.torch = torch
        self.device = torch.device(device)

    def arange(self, start, stop):
        return self.torch.arange(start, stop, dtype=self.torch.int64, device=self.device)

    def asarray(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.int64)
        return t.as_tensor(np.asarray(a).astype(np.int64), device=self.device)

    def const(self, c):
        c &= _MASK64
        return c - (1 << 64) if c >= (1 << 63) else c

    def shr(self, x, k):
        return (x >> k) & ((1 << (64 - k)) - 1)

    def shl(self, x, k):
        return x << k

    def to_i64(self, x):
        return x


def _backend(backend: str, device=None):
    if backend == "numpy":
        return _Numpy()
    if backend == "torch":
        return _Torch(device or "cpu")
    raise ValueError(f"unknown backend {backend!r}")


def _mix64(xp, z):
    z = (z ^ xp.shr(z, 30)) * xp.const(_MIX1)
    z = (z ^ xp.shr(z, 27)) * xp.const(_MIX2)
    return z ^ xp.shr(z, 31)


def _words(xp, key: int, idx):
    # i-th splitmix64 output from state `key`: mix(key + (i + 1) * golden)
    return _mix64(xp, xp.const(key) + (idx + 1) * xp.const(_GOLDEN))


def words(seed: int, stream: int, idx, backend="numpy", device=None):
    """splitmix64 words at indices ``idx`` (uint64 for numpy, int64 bits for torch)."""
    xp = _backend(backend, device)
    return _words(xp, stream_key(seed, stream), xp.asarray(idx))


# --------------------------------------------------------------------------
# Byte records
# --------------------------------------------------------------------------
def _as_bytes(xp, w):
    if xp.name == "numpy":
        return np.ascontiguousarray(w).view(np.uint8)
    return w.contiguous().view(xp.torch.uint8)


def record_bytes(n: int, rec_bytes: int, seed: int, stream: int = STREAM_RECORDS, first: int = 0,
                 backend="numpy", device=None, out=None, chunk_records: int = 1 << 22):
    """Records first .. first+n-1 of the byte stream, as an (n, rec_bytes) uint8 array.

    Record r is bytes [r*rec_bytes, (r+1)*rec_bytes) of the little-endian byte
    stream of ``word(seed, stream, 0), word(seed, stream, 1), ...``.  With the
    torch backend, ``out`` may be a preallocated (n, rec_bytes) uint8 tensor;
    generation then proceeds in chunks to bound temporary memory.
    """
    xp = _backend(backend, device)
    key = stream_key(seed, stream)
    if out is None:
        if xp.name == "numpy":
            out = np.empty((n, rec_bytes), dtype=np.uint8)
        else:
            out = xp.torch.empty((n, rec_bytes), dtype=xp.torch.uint8, device=xp.device)
    for c0 in range(0, n, chunk_records):
        c1 = min(n, c0 + chunk_records)
        b0 = (first + c0) * rec_bytes
        b1 = (first + c1) * rec_bytes
        w0, w1 = b0 // 8, -(-b1 // 8)
        w = _words(xp, key, xp.arange(w0, w1))
        by = _as_bytes(xp, w)[b0 - w0 * 8: b1 - w0 * 8]
        out[c0:c1] = by.reshape(c1 - c0, rec_bytes)
    return out


def records_at(idx, rec_bytes: int, seed: int, stream: int = STREAM_RECORDS) -> np.ndarray:
    """Records at arbitrary indices (numpy), without generating the others."""
    idx = np.asarray(idx, dtype=np.int64).reshape(-1)
    xp = _Numpy()
    key = stream_key(seed, stream)
    nw = rec_bytes // 8 + 2
    first_word = (idx * rec_bytes) // 8
    widx = (first_word[:, None] + np.arange(nw, dtype=np.int64)[None, :]).astype(np.uint64)
    by = _words(xp, key, widx).view(np.uint8).reshape(idx.size, nw * 8)
    off = (idx * rec_bytes - first_word * 8)
    cols = off[:, None] + np.arange(rec_bytes)[None, :]
    return np.take_along_axis(by, cols, axis=1)


# --------------------------------------------------------------------------
# Permutations and index draws
# --------------------------------------------------------------------------
def _feistel_bits(n: int) -> int:
    k = max(2, (n - 1).bit_length())
    return k + (k & 1)


def permutation_at(n: int, idx, seed: int, stream: int = STREAM_RIDS, backend="numpy", device=None):
    """pi(idx) for a seeded pseudo-random permutation pi of [0, n)."""
    if n <= 0:
        raise ValueError("n must be positive")
    xp = _backend(backend, device)
    k = _feistel_bits(n)
    h = k // 2
    mask = xp.const((1 << h) - 1)
    base = stream_key(seed, stream)
    round_keys = [xp.const(_mix64_int(base + (j + 1) * _GOLDEN)) for j in range(4)]

    def once(x):
        a = xp.shr(x, h)
        b = x & mask
        for rk in round_keys:
            a, b = b, a ^ (_mix64(xp, b ^ rk) & mask)
        return xp.shl(a, h) | b

    y = once(xp.asarray(idx))
    if (1 << k) == n:
        return xp.to_i64(y)
    nn = xp.const(n)
    while True:
        bad = y >= nn
        if not bool(bad.any()):
            break
        y[bad] = once(y[bad])
    return xp.to_i64(y)


def rids_permutation(n: int, seed: int, backend="numpy", device=None, first: int = 0, count: int | None = None):
    """rids[i] = pi(i): a pseudo-random permutation of [0, n), as int32."""
    count = n - first if count is None else count
    xp = _backend(backend, device)
    r = permutation_at(n, xp.arange(first, first + count), seed, STREAM_RIDS, backend, device)
    return r.astype(np.int32) if backend == "numpy" else r.to(xp.torch.int32)


def uniform_at(n: int, idx, seed: int, stream: int, backend="numpy", device=None):
    """Uniform draws in [0, n) at counter indices idx (53-bit word prefix mod n)."""
    xp = _backend(backend, device)
    w = _words(xp, stream_key(seed, stream), xp.asarray(idx))
    return xp.to_i64(xp.shr(w, 11) % xp.const(n))


def rids_uniform(n_src: int, n_rids: int, seed: int, backend="numpy", device=None):
    """n_rids rids drawn uniformly with replacement from [0, n_src), as int32."""
    xp = _backend(backend, device)
    r = uniform_at(n_src, xp.arange(0, n_rids), seed, STREAM_RIDS, backend, device)
    return r.astype(np.int32) if backend == "numpy" else r.to(xp.torch.int32)


def rids_blocked(n: int, rec_bytes: int, seed: int, backend="numpy", device=None):
    """Blocked permutation: the source is cut into runs of floor(4096 / rec_bytes)
    records (the last run may be short); the runs are visited in a seeded random
    order and each run's rids are listed in ascending order."""
    run = max(1, 4096 // rec_bytes)
    n_runs = -(-n // run)
    order = np.asarray(_to_numpy(permutation_at(n_runs, np.arange(n_runs, dtype=np.uint64), seed,
                                                STREAM_RIDS, "numpy")), dtype=np.int64)
    lens = np.minimum(run, n - order * run)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    pos = np.arange(n, dtype=np.int64)
    which = np.repeat(np.arange(n_runs), lens)
    rids = (order[which] * run + (pos - starts[which])).astype(np.int32)
    if backend == "numpy":
        return rids
    import torch

    return torch.as_tensor(rids, device=device)


def _to_numpy(x):
    if isinstance(x, np.ndarray):
        return x
    return x.cpu().numpy()


# --------------------------------------------------------------------------
# Zipf foreign keys and join tables
# --------------------------------------------------------------------------
_ZIPF_CACHE: dict = {}


def zipf_thresholds(n: int, s: float) -> np.ndarray:
    """Integer inverse-CDF table for P(rank k) proportional to k**-s, k = 1..n.

    thresholds[j] = floor(2**53 * sum_{k<=j+1} k**-s / sum_{k<=n} k**-s), and the
    last entry is exactly 2**53.  Built in float64 with numpy on the host.
    """
    key = (n, float(s))
    if key not in _ZIPF_CACHE:
        k = np.arange(1, n + 1, dtype=np.float64)
        w = np.ones(n) if s == 0 else k ** (-float(s))
        c = np.cumsum(w)
        t = np.floor(c / c[-1] * float(1 << 53)).astype(np.int64)
        t[-1] = 1 << 53
        _ZIPF_CACHE[key] = t
    return _ZIPF_CACHE[key]


def zipf_fk_at(n_dim: int, s: float, idx, seed: int, permute_ids: bool = True,
               backend="numpy", device=None):
    """Foreign keys at fact row indices idx: rank drawn by Zipf(s), id = pi(rank)."""
    xp = _backend(backend, device)
    u = xp.shr(_words(xp, stream_key(seed, STREAM_FK), xp.asarray(idx)), 11)
    t = zipf_thresholds(n_dim, s)
    if xp.name == "numpy":
        rank = np.searchsorted(t, u.astype(np.int64), side="right").astype(np.int64)
    else:
        tt = xp.torch.as_tensor(t, device=xp.device)
        rank = xp.torch.searchsorted(tt, u, right=True)
    if not permute_ids:
        return rank
    return permutation_at(n_dim, rank, seed, STREAM_ZIPF_PERM, backend, device)


def fact_table(n_fact: int, n_dim: int, s: float, seed: int, fact_bytes: int = 16,
               permute_ids: bool = True, backend="numpy", device=None, chunk: int = 1 << 24):
    """Fact rows: [uint32 foreign key, little-endian][payload bytes from stream 6]."""
    xp = _backend(backend, device)
    out = record_bytes(n_fact, fact_bytes, seed, STREAM_FACT, backend=backend, device=device)
    for c0 in range(0, n_fact, chunk):
        c1 = min(n_fact, c0 + chunk)
        fk = zipf_fk_at(n_dim, s, xp.arange(c0, c1), seed, permute_ids, backend, device)
        if xp.name == "numpy":
            out[c0:c1, 0:4] = fk.astype(np.uint32).view(np.uint8).reshape(-1, 4)
        else:
            out[c0:c1, 0:4] = fk.to(xp.torch.int32).view(xp.torch.uint8).reshape(-1, 4)
    return out


def dim_table(n_dim: int, seed: int, dim_bytes: int = 64, backend="numpy", device=None):
    """Dimension rows: [uint32 id = row index, little-endian][payload bytes from stream 7]."""
    xp = _backend(backend, device)
    out = record_bytes(n_dim, dim_bytes, seed, STREAM_DIM, backend=backend, device=device)
    ids = xp.arange(0, n_dim)
    if xp.name == "numpy":
        out[:, 0:4] = ids.astype(np.uint32).view(np.uint8).reshape(-1, 4)
    else:
        out[:, 0:4] = ids.to(xp.torch.int32).view(xp.torch.uint8).reshape(-1, 4)
    return out


def log_uniform_int(lo: int, hi: int, u: float) -> int:
    """Map u in [0, 1) to an integer log-uniform in [lo, hi]."""
    return int(min(hi, max(lo, math.floor(math.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))))))
