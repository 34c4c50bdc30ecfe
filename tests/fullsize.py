"""Chunked comparison of full-size GPU results with the CPU oracle.

A full-size result (gigabytes) is cut into chunks.  Each chunk is copied from
the device in the main thread, and the oracle computes the same chunk in a
worker thread; the oracle's C routines release the GIL (ctypes), so the chunks
run on all host cores at once.  Every byte of the result is compared.

Only the chunking lives here: which rows form a chunk and where they sit in
the result.  The expected bytes always come from the oracle.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import sys
import time

import numpy as np


def host_workers() -> int:
    """Worker threads: the host cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def note(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def compare_chunks(name: str, chunks, fetch, expect, workers: int | None = None) -> None:
    """For every chunk c: fetch(c) (main thread, the device's bytes as a numpy
    array) must equal expect(c) (worker thread, the oracle's bytes).  At most
    `workers` chunks are held at once.  Fails naming the first chunk and row
    that differ."""
    workers = workers or host_workers()
    chunks = list(chunks)
    t0 = time.perf_counter()

    def job(c, got):
        want = expect(c)
        if isinstance(want, tuple):
            assert isinstance(got, tuple) and len(got) == len(want)
            pairs = list(zip(got, want))
        else:
            pairs = [(got, want)]
        for k, (g, w) in enumerate(pairs):
            if g.shape != w.shape:
                return f"chunk {c}: part {k} shape {g.shape} != oracle {w.shape}"
            if not np.array_equal(g, w):
                diff = np.flatnonzero((g != w).reshape(g.shape[0], -1).any(axis=1)) if g.ndim else [0]
                return f"chunk {c}: part {k} differs from the oracle first at row {int(diff[0])} ({diff.size} rows)"
        return None

    errors = []
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        pending = []
        for c in chunks:
            got = fetch(c)
            pending.append(ex.submit(job, c, got))
            while len(pending) >= workers:
                done, rest = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
                errors += [f.result() for f in done]
                pending = list(rest)
        errors += [f.result() for f in pending]
    errors = [e for e in errors if e]
    note(f"{name}: {len(chunks)} chunks compared with the oracle in {time.perf_counter() - t0:.1f} s "
         f"on {workers} threads")
    assert not errors, f"{name}: " + "; ".join(errors[:4])


def groups_by_small_key(small_key: np.ndarray, n_groups: int):
    """Stable partition of row indices by an integer key in [0, n_groups):
    returns (order, starts) with the rows of group g at order[starts[g]:
    starts[g + 1]] in ascending row order."""
    order = np.argsort(small_key, kind="stable")
    counts = np.bincount(small_key, minlength=n_groups)
    starts = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return order, starts
