"""The serving engine on the GPU: continuous batching under an HBM budget.
Every request's output must be the same alone and in the mix (bit for bit),
and equal the oracle; the arena is never exceeded; oversize and invalid
requests fail cleanly."""
import threading
import time

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


def build_requests(n_req, seed, max_log2=15, sizes=None):
    """n_req requests of N log-uniform in [1, 2^max_log2] (or N = sizes[k])."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_req):
        n = int(np.exp(rng.uniform(0, np.log(1 << max_log2))))
        if sizes is not None:
            n = sizes[k]
        if rng.random() < 0.75:
            rec = int(rng.choice([16, 64, 100, 256]))
            n_src = max(1, n)
            src = synth.record_bytes(n_src, rec, seed=seed * 7919 + k)
            rids = synth.rids_permutation(n_src, seed=seed * 7919 + k)
            want = oracle.retrieve(src, rids)
            s_t, r_t = torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV)
            algo = int(rng.choice([dpg.ALGO_AUTO, dpg.ALGO_DIRECT, dpg.ALGO_DPG]))
            req = dpg.Request(dpg.REQ_RETRIEVE, algo, s_t.data_ptr(), n_src, rec, 0, r_t.data_ptr(), None, n, 0, 0,
                              None)
            out.append((req, (s_t, r_t), want))
        else:
            n_dim = max(1, n // 16)
            rec = int(rng.choice([16, 64, 100, 256]))
            order = int(rng.integers(0, 2))
            fact = synth.fact_table(n, n_dim, 0.0, seed=seed * 7919 + k)
            dim = synth.dim_table(n_dim, seed=seed * 7919 + k, dim_bytes=rec)
            fn = oracle.fk_join_fact_order if order == 0 else oracle.fk_join_dim_order
            want = fn(fact, dim, 0)
            f_t, d_t = torch.from_numpy(fact).to(DEV), torch.from_numpy(dim).to(DEV)
            algo = int(rng.choice([dpg.ALGO_AUTO, dpg.ALGO_DIRECT, dpg.ALGO_DPG]))
            req = dpg.Request(dpg.REQ_FK_JOIN, algo, d_t.data_ptr(), n_dim, rec, 16, None, f_t.data_ptr(), n, 0,
                              order, None)
            out.append((req, (f_t, d_t), want))
    torch.cuda.synchronize()
    return out


def run_all(server, reqs, gap_s=0.0, many=False):
    """Submit (optionally spaced in time, or all in one submit_many call),
    collect every output by polling its own tickets (safe with several
    submitting threads), release."""
    tickets = {}
    if many:
        for i, t in enumerate(server.submit_many([req for req, _, _ in reqs])):
            tickets[t] = i
    for i, (req, _, _) in enumerate([] if many else reqs):
        tickets[server.submit(req)] = i
        if gap_s:
            time.sleep(gap_s)
    got = {}
    waiting = set(tickets)
    deadline = time.time() + 120
    while waiting:
        assert time.time() < deadline, "server did not finish"
        for t in list(waiting):
            state, status, dst, lat = server.poll(t)
            if state < dpg.TICKET_DONE:
                continue
            i = tickets[t]
            assert state == dpg.TICKET_DONE, (i, state, status)
            assert lat > 0
            nbytes = reqs[i][2].nbytes
            got[i] = dpg.copy_device_bytes(dst, nbytes).cpu().numpy().reshape(reqs[i][2].shape)
            server.release(t)
            waiting.discard(t)
        time.sleep(0.0005)
    return got


@pytest.mark.parametrize("mode", ["graph", "batch", "per-request"])
def test_server_outputs_match_oracle(ctx, mode):
    reqs = build_requests(160, seed=1)
    kw = dict(graph=dict(max_batch_requests=64, use_graph=True, batch_max_kib=1 << 20),
              batch=dict(max_batch_requests=64, use_graph=False, batch_max_kib=256),
              **{"per-request": dict(max_batch_requests=1, use_graph=False)})[mode]
    server = dpg.Server(ctx, 1 << 30, max_inflight=3, **kw)
    try:
        got = run_all(server, reqs)
        for i, (_, _, want) in enumerate(reqs):
            assert np.array_equal(got[i], want), i
        st = server.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["arena_high_water"] <= 1 << 30
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        if mode != "per-request":
            assert st["batches"] < len(reqs)
    finally:
        server.close()


@pytest.mark.parametrize("mode", ["graph", "per-request"])
def test_submit_many_matches_oracle(ctx, mode):
    """A burst of requests handed over in one submit_many call: tickets in
    request order, every output equals the oracle's; an empty burst queues
    nothing."""
    reqs = build_requests(120, seed=21)
    kw = dict(graph=dict(max_batch_requests=64, use_graph=True),
              **{"per-request": dict(max_batch_requests=1, use_graph=False)})[mode]
    server = dpg.Server(ctx, 1 << 30, max_inflight=4, **kw)
    try:
        assert server.submit_many([]) == []
        got = run_all(server, reqs, many=True)
        for i, (_, _, want) in enumerate(reqs):
            assert np.array_equal(got[i], want), i
        st = server.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
    finally:
        server.close()


def test_server_requests_up_to_2p22_rows_match_oracle(ctx):
    """Requests of the serving mix's full size range (up to 2^22 rows): the
    large ones run alone through their single-request entry points, the
    small ones in graph batches beside them; every output equals the
    oracle's."""
    sizes = [1 << 22, (1 << 21) + 77, 1 << 20, 3 << 18, 1000, 1 << 14, 5000, 1 << 16, (1 << 22) - 3, 1 << 19,
             300, 1 << 12]
    reqs = build_requests(len(sizes), seed=11, sizes=sizes)
    server = dpg.Server(ctx, 8 << 30, max_inflight=4, max_batch_requests=64, use_graph=True)
    try:
        got = run_all(server, reqs)
        for i, (_, _, want) in enumerate(reqs):
            assert np.array_equal(got[i], want), (i, sizes[i])
        st = server.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
    finally:
        server.close()


def test_alone_equals_in_the_mix(ctx):
    """Each request submitted on its own, then all of them at once while a
    second thread keeps submitting: outputs identical."""
    reqs = build_requests(60, seed=2)
    server = dpg.Server(ctx, 1 << 30, max_inflight=4, max_batch_requests=32)
    try:
        alone = {}
        for i in range(len(reqs)):
            alone[i] = run_all(server, [reqs[i]])[0]
        mix_a, mix_b = {}, {}

        def second():
            mix_b.update(run_all(server, reqs[30:], gap_s=0.0005))

        th = threading.Thread(target=second)
        th.start()
        mix_a.update(run_all(server, reqs[:30], gap_s=0.0003))
        th.join()
        for i in range(len(reqs)):
            mixed = mix_a[i] if i < 30 else mix_b[i - 30]
            assert np.array_equal(alone[i], mixed), i
            assert np.array_equal(alone[i], reqs[i][2]), i
    finally:
        server.close()


def test_budget_backpressure_and_failures(ctx):
    """A small arena: requests wait for memory (never exceeding it), a request
    larger than the arena fails with BUSY, an invalid one with INVALID_ARG."""
    budget = 8 << 20
    reqs = build_requests(40, seed=3, max_log2=13)
    server = dpg.Server(ctx, budget, max_inflight=2, max_batch_requests=8)
    try:
        big_src = torch.zeros((1 << 17, 100), dtype=torch.uint8, device=DEV)
        big_rids = torch.zeros(1 << 17, dtype=torch.int32, device=DEV)
        big = dpg.Request(dpg.REQ_RETRIEVE, dpg.ALGO_DIRECT, big_src.data_ptr(), 1 << 17, 100, 0,
                          big_rids.data_ptr(), None, 1 << 17, 0, 0, None)
        bad = dpg.Request.from_buffer_copy(reqs[0][0])
        bad.rec_bytes = 6
        tb = server.submit(big)
        tbad = server.submit(bad)
        got = run_all(server, reqs)
        for i, (_, _, want) in enumerate(reqs):
            assert np.array_equal(got[i], want)
        for t, status in ((tb, dpg.ERR_BUSY), (tbad, dpg.ERR_INVALID_ARG)):
            state, st, dst, _ = server.poll(t)
            assert state == dpg.TICKET_FAILED and st == status and dst is None
            server.release(t)
        st = server.stats()
        assert st["arena_high_water"] <= budget
        assert st["failed"] == 2
    finally:
        server.close()


def test_request_between_capacity_and_arena_size_fails(ctx):
    """The slot workspaces take part of the arena for good: a request whose
    output fits the arena but not what is left for requests fails with BUSY
    at once instead of blocking the queue, the requests behind it are served,
    and closing the server with an output still held does not wait for it."""
    budget = 16 << 20
    server = dpg.Server(ctx, budget, max_inflight=2, max_batch_requests=8)
    slot_ws = dpg.lib().dpg_batch_graph_workspace_bytes(ctx.handle, 8)
    capacity = budget - 2 * ((slot_ws + 255) // 256 * 256)
    assert capacity < budget
    try:
        n = (capacity + budget) // 2 // 100  # output between the capacity and the arena size
        assert capacity < n * 100 <= budget
        src = torch.zeros((n, 100), dtype=torch.uint8, device=DEV)
        rids = torch.zeros(n, dtype=torch.int32, device=DEV)
        big = dpg.Request(dpg.REQ_RETRIEVE, dpg.ALGO_DIRECT, src.data_ptr(), n, 100, 0, rids.data_ptr(), None, n,
                          0, 0, None)
        tb = server.submit(big)
        reqs = build_requests(12, seed=11, max_log2=12)
        got = run_all(server, reqs)
        for i, (_, _, want) in enumerate(reqs):
            assert np.array_equal(got[i], want)
        state, st, dst, _ = server.poll(tb)
        assert state == dpg.TICKET_FAILED and st == dpg.ERR_BUSY and dst is None
        # an output held while the server closes: a queued request that can
        # then never be admitted fails instead of keeping close() waiting
        half = capacity // 2 // 100 + 1
        hold = dpg.Request(dpg.REQ_RETRIEVE, dpg.ALGO_DIRECT, src.data_ptr(), half, 100, 0, rids.data_ptr(), None,
                           half, 0, 0, None)
        t1 = server.submit(hold)
        while server.poll(t1)[0] not in (dpg.TICKET_DONE, dpg.TICKET_FAILED):
            time.sleep(0.001)
        assert server.poll(t1)[0] == dpg.TICKET_DONE
        t2 = server.submit(hold)
        t0 = time.perf_counter()
        server.close()
        assert time.perf_counter() - t0 < 10.0
    finally:
        server.close()
