"""Batches: many retrieval and join requests of uneven size in one call (one
persistent launch for the direct work), and the captured-graph variant.  Every
request's output must equal the same request run alone, and the oracle."""
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


def make_mix(n_req, seed, kinds=("retrieve", "join"), algos=(dpg.ALGO_DIRECT, dpg.ALGO_DPG, dpg.ALGO_AUTO),
             orders=(0, 1), max_log2=16):
    """Requests with log-uniform sizes and record sizes from {16, 64, 100, 256}."""
    rng = np.random.default_rng(seed)
    reqs, keep, expects = [], [], []
    for k in range(n_req):
        kind = kinds[rng.integers(0, len(kinds))]
        algo = int(algos[rng.integers(0, len(algos))])
        n = int(np.exp(rng.uniform(np.log(1), np.log(1 << max_log2))))
        if kind == "retrieve":
            rec = int(rng.choice([4, 12, 16, 64, 100, 256]))
            n_src = max(1, int(n * rng.uniform(0.5, 2.0)))
            src = synth.record_bytes(n_src, rec, seed=seed * 1000 + k)
            rids = synth.rids_uniform(n_src, n, seed=seed * 1000 + k)
            expects.append(oracle.retrieve(src, rids))
            s_t, r_t = torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV)
            dst = torch.empty((n, rec), dtype=torch.uint8, device=DEV)
            reqs.append(dpg.retrieve_request(s_t, r_t, dst, algo))
            keep.append((s_t, r_t, dst))
        else:
            order = int(orders[rng.integers(0, len(orders))])
            n_dim = max(1, n // 8)
            fact = synth.fact_table(n, n_dim, 0.8, seed=seed * 1000 + k)
            dim = synth.dim_table(n_dim, seed=seed * 1000 + k)
            fn = oracle.fk_join_fact_order if order == 0 else oracle.fk_join_dim_order
            expects.append(fn(fact, dim, 0))
            f_t, d_t = torch.from_numpy(fact).to(DEV), torch.from_numpy(dim).to(DEV)
            dst = torch.empty((n, 80), dtype=torch.uint8, device=DEV)
            reqs.append(dpg.join_request(f_t, d_t, dst, 0, order, algo))
            keep.append((f_t, d_t, dst))
    return reqs, keep, expects


def test_batch_matches_alone_and_oracle(ctx):
    reqs, keep, expects = make_mix(120, seed=7)
    ctx.batch_run(reqs)
    torch.cuda.synchronize()
    batched = [k[2].clone() for k in keep]
    for k, want in zip(keep, expects):
        assert np.array_equal(k[2].cpu().numpy(), want)
    # each request alone, through the single-request entry points
    for q, k, got in zip(reqs, keep, batched):
        k[2].fill_(0)
        if q.kind == dpg.REQ_RETRIEVE:
            ctx.retrieve(k[0], k[1], dst=k[2], algo=q.algo)
        else:
            ctx.fk_join(k[0], k[1], 0, q.order, out=k[2], algo=q.algo)
        torch.cuda.synchronize()
        assert torch.equal(k[2], got)


def test_batch_single_and_empty(ctx):
    reqs, keep, expects = make_mix(1, seed=3, kinds=("retrieve",))
    ctx.batch_run(reqs)
    torch.cuda.synchronize()
    assert np.array_equal(keep[0][2].cpu().numpy(), expects[0])
    ctx.batch_run([])


def test_batch_rejects_invalid_request(ctx):
    reqs, keep, _ = make_mix(5, seed=4, kinds=("retrieve",))
    bad = list(reqs)
    q = dpg.Request.from_buffer_copy(bad[2])
    q.rec_bytes = 6
    bad[2] = q
    for k in keep:
        k[2].fill_(3)
    with pytest.raises(dpg.DPGError) as e:
        ctx.batch_run(bad, workspace=torch.empty(1 << 20, dtype=torch.uint8, device=DEV))
    assert e.value.status == dpg.ERR_INVALID_ARG
    torch.cuda.synchronize()
    for k in keep:
        assert bool((k[2] == 3).all())


def with_scratch(ctx, reqs):
    """Give every request the scratch its steps need in a graph batch (none
    for direct work).  Returns the buffers (keep them alive)."""
    bufs = []
    for q in reqs:
        need = ctx.batch_request_workspace_bytes(q)
        sorts = q.kind == dpg.REQ_FK_JOIN and q.order == 1 and q.n > 0
        assert (need > 0) == (q.algo == dpg.ALGO_DPG or sorts) or q.algo == dpg.ALGO_AUTO or q.n == 0
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=DEV)
        q.workspace, q.workspace_bytes = ws.data_ptr(), need
        bufs.append(ws)
    return bufs


def test_graph_replays_match_eager(ctx):
    """Replays of one captured persistent batch with new requests: direct and
    DPG retrievals, fact-order and dimension-order joins, every replay against
    the oracle, with the program's own eager work between replays.  Every
    request's completion word is set once the stream has finished."""
    stream = torch.cuda.Stream()
    graph = dpg.BatchGraph(ctx, 256, stream)
    for round_, (n_req, seed) in enumerate([(200, 11), (37, 12), (200, 11), (5, 13), (60, 15)]):
        reqs, keep, expects = make_mix(n_req, seed, algos=(dpg.ALGO_DIRECT, dpg.ALGO_DPG, dpg.ALGO_AUTO))
        scratch = with_scratch(ctx, reqs)
        torch.cuda.synchronize()  # inputs were uploaded on the default stream
        with torch.cuda.stream(stream):
            graph.launch(reqs, stream)
        stream.synchronize()
        for i, (k, want) in enumerate(zip(keep, expects)):
            assert np.array_equal(k[2].cpu().numpy(), want), f"replay {round_}, request {i}"
            assert graph.request_done(i), f"replay {round_}, request {i}"
        del scratch
        # eager work of the program's own between replays
        x = torch.randn(1 << 20, device=DEV)
        torch.cuda.synchronize()
        assert float(x.abs().sum()) > 0
    # a DPG request, or a dimension-order join, without scratch is refused
    reqs, keep, _ = make_mix(3, seed=14, algos=(dpg.ALGO_DPG,), kinds=("retrieve",))
    with pytest.raises(dpg.DPGError) as e:
        graph.launch(reqs, stream)
    assert e.value.status == dpg.ERR_WORKSPACE_TOO_SMALL
    reqs, keep, _ = make_mix(2, seed=16, algos=(dpg.ALGO_DIRECT,), kinds=("join",), orders=(1,))
    with pytest.raises(dpg.DPGError) as e:
        graph.launch(reqs, stream)
    assert e.value.status == dpg.ERR_WORKSPACE_TOO_SMALL
    graph.close()


def test_batch_dpg_one_tile_boundary(ctx):
    """DPG retrievals around the size where the whole distribute is one item
    (at most 4096 rids) and where it takes the clear, count, scan and
    distribute steps: permutations, repeated rids and out-of-order duplicates
    over sources with 1, 5 and 33 runs, eagerly and by graph replay; each
    output equals the oracle's."""
    reqs, keep, expects = [], [], []
    cases = [(1, 1, "perm"), (63, 63, "perm"), (4095, 4095, "perm"), (4096, 4096, "perm"), (4097, 4097, "perm"),
             (8191, 8191, "perm"), (4096, 300, "repeat"), (4096, 1 << 20, "uniform"), (3000, 1 << 22, "uniform"),
             (4097, 1 << 20, "uniform")]
    for k, (n, n_src, kind) in enumerate(cases):
        src = synth.record_bytes(n_src, 100, seed=500 + k)
        if kind == "perm":
            rids = synth.rids_permutation(n, seed=500 + k)
        else:
            rids = synth.rids_uniform(n_src, n, seed=500 + k)
        expects.append(oracle.retrieve(src, rids))
        s_t, r_t = torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV)
        dst = torch.empty((n, 100), dtype=torch.uint8, device=DEV)
        reqs.append(dpg.retrieve_request(s_t, r_t, dst, dpg.ALGO_DPG))
        keep.append((s_t, r_t, dst))
    ctx.batch_run(reqs)
    torch.cuda.synchronize()
    for i, want in enumerate(expects):
        assert np.array_equal(keep[i][2].cpu().numpy(), want), cases[i]
    stream = torch.cuda.Stream()
    graph = dpg.BatchGraph(ctx, 64, stream)
    scratch = with_scratch(ctx, reqs)
    for _ in range(2):
        for _, _, dst in keep:
            dst.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.launch(reqs, stream)
        stream.synchronize()
        for i, want in enumerate(expects):
            assert np.array_equal(keep[i][2].cpu().numpy(), want), cases[i]
    del scratch
    graph.close()


@pytest.mark.parametrize("n_dim_log2", [0, 8, 9, 17, 25])
def test_batch_dim_order_passes(ctx, n_dim_log2):
    """Dimension-order joins inside the persistent launch with 1 to 4 stable
    passes (dimension tables of 1, 2^8, 2^9, 2^17 and 2^25 rows), uniform and
    heavily repeated keys, DPG and direct moves of the fact rows: each output
    equals the oracle's (foreign-key order, ties in fact order)."""
    n_dim = 1 << n_dim_log2
    reqs, keep, expects = [], [], []
    dim = synth.dim_table(n_dim, seed=n_dim_log2, dim_bytes=64 if n_dim_log2 < 20 else 16)
    d_t = torch.from_numpy(dim).to(DEV)
    for k, (n, skew, algo) in enumerate([(1, 0.0, dpg.ALGO_DPG), (5000, 0.0, dpg.ALGO_DIRECT),
                                         (70000, 1.2, dpg.ALGO_DPG), (200003, 0.0, dpg.ALGO_DPG),
                                         (4096, 2.0, dpg.ALGO_AUTO)]):
        fact = synth.fact_table(n, n_dim, skew, seed=100 * n_dim_log2 + k)
        expects.append(oracle.fk_join_dim_order(fact, dim, 0))
        f_t = torch.from_numpy(fact).to(DEV)
        dst = torch.empty((n, fact.shape[1] + dim.shape[1]), dtype=torch.uint8, device=DEV)
        reqs.append(dpg.join_request(f_t, d_t, dst, 0, 1, algo))
        keep.append((f_t, d_t, dst))
    ctx.batch_run(reqs)
    torch.cuda.synchronize()
    for i, (k, want) in enumerate(zip(keep, expects)):
        assert np.array_equal(k[2].cpu().numpy(), want), i


def test_batch_dim_order_large(ctx):
    """Two dimension-order joins of 2^22 + 3 fact rows (1025 sort tiles, so
    the count-matrix scan walks a long column) in one batch, with the DPG
    and the direct move of the fact rows, Zipf(1.2) keys over 2^20
    dimension rows: each output equals the oracle's."""
    n, n_dim = (1 << 22) + 3, 1 << 20
    dim = synth.dim_table(n_dim, seed=61, dim_bytes=16)
    fact = synth.fact_table(n, n_dim, 1.2, seed=62)
    want = oracle.fk_join_dim_order(fact, dim, 0)
    d_t, f_t = torch.from_numpy(dim).to(DEV), torch.from_numpy(fact).to(DEV)
    outs = [torch.empty((n, fact.shape[1] + dim.shape[1]), dtype=torch.uint8, device=DEV) for _ in range(2)]
    reqs = [dpg.join_request(f_t, d_t, outs[0], 0, 1, dpg.ALGO_DPG),
            dpg.join_request(f_t, d_t, outs[1], 0, 1, dpg.ALGO_DIRECT)]
    ctx.batch_run(reqs)
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), want)


@pytest.mark.parametrize("log2_run", [0, 2, 5])
def test_batch_dpg_steps_many_runs(ctx, log2_run):
    """DPG requests inside the persistent launch with forced short runs (up to
    the 2048 runs one distribute step takes; longer runs beyond that), empty
    and single-row requests among them: each output equals the oracle's."""
    ctx.set_option(dpg.OPT_LOG2_RUN, log2_run)
    try:
        reqs, keep, expects = make_mix(40, seed=30 + log2_run, algos=(dpg.ALGO_DPG,), orders=(0,), max_log2=15)
        extra, keep2, exp2 = make_mix(6, seed=40 + log2_run, algos=(dpg.ALGO_DPG,), kinds=("retrieve",), max_log2=1)
        # an empty request between them
        s_t, r_t, d_t = keep2[0]
        empty = dpg.retrieve_request(s_t, r_t[:0], d_t[:0], dpg.ALGO_DPG)
        ctx.batch_run(reqs + [empty] + extra)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(dpg.OPT_LOG2_RUN, 0)
    for i, (k, want) in enumerate(zip(keep + keep2, expects + exp2)):
        assert np.array_equal(k[2].cpu().numpy(), want), i


def test_batch_large_mixed_sizes(ctx):
    """A batch shaped like the serving workload: sizes up to 2^22 records."""
    reqs, keep, expects = make_mix(12, seed=21, kinds=("retrieve",), algos=(dpg.ALGO_AUTO,), max_log2=22)
    ctx.batch_run(reqs)
    torch.cuda.synchronize()
    for k, want in zip(keep, expects):
        assert np.array_equal(k[2].cpu().numpy(), want)
