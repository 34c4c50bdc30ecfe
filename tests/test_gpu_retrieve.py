"""Retrieval on the GPU through the C ABI, compared byte for byte with the CPU
oracle on the same seeded inputs (Section 2's definition; Figure 1's phases)."""
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


def configure(ctx, probe=0, log2_run=0, dist_tile=0, xcd=1, dist=0, gather=0):
    ctx.set_option(dpg.OPT_DISTRIBUTE, dist)
    ctx.set_option(dpg.OPT_PROBE, probe)
    ctx.set_option(dpg.OPT_LOG2_RUN, log2_run)
    ctx.set_option(dpg.OPT_DIST_TILE, dist_tile)
    ctx.set_option(dpg.OPT_XCD_REMAP, xcd)
    ctx.set_option(dpg.OPT_GATHER, gather)


def make_rids(kind, n_src, n_rids, rec_bytes, seed):
    if kind == "perm":
        assert n_rids == n_src
        return synth.rids_permutation(n_src, seed)
    if kind == "uniform":
        return synth.rids_uniform(n_src, n_rids, seed)
    if kind == "blocked":
        return synth.rids_blocked(n_src, rec_bytes, seed)
    if kind == "same":
        return np.full(n_rids, n_src // 2, dtype=np.int32)
    if kind == "zipf":  # Zipf(1.2) ranks as ids: the hot records sit together at the start
        return synth.zipf_fk_at(n_src, 1.2, np.arange(n_rids), seed, permute_ids=False).astype(np.int32)
    if kind == "identity":
        return np.arange(n_rids, dtype=np.int32) % n_src
    if kind == "reverse":
        return (n_src - 1 - np.arange(n_rids, dtype=np.int64) % n_src).astype(np.int32)
    raise ValueError(kind)


VARIANTS = {
    "direct": (dpg.ALGO_DIRECT, {}),
    "dpg-cached": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED)),
    "dpg-lds": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_LDS)),
    "dpg-short-runs": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, log2_run=3)),
    "dpg-lds-short-runs": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_LDS, log2_run=4)),
    "dpg-small-tiles": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, log2_run=6, dist_tile=128)),
    "dpg-no-xcd-remap": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, xcd=2)),
    "dpg-append": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, dist=dpg.DIST_APPEND)),
    "dpg-lds-append": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_LDS, dist=dpg.DIST_APPEND)),
    "dpg-partition-long-runs": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, log2_run=12, dist=dpg.DIST_PARTITION)),
    # 257..4096 runs: the 12-bit partition pass
    "dpg-wide-partition": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, log2_run=4, dist=dpg.DIST_PARTITION)),
    # distribute tiles of 32768 rids (32 per thread of a 1024-thread pass)
    "dpg-partition-tile-32768": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, log2_run=6, dist=dpg.DIST_PARTITION,
                                                    gather=1, dist_tile=32768)),
    # Phase III forms: through the caches, or a distribute tile staged in LDS
    # (the latter applies to 4..16-byte records with the partition distribute)
    "dpg-cached-gather": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, dist=dpg.DIST_PARTITION, gather=1)),
    "dpg-lds-gather": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, dist=dpg.DIST_PARTITION, gather=2)),
    "dpg-lds-gather-wide": (dpg.ALGO_DPG, dict(probe=dpg.PROBE_CACHED, log2_run=3, dist=dpg.DIST_PARTITION,
                                               gather=2)),
    # two phases: the probe writes every record to its place in dst
    "dpg-scatter": (dpg.ALGO_DPG, dict(gather=dpg.GATHER_NONE)),
    "dpg-scatter-short-runs": (dpg.ALGO_DPG, dict(gather=dpg.GATHER_NONE, log2_run=6)),
    # skew-balanced runs from a sorted sample (Section 2.3)
    "dpg-sampled": (dpg.ALGO_DPG, dict(dist=dpg.DIST_SAMPLED)),
    "dpg-sampled-short-runs": (dpg.ALGO_DPG, dict(dist=dpg.DIST_SAMPLED, log2_run=3)),
    # two partition passes and a two-pass gather (multi-pass DPG, Section 7)
    "dpg-two-pass": (dpg.ALGO_DPG, dict(dist=dpg.DIST_TWO_PASS)),
    "dpg-two-pass-short-runs": (dpg.ALGO_DPG, dict(dist=dpg.DIST_TWO_PASS, log2_run=1)),
    # the same two passes with every run staged in LDS for the probe (run
    # boundaries found from the sorted list; Phase III in one pass)
    "dpg-two-pass-lds": (dpg.ALGO_DPG, dict(dist=dpg.DIST_TWO_PASS, probe=dpg.PROBE_LDS)),
    "dpg-two-pass-lds-short-runs": (dpg.ALGO_DPG, dict(dist=dpg.DIST_TWO_PASS, probe=dpg.PROBE_LDS, log2_run=1)),
    "auto": (dpg.ALGO_AUTO, {}),
}

CASES = [
    # (n_src, n_rids, rec_bytes, rid kind)
    (1000, 1000, 100, "perm"),
    (4099, 4099, 100, "perm"),
    (65537, 65537, 100, "perm"),
    (20000, 50000, 100, "uniform"),
    (30011, 30011, 100, "blocked"),
    (5000, 7000, 100, "same"),
    (10000, 10000, 8, "perm"),
    (12345, 30000, 16, "uniform"),
    (7777, 7777, 4, "perm"),
    (3001, 3001, 12, "reverse"),
    (40009, 50021, 12, "uniform"),  # 12-byte records over several distribute tiles
    (9000, 9000, 36, "perm"),
    (8192, 8192, 64, "blocked"),
    (4000, 4000, 128, "identity"),
    (2500, 6000, 256, "uniform"),
    (300, 700, 4096, "uniform"),
    (9001, 9001, 120, "perm"),
    (5003, 7001, 96, "uniform"),
    (2000, 3000, 1000, "uniform"),
    (6007, 6007, 32, "reverse"),
    (1, 5, 100, "same"),
    (3, 1, 24, "uniform"),
    (50000, 80000, 100, "zipf"),
    (20000, 30000, 8, "zipf"),
]


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-M{c[1]}-R{c[2]}-{c[3]}")
def test_retrieve_matches_oracle(ctx, case, variant):
    n_src, n_rids, rec_bytes, kind = case
    algo, opts = VARIANTS[variant]
    seed = synth.SEED_BASE + n_src + rec_bytes
    src = synth.record_bytes(n_src, rec_bytes, seed)
    rids = make_rids(kind, n_src, n_rids, rec_bytes, seed)
    expect = oracle.retrieve(src, rids)
    configure(ctx, **opts)
    try:
        got = ctx.retrieve(torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV), algo=algo)
        torch.cuda.synchronize()
    finally:
        configure(ctx)
    assert np.array_equal(got.cpu().numpy(), expect), f"{variant} {case}"


def test_partition_tile_option_takes_effect(ctx):
    """The 32768-rid distribute tile is planned when asked for (up to 2^11
    runs, not with the two-phase scatter) -- the variant above runs it."""
    configure(ctx, **VARIANTS["dpg-partition-tile-32768"][1])
    try:
        assert ctx.plan_retrieve(65537, 100, 80000, dpg.ALGO_DPG).dist_tile == 32768
        ctx.set_option(dpg.OPT_LOG2_RUN, 5)  # 2049 runs (12-bit digits): 16384-rid tiles
        assert ctx.plan_retrieve(65537, 100, 80000, dpg.ALGO_DPG).dist_tile == 16384
    finally:
        configure(ctx)


@pytest.mark.parametrize("variant", ["dpg-two-pass-lds", "dpg-two-pass", "dpg-cached"])
def test_unchecked_out_of_range_rids_leave_valid_rows_exact(ctx, variant):
    """Without the rid check, an rid outside the source gives an undefined
    row but touches nothing outside the buffers: every row of a valid rid
    still equals the oracle's (the two-pass distribute drops invalid rids in
    its first pass and fills the slots it leaves)."""
    n_src, n_rids, rec = 40000, 70001, 100
    seed = synth.SEED_BASE + 77
    src = synth.record_bytes(n_src, rec, seed)
    rids = synth.rids_uniform(n_src, n_rids, seed)
    bad = np.arange(0, n_rids, 97)
    rids[bad] = np.where(bad % 2 == 0, n_src + bad, -1 - bad).astype(np.int32)
    ok = np.ones(n_rids, dtype=bool)
    ok[bad] = False
    algo, opts = VARIANTS[variant]
    configure(ctx, **opts)
    try:
        got = ctx.retrieve(torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV), algo=algo)
        torch.cuda.synchronize()
    finally:
        configure(ctx)
    assert np.array_equal(got.cpu().numpy()[ok], oracle.retrieve(src, rids[ok]))


def test_two_pass_lds_plan(ctx):
    """The LDS probe over two-pass runs: regions of at most 64 KiB (512
    records of 100 B), 2^17 runs at 2^26 records, no intermediate array."""
    configure(ctx, **VARIANTS["dpg-two-pass-lds"][1])
    try:
        p = ctx.plan_retrieve(1 << 26, 100, 1 << 26, dpg.ALGO_DPG)
        assert (p.probe, p.distribute, p.log2_run, p.n_runs) == (dpg.PROBE_LDS, dpg.DIST_TWO_PASS, 9, 1 << 17)
        q = ctx.plan_retrieve(1 << 26, 100, 1 << 26, dpg.ALGO_DPG)
        configure(ctx, dist=dpg.DIST_TWO_PASS)
        c = ctx.plan_retrieve(1 << 26, 100, 1 << 26, dpg.ALGO_DPG)
        assert c.probe == dpg.PROBE_CACHED and q.workspace_bytes < c.workspace_bytes
    finally:
        configure(ctx)


def test_empty_rid_list(ctx):
    src = torch.zeros((10, 8), dtype=torch.uint8, device=DEV)
    rids = torch.zeros(0, dtype=torch.int32, device=DEV)
    for algo in (dpg.ALGO_DIRECT, dpg.ALGO_DPG):
        out = ctx.retrieve(src, rids, algo=algo)
        assert out.shape == (0, 8)


@pytest.mark.parametrize("algo", [dpg.ALGO_DIRECT, dpg.ALGO_DPG])
def test_check_rids_rejects_and_leaves_dst(ctx, algo):
    src = torch.arange(400, dtype=torch.int32, device=DEV).view(torch.uint8).reshape(100, 16)
    for bad in (100, -1, 1 << 30):
        rids = torch.arange(50, dtype=torch.int32, device=DEV)
        rids[37] = bad
        dst = torch.full((50, 16), 7, dtype=torch.uint8, device=DEV)
        with pytest.raises(dpg.DPGError) as e:
            ctx.retrieve(src, rids, dst=dst, algo=algo, check_rids=True)
        assert e.value.status == dpg.ERR_RID_OUT_OF_RANGE
        assert bool((dst == 7).all())
    rids = torch.arange(50, dtype=torch.int32, device=DEV)
    out = ctx.retrieve(src, rids, algo=algo, check_rids=True)
    assert torch.equal(out, src[:50])


def test_phase_products_match_figure1(ctx):
    """The distribute and probe intermediates against the oracle's Figure 1
    run.  Run boundaries are unique and must be equal.  The append distribute
    (dist=1) keeps RID order inside a run, so its runs and INTERNAL must equal
    Figure 1's exactly; the one-pass partition distribute leaves the order
    inside a run unspecified, so there every run must hold the same rids (as
    a multiset) and INTERNAL[k] must be the record of RID_RUN[k]."""
    for (n, m, rec, kind, probe, lg, dist) in [(5000, 5000, 100, "perm", dpg.PROBE_CACHED, 8, 0),
                                               (5000, 5000, 100, "perm", dpg.PROBE_CACHED, 4, 0),
                                               (3000, 9000, 16, "uniform", dpg.PROBE_LDS, 0, 0),
                                               (3000, 9000, 16, "uniform", dpg.PROBE_LDS, 0, 1),
                                               (70000, 70000, 64, "perm", dpg.PROBE_CACHED, 0, 0),
                                               (70000, 70000, 64, "perm", dpg.PROBE_CACHED, 0, 1),
                                               (4096, 4096, 8, "same", dpg.PROBE_LDS, 5, 0),
                                               (20000, 20000, 32, "perm", dpg.PROBE_CACHED, 4, 2),
                                               (3000, 9000, 16, "uniform", dpg.PROBE_CACHED, 2, 2),
                                               (50000, 50000, 8, "same", dpg.PROBE_CACHED, 4, 2)]:
        src = synth.record_bytes(n, rec, seed=n)
        rids = make_rids(kind, n, m, rec, seed=n)
        # INTERNAL is the product checked here: a Phase III that reads it
        configure(ctx, probe=probe, log2_run=lg, dist=dist, gather=dpg.GATHER_CACHED)
        try:
            plan = ctx.plan_retrieve(n, rec, m, dpg.ALGO_DPG)
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=DEV)
            out = ctx.retrieve(torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV), algo=dpg.ALGO_DPG,
                               workspace=ws)
            torch.cuda.synchronize()
        finally:
            configure(ctx)
        rid_run, run_off, record_run, dst = oracle.dpg_phases(src, rids, 1 << plan.log2_run)
        w = ws.cpu().numpy()
        g_off = w[plan.ws_run_off: plan.ws_run_off + 4 * (plan.n_runs + 1)].view(np.int32)
        g_run = w[plan.ws_rid_run: plan.ws_rid_run + 4 * m].view(np.int32)
        g_int = w[plan.ws_internal: plan.ws_internal + rec * m].reshape(m, rec)
        assert np.array_equal(g_off.astype(np.int64), run_off)
        if dist == 1:
            assert np.array_equal(g_run, rid_run)
            assert np.array_equal(g_int, record_run)
        else:
            run_of_slot = np.repeat(np.arange(plan.n_runs), np.diff(run_off))
            assert np.array_equal(g_run.astype(np.int64) >> plan.log2_run, run_of_slot)
            assert np.array_equal(np.sort(g_run), np.sort(rid_run))
            assert np.array_equal(g_int, src[g_run])
        assert np.array_equal(out.cpu().numpy(), dst)


def test_deterministic_and_variant_independent(ctx):
    n, rec = 200003, 100
    src = torch.from_numpy(synth.record_bytes(n, rec, seed=1)).to(DEV)
    rids = torch.from_numpy(synth.rids_uniform(n, 300000, seed=1)).to(DEV)
    outs = []
    for algo, opts in VARIANTS.values():
        configure(ctx, **opts)
        try:
            outs.append(ctx.retrieve(src, rids, algo=algo))
            outs.append(ctx.retrieve(src, rids, algo=algo))
        finally:
            configure(ctx)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


def test_torch_generator_matches_numpy_on_gpu():
    a = synth.record_bytes(5000, 100, seed=3, first=11)
    b = synth.record_bytes(5000, 100, seed=3, first=11, backend="torch", device=DEV, chunk_records=1234)
    assert np.array_equal(a, b.cpu().numpy())
    for n in (1 << 16, 100003):
        pa = synth.rids_permutation(n, seed=4)
        pb = synth.rids_permutation(n, seed=4, backend="torch", device=DEV)
        assert np.array_equal(pa, pb.cpu().numpy())
    fa = synth.fact_table(10000, 1 << 12, 1.2, seed=5)
    fb = synth.fact_table(10000, 1 << 12, 1.2, seed=5, backend="torch", device=DEV)
    assert np.array_equal(fa, fb.cpu().numpy())


def test_2p20_records_of_100B_full_oracle(ctx):
    """2^20 records of 100 B, random permutation: every output byte vs the oracle."""
    n, rec = 1 << 20, 100
    seed = synth.SEED_BASE
    src = synth.record_bytes(n, rec, seed)
    rids = synth.rids_permutation(n, seed)
    expect = oracle.retrieve(src, rids)
    for algo in (dpg.ALGO_DIRECT, dpg.ALGO_DPG):
        got = ctx.retrieve(torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV), algo=algo)
        assert np.array_equal(got.cpu().numpy(), expect)


@pytest.mark.parametrize("kind", ["uniform", "zipf"])
def test_sampled_runs_are_ordered_ranges(ctx, kind):
    """Runs bounded by splitters from a sorted sample (Section 2.3): run b's
    rids all lie below run b+1's, the runs hold the rid multiset, and with
    uniform rids no run holds more than twice its share."""
    n, m, rec = 200003, 300000, 16
    src = synth.record_bytes(n, rec, seed=4)
    rids = make_rids(kind, n, m, rec, seed=4)
    configure(ctx, dist=dpg.DIST_SAMPLED, log2_run=6)
    try:
        plan = ctx.plan_retrieve(n, rec, m, dpg.ALGO_DPG)
        assert plan.distribute == dpg.DIST_SAMPLED and plan.n_runs > 1000
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=DEV)
        out = ctx.retrieve(torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV), algo=dpg.ALGO_DPG,
                           workspace=ws)
        torch.cuda.synchronize()
    finally:
        configure(ctx)
    assert np.array_equal(out.cpu().numpy(), oracle.retrieve(src, rids))
    w = ws.cpu().numpy()
    off = w[plan.ws_run_off: plan.ws_run_off + 4 * (plan.n_runs + 1)].view(np.int32).astype(np.int64)
    run = w[plan.ws_rid_run: plan.ws_rid_run + 4 * m].view(np.int32)
    assert off[0] == 0 and off[-1] == m and np.all(np.diff(off) >= 0)
    assert np.array_equal(np.sort(run), np.sort(rids))
    runs = [run[off[b]:off[b + 1]] for b in range(plan.n_runs) if off[b + 1] > off[b]]
    for a, b in zip(runs, runs[1:]):
        assert a.max() < b.min()
    if kind == "uniform":
        assert np.diff(off).max() <= 2 * m / plan.n_runs


def test_two_pass_runs_in_run_order(ctx):
    """Two partition passes (fine run bits, then coarse bits, stable): the
    final RID list is ordered by run index and holds the rid multiset."""
    n, m, rec = 300007, 400000, 8
    src = synth.record_bytes(n, rec, seed=5)
    rids = make_rids("uniform", n, m, rec, seed=5)
    configure(ctx, dist=dpg.DIST_TWO_PASS, log2_run=2)   # 75002 runs: 12 fine bits + 5 coarse bits
    try:
        plan = ctx.plan_retrieve(n, rec, m, dpg.ALGO_DPG)
        assert plan.distribute == dpg.DIST_TWO_PASS and plan.n_runs > 4096 and plan.ws_run_off == 0
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=DEV)
        out = ctx.retrieve(torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV), algo=dpg.ALGO_DPG,
                           workspace=ws)
        torch.cuda.synchronize()
    finally:
        configure(ctx)
    assert np.array_equal(out.cpu().numpy(), oracle.retrieve(src, rids))
    run = ws.cpu().numpy()[plan.ws_rid_run: plan.ws_rid_run + 4 * m].view(np.int32)
    assert np.all(np.diff(run.astype(np.int64) >> plan.log2_run) >= 0)
    assert np.array_equal(np.sort(run), np.sort(rids))


@pytest.mark.parametrize("rec", [4, 8, 16])
@pytest.mark.parametrize("log2_run", [0, 1, 3])
def test_lds_probe_unaligned_source(ctx, rec, log2_run):
    """The LDS probes stage a region with 16-byte loads only when the source
    and every region start allow it: a source 4 bytes past an aligned address,
    and runs of 2 or 8 records, take the element-wise path."""
    n, m = 20001, 30000
    base = torch.from_numpy(synth.record_bytes(n + 1, rec, seed=rec)).to(DEV)
    src = base.view(-1)[4: 4 + n * rec].view(n, rec)  # 4 bytes past the allocation
    rids = torch.from_numpy(synth.rids_uniform(n, m, seed=rec + 1)).to(DEV)
    want = oracle.retrieve(src.cpu().numpy(), rids.cpu().numpy())
    configure(ctx, probe=dpg.PROBE_LDS, log2_run=log2_run)
    try:
        got = ctx.retrieve(src, rids, algo=dpg.ALGO_DPG)
        torch.cuda.synchronize()
    finally:
        configure(ctx)
    assert np.array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("per", [2, 4, 8, 16])
@pytest.mark.parametrize("nt", [True, False], ids=["nt", "plain"])
def test_stream_copy(ctx, per, nt):
    """The copy-ceiling kernel: three whole tiles and a partial one, copied
    exactly; misaligned or unequal buffers are refused."""
    n = 16 * (256 * per * 3 + 17)
    a = torch.from_numpy(synth.record_bytes(n // 16, 16, seed=per).reshape(-1)).to(DEV)
    b = torch.zeros_like(a)
    ctx.stream_copy(a, b, per, nt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(dpg.DPGError) as e:
        ctx.stream_copy(a[4:n - 12], b[:n - 16], per, nt)
    assert e.value.status == dpg.ERR_INVALID_ARG
