"""Benchmark: DPG record retrieval on one MI355X, plus the operators built on it.

Headline workload (the metric's configuration): 2^26 source records of 100 B
(10-byte uniform key + 90-byte payload), rids a pseudo-random permutation of
[0, 2^26), 2^26 outputs.  One step is one full DPG retrieval (distribute,
probe, gather) with the planner's DPG plan; the autotuner's best plan and
its time are reported beside it, and the direct gather is timed on the same
inputs.  Inputs are resident in HBM before timing starts.

Secondary measurements reported in the same JSON line (each on its own
synthetic inputs): the key-pointer sort of 10^8 x 100 B records, the DPG-Move
and DPG-Sort joins of 2^28 x 16 B fact rows with 2^24 x 64 B dimension rows
under Zipf(0 / 0.8 / 1.2) keys, the batch lookup of 2^26 keys in a hash index
of 2^24 keys, and the serving workload (4096 retrieval /
join requests, log-uniform sizes, Poisson arrivals, 64 GiB HBM budget):
batched server vs per-request launches, p50 / p99 latency.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "retrieval GB/s, DPG vs direct gather @100B records; p50/p99 batched latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--rec-bytes", type=int, default=100)
    ap.add_argument("--pattern", default="perm", choices=["perm", "uniform", "blocked"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--log2-run", type=int, default=0, help="force L = 2^v records per run (0: planner's choice)")
    ap.add_argument("--probe", type=int, default=0, help="1 cached, 2 LDS (0: planner's choice)")
    ap.add_argument("--dist", type=int, default=0, help="Phase I: 1 append, 2 partition (0: planner's choice)")
    ap.add_argument("--gather", type=int, default=0,
                    help="Phase III: 1 cached, 2 LDS, 3 none (the probe writes dst) (0: planner's choice)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: also run the autotuner over the DPG plans and report its pick")
    ap.add_argument("--only", default="",
                    help="comma list of sections: retrieve,lds,small,sweep,sort,join,smj,hash,btree,skew,serve "
                         "(default all)")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--join-zipf", default="0,0.8,1.2", help="Zipf exponents of the join section")
    ap.add_argument("--join-variants", default="move_dpg,move_direct,sort_dpg,sort_direct,keyed",
                    help="join variants to time: move_dpg, move_direct, sort_dpg, sort_direct, keyed")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (calibrates rocprofv3 byte counters)")
    ap.add_argument("--counters", default=os.path.join(ROOT, "profiles", "counters.json"),
                    help="HBM byte counts per launch measured with rocprofv3 --pmc (optional)")
    return ap.parse_args()


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_and_profile(ctx, fn, steps, warmup, torch):
    """Time `steps` calls with per-kernel profiling off (the reported
    ms/step), then run the same number of calls again with HIP events around
    every launch for the per-kernel durations.  Returns (ms, wall_s, prof)."""
    ms, wall = time_steps(fn, steps, warmup, torch)
    ctx.profile_enable(True)
    ctx.profile_reset()
    try:
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        prof = ctx.profile_collect()
    finally:
        ctx.profile_enable(False)
        ctx.profile_reset()
    return ms, wall, prof


def host_threads() -> int:
    """Host cores this process may use (at most 16, the GPU machine's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def timed_oracle(fn, items, threads):
    """Wall time of fn over every item, on `threads` host threads (the
    oracle's C routines release the GIL, so the items run in parallel)."""
    import concurrent.futures as cf

    t0 = time.perf_counter()
    if threads == 1:
        for it in items:
            fn(it)
    else:
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(fn, items))
    return time.perf_counter() - t0


def cpu_baseline(src_dev, rids_np, rec_bytes, target_s):
    """The oracle's retrieval loop, as it stands, on a bounded prefix of the
    rid list against the full source copied to host memory: once on one
    core, and once with the prefix cut into disjoint slices run on every host
    core at the same time."""
    import oracle

    src = src_dev.cpu().numpy()
    m_total = rids_np.size
    m = min(m_total, 1 << 20)
    dt = timed_oracle(lambda r: oracle.retrieve(src, r), [rids_np[:m]], 1)
    if dt < target_s and m < m_total:
        m = int(min(m_total, m * max(1.0, target_s / max(dt, 1e-3))))
    threads = host_threads()
    step = -(-m // (4 * threads))
    slices = [rids_np[a:min(m, a + step)] for a in range(0, m, step)]
    # medians of three runs each
    dts = sorted(timed_oracle(lambda r: oracle.retrieve(src, r), [rids_np[:m]], 1) for _ in range(3))
    dts_all = sorted(timed_oracle(lambda r: oracle.retrieve(src, r), slices, threads) for _ in range(3))
    dt, dt_all = dts[1], dts_all[1]
    del src
    return {
        "value": round(m * rec_bytes / dt_all / 1e9, 3),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {m} of {m_total} rids over the full {rec_bytes}-byte source, cut into "
                  f"{len(slices)} slices on {threads} threads: median of 3 runs {dt_all:.2f} s ({host_desc()})",
        "single_core": {"value": round(m * rec_bytes / dt / 1e9, 3), "unit": "GB/s", "cores": 1,
                        "sample": f"the same {m} rids on one thread: median of 3 runs {dt:.2f} s"},
    }


def host_desc() -> str:
    """CPU model, logical CPUs and RAM of the host the oracle ran on."""
    model = platform.processor() or platform.machine()
    mem = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = f", {int(line.split()[1]) / 2 ** 20:.0f} GiB RAM"
                    break
    except OSError:
        pass
    return f"{model}; host reports {os.cpu_count()} logical CPUs{mem}"


NO_CPU = False  # --no-cpu: no oracle timings (their entries are null)


def oracle_rate(fn, units: float, unit: str, sample: str):
    """The oracle timed on a bounded sample of a section's workload: one call
    of fn on one core, then one call per host core, all at once (independent
    copies of the same work; the throughput counts every copy)."""
    if NO_CPU:
        return None
    dt1 = timed_oracle(lambda _: fn(), [None], 1)
    threads = host_threads()
    dtn = timed_oracle(lambda _: fn(), [None] * threads, threads)
    return {"value": round(threads * units / dtn, 1), "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"{sample}: {threads} copies at once on {threads} threads, {dtn:.2f} s",
            "single_core": {"value": round(units / dt1, 1), "unit": unit, "cores": 1,
                            "sample": f"one copy on one thread, {dt1:.2f} s"}}


# Sources of the retrieval kernels and their launch shapes: counter data
# taken before a change to any of them no longer describe the kernels.
RETRIEVAL_SOURCES = ("copy.hip", "partition.hip", "partition.h", "scan.hip", "distribute.hip", "plan.cpp",
                     "dev_common.h")


def retrieval_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in RETRIEVAL_SOURCES:
        with open(os.path.join(ROOT, "paper_cs_0308004_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:12]


def roofline_entry(prof: dict, kernels: list[str], counters: dict | None, workload_key: str | None = None):
    """The dominant kernel: algorithmic bytes per launch over its average
    launch duration (HIP events on the kernel's own stream)."""
    cand = {k: v for k, v in prof.items() if k in kernels}
    name = max(cand, key=lambda k: cand[k]["ms"])
    v = cand[name]
    avg_ms = v["ms"] / v["launches"]
    bytes_per_launch = v["bytes"] / v["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    if counters and workload_key and counters.get("workload") == workload_key:
        traffic = counters.get("kernels", {}).get(name, {}).get("hbm_bytes_per_launch")
    return {
        "kernel": name,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_key": workload_key,
        "avg_launch_ms": round(avg_ms, 4),
        "alg_bytes_per_launch": bytes_per_launch,
    }


# ---------------------------------------------------------------------------
def bench_retrieve(args, ctx, dpg, synth, torch, np, counters):
    dev = "cuda:0"
    n = 1 << args.log2n
    R = args.rec_bytes
    seed = synth.SEED_BASE + 1
    log(f"bench: generating {n} x {R} B records and {args.pattern} rids on {dev}")
    src = synth.record_bytes(n, R, seed, backend="torch", device=dev)
    if args.pattern == "perm":
        rids = synth.rids_permutation(n, seed, backend="torch", device=dev)
    elif args.pattern == "uniform":
        rids = synth.rids_uniform(n, n, seed, backend="torch", device=dev)
    else:
        rids = synth.rids_blocked(n, R, seed, backend="torch", device=dev)
    m = rids.numel()
    dst = torch.empty((m, R), dtype=torch.uint8, device=dev)
    tuned = None
    if args.log2_run or args.probe or args.dist or args.gather:
        ctx.set_option(dpg.OPT_LOG2_RUN, args.log2_run)
        ctx.set_option(dpg.OPT_PROBE, args.probe)
        ctx.set_option(dpg.OPT_DISTRIBUTE, args.dist)
        ctx.set_option(dpg.OPT_GATHER, args.gather)
    elif args.autotune:
        # the autotuner's pick is reported next to the planner's default plan,
        # which is what is timed (a fixed plan keeps profiles comparable)
        log("bench: autotuning the DPG configuration")
        best, tuned_ms = ctx.autotune_retrieve(src, rids, dst, reps=2, dpg_only=True)
        tuned = {"ms": round(tuned_ms, 4), "log2_run": best.log2_run, "n_runs": best.n_runs,
                 "probe": {1: "cached", 2: "lds"}.get(best.probe, "?"),
                 "distribute": {1: "append", 2: "partition", 3: "sampled", 4: "two-pass"}.get(best.distribute, "?"),
                 "gather": {1: "cached", 2: "lds", 3: "none (probe scatters)"}.get(best.gather, "?")}
        ctx.tune_clear()
    plan = ctx.plan_retrieve(n, R, m, dpg.ALGO_DPG)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    ws_direct = torch.empty(256, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step_dpg():
        ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DPG, workspace=ws, stream=stream)

    def step_direct():
        ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DIRECT, workspace=ws_direct, stream=stream)

    log(f"bench: plan L=2^{plan.log2_run} runs={plan.n_runs} tile={plan.dist_tile} probe={plan.probe}")
    ms_dpg, wall_dpg, prof_dpg = time_and_profile(ctx, step_dpg, args.steps, args.warmup, torch)
    ms_direct, _, prof_direct = time_and_profile(ctx, step_direct, args.steps, args.warmup, torch)
    log(f"bench: dpg {ms_dpg:.3f} ms/step, direct {ms_direct:.3f} ms/step")
    # the timed output, spot-checked against the generator
    sample = np.random.default_rng(0).integers(0, m, 256)
    rids_np = rids.cpu().numpy()
    step_dpg()
    torch.cuda.synchronize()
    got = dst[torch.from_numpy(sample).to(dev)].cpu().numpy()
    if not np.array_equal(got, synth.records_at(rids_np[sample], R, seed)):
        raise SystemExit("bench: DPG output differs from the generator's records")
    delivered = m * R
    # counter data apply only to the same shape, DPG plan and kernel sources
    wkey = (f"{n}x{R}:{args.pattern}:L{plan.log2_run}:probe{plan.probe}:runs{plan.n_runs}:dist{plan.distribute}"
            f":tile{plan.dist_tile}:gather{plan.gather}:src{retrieval_source_hash()}")
    dpg_kernels = ["k_part_hist", "k_part_scatter", "k_part_hist_wide", "k_part_scatter_unstable", "k_dist_hist",
                   "k_dist_scatter", "k_probe_cached", "k_probe_lds", "k_gather_phase", "k_gather_lds",
                   "k_probe_scatter"]
    out = {
        "value": round(delivered / (ms_dpg * 1e-3) / 1e9, 2),
        "ms_per_step": round(ms_dpg, 4),
        "config": {
            "workload": f"DPG record retrieval, N=M=2^{args.log2n}, {R}-byte records, rids {args.pattern}",
            "n_src": n, "n_rids": m, "rec_bytes": R, "rid_pattern": args.pattern,
            "algo": "dpg", "log2_run": plan.log2_run, "n_runs": plan.n_runs, "dist_tile": plan.dist_tile,
            "distribute": {1: "append", 2: "partition", 3: "sampled", 4: "two-pass"}.get(plan.distribute, "?"),
            "probe": {1: "cached", 2: "lds"}.get(plan.probe, "?"),
            "gather": {1: "cached", 2: "lds", 3: "none (probe scatters)"}.get(plan.gather, "?"),
            "autotuned": tuned,
        },
        "roofline": roofline_entry(prof_dpg, dpg_kernels, counters, wkey),
        "direct": {
            "value": round(delivered / (ms_direct * 1e-3) / 1e9, 2),
            "unit": "GB/s",
            "ms_per_step": round(ms_direct, 4),
            "roofline": roofline_entry(prof_direct, ["k_direct_gather"], counters, wkey),
        },
        "dpg_over_direct": round(ms_direct / ms_dpg, 4),
        "kernels_ms_per_step": {k: round(v["ms"] / v["launches"], 4) for k, v in prof_dpg.items()},
        "wall_s_timed": round(wall_dpg, 4),
    }
    # the problem's floor for any method, B_min = 4M + R * (records touched) +
    # R * M, over each method's whole step; and a plain device copy of 4 GiB
    # as the practical read + write ceiling
    touched = int(torch.unique(rids).numel()) if args.pattern == "uniform" else min(n, m)
    b_min = 4.0 * m + R * touched + R * m
    out["eta_min"] = {"bytes": b_min, "dpg": round(b_min / (ms_dpg * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                      "direct": round(b_min / (ms_direct * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
    # each method's own algorithmic bytes over its whole step:
    #   DPG, three phases: 24M + R*N + 3R*M (distribute: rids read twice and
    #     run + inv written, 16M; probe: run 4M + source R*N + INTERNAL R*M;
    #     gather: inv 4M + INTERNAL R*M + dst R*M)
    #   DPG, two phases (the probe writes dst): 24M + R*N + R*M
    #   direct: 4M + f*M + R*M, f = bytes of the 64-byte sectors a record
    #     touches, on average over the record offsets
    f_r = 64.0 * sum(((j * R) % 64 + R + 63) // 64 for j in range(64)) / 64.0
    two_phase = plan.gather == 3
    b_dpg = 24.0 * m + R * touched + (1 if two_phase else 3) * R * m
    b_direct = 4.0 * m + f_r * m + R * m
    out["eta_alg"] = {
        "dpg": {"form": "two phases" if two_phase else "three phases", "bytes": b_dpg,
                "frac": round(b_dpg / (ms_dpg * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)},
        "direct": {"sector_bytes_per_record": f_r, "bytes": b_direct,
                   "frac": round(b_direct / (ms_direct * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}}
    out["copy_ceiling"] = copy_ceiling(ctx, torch)
    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle baseline")
        cpu = cpu_baseline(src, rids_np, R, args.cpu_seconds)
    for opt in (dpg.OPT_LOG2_RUN, dpg.OPT_PROBE, dpg.OPT_DISTRIBUTE, dpg.OPT_GATHER):
        ctx.set_option(opt, 0)
    del src, rids, dst, ws
    torch.cuda.empty_cache()
    return out, cpu


def bench_lds_probe(args, ctx, dpg, synth, torch, np):
    """The headline workload with Phase II as the paper states it: every
    source run loaded whole into LDS (runs of <= 64 KiB from two partition
    passes), then the gather through the composed slots.  A section of its
    own, so that profiles of the headline section see the default plan only."""
    dev = "cuda:0"
    n = 1 << args.log2n
    R = args.rec_bytes
    seed = synth.SEED_BASE + 1
    log(f"bench: LDS-staged probe over two-pass runs, {n} x {R} B")
    src = synth.record_bytes(n, R, seed, backend="torch", device=dev)
    rids = synth.rids_permutation(n, seed, backend="torch", device=dev)
    dst = torch.empty((n, R), dtype=torch.uint8, device=dev)
    ctx.set_option(dpg.OPT_DISTRIBUTE, dpg.DIST_TWO_PASS)
    ctx.set_option(dpg.OPT_PROBE, dpg.PROBE_LDS)
    try:
        plan = ctx.plan_retrieve(n, R, n, dpg.ALGO_DPG)
        if plan.probe != dpg.PROBE_LDS:
            return None
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream()
        ms, _, prof = time_and_profile(
            ctx, lambda: ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DPG, workspace=ws, stream=stream),
            args.steps, args.warmup, torch)
    finally:
        ctx.set_option(dpg.OPT_DISTRIBUTE, 0)
        ctx.set_option(dpg.OPT_PROBE, 0)
    sample = np.random.default_rng(0).integers(0, n, 256)
    rids_np = rids.cpu().numpy()
    if not np.array_equal(dst[torch.from_numpy(sample).to(dev)].cpu().numpy(),
                          synth.records_at(rids_np[sample], R, seed)):
        raise SystemExit("bench: the LDS-probe DPG output differs from the generator's records")
    res = {
        "what": "the headline retrieval with Phase II staged in LDS: two partition passes into "
                f"{plan.n_runs} runs of 2^{plan.log2_run} records, each loaded whole into LDS",
        "value": round(n * R / (ms * 1e-3) / 1e9, 2), "unit": "GB/s", "ms_per_step": round(ms, 4),
        "kernels_ms_per_launch": {k: round(v["ms"] / v["launches"], 4) for k, v in prof.items()},
        "launches_per_step": {k: round(v["launches"] / args.steps) for k, v in prof.items()},
        "roofline": roofline_entry(prof, ["k_probe_lds"], None),
    }
    del src, rids, dst, ws
    torch.cuda.empty_cache()
    return res


def copy_ceiling(ctx, torch):
    """The library's plain streaming copy (dpg_stream_copy) of 4 GiB, device
    to device, over its launch shapes: the practical read + write ceiling of
    a phase that reads its bytes once and writes them once."""
    a = torch.empty(1 << 32, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    shapes = {}
    for per in (4, 8, 16):
        for nt in (True, False):
            ms, _ = time_steps(lambda: ctx.stream_copy(a, b, per, nt), 5, 2, torch)
            shapes[f"{per}x16B_{'nt' if nt else 'plain'}"] = round(2.0 * a.numel() / (ms * 1e-3) / 1e9, 1)
    if not torch.equal(a[::4099], b[::4099]):
        raise SystemExit("bench: the streaming copy differs from its source")
    torch_ms, _ = time_steps(lambda: b.copy_(a), 5, 2, torch)
    del a, b
    torch.cuda.empty_cache()
    best = max(shapes, key=shapes.get)
    return {"GB_per_s": shapes[best], "shape": best, "shapes_GB_per_s": shapes,
            "torch_copy_GB_per_s": round(2.0 * (1 << 32) / (torch_ms * 1e-3) / 1e9, 1),
            "what": "k_stream_copy of 4 GiB device to device (reads and writes 4 GiB); best launch shape"}


def bench_sweep(args, ctx, dpg, synth, torch, np):
    """The record-size and rid-pattern sweep at 2^26 records: R in {8, 16,
    32, 64, 100, 128, 256} B, rids a permutation, uniform draws with repeats,
    or shuffled 4 KB runs; the default DPG plan against the direct gather,
    each timed over a few steps without per-kernel events (a spot check of
    the output against src[rids] for each)."""
    dev = "cuda:0"
    n = 1 << args.log2n
    steps = max(3, args.steps // 4)
    res = {"workload": f"2^{args.log2n} source records and rids, R in {{8,16,32,64,100,128,256}} B, rids "
                       "perm / uniform / blocked", "ms": {}}
    for R in (8, 16, 32, 64, 100, 128, 256):
        seed = synth.SEED_BASE + 50 + R
        src = synth.record_bytes(n, R, seed, backend="torch", device=dev)
        dst = torch.empty_like(src)
        for pattern in ("perm", "uniform", "blocked"):
            if pattern == "perm":
                rids = synth.rids_permutation(n, seed, backend="torch", device=dev)
            elif pattern == "uniform":
                rids = synth.rids_uniform(n, n, seed, backend="torch", device=dev)
            else:
                rids = synth.rids_blocked(n, R, seed, backend="torch", device=dev)
            plan = ctx.plan_retrieve(n, R, n, dpg.ALGO_DPG)
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
            wsd = torch.empty(256, dtype=torch.uint8, device=dev)
            t_dpg, _ = time_steps(lambda: ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DPG, workspace=ws),
                                  steps, 2, torch)
            pick = torch.arange(0, n, 65537, device=dev)
            if not torch.equal(dst[pick], src[rids[pick].long()]):
                raise SystemExit(f"bench: sweep R={R} {pattern}: DPG output differs from src[rids]")
            t_dir, _ = time_steps(lambda: ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DIRECT, workspace=wsd),
                                  steps, 2, torch)
            form = {1: "three phases, cached gather", 2: "three phases, LDS gather", 3: "two phases"}.get(plan.gather)
            res["ms"][f"{R}B_{pattern}"] = {"dpg": round(t_dpg, 4), "direct": round(t_dir, 4),
                                            "dpg_over_direct": round(t_dir / t_dpg, 3), "dpg_form": form,
                                            "runs": plan.n_runs}
            log(f"bench: sweep {R} B {pattern}: dpg {t_dpg:.3f} ms, direct {t_dir:.3f} ms")
            del rids, ws
        del src, dst
        torch.cuda.empty_cache()
    return res


def bench_small(args, ctx, dpg, synth, torch, np):
    """2^20 records of 100 B and a permutation of 2^20 rids (the paper's
    1M x 100 B workload): source and output fit the 256 MiB Infinity Cache,
    so each call is timed warm (repeated on the same buffers) and cold (a
    1 GiB write before every call evicts the cache).  Median and minimum of
    20 calls, HIP events around each call."""
    dev = "cuda:0"
    n, R = 1 << 20, 100
    seed = synth.SEED_BASE + 1
    src = synth.record_bytes(n, R, seed, backend="torch", device=dev)
    rids = synth.rids_permutation(n, seed, backend="torch", device=dev)
    dst = torch.empty((n, R), dtype=torch.uint8, device=dev)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    log("bench: 2^20 x 100 B retrieval, warm and cold")
    res = {"workload": "2^20 records of 100 B (10-byte key + 90-byte payload), rids a permutation of 2^20; "
                       "cold: a 1 GiB write before each call"}
    reps = 20
    for algo, name in ((dpg.ALGO_DPG, "dpg"), (dpg.ALGO_DIRECT, "direct")):
        plan = ctx.plan_retrieve(n, R, n, algo)
        ws = torch.empty(max(1, plan.workspace_bytes), dtype=torch.uint8, device=dev)
        call = lambda: ctx.retrieve(src, rids, dst=dst, algo=algo, workspace=ws)
        entry = {}
        for mode in ("warm", "cold"):
            for _ in range(3):
                call()
            times = []
            for _ in range(reps):
                if mode == "cold":
                    flush.fill_(1)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                call()
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) * 1e3)
            times.sort()
            med = times[reps // 2]
            entry[mode] = {"median_us": round(med, 1), "min_us": round(times[0], 1),
                           "GB_per_s": round(n * R / (med * 1e-6) / 1e9, 1)}
        pick = torch.arange(0, n, 4099, device=dev)
        if not torch.equal(dst[pick], src[rids[pick].to(torch.int64)]):
            raise SystemExit(f"bench: 2^20 x 100 B {name} retrieval differs from src[rids]")
        res[name] = entry
        del ws
    del src, rids, dst, flush
    torch.cuda.empty_cache()
    return res


def bench_sort(args, ctx, dpg, synth, torch, np):
    dev = "cuda:0"
    n, R = 100_000_000, 100
    seed = synth.SEED_BASE + 2
    log("bench: sort 10^8 x 100 B records")
    src = synth.record_bytes(n, R, seed, backend="torch", device=dev)
    dst = torch.empty_like(src)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    res = {}
    steps = max(2, args.steps // 3)
    for name, algo in (("dpg", dpg.ALGO_DPG), ("direct", dpg.ALGO_DIRECT)):
        ws = torch.empty(ctx.sort_workspace_bytes(n, R, 0, 10, algo), dtype=torch.uint8, device=dev)
        ms, _, prof = time_and_profile(
            ctx, lambda: ctx.sort_records(src, 0, 10, dst=dst, perm=perm, algo=algo, workspace=ws), steps, 1, torch)
        calls = steps
        res[name] = {"ms": round(ms, 3), "records_per_s": round(n / (ms * 1e-3), 1),
                     "GB_per_s": round(n * R / (ms * 1e-3) / 1e9, 2),
                     "kernels_ms_per_sort": {k: round(v["ms"] / calls, 4) for k, v in prof.items()},
                     "roofline": roofline_entry(prof, list(prof), None)}
        del ws
    k8 = dst[:2000, 0:10].cpu().numpy()
    keys = [bytes(r) for r in k8]
    if keys != sorted(keys):
        raise SystemExit("bench: sort output not sorted")
    host = src[: 1 << 20].cpu().numpy()  # the oracle's sample, uniform keys
    # the same records with the first four key bytes drawn from 4096 values:
    # groups of about 24,000 equal prefixes send the pairs through the
    # full-key passes (the device raises the flag, the gated passes run)
    pool = synth.record_bytes(4096, 4, seed, stream=synth.STREAM_MIX, backend="torch", device=dev)
    pick = synth.uniform_at(4096, torch.arange(n, device=dev), seed, synth.STREAM_FK, backend="torch", device=dev)
    src[:, 0:4] = pool[pick]
    del pool, pick
    ws = torch.empty(ctx.sort_workspace_bytes(n, R, 0, 10, dpg.ALGO_DPG), dtype=torch.uint8, device=dev)
    ms, _, prof = time_and_profile(
        ctx, lambda: ctx.sort_records(src, 0, 10, dst=dst, perm=perm, algo=dpg.ALGO_DPG, workspace=ws), steps, 1,
        torch)
    if int(ws[:4].view(torch.int32).item()) != 1:
        raise SystemExit("bench: the tied-prefix sort did not take the full-key passes")
    k8 = dst[::99991, 0:10].cpu().numpy()
    keys = [bytes(r) for r in k8]
    if keys != sorted(keys):
        raise SystemExit("bench: tied-prefix sort output not sorted")
    res["dpg_full_key_passes"] = {
        "workload": "the same 10^8 records with key bytes 0-3 drawn from 4096 values (groups of ~24,000 equal "
                    "prefixes: the full-key LSD passes run)",
        "ms": round(ms, 3), "records_per_s": round(n / (ms * 1e-3), 1),
        "kernels_ms_per_sort": {k: round(v["ms"] / steps, 4) for k, v in prof.items()}}
    del ws
    import oracle

    res["cpu_oracle"] = oracle_rate(lambda: oracle.sort_records(host, 0, 10), 1 << 20, "records/s",
                                    "the first 2^20 of the records")
    del src, dst, perm, host
    torch.cuda.empty_cache()
    return {"workload": "10^8 records x 100 B, 10-byte uniform key; key-pointer LSD radix sort + copy",
            **res, "dpg_over_direct": round(res["direct"]["ms"] / res["dpg"]["ms"], 4)}


def bench_join(args, ctx, dpg, synth, torch, np):
    dev = "cuda:0"
    n_dim, n_fact = 1 << 24, 1 << 28
    seed = synth.SEED_BASE + 3
    log("bench: joins 2^28 x 16 B fact rows with 2^24 x 64 B dimension rows")
    dim = synth.dim_table(n_dim, seed, backend="torch", device=dev)
    out = torch.empty((n_fact, 80), dtype=torch.uint8, device=dev)
    res = {}
    steps = max(2, args.steps // 3)
    variants = set(v for v in args.join_variants.split(",") if v)
    for s in (float(z) for z in args.join_zipf.split(",") if z):
        fact = synth.fact_table(n_fact, n_dim, s, seed, backend="torch", device=dev)
        for order, oname in ((dpg.JOIN_FACT_ORDER, "dpg_move"), (dpg.JOIN_DIM_ORDER, "dpg_sort")):
            for algo, aname in ((dpg.ALGO_DPG, "dpg"), (dpg.ALGO_DIRECT, "direct")):
                if f"{oname[4:]}_{aname}" not in variants:
                    continue
                ws = torch.empty(max(1, ctx.fk_join_workspace_bytes(n_fact, 16, 0, n_dim, 64, order, algo)),
                                 dtype=torch.uint8, device=dev)
                ms, _, prof = time_and_profile(
                    ctx, lambda: ctx.fk_join(fact, dim, 0, order, out=out, algo=algo, workspace=ws), steps, 1, torch)
                res[f"zipf{s}_{oname}_{aname}"] = {"ms": round(ms, 3),
                                                   "out_GB_per_s": round(n_fact * 80 / (ms * 1e-3) / 1e9, 2),
                                                   "roofline": roofline_entry(prof, list(prof), None)}
                del ws
        if s == 0.0 and "keyed" in variants:
            # the same join over non-dense keys: dimension keys are distinct
            # odd uint32, and the fk column holds the key of the row it names
            keys = (2 * synth.rids_permutation(1 << 30, seed, backend="torch", device=dev, count=n_dim).to(torch.int64)
                    + 1).to(torch.int32)
            dim_k = dim.clone()
            dim_k[:, 4:8] = keys.view(torch.uint8).reshape(-1, 4)
            fact_k = fact.clone()
            fact_k[:, 0:4] = keys[fact[:, 0:4].contiguous().view(torch.int32).view(-1).to(torch.int64)].view(
                torch.uint8).reshape(-1, 4)
            lg_slots = 25
            index = ctx.hash_build(keys, lg_slots)
            for order, oname in ((dpg.JOIN_FACT_ORDER, "move"), (dpg.JOIN_DIM_ORDER, "sort")):
                for algo, aname in ((dpg.ALGO_DPG, "dpg"), (dpg.ALGO_DIRECT, "direct"), (dpg.ALGO_AUTO, "auto")):
                    ws = torch.empty(ctx.key_join_workspace_bytes(n_fact, 16, 0, n_dim, 64, lg_slots, order, algo),
                                     dtype=torch.uint8, device=dev)
                    # unchecked keys: no stream synchronization inside the timed calls
                    ms, _ = time_steps(lambda: ctx.key_join(fact_k, dim_k, 0, index, lg_slots, order, out=out,
                                                            algo=algo, workspace=ws, check_fk=False), steps, 1,
                                       torch)
                    res[f"keyed_{oname}_{aname}"] = {"ms": round(ms, 3),
                                                     "out_GB_per_s": round(n_fact * 80 / (ms * 1e-3) / 1e9, 2)}
                    del ws
            del dim_k, fact_k, keys, index
        if s == 0.0:
            import oracle

            f_host, d_host = fact[: 1 << 22].cpu().numpy(), dim.cpu().numpy()
            res["cpu_oracle"] = oracle_rate(lambda: oracle.fk_join_fact_order(f_host, d_host, 0), 1 << 22,
                                            "fact rows/s", "the first 2^22 fact rows (Zipf 0) of the fact-order join")
            del f_host, d_host
        del fact
        torch.cuda.empty_cache()
    del dim, out
    torch.cuda.empty_cache()
    return {"workload": "fact 2^28 x 16 B (uint32 fk, Zipf s over 2^24 ids) joined with dimension 2^24 x 64 B; "
                        "keyed_*: the same join (s = 0) over distinct non-dense uint32 keys, through a hash index "
                        "of 2^25 slots (auto: DPG lookup, planner's move); "
                        "output 2^28 x 80 B rows", **res}


def bench_smj(args, ctx, dpg, synth, torch, np):
    """Sort-merge join with DPG sort (Section 4.1): two relations of 2^24 x
    100 B rows, joined on a 4-byte key uniform over 2^24 values; both sorted by
    the key-pointer sort (copy phase DPG or direct), then merged."""
    dev = "cuda:0"
    n, R, n_keys = 1 << 24, 100, 1 << 24
    seed = synth.SEED_BASE + 7
    log("bench: sort-merge join of 2^24 x 100 B with 2^24 x 100 B rows")
    rel, counts = [], []
    for side in range(2):
        rows = synth.record_bytes(n, R, seed + side, backend="torch", device=dev)
        k = synth.uniform_at(n_keys, torch.arange(n, device=dev), seed + side, synth.STREAM_FK, backend="torch",
                             device=dev).to(torch.int32)
        rows[:, 0:4] = k.view(torch.uint8).reshape(-1, 4)
        rel.append(rows)
        counts.append(torch.bincount(k.to(torch.int64), minlength=n_keys))
    want_rows = int((counts[0] * counts[1]).sum())
    del counts
    cap = want_rows + 1024
    out = torch.empty((cap, 2 * R), dtype=torch.uint8, device=dev)
    res = {"workload": "R, S: 2^24 x 100 B rows each, 4-byte join key uniform over 2^24 values; "
                       f"{want_rows} result rows of 200 B", "result_rows": want_rows}
    steps = max(2, args.steps // 3)
    for name, algo in (("dpg", dpg.ALGO_DPG), ("direct", dpg.ALGO_DIRECT)):
        ws = torch.empty(ctx.sort_merge_join_workspace_bytes(n, R, 0, n, R, 0, 4, algo), dtype=torch.uint8,
                         device=dev)
        got = []
        ms, _, prof = time_and_profile(
            ctx, lambda: got.append(ctx.sort_merge_join(rel[0], rel[1], 0, 0, 4, algo=algo, out=out, workspace=ws)),
            steps, 1, torch)
        rows = got[-1]
        if rows.shape[0] != want_rows or not torch.equal(rows[:, 0:4], rows[:, R:R + 4]):
            raise SystemExit(f"bench: {name} sort-merge join result is wrong")
        kk = rows[:, 0:4].flip(1).contiguous().view(torch.int32).view(-1).to(torch.int64) & 0xFFFFFFFF
        if not bool((kk[1:] >= kk[:-1]).all()):
            raise SystemExit(f"bench: {name} sort-merge join result is not in key order")
        calls = steps
        res[name] = {"ms": round(ms, 3), "input_rows_per_s": round(2 * n / (ms * 1e-3), 1),
                     "kernels_ms_per_join": {k: round(v["ms"] / calls, 4) for k, v in prof.items()},
                     "roofline": roofline_entry(prof, list(prof), None)}
        del ws, got, rows, kk
    res["dpg_over_direct"] = round(res["direct"]["ms"] / res["dpg"]["ms"], 4)
    import oracle

    r_host, s_host = rel[0][: 1 << 20].cpu().numpy(), rel[1][: 1 << 20].cpu().numpy()
    res["cpu_oracle"] = oracle_rate(lambda: oracle.sort_merge_join(r_host, s_host, 0, 0, 4), 2 << 20,
                                    "input rows/s", "the first 2^20 rows of each relation")
    del rel, out, r_host, s_host
    torch.cuda.empty_cache()
    return res


def bench_hash(args, ctx, dpg, synth, torch, np):
    """Batch lookup in a hash index (Section 4.2.3): 2^24 distinct uint32 keys
    in 2^25 slots, 2^26 query keys of which 80 % are stored; DPG (distribute
    by index partition, probe, gather) vs one direct probe per query."""
    dev = "cuda:0"
    n, s, m = 1 << 24, 25, 1 << 26
    seed = synth.SEED_BASE + 6
    log(f"bench: hash index of {n} keys in 2^{s} slots, {m} lookups")
    keys = 2 * synth.rids_permutation(1 << 25, seed, backend="torch", device=dev)[:n].to(torch.int64) + 1
    keys = keys.to(torch.int32)  # odd, distinct (bit patterns of uint32)
    t0 = time.perf_counter()
    index = ctx.hash_build(keys, s)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    pick = synth.uniform_at(n, torch.arange(m, device=dev), seed, synth.STREAM_RIDS, backend="torch", device=dev)
    queries = keys[pick.to(torch.int64)].clone()
    hit = synth.uniform_at(10, torch.arange(m, device=dev), seed, synth.STREAM_MIX, backend="torch", device=dev) < 8
    queries[~hit] = 2 * (pick[~hit].to(torch.int32) + 1)  # even: never stored
    out = torch.empty(m, dtype=torch.int32, device=dev)
    ws = torch.empty(ctx.hash_lookup_workspace_bytes(n, s, m, dpg.ALGO_DPG), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    res = {"workload": f"batch lookup of 2^26 uint32 keys (80% stored) in a hash index of 2^24 distinct keys, "
                       f"2^{s} slots + overflow array", "build_s": round(build_s, 4)}
    for name, algo in (("dpg", dpg.ALGO_DPG), ("direct", dpg.ALGO_DIRECT)):
        ms, _, prof = time_and_profile(
            ctx, lambda: ctx.hash_lookup(index, n, s, queries, out, algo=algo, workspace=ws, stream=stream),
            args.steps, args.warmup, torch)
        got = out.cpu().numpy()
        want = np.where(hit.cpu().numpy(), pick.cpu().numpy(), -1)
        if not np.array_equal(got, want):
            raise SystemExit(f"bench: {name} hash lookup differs from the stored rids")
        res[name] = {"ms": round(ms, 4), "lookups_per_s": round(m / (ms * 1e-3), 1),
                     "kernels_ms": {k: round(v["ms"] / v["launches"], 4) for k, v in prof.items()},
                     "roofline": roofline_entry(prof, list(prof), None)}
    res["dpg_over_direct"] = round(res["direct"]["ms"] / res["dpg"]["ms"], 4)
    # what bounds the probe, from its LDS and instruction counters
    # (profiles/lookups_probe_counters.md)
    res["dpg"]["roofline"]["limiter"] = ("latency of dependent reads (query, slot, overflow range) at 13.5 "
                                         "waves per CU: LDS busy <10 %, VALU 19 %, waves waiting 75 %")
    import oracle

    k_host = keys.cpu().numpy().view(np.uint32)
    q_host = queries[: 1 << 22].cpu().numpy().view(np.uint32)
    res["cpu_oracle"] = oracle_rate(lambda: oracle.hash_lookup(k_host, q_host), 1 << 22, "lookups/s",
                                    "the first 2^22 queries against all 2^24 keys")
    del keys, index, queries, out, ws, k_host, q_host
    torch.cuda.empty_cache()
    return res


def bench_btree(args, ctx, dpg, synth, torch, np):
    """Batch lookup in an enhanced B+ tree (Section 4.2.3): 2^26 distinct
    uint32 keys (a 516 MiB tree, twice the Infinity Cache), 2^26 query keys of
    which 80 % are stored; DPG (top-of-tree partition, walks finished with
    each run's leaves in LDS, gather) vs one root-to-leaf walk per query."""
    dev = "cuda:0"
    n, m = 1 << 26, 1 << 26
    seed = synth.SEED_BASE + 8
    log(f"bench: B+ tree of {n} keys, {m} lookups")
    keys = 2 * synth.rids_permutation(1 << 27, seed, backend="torch", device=dev)[:n].to(torch.int64) + 1
    keys = keys.to(torch.int32)  # odd, distinct (bit patterns of uint32)
    t0 = time.perf_counter()
    tree = ctx.btree_build(keys)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    pick = synth.uniform_at(n, torch.arange(m, device=dev), seed, synth.STREAM_RIDS, backend="torch", device=dev)
    queries = keys[pick.to(torch.int64)].clone()
    hit = synth.uniform_at(10, torch.arange(m, device=dev), seed, synth.STREAM_MIX, backend="torch", device=dev) < 8
    queries[~hit] = 2 * (pick[~hit].to(torch.int32) + 1)  # even: never stored
    out = torch.empty(m, dtype=torch.int32, device=dev)
    ws = torch.empty(ctx.btree_lookup_workspace_bytes(n, m, dpg.ALGO_DPG), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    res = {"workload": "batch lookup of 2^26 uint32 keys (80% stored) in an enhanced B+ tree (fanout 32) of "
                       "2^26 distinct keys", "tree_MiB": round(tree.numel() / 2 ** 20, 1),
           "build_s": round(build_s, 4)}
    want = np.where(hit.cpu().numpy(), pick.cpu().numpy(), -1)
    for name, algo in (("dpg", dpg.ALGO_DPG), ("direct", dpg.ALGO_DIRECT)):
        ms, _, prof = time_and_profile(
            ctx, lambda: ctx.btree_lookup(tree, n, queries, out, algo=algo, workspace=ws, stream=stream),
            args.steps, args.warmup, torch)
        if not np.array_equal(out.cpu().numpy(), want):
            raise SystemExit(f"bench: {name} B+ tree lookup differs from the stored rids")
        res[name] = {"ms": round(ms, 4), "lookups_per_s": round(m / (ms * 1e-3), 1),
                     "kernels_ms": {k: round(v["ms"] / v["launches"], 4) for k, v in prof.items()},
                     "roofline": roofline_entry(prof, list(prof), None)}
    res["dpg_over_direct"] = round(res["direct"]["ms"] / res["dpg"]["ms"], 4)
    # what bounds the probe, from its LDS and instruction counters
    # (profiles/lookups_probe_counters.md)
    res["dpg"]["roofline"]["limiter"] = ("instruction issue and LDS latency: VALU busy 46 %, LDS busy 28 % "
                                         "(1.5 bank conflicts per access with swizzled nodes), waves waiting 70 %")
    import oracle

    k_host = keys[: 1 << 22].cpu().numpy().view(np.uint32)
    q_host = queries[: 1 << 22].cpu().numpy().view(np.uint32)

    def walk():
        oracle.btree_lookup(oracle.btree_build(k_host), k_host.size, q_host)

    res["cpu_oracle"] = oracle_rate(walk, 1 << 22, "lookups/s",
                                    "build over the first 2^22 keys, then 2^22 walks")
    del keys, tree, queries, out, ws, pick, hit, k_host, q_host
    torch.cuda.empty_cache()
    return res


def bench_skew_multipass(args, ctx, dpg, synth, torch, np):
    """The two Phase I forms for extreme cases (Sections 2.3 and 7):
    skew-balanced runs from a sorted sample, on 2^26 Zipf(1.2) rids over
    2^26 x 100 B records whose hot records sit together; and two-pass DPG on a
    64 GiB source (2^30 x 64 B, 2^27 uniform rids), against the one-pass
    partition with longer runs and the direct gather."""
    dev = "cuda:0"
    steps = max(2, args.steps // 3)
    res = {}

    def timed(name, src, rids, algo, dist=0, lg=0):
        ctx.set_option(dpg.OPT_DISTRIBUTE, dist)
        ctx.set_option(dpg.OPT_LOG2_RUN, lg)
        try:
            plan = ctx.plan_retrieve(src.shape[0], src.shape[1], rids.numel(), algo)
            ws = torch.empty(max(1, plan.workspace_bytes), dtype=torch.uint8, device=dev)
            dst = torch.empty((rids.numel(), src.shape[1]), dtype=torch.uint8, device=dev)
            ms, _ = time_steps(lambda: ctx.retrieve(src, rids, dst=dst, algo=algo, workspace=ws), steps, 1, torch)
            pick = torch.arange(0, rids.numel(), 997, device=dev)
            if not torch.equal(dst[pick], src[rids[pick].to(torch.int64)]):
                raise SystemExit(f"bench: {name} retrieval differs from src[rids]")
            res[name] = {"ms": round(ms, 3), "log2_run": plan.log2_run, "runs": plan.n_runs,
                         "distribute": plan.distribute}
            del ws, dst
        finally:
            ctx.set_option(dpg.OPT_DISTRIBUTE, 0)
            ctx.set_option(dpg.OPT_LOG2_RUN, 0)

    n, R = 1 << 26, 100
    log("bench: skewed rids (Zipf 1.2, hot records together), 2^26 x 100 B")
    src = synth.record_bytes(n, R, synth.SEED_BASE + 9, backend="torch", device=dev)
    rids = synth.zipf_fk_at(n, 1.2, torch.arange(n, device=dev), synth.SEED_BASE + 9, permute_ids=False,
                            backend="torch", device=dev).to(torch.int32)
    timed("zipf1.2_direct", src, rids, dpg.ALGO_DIRECT)
    timed("zipf1.2_dpg_partition", src, rids, dpg.ALGO_DPG, dpg.DIST_PARTITION)
    timed("zipf1.2_dpg_sampled", src, rids, dpg.ALGO_DPG, dpg.DIST_SAMPLED)
    del src, rids
    torch.cuda.empty_cache()
    n, R, m = 1 << 30, 64, 1 << 27
    log("bench: 64 GiB source (2^30 x 64 B), 2^27 uniform rids")
    src = torch.empty((n, R), dtype=torch.uint8, device=dev)
    synth.record_bytes(n, R, synth.SEED_BASE + 10, backend="torch", device=dev, out=src)
    rids = synth.uniform_at(n, torch.arange(m, device=dev), synth.SEED_BASE + 10, synth.STREAM_RIDS,
                            backend="torch", device=dev).to(torch.int32)
    timed("big_direct", src, rids, dpg.ALGO_DIRECT)
    timed("big_dpg_one_pass", src, rids, dpg.ALGO_DPG)
    timed("big_dpg_two_pass", src, rids, dpg.ALGO_DPG, dpg.DIST_TWO_PASS, 16)
    del src, rids
    torch.cuda.empty_cache()
    res["workload"] = ("zipf: 2^26 Zipf(1.2) rank-ordered rids over 2^26 x 100 B; big: 2^27 uniform rids over "
                       "2^30 x 64 B (64 GiB)")
    return res


def bench_serve(args, ctx, dpg, synth, torch, np, max_log2=22, seed_off=0, algo=None, mode_names=None):
    """4096 requests (75 % retrievals, 25 % fact-order or dimension-order
    joins), N log-uniform in [2^10, 2^max_log2], record size uniform over
    {16, 64, 100, 256} B, rids a random permutation of [0, N); tables resident;
    Poisson arrivals; admission under a 64 GiB arena.  algo: the requests'
    algorithm (default AUTO); mode_names: the server modes to run (default
    all)."""
    algo = dpg.ALGO_AUTO if algo is None else algo
    dev = "cuda:0"
    n_req = args.serve_requests
    seed = synth.SEED_BASE + 4 + seed_off
    rng = np.random.default_rng(seed)
    sizes = (16, 64, 100, 256)
    log(f"bench: serving workload, {n_req} requests")
    tables = {R: synth.record_bytes(1 << 22, R, seed + R, backend="torch", device=dev) for R in sizes}
    bases = [synth.rids_permutation(1 << 22, seed + 100 + k, backend="torch", device=dev) for k in range(4)]
    reqs, keep, shapes = [], [], []
    for k in range(n_req):
        u = rng.uniform(math.log(1 << 10), math.log((1 << max_log2) + 1))
        n = int(min(1 << max_log2, max(1 << 10, math.floor(math.exp(u)))))
        R = int(sizes[rng.integers(0, 4)])
        if rng.random() < 0.75:
            base = bases[rng.integers(0, 4)]
            rids = base[base < n].contiguous()  # a uniformly random permutation of [0, n)
            reqs.append(dpg.Request(dpg.REQ_RETRIEVE, algo, tables[R].data_ptr(), n, R, 0,
                                    rids.data_ptr(), None, n, 0, 0, None))
            keep.append(rids)
            shapes.append(("retrieve", n, R))
        else:
            n_dim = max(1, n // 16)
            fk = synth.uniform_at(n_dim, torch.arange(n, device=dev), seed * 7 + k, synth.STREAM_FK,
                                  backend="torch", device=dev).to(torch.int32)
            fact = synth.record_bytes(n, 16, seed * 7 + k, synth.STREAM_FACT, backend="torch", device=dev)
            fact[:, 0:4] = fk.view(torch.uint8).reshape(-1, 4)
            order = int(rng.integers(0, 2))
            reqs.append(dpg.Request(dpg.REQ_FK_JOIN, algo, tables[R].data_ptr(), n_dim, R, 16, None,
                                    fact.data_ptr(), n, 0, order, None))
            keep.append(fact)
            shapes.append(("join", n, R))
    torch.cuda.synchronize()
    out_bytes = sum(n * (R if kind == "retrieve" else R + 16) for kind, n, R in shapes)
    arrivals = np.cumsum(rng.exponential(1.0, n_req))  # unit-rate Poisson process, scaled by the rate

    def run(server, rate):
        """Submit at Poisson arrival times (rate requests/s; None: all at once,
        in one submit_many call), release outputs as they complete; returns
        the server's stats."""
        server.reset_stats()
        pending = {}
        t0 = time.perf_counter()
        k = done = checked = 0
        if rate is None:
            # saturation: the whole queue handed over as one burst
            for i, t in enumerate(server.submit_many(reqs)):
                pending[t] = i
            k = n_req
        while done < n_req:
            now = time.perf_counter() - t0
            while k < n_req and arrivals[k] / rate <= now:
                pending[server.submit(reqs[k])] = k
                k += 1
            t = server.next_completed(0 if k < n_req else 50)
            while t is not None:
                state, status, dst, _ = server.poll(t)
                if state != dpg.TICKET_DONE:
                    raise SystemExit(f"bench: serving request failed with status {status}")
                i = pending.pop(t)
                if checked < 8 and shapes[i][0] == "retrieve":
                    n, R = shapes[i][1], shapes[i][2]
                    j = n // 2
                    row = dpg.copy_device_bytes(dst + j * R, R).cpu().numpy()
                    if not np.array_equal(row, tables[R][int(keep[i][j])].cpu().numpy()):
                        raise SystemExit("bench: served output differs")
                    checked += 1
                server.release(t)
                done += 1
                t = server.next_completed(0)
        return server.stats()

    algo_name = {dpg.ALGO_AUTO: "AUTO", dpg.ALGO_DPG: "DPG", dpg.ALGO_DIRECT: "direct"}[algo]
    res = {"workload": f"{n_req} requests: 75% retrieval, 25% FK join (either order); N log-uniform "
                       f"[2^10, 2^{max_log2}]; record size uniform over {{16,64,100,256}} B; random-permutation rids; "
                       f"resident tables; Poisson arrivals; 64 GiB HBM budget; algorithm {algo_name}",
           "output_GB_total": round(out_bytes / 1e9, 2)}
    budget = 64 << 30
    modes = {"batched_graph": dict(max_inflight=4, max_batch_requests=256, use_graph=True),
             "batched_eager": dict(max_inflight=4, max_batch_requests=256, use_graph=False),
             "batched_window": dict(max_inflight=4, max_batch_requests=256, use_graph=False, batch_window_us=50),
             "per_request": dict(max_inflight=4, max_batch_requests=1, use_graph=False)}
    if mode_names:
        modes = {k: v for k, v in modes.items() if k in mode_names}
    servers = {}
    try:
        sat = {}
        for name, kw in modes.items():
            servers[name] = dpg.Server(ctx, budget, **kw)
            log(f"bench: serving saturation run, {name}")
            # the better of two runs: a single one varies by about 10 %
            st = min((run(servers[name], None) for _ in range(2)), key=lambda t: t["span_s"])
            sat[name] = n_req / st["span_s"]
            res[f"{name}_saturation"] = {"req_per_s": round(sat[name], 1),
                                         "GB_per_s": round(st["bytes_delivered"] / st["span_s"] / 1e9, 2),
                                         "batches": st["batches"], "host_launch_s": round(st["launch_s"], 4),
                                         "span_s": round(st["span_s"], 4)}
            servers[name].close()
            del servers[name]
        # common arrival rates: 50, 80, 95 and 110 % of what per-request
        # launches sustain; every mode sees the same arrival times at each rate
        res["load_points"] = []
        for frac in (0.5, 0.8, 0.95, 1.1):
            rate = frac * sat["per_request"]
            point = {"fraction_of_per_request_saturation": frac, "arrival_rate_req_per_s": round(rate, 1)}
            for name, kw in modes.items():
                servers[name] = dpg.Server(ctx, budget, **kw)
                log(f"bench: serving at {rate:.0f} req/s, {name}")
                st = run(servers[name], rate)
                point[name] = {"p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                               "max_ms": round(st["max_ms"], 3), "req_per_s": round(n_req / st["span_s"], 1),
                               "GB_per_s": round(st["bytes_delivered"] / st["span_s"] / 1e9, 2),
                               "batches": st["batches"],
                               "arena_high_water_GB": round(st["arena_high_water"] / 1e9, 2)}
                servers[name].close()
                del servers[name]
            res["load_points"].append(point)
    finally:
        for srv in servers.values():
            srv.close()
    del tables, bases, keep
    torch.cuda.empty_cache()
    return res


def main():
    global NO_CPU
    args = parse()
    NO_CPU = args.no_cpu
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_cs_0308004_amd import dpg, synth

    only = set(s for s in args.only.split(",") if s) or {"retrieve", "lds", "small", "sweep", "sort", "join", "smj",
                                                          "hash", "btree", "skew", "serve"}
    counters = None
    if os.path.exists(args.counters):
        with open(args.counters) as f:
            counters = json.load(f)
    ctx = dpg.Context(0)
    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, b
    out = {"metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic"}
    cpu = None
    if "retrieve" in only:
        r, cpu = bench_retrieve(args, ctx, dpg, synth, torch, np, counters)
        out.update(r)
    if "lds" in only:
        out["dpg_lds_probe"] = bench_lds_probe(args, ctx, dpg, synth, torch, np)
        if out["dpg_lds_probe"] and out.get("ms_per_step"):
            out["dpg_lds_probe"]["over_default_dpg"] = round(out["ms_per_step"] / out["dpg_lds_probe"]["ms_per_step"], 4)
    if "small" in only:
        out["small_1m_x_100B"] = bench_small(args, ctx, dpg, synth, torch, np)
    if "sweep" in only:
        out["sweep_2p26"] = bench_sweep(args, ctx, dpg, synth, torch, np)
    if "sort" in only:
        out["sort"] = bench_sort(args, ctx, dpg, synth, torch, np)
    if "join" in only:
        out["join"] = bench_join(args, ctx, dpg, synth, torch, np)
    if "smj" in only:
        out["sort_merge_join"] = bench_smj(args, ctx, dpg, synth, torch, np)
    if "hash" in only:
        out["hash_lookup"] = bench_hash(args, ctx, dpg, synth, torch, np)
    if "btree" in only:
        out["btree_lookup"] = bench_btree(args, ctx, dpg, synth, torch, np)
    if "skew" in only:
        out["skew_multipass"] = bench_skew_multipass(args, ctx, dpg, synth, torch, np)
    if "serve" in only:
        out["serving"] = bench_serve(args, ctx, dpg, synth, torch, np)
        # the same mix restricted to small requests (N up to 2^14), where
        # launch cost rather than HBM bandwidth decides throughput
        out["serving_small"] = bench_serve(args, ctx, dpg, synth, torch, np, max_log2=14, seed_off=1)
        # the small-request mix with every retrieval and fact-order join
        # planned as DPG: the batch runs their phases as steps of the
        # persistent launch, per-request launches run each phase alone
        out["serving_small_dpg"] = bench_serve(args, ctx, dpg, synth, torch, np, max_log2=14, seed_off=1,
                                               algo=dpg.ALGO_DPG, mode_names=("batched_graph", "per_request"))
    if cpu is not None:
        out["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
