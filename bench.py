"""Benchmark: DPG record retrieval on one MI355X.

Default workload: 2^26 source records of 100 B (10-byte uniform key + 90-byte
payload), rids a pseudo-random permutation of [0, 2^26), 2^26 outputs.  One
step is one full DPG retrieval (distribute, probe, gather); the direct-gather
kernel is timed beside it on the same inputs.  Inputs are resident in HBM
before timing starts.

Prints one JSON line (see README/DESIGN for the fields).
"""
from __future__ import annotations

import argparse
import json
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
    ap.add_argument("--log2-run", type=int, default=0, help="force L = 2^v records per run (0: planner)")
    ap.add_argument("--probe", type=int, default=0, help="1 cached, 2 LDS (0: planner)")
    ap.add_argument("--dist", type=int, default=0, help="Phase I: 1 append, 2 partition (0: planner)")
    ap.add_argument("--counters", default=os.path.join(ROOT, "profiles", "counters.json"),
                    help="HBM byte counts measured with rocprofv3 --pmc (optional)")
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


def cpu_baseline(src_dev, rids_np, rec_bytes, target_s, torch):
    """The oracle (single-threaded C loop) on a bounded prefix of the rid list,
    against the full source copied to host memory."""
    import numpy as np

    import oracle

    src = src_dev.cpu().numpy()
    m_total = rids_np.size
    m = min(m_total, 1 << 20)
    t0 = time.perf_counter()
    oracle.retrieve(src, rids_np[:m])
    dt = time.perf_counter() - t0
    if dt < target_s and m < m_total:
        m = int(min(m_total, m * max(1.0, target_s / max(dt, 1e-3))))
        t0 = time.perf_counter()
        oracle.retrieve(src, rids_np[:m])
        dt = time.perf_counter() - t0
    del src
    return {
        "value": round(m * rec_bytes / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {m} of {m_total} rids over the full {rec_bytes}-byte source; "
                  f"{dt:.2f} s single-threaded on {platform.processor() or platform.machine()} "
                  f"(host has {os.cpu_count()} logical CPUs)",
    }


def roofline_entry(prof: dict, kernels: list[str], counters: dict | None):
    """The dominant kernel of the step: algorithmic bytes per launch over its
    average launch duration (HIP events on the kernel's stream)."""
    cand = {k: v for k, v in prof.items() if k in kernels}
    name = max(cand, key=lambda k: cand[k]["ms"])
    v = cand[name]
    avg_ms = v["ms"] / v["launches"]
    bytes_per_launch = v["bytes"] / v["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    if counters and name in counters.get("kernels", {}):
        traffic = counters["kernels"][name].get("hbm_bytes_per_launch")
    return {
        "kernel": name,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "avg_launch_ms": round(avg_ms, 4),
        "alg_bytes_per_launch": bytes_per_launch,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_cs_0308004_amd import dpg, synth

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
    ctx = dpg.Context(0)
    ctx.set_option(dpg.OPT_LOG2_RUN, args.log2_run)
    ctx.set_option(dpg.OPT_PROBE, args.probe)
    ctx.set_option(dpg.OPT_DISTRIBUTE, args.dist)
    plan = ctx.plan_retrieve(n, R, m, dpg.ALGO_DPG)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    ws_direct = torch.empty(256, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step_dpg():
        ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DPG, workspace=ws, stream=stream)

    def step_direct():
        ctx.retrieve(src, rids, dst=dst, algo=dpg.ALGO_DIRECT, workspace=ws_direct, stream=stream)

    log(f"bench: plan L=2^{plan.log2_run} runs={plan.n_runs} tile={plan.dist_tile} probe={plan.probe}")
    # timed region, with per-kernel HIP events on the library's stream
    ctx.profile_enable(True)
    step_dpg()
    torch.cuda.synchronize()
    ctx.profile_reset()
    ms_dpg, wall_dpg = time_steps(step_dpg, args.steps, args.warmup, torch)
    prof_dpg = ctx.profile_collect()
    # the warmup launches are in the profile too; per-launch averages are unaffected
    ctx.profile_reset()
    ms_direct, _ = time_steps(step_direct, args.steps, args.warmup, torch)
    prof_direct = ctx.profile_collect()
    ctx.profile_enable(False)
    log(f"bench: dpg {ms_dpg:.3f} ms/step, direct {ms_direct:.3f} ms/step")

    # a spot check of the timed output against the generator (not the oracle)
    sample = np.random.default_rng(0).integers(0, m, 256)
    rids_np = rids.cpu().numpy()
    step_dpg()
    torch.cuda.synchronize()
    got = dst[torch.from_numpy(sample).to(dev)].cpu().numpy()
    if not np.array_equal(got, synth.records_at(rids_np[sample], R, seed)):
        raise SystemExit("bench: DPG output differs from the generator's records")

    delivered = m * R
    counters = None
    if os.path.exists(args.counters):
        with open(args.counters) as f:
            counters = json.load(f)
    dpg_kernels = ["k_dist_hist", "k_dist_scatter", "k_probe_cached", "k_probe_lds", "k_gather_phase"]
    out = {
        "metric": METRIC,
        "value": round(delivered / (ms_dpg * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_dpg, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": f"DPG record retrieval, N=M=2^{args.log2n}, {R}-byte records, rids {args.pattern}",
            "n_src": n, "n_rids": m, "rec_bytes": R, "rid_pattern": args.pattern,
            "algo": "dpg", "log2_run": plan.log2_run, "n_runs": plan.n_runs, "dist_tile": plan.dist_tile,
            "probe": {1: "cached", 2: "lds"}.get(plan.probe, "?"),
        },
        "roofline": roofline_entry(prof_dpg, dpg_kernels, counters),
        "direct": {
            "value": round(delivered / (ms_direct * 1e-3) / 1e9, 2),
            "unit": "GB/s",
            "ms_per_step": round(ms_direct, 4),
            "roofline": roofline_entry(prof_direct, ["k_direct_gather"], counters),
        },
        "dpg_over_direct": round(ms_direct / ms_dpg, 4),
        "kernels_ms_per_step": {k: round(v["ms"] / v["launches"], 4) for k, v in prof_dpg.items()},
        "wall_s_timed": round(wall_dpg, 4),
    }
    if not args.no_cpu:
        log("bench: timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(src, rids_np, R, args.cpu_seconds, torch)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
