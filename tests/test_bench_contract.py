"""bench.py's output contract: one JSON line with the metric, the whole-job
throughput, the roofline of the dominant kernel and the oracle's CPU rate;
several GPUs are refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.gpu
def test_bench_line_contract():
    """A 2^20-record retrieval run: every field of the line, the roofline's
    fraction against its own achieved rate, and no HBM traffic figure (the
    stored counters belong to the 2^26 workload)."""
    cmd = [sys.executable, "-u", BENCH, "--only", "retrieve", "--log2n", "20", "--steps", "3", "--warmup", "1",
           "--autotune", "0", "--cpu-seconds", "0.5"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert d["metric"] == "retrieval GB/s, DPG vs direct gather @100B records; p50/p99 batched latency"
    assert d["unit"] == "GB/s" and d["value"] > 0
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["scaling"] in ("weak", "strong") and d["vs_baseline"] is None
    assert d["dtype"] == "u8" and d["data"] == "synthetic"
    # value is the delivered bytes of one step over its time
    assert d["value"] == pytest.approx((1 << 20) * 100 / (d["ms_per_step"] * 1e-3) / 1e9, rel=0.01)
    cfg = d["config"]
    assert "2^20" in cfg["workload"] and cfg["n_src"] == cfg["n_rids"] == 1 << 20 and cfg["rec_bytes"] == 100
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["achieved"] > 0 and roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], abs=1e-4)
    assert roof["traffic"] is None
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1
    assert cpu["unit"] == "GB/s" and cpu["sample"]
    assert cpu["single_core"]["cores"] == 1 and cpu["single_core"]["value"] > 0
    # the timed steps run without per-kernel events; the kernels come from a
    # second, profiled pass
    # (2^20 records of 100 B take the two-phase form: the probe scatters)
    ks = set(d["kernels_ms_per_step"])
    assert "k_part_scatter_unstable" in ks and "k_probe_scatter" in ks and "k_gather_phase" not in ks
    ceil = d["copy_ceiling"]
    assert ceil["GB_per_s"] == max(ceil["shapes_GB_per_s"].values()) > 0
