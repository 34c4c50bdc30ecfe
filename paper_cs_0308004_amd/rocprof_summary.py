"""Summarize rocprofv3 CSV output into the short reports kept with the project.

  python -m paper_cs_0308004_amd.rocprof_summary stats <kernel_stats.csv> <out.md> -- <command...>
  python -m paper_cs_0308004_amd.rocprof_summary bytes <fetch_dir> <write_dir> <reqsize_dir> <out.md>
         <counters.json> <workload key> -- <command...>

  python -m paper_cs_0308004_amd.rocprof_summary counters <out.md> <kernel,kernel,...> <dir> [<dir>...]
         -- <command...>

`counters` averages every counter of each run directory (rocprofv3 --pmc
<counters>) per dispatch of the named kernels, and derives the LDS and
instruction ratios the counters allow (CU_NUM = 256 compute units).

`bytes` reads three counter runs of the same command (rocprofv3 --pmc
FETCH_SIZE; --pmc WRITE_SIZE; --pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum
TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_DRAM_sum).  The command must include a
plain 1 GiB device-to-device copy (bench.py --calib-copy): FETCH_SIZE and
WRITE_SIZE of every kernel are divided by what the counter reads for that
copy per GiB, so the counters' request-size assumptions cancel.  The request-
size run gives the exact L2-to-fabric read bytes as a cross-check, and the DRAM
request count shows how many reads the Infinity Cache did not serve.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import re
import sys
from collections import defaultdict

GIB = 1 << 30


def short_name(name: str) -> str:
    """'void dpg::k_gather_phase<unsigned int, 25, true>(...)' -> 'k_gather_phase'."""
    m = re.search(r"dpg::(k_[a-z0-9_]+)", name)
    if m:
        return m.group(1)
    return name.split("(")[0][:80]


def template_args(name: str) -> str:
    """'void dpg::k_probe_cached<unsigned int __vector(4), 4, true>(...)' -> 'u32x4, 4, true'."""
    m = re.search(r"dpg::k_[a-z0-9_]+<(.*?)>\(", name)
    if not m:
        return ""
    s = m.group(1)
    for a, b in (("unsigned int __vector(4)", "u32x4"), ("unsigned int __vector(2)", "u32x2"),
                 ("unsigned long", "u64"), ("unsigned int", "u32")):
        s = s.replace(a, b)
    return s


def read_csv(path: str) -> list[dict]:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def find(dir_: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dir_, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {dir_}")
    return hits[0]


def stats_report(stats_csv: str, out_md: str, command: str):
    rows = read_csv(stats_csv)
    lines = ["# Kernel durations (rocprofv3 --kernel-trace --stats)", "", f"Command: `{command}`", "",
             "| kernel | template arguments | calls | average (us) | total (ms) | % of GPU time |",
             "|---|---|---:|---:|---:|---:|"]
    for r in rows:
        name = r.get("Name") or r.get("Kernel_Name") or ""
        if not short_name(name).startswith("k_"):
            continue
        lines.append(f"| {short_name(name)} | {template_args(name)} | {int(r['Calls'])} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['Percentage']):.2f} |")
    lines += ["", "Kernels of other libraries (input generation by torch, runtime copies) are omitted."]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def dispatch_counters(dir_: str) -> dict:
    """{dispatch id: (kernel name, {counter: value})}"""
    out = {}
    for r in read_csv(find(dir_, "counter_collection.csv")):
        d = out.setdefault(int(r["Dispatch_Id"]), (r["Kernel_Name"], {}))
        d[1][r["Counter_Name"]] = float(r["Counter_Value"])
    return out


def per_kernel(disp: dict, fn) -> dict:
    acc = defaultdict(list)
    for name, c in disp.values():
        v = fn(c)
        if v is not None:
            acc[name].append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def calibration(fetch: dict, write: dict):
    """The copy kernel dispatch that wrote (close to) 1 GiB."""
    best = None
    for did, (name, c) in write.items():
        if "copyBuffer" not in name or "WRITE_SIZE" not in c:
            continue
        err = abs(c["WRITE_SIZE"] * 1024 - GIB)
        if best is None or err < best[0]:
            best = (err, did)
    if best is None or best[0] > 0.01 * GIB:
        raise SystemExit("no 1 GiB calibration copy found (run the command with --calib-copy)")
    did = best[1]
    # both runs execute the same command, so dispatch ids correspond
    if did not in fetch or "copyBuffer" not in fetch[did][0] or "FETCH_SIZE" not in fetch[did][1]:
        raise SystemExit("the calibration copy has no matching dispatch in the FETCH_SIZE run")
    return fetch[did][1]["FETCH_SIZE"] * 1024 / GIB, write[did][1]["WRITE_SIZE"] * 1024 / GIB


def bytes_report(fetch_dir, write_dir, req_dir, out_md, out_json, workload, command):
    fetch_d, write_d = dispatch_counters(fetch_dir), dispatch_counters(write_dir)
    req_d = dispatch_counters(req_dir) if req_dir != "-" else {}
    f_scale, w_scale = calibration(fetch_d, write_d)
    fetch = per_kernel(fetch_d, lambda c: c.get("FETCH_SIZE"))
    write = per_kernel(write_d, lambda c: c.get("WRITE_SIZE"))
    exact = per_kernel(req_d, lambda c: 32 * c.get("TCC_EA0_RDREQ_32B_sum", 0) + 64 * c.get("TCC_EA0_RDREQ_64B_sum", 0)
                       + 128 * c.get("TCC_EA0_RDREQ_128B_sum", 0) if "TCC_EA0_RDREQ_128B_sum" in c else None)
    dram = per_kernel(req_d, lambda c: c.get("TCC_EA0_RDREQ_DRAM_sum"))
    lines = ["# HBM bytes per dispatch", "",
             f"Command (once per counter set): `{command}`", "",
             "Runs: `rocprofv3 --pmc FETCH_SIZE`, `rocprofv3 --pmc WRITE_SIZE`, and `rocprofv3 --pmc "
             "TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_DRAM_sum`, each "
             "with `--output-format csv` and the command above.", "",
             f"Calibration: a plain 1 GiB device copy (`__amd_rocclr_copyBuffer`) reads {f_scale:.4f} GiB by "
             f"FETCH_SIZE and writes {w_scale:.4f} GiB by WRITE_SIZE.  Scaled traffic below = FETCH_SIZE / "
             f"{f_scale:.4f} + WRITE_SIZE / {w_scale:.4f}.  (FETCH_SIZE counts every read request as 64 B; "
             "gfx950 fills 128-byte lines, hence the factor.)", "",
             "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | scaled traffic (GB) | exact reads by request size (GB) "
             "| DRAM read requests (M) |",
             "|---|---:|---:|---:|---:|---:|"]
    kernels = {}
    for k in sorted(set(fetch) & set(write), key=lambda x: -(fetch[x] + write[x])):
        name = short_name(k)
        if not name.startswith("k_") or name in kernels:
            continue
        hbm = fetch[k] * 1024 / f_scale + write[k] * 1024 / w_scale
        kernels[name] = {"fetch_kib_per_dispatch": round(fetch[k], 1), "write_kib_per_dispatch": round(write[k], 1),
                         "hbm_bytes_per_launch": round(hbm), "exact_read_bytes": round(exact.get(k, 0)),
                         "dram_read_requests": round(dram.get(k, 0))}
        lines.append(f"| {name} | {fetch[k]:.0f} | {write[k]:.0f} | {hbm / 1e9:.3f} | "
                     f"{exact.get(k, 0) / 1e9:.3f} | {dram.get(k, 0) / 1e6:.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(out_json, "w") as f:
        json.dump({"workload": workload, "command": command,
                   "calibration": {"kernel": "__amd_rocclr_copyBuffer (1 GiB)", "fetch_scale": round(f_scale, 6),
                                   "write_scale": round(w_scale, 6)},
                   "kernels": kernels}, f, indent=1)


CU_NUM = 256
XCD_NUM = 8  # GRBM_GUI_ACTIVE comes summed over the XCDs: per XCD it is the kernel's cycles


def counters_report(out_md: str, kernels: list[str], dirs: list[str], command: str):
    """Mean of each counter per dispatch, per kernel, over the runs in dirs."""
    per = defaultdict(lambda: defaultdict(list))  # kernel -> counter -> values (one per dispatch)
    passes = []
    for d in dirs:
        names = set()
        for name, c in dispatch_counters(d).values():
            k = short_name(name)
            if k not in kernels:
                continue
            for cn, v in c.items():
                per[k][cn].append(v)
                names.add(cn)
        passes.append(sorted(names))
    lines = ["# Instruction and LDS counters per dispatch", "",
             f"Command: `{command}`", "",
             "Runs (one per counter set, each `rocprofv3 --pmc <set> --output-format csv -- <command>`):", ""]
    lines += [f"* `{' '.join(p)}`" for p in passes]
    lines += ["", "Mean per dispatch:", ""]
    counters = sorted({cn for k in per for cn in per[k]})
    lines.append("| counter | " + " | ".join(kernels) + " |")
    lines.append("|---|" + "---:|" * len(kernels))
    mean = {k: {cn: sum(v) / len(v) for cn, v in per[k].items()} for k in per}
    for cn in counters:
        lines.append(f"| {cn} | " + " | ".join(f"{mean.get(k, {}).get(cn, float('nan')):.4g}" for k in kernels) + " |")

    def ratio(k, a, b, scale=1.0):
        m = mean.get(k, {})
        if a in m and b in m and m[b]:
            return scale * m[a] / m[b]
        return None

    # GRBM_GUI_ACTIVE / 8 = the kernel's cycles; SQ_WAVE_CYCLES and
    # SQ_WAIT_ANY count in units of 4 cycles (the OccupancyPercent and
    # LdsUtil expressions of rocprofv3 -L use the same scales)
    per_cu = XCD_NUM * 100.0 / CU_NUM
    derived = [
        ("LDS busy, % of CU cycles (SQ_LDS_IDX_ACTIVE / (cycles x 256))",
         lambda k: ratio(k, "SQ_LDS_IDX_ACTIVE", "GRBM_GUI_ACTIVE", per_cu)),
        ("LDS bank conflicts per access (SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT))",
         lambda k: (lambda m: m["SQ_LDS_BANK_CONFLICT"] / (m["SQ_LDS_IDX_ACTIVE"] - m["SQ_LDS_BANK_CONFLICT"])
                    if "SQ_LDS_BANK_CONFLICT" in m and m.get("SQ_LDS_IDX_ACTIVE", 0) > m["SQ_LDS_BANK_CONFLICT"]
                    else None)(mean.get(k, {}))),
        ("LDS busy cycles spent in bank conflicts, %",
         lambda k: ratio(k, "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", 100.0)),
        ("waves waiting on anything, % of wave cycles (SQ_WAIT_ANY / SQ_WAVE_CYCLES)",
         lambda k: ratio(k, "SQ_WAIT_ANY", "SQ_WAVE_CYCLES", 100.0)),
        ("LDS instructions per wave", lambda k: ratio(k, "SQ_INSTS_LDS", "SQ_WAVES")),
        ("VALU instructions per wave", lambda k: ratio(k, "SQ_INSTS_VALU", "SQ_WAVES")),
        ("vector memory reads per wave", lambda k: ratio(k, "SQ_INSTS_VMEM_RD", "SQ_WAVES")),
        ("VALU busy, % of CU cycles (SQ_ACTIVE_INST_VALU / (cycles x 256))",
         lambda k: ratio(k, "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE", per_cu)),
        ("mean resident waves per CU (4 SQ_WAVE_CYCLES / (cycles x 256))",
         lambda k: ratio(k, "SQ_WAVE_CYCLES", "GRBM_GUI_ACTIVE", 4.0 * XCD_NUM / CU_NUM)),
    ]
    lines += ["", "Derived:", "", "| ratio | " + " | ".join(kernels) + " |", "|---|" + "---:|" * len(kernels)]
    for label, fn in derived:
        vals = [fn(k) for k in kernels]
        if all(v is None for v in vals):
            continue
        lines.append(f"| {label} | " + " | ".join("-" if v is None else f"{v:.3g}" for v in vals) + " |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv):
    if "--" not in argv:
        raise SystemExit(__doc__)
    cut = argv.index("--")
    args, command = argv[:cut], " ".join(argv[cut + 1:])
    if args[0] == "stats":
        stats_report(args[1], args[2], command)
    elif args[0] == "bytes":
        bytes_report(args[1], args[2], args[3], args[4], args[5], args[6], command)
    elif args[0] == "counters":
        counters_report(args[1], args[2].split(","), args[3:], command)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
