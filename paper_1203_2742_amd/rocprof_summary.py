"""Summarize rocprofv3 CSV output of bench.py runs into profiles/.

    python -m paper_1203_2742_amd.rocprof_summary --workload grid2d_128 \\
        --trace out/prof_trace --fetch out/prof_fetch \\
        --write out/prof_write --command "<the rocprofv3 command lines>"

Writes profiles/kernels_<workload>.md (per-kernel duration statistics from
--kernel-trace --stats, HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE)
and profiles/traffic_<workload>.json, which bench.py reads for the
roofline's "traffic" field.  The byte counters are scaled by what the same
counters report for the run's calibration copy (an elementwise kernel that
reads and writes exactly --calib-mib MiB).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def symbol(name: str) -> str:
    return name.split("(")[0].replace("mfb::", "").replace("void ", "")


def short(name: str) -> str:
    """Operation a kernel symbol serves: the register-front variants
    (k_<op>_reg<shape>) and the blocked kernel k_<op> count as one."""
    return symbol(name).split("<")[0].replace("_reg", "")


def read_counter(d, calib_pat):
    f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    agg = collections.defaultdict(lambda: [0, 0.0])
    calib = None
    for r in csv.DictReader(open(f)):
        nm = r["Kernel_Name"]
        v = float(r["Counter_Value"])  # KiB per dispatch
        if calib_pat in nm:
            calib = v
            continue
        if "mfb::" not in nm:
            continue
        a = agg[short(nm)]
        a[0] += 1
        a[1] += v
    return agg, calib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-mib", type=int, default=256)
    ap.add_argument("--calib-kernel", default="neg_kernel")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    from bench import kernel_source_hash

    stats = glob.glob(os.path.join(args.trace, "*kernel_stats.csv"))[0]
    rows = [r for r in csv.DictReader(open(stats)) if "mfb::" in r["Name"]]
    agg = {}
    for r in rows:
        a = agg.setdefault(short(r["Name"]), {"calls": 0, "total": 0.0, "min": float("inf"), "max": 0.0, "pct": 0.0})
        a["calls"] += int(r["Calls"])
        a["total"] += float(r["TotalDurationNs"])
        a["min"] = min(a["min"], float(r["MinNs"]))
        a["max"] = max(a["max"], float(r["MaxNs"]))
        a["pct"] += float(r["Percentage"])
    lines = [f"# Kernel profile: {args.workload}", "", "Commands:", "", "```", args.command.strip(), "```",
             "", "## rocprofv3 --kernel-trace --stats, per operation", "",
             "Register-front variants and the blocked kernel of one operation are summed.", "",
             "| kernel | calls | total ms | avg us | min us | max us | % of time |",
             "|---|---|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["total"]):
        lines.append(f"| {k} | {a['calls']} | {a['total'] / 1e6:.3f} | {a['total'] / a['calls'] / 1e3:.2f} | "
                     f"{a['min'] / 1e3:.2f} | {a['max'] / 1e3:.2f} | {a['pct']:.2f} |")
    lines += ["", "## per kernel symbol", "",
              "| symbol | calls | total ms | avg us |", "|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| {symbol(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} |")
    traffic = {}
    if args.fetch and args.write:
        fa, fc = read_counter(args.fetch, args.calib_kernel)
        wa, wc = read_counter(args.write, args.calib_kernel)
        known_kib = args.calib_mib * 1024.0
        fs, ws = known_kib / fc, known_kib / wc
        lines += ["", "## HBM bytes per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
                  f"Calibration: an elementwise copy of {args.calib_mib} MiB reads {fc:.1f} KiB by "
                  f"FETCH_SIZE and writes {wc:.1f} KiB by WRITE_SIZE, so the counters are scaled by "
                  f"{fs:.4f} (fetch) and {ws:.4f} (write).", "",
                  "| kernel | dispatches | fetch KiB/dispatch (scaled) | write KiB/dispatch (scaled) | total MB/dispatch |",
                  "|---|---|---|---|---|"]
        for k in sorted(fa, key=lambda k: -(fa[k][1] / fa[k][0])):
            f_kib = fa[k][1] / fa[k][0] * fs
            w_kib = wa[k][1] / wa[k][0] * ws if k in wa else 0.0
            traffic[k] = (f_kib + w_kib) * 1024.0
            lines.append(f"| {k} | {fa[k][0]} | {f_kib:.1f} | {w_kib:.1f} | {traffic[k] / 1e6:.3f} |")
        tj = {"workload": args.workload, "source_hash": kernel_source_hash(), "fetch_scale": fs,
              "write_scale": ws, "bytes_per_launch": {k: round(v, 1) for k, v in traffic.items()}}
        with open(os.path.join(args.out, f"traffic_{args.workload}.json"), "w") as fh:
            json.dump(tj, fh, indent=1)
    lines += ["", f"Kernel sources hash: {kernel_source_hash()}", ""]
    with open(os.path.join(args.out, f"kernels_{args.workload}.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
