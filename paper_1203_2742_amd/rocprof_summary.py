"""Summarize rocprofv3 CSV output of bench.py runs into profiles/.

    python -m paper_1203_2742_amd.rocprof_summary --workload grid3d_40 --steps 2 \\
        --trace out/prof_trace --fetch out/prof_fetch --write out/prof_write \\
        --command "<the rocprofv3 command lines>"

Writes profiles/kernels_<workload>.md (kernel durations from --kernel-trace
--stats, grouped by the operation of the step each kernel serves, with the
time per step of every operation; HBM bytes from FETCH_SIZE / WRITE_SIZE)
and profiles/traffic_<workload>.json, which bench.py reads for the
roofline's "traffic" field (HBM bytes per call of an operation).  The byte
counters are scaled by what the same counters report for the run's
calibration copy (an elementwise kernel that reads and writes exactly
--calib-mib MiB).  --steps is the number of steps of each profiled run, the
warm-up step included (bench.py --profile-run: warmup + steps).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

# kernel symbol (without namespace and arguments) -> operation of the step;
# the template tags of the wide-front and gather kernels name their caller
OP_OF = [
    (r"^k_factor", "factor"), (r"^k_wide_update<0>", "factor"), (r"^k_fat_panel<0>", "factor"),
    (r"^k_fat_(potrf_diag|potrf_panel|potrf_trail|trtri_row)<0>", "factor"), (r"^k_fat_factor_fin", "factor"),
    (r"^k_product", "cholesky_product"), (r"^k_wide_update<3>", "cholesky_product"),
    (r"^k_fat_panel<3>", "cholesky_product"), (r"^k_fat_up_fin<0>", "cholesky_product"),
    (r"^k_projinv", "projected_inverse"), (r"^k_wide_extract<0>", "projected_inverse"),
    (r"^k_wide_projinv", "projected_inverse"),
    (r"^k_hess_", "hessian"), (r"^k_wide_update<1>", "hessian"), (r"^k_wide_hdown", "hessian"),
    (r"^k_fat_panel<1>", "hessian"), (r"^k_fat_up_fin<1>", "hessian"),
    (r"^k_ihess_", "inv_hessian"), (r"^k_wide_update<2>", "inv_hessian"), (r"^k_vinv", "inv_hessian"),
    (r"^k_gather_map<1>", "inv_hessian"), (r"^k_wide_extract<1>", "inv_hessian"),
    (r"^k_fat_panel<2>", "inv_hessian"), (r"^k_fat_up_fin<2>", "inv_hessian"), (r"^k_fat_ihess", "inv_hessian"),
    (r"^k_completion", "completion"), (r"^k_gather_map<2>", "completion"),
    (r"^k_wide_extract<2>", "completion"), (r"^k_fat_compl", "completion"),
    (r"^k_fat_(potrf_diag|potrf_panel|potrf_trail|trtri_row)<1>", "completion"),
    (r"^k_bigv_\w+<0>", "inv_hessian"), (r"^k_bigv_\w+<1>", "completion"), (r"^k_bigv_\w+<2>", "hessian_factor"),
    (r"^k_gamma", "hessian_factor"), (r"^k_hfactor_adj", "hessian_factor_adj"), (r"^k_hfactor", "hessian_factor"),
    (r"^k_gram", "gram"),
    (r"^k_logdet", "logdet (2 calls)"), (r"^k_reset_status", "status reset"),
    (r"^k_export_ldl", "factor_export_ldl"),
    (r"^k_relax_(in|out)", "relaxed-plan maps (X, Y in; S, T out)"),
    (r"^k_up_panel_tiles<0>", "cholesky_product"), (r"^k_up_panel_tiles<1>", "inv_hessian"),
]


def symbol(name: str) -> str:
    return name.split("(")[0].replace("mfb::", "").replace("void ", "").strip()


def op_of(name: str) -> str:
    sym = symbol(name)
    for pat, op in OP_OF:
        if re.match(pat, sym):
            return op
    return sym


def read_counter(d, calib_pat):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
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
        a = agg[op_of(nm)]
        a[0] += 1
        a[1] += v
    return agg, calib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--steps", type=int, required=True, help="steps per profiled run (warm-up included)")
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--counter-steps", type=int, help="steps of the counter runs (default --steps)")
    ap.add_argument("--calib-mib", type=int, default=256)
    ap.add_argument("--calib-kernel", default="neg_kernel")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    from bench import kernel_source_hash

    stats = glob.glob(os.path.join(args.trace, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = [r for r in csv.DictReader(open(stats)) if "mfb::" in r["Name"]]
    agg = {}
    for r in rows:
        a = agg.setdefault(op_of(r["Name"]), {"calls": 0, "total": 0.0, "pct": 0.0})
        a["calls"] += int(r["Calls"])
        a["total"] += float(r["TotalDurationNs"])
        a["pct"] += float(r["Percentage"])
    steps = args.steps
    lines = [f"# Kernel profile: {args.workload}", "", "Commands:", "", "```", args.command.strip(), "```",
             "", "## rocprofv3 --kernel-trace --stats, per operation of the step", "",
             f"Every kernel is attributed to the operation whose call launches it; the time per step is "
             f"the total over the run divided by its {steps} steps.  bench.py's roofline names one "
             f"operation and its time per call (all its launches), which this column reproduces.  "
             f"Operations that the step runs concurrently on two streams (the completion and the "
             f"product beside the Hessian) show their kernels' durations under that contention, longer "
             f"than alone (bench.py's per_op_ms times every operation alone); the operation named by "
             f"the roofline runs alone.", "",
             "| operation | kernel launches | total ms | ms per step | % of kernel time |",
             "|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["total"]):
        lines.append(f"| {k} | {a['calls']} | {a['total'] / 1e6:.3f} | {a['total'] / 1e6 / steps:.3f} | "
                     f"{a['pct']:.2f} |")
    lines += ["", "## per kernel symbol", "",
              "| symbol | operation | calls | total ms | avg us |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| {symbol(r['Name'])} | {op_of(r['Name'])} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.2f} |")
    if args.fetch and args.write:
        csteps = args.counter_steps or steps
        fa, fc = read_counter(args.fetch, args.calib_kernel)
        wa, wc = read_counter(args.write, args.calib_kernel)
        known_kib = args.calib_mib * 1024.0
        fs, ws = known_kib / fc, known_kib / wc
        lines += ["", "## HBM bytes per step (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
                  f"Calibration: an elementwise copy of {args.calib_mib} MiB reads {fc:.1f} KiB by "
                  f"FETCH_SIZE and writes {wc:.1f} KiB by WRITE_SIZE, so the counters are scaled by "
                  f"{fs:.4f} (fetch) and {ws:.4f} (write).  Each counter run has {csteps} steps.", "",
                  "| operation | dispatches | fetch MB/step (scaled) | write MB/step (scaled) | total MB/step |",
                  "|---|---|---|---|---|"]
        traffic = {}
        for k in sorted(fa, key=lambda k: -fa[k][1]):
            f_mb = fa[k][1] * fs * 1024.0 / csteps / 1e6
            w_mb = (wa[k][1] * ws * 1024.0 / csteps / 1e6) if k in wa else 0.0
            traffic[k] = (f_mb + w_mb) * 1e6
            lines.append(f"| {k} | {fa[k][0]} | {f_mb:.2f} | {w_mb:.2f} | {f_mb + w_mb:.2f} |")
        tj = {"workload": args.workload, "source_hash": kernel_source_hash(), "fetch_scale": fs,
              "write_scale": ws, "steps": csteps,
              "bytes_per_call": {k: round(v, 1) for k, v in traffic.items()}}
        with open(os.path.join(args.out, f"traffic_{args.workload}.json"), "w") as fh:
            json.dump(tj, fh, indent=1)
    lines += ["", f"Kernel sources hash: {kernel_source_hash()}", ""]
    with open(os.path.join(args.out, f"kernels_{args.workload}.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
