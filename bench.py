"""Benchmark of the barrier hot path on one MI355X.

One step = one pass over every stage of the path on one input: factor X
(Algorithm 7.1), log det, projected inverse S = P(X^-1) (Algorithm 7.2),
Hessian T = P(X^-1 Y X^-1) for k right-hand sides, inverse Hessian of T,
completion of S (Algorithm 7.3) with log det X-hat, and the values of X-hat
(Cholesky product).  Inputs are resident in HBM before timing starts; CCS
ingest and egress are fused into the kernels.

Output: one JSON line (metric, value = Hessian evaluations per second of the
whole step, roofline of the dominant kernel, CPU-oracle baseline, latency
percentiles, per-operation times, batched-versus-plain Hessian throughput,
and the measured error against the oracle).

    python bench.py [--steps K] [--warmup W] [--workload grid2d_128] [--k 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hessian evals/s + FP64 GB/s·GFLOP/s vs plain path; p50/p99 latency, 1 GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{workload}.json")
KERNEL_SOURCES = ["paper_1203_2742_amd/csrc/kernels.hip", "paper_1203_2742_amd/csrc/wg_dense.h",
                  "paper_1203_2742_amd/csrc/reg_front.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid2d_128")
    ap.add_argument("--k", type=int, default=1, help="Hessian right-hand sides per step")
    ap.add_argument("--batch-k", type=int, default=16, help="k for the batched-vs-plain comparison")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="timed steps only (for runs under rocprofv3): no per-op pass, no "
                         "batched-vs-plain pass, no oracle")
    ap.add_argument("--calibrate-mib", type=int, default=0,
                    help="first run one elementwise copy of this many MiB (reads and writes "
                         "exactly that much), to scale hardware byte counters")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_1203_2742_amd import mfb
    from workloads import get_config, values as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pat = get_config(args.workload)
    n, cp, ri = pat
    nnz = int(cp[-1])
    k = args.k
    log(args, f"workload {args.workload}: n={n} nnz={nnz} k={k}")
    x_h = V.make_x(*pat, seed=0)
    y_h = V.make_ys(*pat, k, seed=0)
    t0 = time.perf_counter()
    b = mfb.SparseBarrier(pat, device=dev)
    plan_s = time.perf_counter() - t0
    info = b.info
    x = torch.from_numpy(x_h).to(dev)
    y = torch.from_numpy(y_h).to(dev)
    s = torch.empty(nnz, dtype=torch.float64, device=dev)
    t = torch.empty_like(y)
    y2 = torch.empty_like(y)
    xhat = torch.empty(nnz, dtype=torch.float64, device=dev)
    ld = torch.empty(2, dtype=torch.float64, device=dev)
    arena = b.arena(max(k, args.batch_k))
    f = b.f

    ops = [
        ("factor", lambda: mfb.factor(f, x)),
        ("logdet", lambda: mfb.logdet(f, ld[0:1])),
        ("projected_inverse", lambda: mfb.projected_inverse(f, s)),
        ("hessian", lambda: mfb.hessian(f, y, t, arena, k=k)),
        ("inv_hessian", lambda: mfb.inv_hessian(f, t, y2, arena, k=k)),
        ("completion", lambda: mfb.completion(f, s)),
        ("logdet_completion", lambda: mfb.logdet(f, ld[1:2])),
        ("cholesky_product", lambda: mfb.cholesky_product(f, xhat)),
    ]

    def step():
        for _, op in ops:
            op()

    if args.calibrate_mib:
        m = args.calibrate_mib * (1 << 20) // 8
        src = torch.ones(m, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K steps, per-step events for the latency percentiles
    K = args.steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    evs[0].record()
    for i in range(K):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(K)])
    total_ms = float(evs[0].elapsed_time(evs[K]))
    log(args, f"timed {K} steps: {total_ms:.3f} ms (wall {wall * 1e3:.3f} ms)")
    status = b.status()

    if args.profile_run:
        print(json.dumps({"metric": METRIC, "value": round(k * K / (total_ms * 1e-3), 3),
                          "unit": "Hessian evals/s", "ms_per_step": round(total_ms / K, 4),
                          "steps": K, "profile_run": True, "status": status[0]}), flush=True)
        return

    # ---- per-operation breakdown (separate pass, events around every op)
    per_op = {name: [] for name, _ in ops}
    for _ in range(max(3, K // 2)):
        for name, op in ops:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            op()
            e1.record()
            per_op[name].append((e0, e1))
    torch.cuda.synchronize()
    per_op_ms = {name: float(np.median([a.elapsed_time(c) for a, c in v])) for name, v in per_op.items()}

    # ---- kernel-level roofline: the library's HIP events around every launch
    mfb.profile_enable(f, True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - p0
    recs = mfb.profile_read(f)
    mfb.profile_enable(f, False)
    agg = {}
    for r in recs:
        a = agg.setdefault(r["kernel"], {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0})
        a["ms"] += r["ms"]
        a["bytes"] += r["bytes"]
        a["flops"] += r["flops"]
        a["launches"] += 1
    dom = max(agg, key=lambda kk: agg[kk]["ms"])
    d = agg[dom]
    avg_launch_ms = d["ms"] / d["launches"]
    bytes_per_launch = d["bytes"] / d["launches"]
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    traffic = None
    tf = TRAFFIC_FILE.format(workload=args.workload)
    if os.path.exists(tf):
        with open(tf) as fh:
            tj = json.load(fh)
        if tj.get("source_hash") == kernel_source_hash():
            traffic = tj.get("bytes_per_launch", {}).get(dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                "kernel": dom, "launches": d["launches"], "avg_launch_us": round(avg_launch_ms * 1e3, 3),
                "algorithmic_bytes_per_launch": round(bytes_per_launch, 1),
                "achieved_gflops": round(d["flops"] / (d["ms"] * 1e-3) / 1e9, 3)}
    kernels = {kk: {"launches": v["launches"], "total_ms_per_step": round(v["ms"] / K, 4),
                    "avg_launch_us": round(v["ms"] / v["launches"] * 1e3, 3),
                    "GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 2),
                    "GFLOPs": round(v["flops"] / (v["ms"] * 1e-3) / 1e9, 2)} for kk, v in agg.items()}

    # ---- batched versus plain Hessian (same workload, k = batch_k)
    kb = args.batch_k
    yb = torch.from_numpy(V.make_ys(*pat, kb, seed=1)).to(dev)
    tb = torch.empty_like(yb)
    reps = 5
    mfb.factor(f, x)
    mfb.hessian(f, yb, tb, arena, k=kb)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(reps):
        mfb.hessian(f, yb, tb, arena, k=kb)
    e1.record()
    for _ in range(reps):
        for r in range(kb):
            mfb.hessian(f, yb[r], tb[r], arena, k=1)
    e2.record()
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / reps
    plain_ms = e1.elapsed_time(e2) / reps
    hess_flops = info["flops_hessian"]

    # ---- correctness of the timed outputs and the CPU-oracle baseline
    cpu = None
    err = None
    if not args.no_cpu:
        import oracle
        res = {}
        c0 = time.perf_counter()
        steps_done = 0
        while True:
            ldl = oracle.factor(pat, x_h)
            res["logdet"] = oracle.logdet(pat, ldl)
            res["s"] = oracle.projinv(pat, ldl)
            res["t"] = [oracle.hessian(pat, ldl, res["s"], y_h[r]) for r in range(k)]
            res["y2"] = [oracle.inv_hessian(pat, ldl, res["s"], res["t"][r]) for r in range(k)]
            lh = oracle.completion(pat, res["s"])
            res["logdet_hat"] = oracle.logdet(pat, lh)
            res["xhat"] = oracle.product(pat, lh)
            steps_done += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        cpu_s = time.perf_counter() - c0
        cpu = {"value": round(k * steps_done / cpu_s, 4), "unit": "Hessian evals/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{steps_done} full steps of the {args.workload} workload (k={k}), "
                         f"single-threaded C oracle, {cpu_s:.1f} s"}
        w = np.where(np.asarray(ri) == V.column_index(n, cp), 1.0, 2.0)

        def rel(a, bb):
            return float(np.sqrt(np.sum(w * (a - bb) ** 2)) / np.sqrt(np.sum(w * bb ** 2)))
        lds = ld.cpu().numpy()
        err = {
            "projected_inverse": rel(s.cpu().numpy(), res["s"]),
            "hessian": max(rel(t[r].cpu().numpy(), res["t"][r]) for r in range(k)),
            "inv_hessian": max(rel(y2[r].cpu().numpy(), res["y2"][r]) for r in range(k)),
            "xhat_vs_oracle": rel(xhat.cpu().numpy(), res["xhat"]),
            "xhat_vs_x": rel(xhat.cpu().numpy(), x_h),
            "logdet": abs(lds[0] - res["logdet"]) / max(1.0, abs(res["logdet"])),
            "logdet_completion": abs(lds[1] - res["logdet_hat"]) / max(1.0, abs(res["logdet_hat"])),
        }
        err = {kk: float(f"{v:.3e}") for kk, v in err.items()}

    value = k * K / (total_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Hessian evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": int(n), "nnz": nnz, "k": k,
                   "nsuper": info["nsuper"], "levels": info["nlevels_up"],
                   "max_front": info["max_front"],
                   "step": "factor+logdet+projected_inverse+hessian(k)+inv_hessian(k)+completion+logdet+product"},
        "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
        "per_op_ms": {kk: round(v, 4) for kk, v in per_op_ms.items()},
        "roofline": roofline,
        "kernels": kernels,
        "profiled_pass_ms_per_step": round(prof_wall * 1e3 / K, 4),
        "batched_vs_plain": {"k": kb, "batched_ms": round(batched_ms, 4), "plain_ms": round(plain_ms, 4),
                             "batched_evals_per_s": round(kb / (batched_ms * 1e-3), 2),
                             "plain_evals_per_s": round(kb / (plain_ms * 1e-3), 2),
                             "batched_gflops": round(kb * hess_flops / (batched_ms * 1e-3) / 1e9, 3)},
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": err,
        "status": status[0],
        "plan_symbolic_s": round(plan_s, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
