"""Benchmark of the barrier hot path on one MI355X.

One step = one pass over every stage of the path on one input: factor X
(Algorithm 7.1), log det, projected inverse S = P(X^-1) (Algorithm 7.2),
Hessian T = P(X^-1 Y X^-1) for k right-hand sides, completion of S
(Algorithm 7.3) with log det X-hat, inverse Hessian of T at X-hat (the
Hessian of the dual barrier at S), and the values of X-hat (Cholesky
product).  Factor, log det, gradient and Hessian run on a relaxed plan
(supernodes merged up to --relax explicit zeros; exact for these
operations); completion, inverse Hessian and product run on the
fundamental plan, whose handle the completion fills with the factor of
X-hat = X.  --relax -1 runs every operation on the fundamental plan, with
the inverse Hessian at X before the completion.  Inputs are resident in HBM
before timing starts.

The headline workload is the filled 3D 7-point grid 40^3 under nested
dissection (n = 64000, fronts up to 2360) with k = 16 right-hand sides.  The
JSON line also carries the other measured workloads:

* batched: block-arrow, 64 diagonal blocks of 32-256 plus an arrow of 128,
  Hessian and inverse Hessian of 64 right-hand sides in one call against 64
  single-RHS calls;
* latency: band n = 200, half-bandwidth 5 (a 195-level chain), p50/p99 of
  one log det + gradient + Hessian call sequence;
* grid2d_128: the 2D 5-point grid 128^2 under nested dissection, one step;
* attainable peaks: a device copy (HBM) and an FP64 matrix product.

    python bench.py [--steps K] [--warmup W] [--workload grid3d_40] [--k 16]
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
BALANCE = FP64_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS  # flop per byte at the ridge point
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{workload}.json")
KERNEL_SOURCES = ["paper_1203_2742_amd/csrc/kernels.hip", "paper_1203_2742_amd/csrc/wide.hip",
                  "paper_1203_2742_amd/csrc/wg_dense.h", "paper_1203_2742_amd/csrc/reg_front.h",
                  "paper_1203_2742_amd/csrc/front.h"]
OPS = ("factor", "logdet", "projected_inverse", "hessian", "inv_hessian", "completion",
       "logdet_completion", "cholesky_product")
# profile kernel name -> operation of the step (a launch record belongs to one call)
KERNEL_OP = {"k_factor": "factor", "k_projinv": "projected_inverse", "k_hess_up": "hessian",
             "k_hess_down": "hessian", "k_ihess_down": "inv_hessian", "k_ihess_up": "inv_hessian",
             "k_vinv": "inv_hessian", "k_gather": None, "k_completion": "completion",
             "k_product": "cholesky_product", "k_bigv": "completion"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid3d_40")
    ap.add_argument("--k", type=int, default=16, help="Hessian right-hand sides per step")
    ap.add_argument("--relax", type=float, default=None,
                    help="zero budget of the relaxed plan of the forward operations (-1: none; default: the "
                         "autotuner's cached choice, else 0.05)")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the autotuner cache (default options)")
    ap.add_argument("--batch-workload", default="arrow64")
    ap.add_argument("--batch-k", type=int, default=64)
    ap.add_argument("--cpu-columns", type=int, default=5000,
                    help="leading columns of the workload the oracle baseline runs on")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, latency, grid2d_128 and peak measurements")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="timed steps only (for runs under rocprofv3)")
    ap.add_argument("--calibrate-mib", type=int, default=0,
                    help="first run one elementwise copy of this many MiB (reads and writes "
                         "exactly that much), to scale hardware byte counters")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def ev(torch):
    return torch.cuda.Event(enable_timing=True)


class Step:
    """Device buffers and the operation list of one step on one workload."""

    def __init__(self, torch, mfb, V, pat, k, dev, seed=0, relax=None, fwd_opts=None, fund_opts=None):
        n, cp, ri = pat
        self.pat, self.k, self.nnz = pat, k, int(cp[-1])
        self.relax = relax
        fo = {kk: int(v) for kk, v in (fund_opts or {}).items() if kk in ("wide_j", "big_a")}
        wo = {kk: int(v) for kk, v in (fwd_opts or {}).items() if kk == "wide_j"}
        self.b = mfb.SparseBarrier(pat, device=dev, **fo)
        self.info = self.b.info
        # the forward operations' handle (the same one without relaxation)
        self.fw = mfb.SparseBarrier(pat, device=dev, relax=relax, **wo) if relax is not None else self.b
        self.info_fw = self.fw.info
        self.x_h = V.make_x(*pat, seed=seed)
        self.y_h = V.make_ys(*pat, k, seed=seed)
        self.x = torch.from_numpy(self.x_h).to(dev)
        self.y = torch.from_numpy(self.y_h).to(dev)
        self.s = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        self.t = torch.empty_like(self.y)
        self.y2 = torch.empty_like(self.y)
        self.xhat = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        self.ld = torch.empty(2, dtype=torch.float64, device=dev)
        # one arena serves both handles (their calls run one after another)
        self.arena = self.b.arena(k)
        f, g = self.b.f, self.fw.f
        fwd = [
            ("factor", lambda: mfb.factor(g, self.x)),
            ("logdet", lambda: mfb.logdet(g, self.ld[0:1])),
            ("projected_inverse", lambda: mfb.projected_inverse(g, self.s)),
            ("hessian", lambda: mfb.hessian(g, self.y, self.t, self.arena, k=k)),
        ]
        inv = ("inv_hessian", lambda: mfb.inv_hessian(f, self.t, self.y2, self.arena, k=k))
        compl = [
            ("completion", lambda: mfb.completion(f, self.s)),
            ("logdet_completion", lambda: mfb.logdet(f, self.ld[1:2])),
        ]
        prod = ("cholesky_product", lambda: mfb.cholesky_product(f, self.xhat))
        if relax is None:
            self.ops = fwd + [inv] + compl + [prod]
        else:
            self.ops = fwd + compl + [inv, prod]
        self.handles = [self.b] if relax is None else [self.fw, self.b]
        self.torch = torch
        self.fwd, self.compl, self.inv, self.prod = fwd, compl, inv, prod
        # with two handles: a second stream (default priority) for the
        # fundamental handle's chain, which needs S after the gradient and T
        # after the Hessian, so the completion runs beside the Hessian
        self.side = torch.cuda.Stream(device=dev) if relax is not None else None

    def run(self):
        if self.side is None:
            for _, op in self.ops:
                op()
            return
        torch = self.torch
        main = torch.cuda.current_stream()
        for _, op in self.fwd[:3]:  # factor, log det, gradient (relaxed handle)
            op()
        e_s = torch.cuda.Event()
        e_s.record(main)
        self.side.wait_event(e_s)
        with torch.cuda.stream(self.side):
            for _, op in self.compl:  # completion of S, log det of X-hat, X-hat values
                op()
            self.prod[1]()
        self.fwd[3][1]()  # Hessian, beside the completion
        e_t = torch.cuda.Event()
        e_t.record(main)
        self.side.wait_event(e_t)
        with torch.cuda.stream(self.side):
            self.inv[1]()  # inverse Hessian of T at X-hat (the arena is free again)
        e_end = torch.cuda.Event()
        e_end.record(self.side)
        main.wait_event(e_end)


def timed_steps(torch, st, steps):
    evs = [ev(torch) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record()
    for i in range(steps):
        st.run()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    return float(evs[0].elapsed_time(evs[steps])), per, wall


def per_op_times(torch, st, reps):
    rec = {name: [] for name, _ in st.ops}
    for _ in range(reps):
        for name, op in st.ops:
            a, c = ev(torch), ev(torch)
            a.record()
            op()
            c.record()
            rec[name].append((a, c))
    torch.cuda.synchronize()
    return {name: float(np.median([a.elapsed_time(c) for a, c in v])) for name, v in rec.items()}


def profiled_step(torch, mfb, st):
    """One step with the library's launch records (HIP events on the step's
    stream around every level launch)."""
    for h in st.handles:
        mfb.profile_enable(h.f, True)
    torch.cuda.synchronize()
    st.run()
    torch.cuda.synchronize()
    recs = []
    for h in st.handles:
        recs += mfb.profile_read(h.f)
        mfb.profile_enable(h.f, False)
    return recs


def roofline_of(recs, workload, k):
    """Per operation of the step: canonical bytes and flops of its launches
    and their total time; the dominant operation's roofline; and per level
    (launch record) the fraction of min(FP64 peak, AI * HBM peak)."""
    agg = {}
    for r in recs:
        op = KERNEL_OP.get(r["kernel"])
        if op is None:  # the gathers serve the inverse Hessian (k RHS) and the completion (1)
            op = ("inv_hessian" if r["k"] == k else "completion") if k > 1 else "gather"
        a = agg.setdefault(op, {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "records": 0})
        a["ms"] += r["ms"]
        a["bytes"] += r["bytes"]
        a["flops"] += r["flops"]
        a["records"] += 1
    dom = max((o for o in agg if o != "gather"), key=lambda o: agg[o]["ms"])
    d = agg[dom]
    ai = d["flops"] / max(1.0, d["bytes"])
    sec = d["ms"] * 1e-3
    gbs = d["bytes"] / sec / 1e9
    tfs = d["flops"] / sec / 1e12
    if ai > BALANCE:
        bound, achieved, peak, unit = "mfma", tfs, FP64_PEAK_TFLOPS, "TFLOP/s"
    else:
        bound, achieved, peak, unit = "hbm", gbs, HBM_PEAK_GBS, "GB/s"
    traffic = None
    tf = TRAFFIC_FILE.format(workload=workload)
    if os.path.exists(tf):
        with open(tf) as fh:
            tj = json.load(fh)
        if tj.get("source_hash") == kernel_source_hash():
            traffic = tj.get("bytes_per_call", {}).get(dom)
    roof = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 6), "traffic": traffic,
            "kernel": dom, "launch": "one call of the operation (all its kernel launches)",
            "avg_launch_us": round(d["ms"] * 1e3, 3), "launch_records": d["records"],
            "algorithmic_bytes_per_launch": round(d["bytes"], 1),
            "algorithmic_flops_per_launch": round(d["flops"], 1),
            "achieved_GBps": round(gbs, 3), "achieved_TFLOPs": round(tfs, 4),
            "arithmetic_intensity": round(ai, 3)}
    ops = {o: {"ms": round(a["ms"], 4), "GBps": round(a["bytes"] / (a["ms"] * 1e-3) / 1e9, 2),
               "TFLOPs": round(a["flops"] / (a["ms"] * 1e-3) / 1e12, 4), "records": a["records"]}
           for o, a in agg.items()}
    levels = []
    for r in recs:
        if r["ms"] <= 0 or r["flops"] <= 0:
            continue
        ai_l = r["flops"] / max(1.0, r["bytes"])
        roof_tf = min(FP64_PEAK_TFLOPS, ai_l * HBM_PEAK_GBS / 1e3)
        tf_l = r["flops"] / (r["ms"] * 1e-3) / 1e12
        levels.append({"kernel": r["kernel"], "level": r["level"], "fronts": r["nsuper"], "k": r["k"],
                       "ms": round(r["ms"], 4), "gflop": round(r["flops"] / 1e9, 3),
                       "AI": round(ai_l, 2), "TFLOPs": round(tf_l, 3),
                       "roof_TFLOPs": round(roof_tf, 3), "frac": round(tf_l / roof_tf, 4)})
    levels.sort(key=lambda z: -z["gflop"])
    top = levels[:12]
    tot_fl = sum(z["gflop"] for z in top)
    tot_roof_ms = sum(z["gflop"] / z["roof_TFLOPs"] for z in top)  # ms at the roofline
    tot_ms = sum(z["ms"] for z in top)
    summary = {"levels": len(top), "gflop": round(tot_fl, 2), "ms": round(tot_ms, 3),
               "ms_at_roofline": round(tot_roof_ms, 3), "frac": round(tot_roof_ms / tot_ms, 4)}
    return roof, ops, {"largest_levels": top, "largest_levels_summary": summary}


def golden_check(pat, st, host):
    """Entry-wise relative errors of the step's outputs against oracle values
    (sampled positions stored for the workload) and against properties that
    hold at any size.  Returns None when no stored values exist."""
    path = os.path.join(ROOT, "tests", "golden", "grid3d_40_samples.npz")
    if st.nnz != 21288984 or not os.path.exists(path):
        return None
    g = np.load(path)
    idx = g["idx"]
    n, cp, ri = pat

    def ent(a, b):
        b = np.asarray(b)
        return float(np.max(np.abs(np.asarray(a) - b) / (np.abs(b) + 1e-2 * np.abs(b).max())))

    w = np.where(np.asarray(ri) == np.repeat(np.arange(n), np.diff(cp)), 1.0, 2.0)

    def rel(a, b):
        return float(np.sqrt(np.sum(w * (a - b) ** 2)) / np.sqrt(np.sum(w * b * b)))
    st.fw.factor(st.x)
    ldl = host(st.fw.export_ldl())
    s = host(st.fw.projected_inverse())
    ld = float(host(st.fw.logdet())[0])
    t0 = host(st.t[0])  # from the timed step, same X and Y_0
    y0 = host(st.y2[0])
    xhat = host(st.xhat)
    lds = host(st.ld)
    out = {"factor_entrywise": ent(ldl[idx], g["ldl"]),
           "projected_inverse_entrywise": ent(s[idx], g["s"]),
           "hessian_entrywise": ent(t0[idx], g["t0"]),
           "logdet": abs(ld - float(g["logdet"])) / abs(float(g["logdet"])),
           "inv_hessian_vs_y": rel(y0, st.y_h[0]),
           "xhat_vs_x": rel(xhat, st.x_h),
           "logdet_completion": abs(lds[1] - float(g["logdet"])) / abs(float(g["logdet"])),
           "reference": "oracle values at 6712 sampled positions (tests/golden) for the factor, "
                        "gradient and Hessian; H^-1(H(Y)) = Y and X-hat = X on the whole arrays"}
    return {kk: (float(f"{v:.3e}") if isinstance(v, float) else v) for kk, v in out.items()}


def full_oracle_check(pat, st, host):
    """Entry-wise errors against the full oracle arrays (small workloads)."""
    import oracle
    x_h, y_h = st.x_h, st.y_h
    ldl = oracle.factor(pat, x_h)
    s = oracle.projinv(pat, ldl)
    t = [oracle.hessian(pat, ldl, s, y_h[r]) for r in range(min(st.k, 2))]
    ld = oracle.logdet(pat, ldl)

    def ent(a, b):
        return float(np.max(np.abs(np.asarray(a) - b) / (np.abs(b) + 1e-2 * np.abs(b).max())))
    out = {"projected_inverse_entrywise": ent(host(st.s), s),
           "hessian_entrywise": max(ent(host(st.t[r]), t[r]) for r in range(len(t))),
           "inv_hessian_vs_y_entrywise": max(ent(host(st.y2[r]), y_h[r]) for r in range(len(t))),
           "xhat_vs_x_entrywise": ent(host(st.xhat), x_h),
           "logdet": abs(float(host(st.ld)[1]) - ld) / max(1.0, abs(ld))}
    return {kk: float(f"{v:.3e}") for kk, v in out.items()}


def leading(pat, m):
    """Leading principal m x m pattern (whole subtrees of the elimination
    order, so it is filled in the same order)."""
    n, cp, ri = pat
    rows, cpn = [], [0]
    for j in range(m):
        r = ri[cp[j]:cp[j + 1]]
        r = r[r < m]
        rows.append(r)
        cpn.append(cpn[-1] + len(r))
    return m, np.array(cpn, np.int64), np.concatenate(rows).astype(np.int32)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, pat, full_info, k, mfb, V):
    """The oracle (single thread, pinned to one core) on the leading
    `cpu_columns` columns of the workload: factor, gradient, one Hessian,
    one inverse Hessian, completion and product, each scaled to the full
    workload by its canonical flop count (the Hessian and inverse Hessian
    also by k)."""
    import oracle
    m = min(args.cpu_columns, pat[0])
    sub = leading(pat, m)
    info = mfb.plan_symbolic(*sub).info
    x = V.make_x(*sub, seed=0)
    y = V.make_y(*sub, seed=0)
    try:
        cpus = sorted(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {cpus[-1]})
        pinned = cpus[-1]
    except (AttributeError, OSError):
        pinned = None
    tm = {}
    c0 = time.perf_counter()
    ldl = oracle.factor(sub, x)
    tm["factor"] = time.perf_counter() - c0
    c = time.perf_counter()
    s = oracle.projinv(sub, ldl)
    tm["projinv"] = time.perf_counter() - c
    c = time.perf_counter()
    t = oracle.hessian(sub, ldl, s, y)
    tm["hessian"] = time.perf_counter() - c
    c = time.perf_counter()
    oracle.inv_hessian(sub, ldl, s, t)
    tm["inv_hessian"] = time.perf_counter() - c
    c = time.perf_counter()
    lh = oracle.completion(sub, s)
    tm["completion"] = time.perf_counter() - c
    c = time.perf_counter()
    oracle.product(sub, lh)
    tm["product"] = time.perf_counter() - c
    wall = time.perf_counter() - c0
    if pinned is not None:
        os.sched_setaffinity(0, set(cpus))

    def ratio(key, extra=None):
        num = full_info[key] + (full_info[extra] if extra else 0.0)
        den = info[key] + (info[extra] if extra else 0.0)
        return num / max(den, 1.0)
    step = (tm["factor"] * ratio("flops_factor") + tm["projinv"] * ratio("flops_projinv")
            + k * tm["hessian"] * ratio("flops_hessian")
            + k * tm["inv_hessian"] * ratio("flops_inv_hessian", "flops_inv_hessian_x")
            + tm["completion"] * ratio("flops_completion") + tm["product"] * ratio("flops_product"))
    return {"value": round(k / step, 6), "unit": "Hessian evals/s", "cores": 1, "kind": "oracle",
            "sample": f"leading {m} columns of the workload (whole subtrees of its nested dissection; "
                      f"nnz {int(sub[1][-1])}, max front {info['max_front']}): oracle factor, gradient, one "
                      f"Hessian, one inverse Hessian, completion and product in {wall:.1f} s, each scaled to "
                      f"the full workload by its canonical flop count and the Hessian and inverse Hessian "
                      f"by k = {k}; estimated full step {step:.0f} s",
            "cpu": cpu_model(), "nproc": os.cpu_count(), "pinned_core": pinned,
            "sample_seconds": {kk: round(v, 3) for kk, v in tm.items()}}


def peaks(torch, dev):
    """Attainable HBM bandwidth (device-to-device copy of 2 GiB: 4 GiB moved)
    and FP64 matrix-product rate (8192^3 through torch.matmul)."""
    out = {}
    m = (2 << 30) // 8
    a = torch.ones(m, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = ev(torch), ev(torch)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    out["copy_GBps"] = round(5 * 2 * m * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    nn = 8192
    a = torch.randn(nn, nn, dtype=torch.float64, device=dev)
    b = torch.randn(nn, nn, dtype=torch.float64, device=dev)
    c = a @ b
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        c = a @ b
    e1.record()
    torch.cuda.synchronize()
    out["dgemm_TFLOPs"] = round(3 * 2 * nn ** 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12, 2)
    out["datasheet"] = {"hbm_GBps": HBM_PEAK_GBS, "fp64_TFLOPs": FP64_PEAK_TFLOPS}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def batched_vs_plain(torch, mfb, V, get_config, name, kb, dev, log_args):
    """Hessian and inverse Hessian of kb right-hand sides in one call against
    kb single-RHS calls (the plain path), same workload and X."""
    pat = get_config(name)
    b = mfb.SparseBarrier(pat, device=dev)
    x = torch.from_numpy(V.make_x(*pat, seed=0)).to(dev)
    y = torch.from_numpy(V.make_ys(*pat, kb, seed=1)).to(dev)
    t = torch.empty_like(y)
    y2 = torch.empty_like(y)
    arena = b.arena(kb)
    f = b.f
    mfb.factor(f, x)
    mfb.hessian(f, y, t, arena, k=kb)
    mfb.inv_hessian(f, t, y2, arena, k=kb)
    torch.cuda.synchronize()
    reps = 3
    out = {"workload": name, "k": kb}
    for op, fn in (("hessian", mfb.hessian), ("inv_hessian", mfb.inv_hessian)):
        src, dst = (y, t) if op == "hessian" else (t, y2)
        e0, e1, e2 = ev(torch), ev(torch), ev(torch)
        e0.record()
        for _ in range(reps):
            fn(f, src, dst, arena, k=kb)
        e1.record()
        for _ in range(reps):
            for r in range(kb):
                fn(f, src[r], dst[r], arena, k=1)
        e2.record()
        torch.cuda.synchronize()
        bm = e0.elapsed_time(e1) / reps
        pm = e1.elapsed_time(e2) / reps
        fl = kb * (b.info["flops_hessian"] if op == "hessian" else b.info["flops_inv_hessian"])
        out[op] = {"batched_ms": round(bm, 4), "plain_ms": round(pm, 4),
                   "batched_evals_per_s": round(kb / (bm * 1e-3), 2),
                   "plain_evals_per_s": round(kb / (pm * 1e-3), 2),
                   "speedup": round(pm / bm, 3),
                   "batched_TFLOPs": round(fl / (bm * 1e-3) / 1e12, 4),
                   "batched_frac_fp64_peak": round(fl / (bm * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 5)}
    log(log_args, f"batched {name} k={kb}: {out['hessian']['batched_evals_per_s']} vs "
                  f"{out['hessian']['plain_evals_per_s']} evals/s")
    return out


def latency(torch, mfb, V, get_config, name, dev, reps=200):
    """p50/p99 of one log det + gradient + Hessian(1) sequence after a
    factor, each call sequence timed with events on the stream."""
    pat = get_config(name)
    b = mfb.SparseBarrier(pat, device=dev)
    x = torch.from_numpy(V.make_x(*pat, seed=0)).to(dev)
    y = torch.from_numpy(V.make_y(*pat, seed=0)).to(dev)
    t = torch.empty_like(y)
    s = torch.empty_like(y)
    ld = torch.empty(1, dtype=torch.float64, device=dev)
    arena = b.arena(1)
    f = b.f
    mfb.factor(f, x)

    def seq():
        mfb.logdet(f, ld)
        mfb.projected_inverse(f, s)
        mfb.hessian(f, y, t, arena, k=1)
    for _ in range(5):
        seq()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = ev(torch), ev(torch)
        e0.record()
        seq()
        e1.record()
        ms.append((e0, e1))
    torch.cuda.synchronize()
    v = np.array([a.elapsed_time(c) for a, c in ms])
    w0 = time.perf_counter()
    for _ in range(reps):
        seq()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) / reps
    # the same sequence, preceded by the factor, captured once as a HIP graph
    # and replayed (no entry point allocates, synchronizes or records a
    # memset once the plan is on the device)

    def gseq():
        mfb.factor(f, x)
        seq()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gseq()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gseq()
    torch.cuda.synchronize()
    t_eager = t.clone()
    g.replay()
    torch.cuda.synchronize()
    graph_same = bool(torch.equal(t, t_eager))
    gm = []
    for _ in range(reps):
        e0, e1 = ev(torch), ev(torch)
        e0.record()
        g.replay()
        e1.record()
        gm.append((e0, e1))
    torch.cuda.synchronize()
    gv = np.array([a.elapsed_time(c) for a, c in gm])
    # the eager factor + sequence, for the graph's like-for-like comparison
    em = []
    for _ in range(reps):
        e0, e1 = ev(torch), ev(torch)
        e0.record()
        gseq()
        e1.record()
        em.append((e0, e1))
    torch.cuda.synchronize()
    evv = np.array([a.elapsed_time(c) for a, c in em])
    return {"workload": name, "calls": "logdet + projected_inverse + hessian(k=1)", "reps": reps,
            "p50_ms": round(float(np.percentile(v, 50)), 4), "p99_ms": round(float(np.percentile(v, 99)), 4),
            "host_wall_ms_per_sequence": round(wall * 1e3, 4), "levels": b.info["nlevels_up"],
            "with_factor": {"eager_p50_ms": round(float(np.percentile(evv, 50)), 4),
                            "eager_p99_ms": round(float(np.percentile(evv, 99)), 4),
                            "graph_p50_ms": round(float(np.percentile(gv, 50)), 4),
                            "graph_p99_ms": round(float(np.percentile(gv, 99)), 4),
                            "graph_replay_bitwise_equal": graph_same}}


def hessian_factor_extra(torch, mfb, V, st, reps=2):
    """The interior-point use of the Hessian factor on the step's workload
    (Sections 1.3 and 5.4): W = R(Y) for the step's k right-hand sides, the
    Gram matrix Y_i . H(Y_j) = W_i . W_j, and R^adj(W) = H(Y).  Times each
    call (the first R call also builds the per-supernode factors of S_AA)
    and checks both identities against the step's own H(Y) on the device."""
    f, k = st.b.f, st.k
    dev = st.y.device
    st.run()  # the step leaves H(Y) in st.t
    w = torch.empty_like(st.y)
    t2 = torch.empty_like(st.y)
    g = torch.empty((k, k), dtype=torch.float64, device=dev)
    garena = torch.empty(max(1, mfb.gram_arena_bytes(f.plan, k)), dtype=torch.uint8, device=dev)
    e = [ev(torch) for _ in range(2)]
    e[0].record()
    mfb.hessian_factor(f, st.y, w, st.arena, k=k)
    e[1].record()
    torch.cuda.synchronize()
    first = e[0].elapsed_time(e[1])
    times = {"hessian_factor": [], "hessian_factor_adj": [], "gram": []}
    for _ in range(reps):
        e = [ev(torch) for _ in range(4)]
        e[0].record()
        mfb.hessian_factor(f, st.y, w, st.arena, k=k)
        e[1].record()
        mfb.hessian_factor_adj(f, w, t2, st.arena, k=k)
        e[2].record()
        mfb.gram(f.plan, w, g, garena, m=k)
        e[3].record()
        torch.cuda.synchronize()
        for i, name in enumerate(times):
            times[name].append(e[i].elapsed_time(e[i + 1]))
    n, cp, ri = st.pat
    # sparse arguments (Section 5.5): A_r = e_i e_i^T for k random columns
    # i, the constraint matrices of a max-cut relaxation; step 1 prunes every
    # front whose subtree misses i
    rng = np.random.default_rng(7)
    ysp = torch.zeros_like(st.y)
    cols = rng.choice(n, size=k, replace=False)
    for r_, i_ in enumerate(cols):
        ysp[r_, int(cp[i_])] = 1.0
    wsp = torch.empty_like(st.y)
    mfb.hessian_factor(f, ysp, wsp, st.arena, k=k)
    sp_ms = []
    for _ in range(reps):
        e = [ev(torch) for _ in range(2)]
        e[0].record()
        mfb.hessian_factor(f, ysp, wsp, st.arena, k=k)
        e[1].record()
        torch.cuda.synchronize()
        sp_ms.append(e[0].elapsed_time(e[1]))
    col = torch.from_numpy(V.column_index(n, cp)).to(dev)
    wt = torch.where(torch.from_numpy(np.asarray(ri)).to(dev) == col, 1.0, 2.0).to(torch.float64)
    gref = (st.y * wt) @ st.t.T
    gref = 0.5 * (gref + gref.T)
    adj_err = float((t2 - st.t).abs().max() / st.t.abs().max())
    gram_err = float((g - gref).abs().max() / gref.abs().max())
    return {"k": k, "first_hessian_factor_ms": round(first, 3),
            "ms": {kk: round(float(np.median(v)), 3) for kk, v in times.items()},
            "evals_per_s_hessian_factor": round(k / (np.median(times["hessian_factor"]) * 1e-3), 3),
            "max_rel_err_adj_of_factor_vs_hessian": adj_err, "max_rel_err_gram_vs_y_dot_hessian": gram_err,
            "sparse_arguments": {"rhs": "e_i e_i^T, one diagonal entry each", "k": k,
                                 "hessian_factor_ms": round(float(np.median(sp_ms)), 3),
                                 "speedup_vs_dense": round(float(np.median(times["hessian_factor"]) /
                                                                 np.median(sp_ms)), 2)}}


def factored_completion(torch, mfb, V, dev, reps=3):
    """The paper's comparison of the primal gradient (projected inverse)
    with the dual gradient computed by the completion, plain and with
    factored update matrices, on band and arrow patterns of order 2000
    (width w): GPU milliseconds per call (median of reps after one warm-up)
    and the largest difference between the two completion factors; also
    the inverse Hessian of 4 right-hand sides with S_AA used through those
    factors and through the cached inverse factors."""
    from workloads import patterns as P
    out = {}
    for kind, w in (("band", 10), ("band", 100), ("arrow", 10), ("arrow", 100), ("arrow", 1000)):
        pat = P.band(2000, w) if kind == "band" else P.block_arrow([1] * (2000 - w), w)
        b = mfb.SparseBarrier(pat, device=dev)
        x = torch.from_numpy(V.make_x(*pat, seed=0)).to(dev)
        b.factor(x)
        s = b.projected_inverse().clone()

        def ms(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return round(float(np.median(ts)), 4)
        t_pi = ms(lambda: mfb.projected_inverse(b.f, s))
        t_c = ms(lambda: b.completion(s))
        l1 = b.export_ldl().cpu().numpy()
        t_f = ms(lambda: b.completion_factored(s))
        l2 = b.export_ldl().cpu().numpy()
        # the inverse Hessian of 4 right-hand sides with S_AA through the
        # R_s of the factored completion, and through the cached inverse
        # factors after the plain completion
        tk = torch.from_numpy(V.make_ys(*pat, 4, seed=1)).to(dev)
        yf = torch.empty_like(tk)
        yp = torch.empty_like(tk)
        ar = b.arena(4)
        t_if = ms(lambda: mfb.inv_hessian_factored(b.f, tk, yf, ar, k=4))
        b.completion(s)
        t_ip = ms(lambda: mfb.inv_hessian(b.f, tk, yp, ar, k=4))
        dy = float((yf - yp).abs().max() / yp.abs().max())
        out[f"{kind}2000_w{w}"] = {"projected_inverse_ms": t_pi, "completion_ms": t_c,
                                   "completion_factored_ms": t_f, "status": b.status()[0],
                                   "max_rel_diff": float(np.max(np.abs(l1 - l2)) / np.max(np.abs(l1))),
                                   "inv_hessian_k4_ms": t_ip, "inv_hessian_factored_k4_ms": t_if,
                                   "inv_hessian_max_rel_diff": dy}
        del b
        torch.cuda.empty_cache()
    return out


def served(torch, dev, nreq=200, npool=12, seed=0):
    """The served pattern: requests (pattern, X, Y_1..k) with k ~ U{1..8}
    over a pool of filled Erdos-Renyi patterns (average degree 6) under
    minimum degree, n log-uniform in [500, 3000], X fresh per request,
    Poisson arrivals at 0.8 times the sequential plain capacity; 4 streams,
    half of the free HBM as admission budget.  The same request stream is
    then served with plans on relaxed supernodes (5% zeros), at the same
    arrival rate."""
    from paper_1203_2742_amd import serve as sv
    from workloads import patterns as P
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(500), np.log(3000), npool)).round().astype(int)
    pool = [P.er_min_degree(int(n), int(seed * 100 + i + 1)) for i, n in enumerate(ns)]
    reqs = sv.make_requests(nreq, pool, seed=seed + 2)

    def one(relax, rate=None):
        srv = sv.Server(device=dev, streams=4, relax=relax)
        warm = sv.make_requests(npool, pool, seed=seed + 1)
        srv.run(warm, realtime=False)  # plans, handles and device index arrays in place
        alone, t_seq = srv.run_sequential(reqs[:48])
        cap = 48 / t_seq
        rate = rate or 0.8 * cap
        arr = np.cumsum(np.random.default_rng(seed + 3).exponential(1.0 / rate, nreq))
        for r, a in zip(reqs, arr):
            r.arrival = float(a)
        mix, lat, makespan, peak = srv.run(reqs)
        same = sv.alone_vs_mix(mix, alone)
        del mix
        _, _, makespan_sat, _ = srv.run(reqs, realtime=False)  # every request queued at once
        v = np.array([lat[r.rid] for r in reqs]) * 1e3
        evals = sum(r.ys.shape[0] for r in reqs)
        return {"relax": relax, "arrival_rate_per_s": round(rate, 2), "sequential_requests_per_s": round(cap, 2),
                "p50_ms": round(float(np.percentile(v, 50)), 3), "p99_ms": round(float(np.percentile(v, 99)), 3),
                "served_requests_per_s": round(nreq / makespan, 2),
                "served_hessian_evals_per_s": round(evals / makespan, 2),
                "saturated_requests_per_s": round(nreq / makespan_sat, 2),
                "peak_admitted_GB": round(peak / 1e9, 3), "bitwise_equal_alone_vs_mix": bool(same)}
    plain = one(None)
    # relaxed plans under the same arrival rate, then alone
    relaxed = one(0.05, rate=plain["arrival_rate_per_s"])
    out = {"requests": nreq, "patterns": npool, "n_range": [int(ns.min()), int(ns.max())],
           "nnz_range": [int(min(p[1][-1] for p in pool)), int(max(p[1][-1] for p in pool))], "streams": 4}
    out.update(plain)
    out["relaxed_plans"] = relaxed
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the path would shard over "
                                   "right-hand sides, requests or subtrees, which is not built here)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_1203_2742_amd import mfb
    from workloads import get_config, values as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def host(tt):
        torch.cuda.synchronize()
        return tt.detach().cpu().numpy()

    if args.calibrate_mib:
        m = args.calibrate_mib * (1 << 20) // 8
        src = torch.ones(m, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    pat = get_config(args.workload)
    n, cp, ri = pat
    k = args.k
    t0 = time.perf_counter()
    from paper_1203_2742_amd import autotune
    devname = torch.cuda.get_device_name(dev)

    def tuning_for(p, kk):
        ent = None if args.no_tuning else autotune.lookup(p, kk, devname)
        if ent is None:
            return {"source": "default", "forward": dict(autotune.DEFAULT_FORWARD),
                    "fundamental": dict(autotune.DEFAULT_FUNDAMENTAL)}
        return {"source": f"autotuner cache ({ent['match']})", "forward": ent["forward"],
                "fundamental": ent["fundamental"]}

    def relax_of(tun):
        r = args.relax if args.relax is not None else tun["forward"]["relax"]
        return r if r >= 0 else None

    tuning = tuning_for(pat, k)
    relax = relax_of(tuning)
    st = Step(torch, mfb, V, pat, k, dev, relax=relax, fwd_opts=tuning["forward"], fund_opts=tuning["fundamental"])
    setup_s = time.perf_counter() - t0
    info = st.info
    st_info_fw = st.info_fw
    log(args, f"workload {args.workload}: n={n} nnz={st.nnz} k={k} (setup {setup_s:.1f} s)")

    for _ in range(args.warmup):
        st.run()
    torch.cuda.synchronize()
    K = args.steps
    total_ms, step_ms, wall = timed_steps(torch, st, K)
    log(args, f"timed {K} steps: {total_ms:.3f} ms (wall {wall * 1e3:.3f} ms)")
    status = max(h.status() for h in st.handles)
    value = k * K / (total_ms * 1e-3)
    if args.profile_run:
        print(json.dumps({"metric": METRIC, "value": round(value, 4), "unit": "Hessian evals/s",
                          "ms_per_step": round(total_ms / K, 4), "steps": K, "profile_run": True,
                          "status": status[0]}), flush=True)
        return

    per_op = per_op_times(torch, st, 1)
    recs = profiled_step(torch, mfb, st)
    roof, op_rates, level_roof = roofline_of(recs, args.workload, k)
    log(args, f"dominant {roof['kernel']}: {roof['achieved']} {roof['unit']} ({roof['frac']:.4f})")
    err = golden_check(pat, st, host)
    if err is None and st.nnz <= 3_000_000:
        st.run()
        err = full_oracle_check(pat, st, host)
    hfac = None
    if not args.no_extras:
        hfac = hessian_factor_extra(torch, mfb, V, st)
        log(args, f"hessian factor {hfac}")
    del st
    torch.cuda.empty_cache()

    extras = {}
    if not args.no_extras:
        extras["attainable_peaks"] = peaks(torch, dev)
        log(args, f"peaks {extras['attainable_peaks']}")
        extras["batched_vs_plain"] = batched_vs_plain(torch, mfb, V, get_config, args.batch_workload,
                                                      args.batch_k, dev, args)
        torch.cuda.empty_cache()
        extras["latency"] = latency(torch, mfb, V, get_config, "band200", dev)
        log(args, f"latency {extras['latency']}")
        extras["served"] = served(torch, dev)
        log(args, f"served {extras['served']}")
        extras["factored_completion"] = factored_completion(torch, mfb, V, dev)
        log(args, f"factored completion {extras['factored_completion']}")
        torch.cuda.empty_cache()
        p2 = get_config("grid2d_128")
        tun2 = tuning_for(p2, 1)
        g2 = Step(torch, mfb, V, p2, 1, dev, relax=relax_of(tun2), fwd_opts=tun2["forward"],
                  fund_opts=tun2["fundamental"])
        for _ in range(3):
            g2.run()
        tot, per, _ = timed_steps(torch, g2, 20)
        extras["grid2d_128"] = {"k": 1, "relax": relax_of(tun2), "tuning": tun2["source"],
                                "ms_per_step": round(tot / 20, 4),
                                "p50_ms": round(float(np.percentile(per, 50)), 4),
                                "p99_ms": round(float(np.percentile(per, 99)), 4),
                                "per_op_ms": {kk: round(v, 4) for kk, v in per_op_times(torch, g2, 5).items()}}
        del g2
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, pat, info, k, mfb, V)
        log(args, f"cpu baseline {cpu['value']} evals/s ({cpu['sample_seconds']})")

    out = {
        "metric": METRIC,
        "value": round(value, 4),
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
        "config": {"workload": args.workload, "n": int(n), "nnz": st_nnz(cp), "k": k,
                   "nsuper": info["nsuper"], "levels": info["nlevels_up"], "max_front": info["max_front"],
                   "relax": relax,
                   "tuning": tuning,
                   "relaxed_plan": None if relax is None else {
                       "nsuper": st_info_fw["nsuper"], "levels": st_info_fw["nlevels_up"],
                       "nnz": st_info_fw["nnz_relaxed"], "update_GB": round(st_info_fw["update_doubles"] * 8e-9, 3),
                       "max_front": st_info_fw["max_front"]},
                   "step": ("factor+logdet+projected_inverse+hessian(k)+inv_hessian(k)+completion+logdet+product"
                            if relax is None else
                            "relaxed plan: factor+logdet+projected_inverse+hessian(k); fundamental plan: "
                            "completion+logdet+product+inv_hessian(k) at X-hat; the completion and the product run "
                            "on a second stream beside the Hessian")},
        "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
        "per_op_ms": {kk: round(v, 4) for kk, v in per_op.items()},
        "roofline": roof,
        "op_rates": op_rates,
        "level_roofline": level_roof,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": err,
        "status": status[0],
        "setup_s": round(setup_s, 2),
    }
    if hfac is not None:
        out["hessian_factor"] = hfac
    out.update(extras)
    print(json.dumps(out), flush=True)


def st_nnz(cp):
    return int(cp[-1])


if __name__ == "__main__":
    main()
