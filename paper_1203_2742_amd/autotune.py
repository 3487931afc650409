"""Autotuner of the plan options, per pattern and number of right-hand sides.

A step of a barrier method on one pattern uses two plans:

* the forward plan (factor, log det, gradient, Hessian of k right-hand
  sides), which may run on relaxed supernodes: its options are the zero
  budget `relax` and the front order `wide_j` above which fronts run
  tile-parallel;
* the fundamental plan (completion, inverse Hessian of k right-hand sides),
  whose options are `wide_j` and `big_a`, the ancestor count above which the
  blocks S_AA are factored tile-parallel.

`tune` times candidate options on the device with the library's own entry
points (coordinate search: the budget first, then the thresholds; each
candidate is a fresh plan and handle, timed as the median of a few calls
after one warm-up; a candidate replaces the current choice only when it is
at least MIN_GAIN faster, so timing noise does not move the defaults) and
stores the choice in a JSON cache.  Entries are keyed by
a hash of the pattern, k and the device name, and carry the plan statistics
(n, nnz, supernodes, levels, largest front); `lookup` finds the exact entry,
or else the entry of the same device and k whose statistics are nearest
(log distance), so related patterns reuse a tuning.  The options change
which kernels run and, for the forward plan, the supernode partition; the
results stay within rounding of each other (the tests hold every plan to
the oracle).

    python -m paper_1203_2742_amd.autotune --workload grid3d_40 --k 16

writes the entry into the cache file (default: tuned.json next to this
module, or $MFB_TUNE_CACHE).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import time

import numpy as np

from . import mfb

CACHE = os.environ.get("MFB_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json"))
DEFAULT_FORWARD = {"relax": 0.05, "wide_j": 0}
DEFAULT_FUNDAMENTAL = {"wide_j": 0, "big_a": 0}
RELAX = (0.0, 0.01, 0.02, 0.05, 0.1, 0.2)
WIDE_J = (96, 128, 192, 256, 384)
BIG_A = (192, 256, 384, 512)
MIN_GAIN = 0.02


def pattern_hash(pattern) -> str:
    n, cp, ri = pattern
    h = hashlib.sha1()
    h.update(np.int64(n).tobytes())
    h.update(np.ascontiguousarray(cp, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(ri, dtype=np.int32).tobytes())
    return h.hexdigest()[:20]


def plan_stats(pattern) -> dict:
    info = mfb.plan_symbolic(*pattern).info
    return {key: int(info[src]) for key, src in (("n", "n"), ("nnz", "nnz"), ("nsuper", "nsuper"),
                                                 ("levels", "nlevels_up"), ("max_front", "max_front"))}


def _key(phash, k, device):
    return f"{phash}:k{int(k)}:{device}"


def load(cache=None) -> dict:
    path = cache or CACHE
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def lookup(pattern, k, device, cache=None, stats=None):
    """The cached entry for (pattern, k, device), else the nearest entry of
    the same k and device by plan statistics, else None."""
    db = load(cache)
    ent = db.get(_key(pattern_hash(pattern), k, device))
    if ent is not None:
        return dict(ent, match="exact")
    same = [e for e in db.values() if e.get("k") == int(k) and e.get("device") == device]
    if not same:
        return None
    st = stats or plan_stats(pattern)

    def dist(e):
        return sum((math.log(max(1, st[f])) - math.log(max(1, e["stats"][f]))) ** 2
                   for f in ("nnz", "nsuper", "max_front"))
    best = min(same, key=dist)
    return dict(best, match="nearest")


def _median_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune(pattern, k, device="cuda", cache=None, reps=2, log=print):
    """Times the candidates on the current device, stores and returns the
    entry {"forward": {...}, "fundamental": {...}, ...}."""
    import torch
    from workloads import values as V
    dev = torch.device(device)
    name = torch.cuda.get_device_name(dev)
    n, cp, ri = pattern
    nnz = int(cp[-1])
    x = torch.from_numpy(V.make_x(*pattern, seed=0)).to(dev)
    y = torch.from_numpy(V.make_ys(*pattern, k, seed=0)).to(dev)
    s = torch.empty(nnz, dtype=torch.float64, device=dev)
    t = torch.empty_like(y)
    y2 = torch.empty_like(y)
    arena = [torch.empty(0, dtype=torch.uint8, device=dev)]
    t0 = time.perf_counter()
    tried = []

    def arena_for(plan):
        need = max(1, k) * plan.info["rhs_arena_bytes"]
        if arena[0].numel() < need:
            arena[0] = torch.empty(0, dtype=torch.uint8, device=dev)
            torch.cuda.empty_cache()
            arena[0] = torch.empty(need, dtype=torch.uint8, device=dev)
        return arena[0]

    def forward_ms(opt):
        plan = mfb.plan_symbolic(n, cp, ri, relax=opt["relax"], wide_j=opt["wide_j"])
        ws = torch.empty(plan.info["factor_workspace_bytes"], dtype=torch.uint8, device=dev)
        f = mfb.factor_create(plan, ws)
        ar = arena_for(plan)

        def run():
            mfb.factor(f, x)
            mfb.projected_inverse(f, s)
            mfb.hessian(f, y, t, ar, k=k)
        ms = _median_ms(torch, run, reps)
        del f, ws
        torch.cuda.empty_cache()
        return ms

    def fundamental_ms(opt):
        plan = mfb.plan_symbolic(n, cp, ri, wide_j=opt["wide_j"], big_a=opt["big_a"])
        ws = torch.empty(plan.info["factor_workspace_bytes"], dtype=torch.uint8, device=dev)
        f = mfb.factor_create(plan, ws)
        ar = arena_for(plan)

        def run():
            mfb.completion(f, s)
            mfb.inv_hessian(f, t, y2, ar, k=k)
        ms = _median_ms(torch, run, reps)
        del f, ws
        torch.cuda.empty_cache()
        return ms

    def search(kind, timer, start, axes):
        best, best_ms = dict(start), timer(start)
        tried.append({"plan": kind, **best, "ms": round(best_ms, 3)})
        log(f"[autotune] {kind} {best} {best_ms:.2f} ms")
        for axis, values in axes:
            for v in values:
                if v == best[axis]:
                    continue
                cand = dict(best, **{axis: v})
                ms = timer(cand)
                tried.append({"plan": kind, **cand, "ms": round(ms, 3)})
                log(f"[autotune] {kind} {cand} {ms:.2f} ms")
                if ms < (1.0 - MIN_GAIN) * best_ms:
                    best, best_ms = cand, ms
        return dict(best, ms=round(best_ms, 3))

    fwd = search("forward", forward_ms, {"relax": 0.05, "wide_j": 192}, [("relax", RELAX), ("wide_j", WIDE_J)])
    # the fundamental plan's inputs: S and T = H(Y) from the forward plan
    fund = search("fundamental", fundamental_ms, {"wide_j": 192, "big_a": 256},
                  [("wide_j", WIDE_J), ("big_a", BIG_A)])
    entry = {"pattern": pattern_hash(pattern), "k": int(k), "device": name, "stats": plan_stats(pattern),
             "forward": fwd, "fundamental": fund, "candidates": tried,
             "seconds": round(time.perf_counter() - t0, 1)}
    path = cache or CACHE
    db = load(path)
    db[_key(entry["pattern"], k, name)] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="grid3d_40")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--cache", default=None)
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args()
    from workloads import get_config
    e = tune(get_config(a.workload), a.k, cache=a.cache, reps=a.reps)
    print(json.dumps({kk: e[kk] for kk in ("pattern", "k", "device", "stats", "forward", "fundamental", "seconds")}))


if __name__ == "__main__":
    main()
