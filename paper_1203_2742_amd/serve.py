"""Serving independent barrier requests on one GPU.

A request is (pattern, X, Y_1..Y_k): factor X, form the gradient
S = P(X^-1) and the Hessian products T_r = P(X^-1 Y_r X^-1), the call
sequence of one interior-point iteration on one cone.  The server keeps

* a plan cache keyed by the pattern's CCS arrays (symbolic analysis and the
  plan's device index arrays are done once per distinct pattern); with
  `relax`, plans on relaxed supernodes (exact for the gradient and the
  Hessian, the calls a request makes);
* a pool of factor handles per plan, each with its own workspace, reused
  across requests;
* HBM admission: a request is started only while the device bytes of the
  requests in flight (factor workspace, right-hand-side arena, inputs and
  outputs) stay within a budget; otherwise it waits in FIFO order;
* continuous batching over streams: every started request runs on one of a
  few HIP streams (default priority), so the kernels of different requests
  overlap on the GPU while the host keeps admitting new arrivals; a request
  completes when an event recorded after its last call has passed.

Every kernel of the library is deterministic, so a request's results do not
depend on what runs beside it (checked by `alone_vs_mix`).  All numerical
work is done by the C ABI (`mfb`); this module only schedules calls.
"""
from __future__ import annotations

import collections
import dataclasses
import hashlib
import time

import numpy as np

from . import mfb


@dataclasses.dataclass
class Request:
    rid: int
    pattern: tuple          # (n, colptr, rowind)
    x: np.ndarray           # nnz values of X
    ys: np.ndarray          # k x nnz right-hand sides
    arrival: float = 0.0    # seconds after the start of the run
    key: str = ""
    host: tuple = ()        # pinned host copies of x and ys (set by the server)


def pattern_key(pattern) -> str:
    n, cp, ri = pattern
    h = hashlib.sha1()
    h.update(np.int64(n).tobytes())
    h.update(np.ascontiguousarray(cp, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(ri, dtype=np.int32).tobytes())
    return h.hexdigest()


class Server:
    def __init__(self, device="cuda:0", streams: int = 4, hbm_budget: int | None = None, relax=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = free // 2
        self.budget = int(hbm_budget)
        self.relax = relax
        self.plans = {}                            # key -> mfb.Plan
        self.pool = collections.defaultdict(list)  # key -> free factor handles

    # -- resources ---------------------------------------------------------
    def plan(self, key, pattern):
        if key not in self.plans:
            n, cp, ri = pattern
            self.plans[key] = mfb.plan_symbolic(n, cp, ri, relax=self.relax)
        return self.plans[key]

    def need_bytes(self, req: Request) -> int:
        info = self.plan(req.key, req.pattern).info
        k, nnz = req.ys.shape[0], info["nnz"]
        return info["factor_workspace_bytes"] + k * info["rhs_arena_bytes"] + 8 * nnz * (2 + 2 * k)

    def _stage(self, req: Request):
        if not req.host:
            torch = self.torch
            req.host = (torch.from_numpy(req.x).pin_memory(), torch.from_numpy(req.ys).pin_memory())

    def _handle(self, key, stream):
        torch = self.torch
        if self.pool[key]:
            return self.pool[key].pop()
        plan = self.plans[key]
        with torch.cuda.stream(stream):
            ws = torch.empty(plan.info["factor_workspace_bytes"], dtype=torch.uint8, device=self.device)
        return mfb.factor_create(plan, ws)

    # -- one request ---------------------------------------------------------
    def _launch(self, req: Request, stream):
        torch = self.torch
        f = self._handle(req.key, stream)
        info = f.plan.info
        k, nnz = req.ys.shape
        with torch.cuda.stream(stream):
            x = req.host[0].to(self.device, non_blocking=True)
            y = req.host[1].to(self.device, non_blocking=True)
            s = torch.empty(nnz, dtype=torch.float64, device=self.device)
            t = torch.empty((k, nnz), dtype=torch.float64, device=self.device)
            arena = torch.empty(max(1, k) * info["rhs_arena_bytes"], dtype=torch.uint8, device=self.device)
            mfb.factor(f, x, stream=stream)
            mfb.projected_inverse(f, s, stream=stream)
            mfb.hessian(f, y, t, arena, k=k, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return {"req": req, "f": f, "event": ev, "out": (s, t), "keep": (x, y, arena)}

    # -- the request loop ----------------------------------------------------
    def run(self, requests, realtime: bool = True):
        """Serve requests (sorted by arrival).  Returns per-request results
        (device tensors S, T), latencies (seconds from arrival to completion),
        the makespan, and the peak admitted bytes."""
        torch = self.torch
        for r in requests:  # the request data is in host memory when it arrives
            r.key = r.key or pattern_key(r.pattern)
            self.plan(r.key, r.pattern)
            self._stage(r)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        inflight = []
        free_streams = list(range(len(self.streams)))
        in_use = peak = 0
        results, latency = {}, {}
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                queue.append(pending.popleft())
            progressed = False
            while queue and free_streams:
                req = queue[0]
                nb = self.need_bytes(req)
                if in_use and in_use + nb > self.budget:
                    break  # admission: wait for requests in flight to finish
                queue.popleft()
                si = free_streams.pop(0)
                item = self._launch(req, self.streams[si])
                item["stream"], item["bytes"] = si, nb
                in_use += nb
                peak = max(peak, in_use)
                inflight.append(item)
                progressed = True
            for item in list(inflight):
                if item["event"].query():
                    done = time.perf_counter() - t0
                    req = item["req"]
                    latency[req.rid] = done - req.arrival if realtime else done
                    results[req.rid] = item["out"]
                    self.pool[req.key].append(item["f"])
                    free_streams.append(item["stream"])
                    in_use -= item["bytes"]
                    inflight.remove(item)
                    progressed = True
            if not progressed:
                time.sleep(2e-5)
        makespan = time.perf_counter() - t0
        torch.cuda.synchronize(self.device)
        return results, latency, makespan, peak

    def run_sequential(self, requests):
        """The plain path: one request at a time on one stream, each call
        completed before the next request starts."""
        torch = self.torch
        results = {}
        for r in requests:
            r.key = r.key or pattern_key(r.pattern)
            self.plan(r.key, r.pattern)
            self._stage(r)
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        for r in requests:
            item = self._launch(r, self.streams[0])
            item["event"].synchronize()
            results[r.rid] = item["out"]
            self.pool[r.key].append(item["f"])
        return results, time.perf_counter() - t0


def alone_vs_mix(mix_results, alone_results) -> bool:
    """Bitwise equality of every request's S and T between two runs."""
    import torch
    for rid, (s, t) in alone_results.items():
        s2, t2 = mix_results[rid]
        if not (torch.equal(s, s2) and torch.equal(t, t2)):
            return False
    return True


def make_requests(count, pool, seed=0, kmax=8, rate=None):
    """Requests over a pool of patterns, X fresh per request (diagonally
    dominant, as workloads.values.make_x), k ~ U{1..kmax} right-hand sides,
    Poisson arrivals at `rate` per second (all at time 0 when None)."""
    from workloads import values as V
    rng = np.random.default_rng(seed)
    reqs, t = [], 0.0
    keys = [pattern_key(p) for p in pool]
    for i in range(count):
        j = int(rng.integers(0, len(pool)))
        pat = pool[j]
        k = int(rng.integers(1, kmax + 1))
        if rate:
            t += float(rng.exponential(1.0 / rate))
        reqs.append(Request(i, pat, V.make_x(*pat, seed=1000 + i), V.make_ys(*pat, k, seed=1000 + i), t, keys[j]))
    return reqs
