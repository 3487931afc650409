"""The served pattern: independent requests (pattern, X, Y_1..k) through a
plan cache, a pool of factor handles, HBM admission and several streams.
Each request's gradient and Hessian products must be bitwise the same in
the mix as alone (the kernels are deterministic), and agree with the
oracle; a budget below two requests' bytes must still finish every request
(admission never deadlocks)."""
import numpy as np
import pytest

import oracle
from tests.test_gpu_parity import close, host
from workloads import patterns as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_2742_amd import serve as sv
    return sv


def _pool():
    return [P.er_min_degree(n, seed) for n, seed in ((300, 1), (600, 2), (900, 3), (1200, 4))]


@pytest.mark.parametrize("relax", [None, 0.05])
def test_mix_matches_alone_and_oracle(serve, relax):
    pool = _pool()
    reqs = serve.make_requests(24, pool, seed=5, kmax=4, rate=2000.0)
    print(f"[gpu-serve] {len(reqs)} requests over {len(pool)} patterns, relax={relax}", flush=True)
    srv = serve.Server(streams=4, relax=relax)
    mix, lat, makespan, peak = srv.run(reqs)
    assert len(mix) == len(reqs) and all(v >= 0 for v in lat.values())
    alone, _ = serve.Server(streams=1, relax=relax).run_sequential(reqs)
    assert serve.alone_vs_mix(mix, alone)
    for r in reqs[:6]:
        ldl = oracle.factor(r.pattern, r.x)
        s = oracle.projinv(r.pattern, ldl)
        close(r.pattern, host(mix[r.rid][0]), s)
        t = host(mix[r.rid][1])
        for j in range(r.ys.shape[0]):
            close(r.pattern, t[j], oracle.hessian(r.pattern, ldl, s, r.ys[j]))


def test_admission_with_a_small_budget(serve):
    pool = _pool()[:2]
    reqs = serve.make_requests(8, pool, seed=6, kmax=3)
    srv = serve.Server(streams=3, hbm_budget=1)
    mix, lat, _, peak = srv.run(reqs, realtime=False)
    assert len(mix) == len(reqs)
    # one request at a time: the peak admitted bytes are a single request's
    assert peak == max(srv.need_bytes(r) for r in reqs)
    alone, _ = serve.Server(streams=1).run_sequential(reqs)
    assert serve.alone_vs_mix(mix, alone)
