"""The entry points under HIP graph capture.

After a plan's first factor handle exists, no compute entry point
allocates, synchronizes or records a memset, so a whole step captured on a
stream replays as one graph.  The captured sequence starts with the factor,
so the handle's cached state (projected inverse, inverse blocks) is rebuilt
inside every replay in the order the eager calls build it.  Each replay is
checked bitwise against the eager results, with eager work and
synchronizations between the replays.
"""
import numpy as np
import pytest

from tests.test_gpu_parity import CASES, dev, host
from workloads import values as V

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mfb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_2742_amd import mfb as m
    return m


@pytest.mark.parametrize("name", ["arrow_small", "grid2d_24"])
def test_step_graph_replays_match_eager(name, mfb):
    pat = CASES[name]()
    k = 2
    print(f"[gpu-graph] {name}: capture", flush=True)
    b = mfb.SparseBarrier(pat)
    f = b.f
    x = dev(V.make_x(*pat, seed=0))
    y = dev(V.make_ys(*pat, k, seed=1))
    out = {
        "ld": torch.empty(2, dtype=torch.float64, device="cuda"),
        "s": torch.empty(pat[1][-1], dtype=torch.float64, device="cuda"),
        "t": torch.empty_like(y),
        "yi": torch.empty_like(y),
        "w": torch.empty_like(y),
        "xhat": torch.empty(pat[1][-1], dtype=torch.float64, device="cuda"),
    }
    arena = b.arena(k)

    def step():
        mfb.factor(f, x)
        mfb.logdet(f, out["ld"][0:1])
        mfb.projected_inverse(f, out["s"])
        mfb.hessian(f, y, out["t"], arena, k=k)
        mfb.inv_hessian(f, out["t"], out["yi"], arena, k=k)
        mfb.hessian_factor(f, y, out["w"], arena, k=k)
        mfb.completion(f, out["s"])
        mfb.logdet(f, out["ld"][1:2])
        mfb.cholesky_product(f, out["xhat"])

    step()
    want = {key: host(v).copy() for key, v in out.items()}
    # warm-up on a side stream, then capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    other = dev(V.make_ys(*pat, k, seed=9))
    scratch = torch.empty_like(other)
    for rep in range(3):
        for v in out.values():
            v.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for key, v in out.items():
            assert np.array_equal(host(v), want[key]), (rep, key)
        # eager work between replays on the same handle
        mfb.hessian(f, other, scratch, arena, k=k)
        torch.cuda.synchronize()
    assert b.status() == (0, -1)


@pytest.mark.parametrize("name", ["arrow_small", "grid3d_8"])
def test_native_step_graph(name, mfb):
    """mfb_step_graph_create: factor, logdet, gradient, Hessian (k = 2) and
    inverse Hessian captured by the library itself; three replays with
    eager work in between, each bitwise equal to the eager step."""
    pat = CASES[name]()
    k = 2
    b = mfb.SparseBarrier(pat, flags=mfb.PLAN_WIDE_LOW)
    f = b.f
    nnz = pat[1][-1]
    x = dev(V.make_x(*pat, seed=0))
    y = dev(V.make_ys(*pat, k, seed=1))
    ld = torch.empty(1, dtype=torch.float64, device="cuda")
    s = torch.empty(nnz, dtype=torch.float64, device="cuda")
    t = torch.empty_like(y)
    yi = torch.empty_like(y)
    arena = b.arena(k)
    ops = mfb.STEP_FACTOR | mfb.STEP_LOGDET | mfb.STEP_PROJINV | mfb.STEP_HESSIAN | mfb.STEP_INV_HESSIAN
    mfb.factor(f, x)
    mfb.logdet(f, ld)
    mfb.projected_inverse(f, s)
    mfb.hessian(f, y, t, arena, k=k)
    mfb.inv_hessian(f, t, yi, arena, k=k)
    want = [host(v).copy() for v in (ld, s, t, yi)]
    g = mfb.step_graph(f, ops, x, logdet=ld, s=s, k=k, y=y, t=t, t_in=t, y_out=yi, arena=arena)
    other = dev(V.make_ys(*pat, k, seed=9))
    scratch = torch.empty_like(other)
    for rep in range(3):
        for v in (ld, s, t, yi):
            v.fill_(np.nan)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, v in enumerate((ld, s, t, yi)):
            assert np.array_equal(host(v), want[i]), (rep, i)
        mfb.hessian(f, other, scratch, arena, k=k)
        torch.cuda.synchronize()
    with pytest.raises(mfb.MfbError):
        mfb.step_graph(f, mfb.STEP_HESSIAN, x, k=k, y=y, t=t, arena=arena)
