"""The autotuner on the device: it times its candidates through the C ABI,
stores an entry, and the plans built from that entry keep oracle parity
(forward operations on the tuned relaxed plan; completion and inverse
Hessian on the tuned fundamental plan)."""
import numpy as np
import pytest

import oracle
from tests.test_gpu_parity import close, dev, host
from workloads import get_config, values as V

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tune_small_pattern(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_2742_amd import autotune, mfb
    pat = get_config("grid3d_8")
    k = 2
    cache = str(tmp_path / "tuned.json")
    print("[gpu-autotune] grid3d_8 k=2", flush=True)
    e = autotune.tune(pat, k, cache=cache, reps=1, log=lambda *a: None)
    assert e["forward"]["relax"] in autotune.RELAX and e["forward"]["ms"] > 0
    assert len(e["candidates"]) >= len(autotune.RELAX) + len(autotune.BIG_A)
    got = autotune.lookup(pat, k, torch.cuda.get_device_name(), cache=cache)
    assert got["match"] == "exact" and got["fundamental"] == e["fundamental"]
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, k, seed=3)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    fw = mfb.SparseBarrier(pat, relax=e["forward"]["relax"], wide_j=e["forward"]["wide_j"])
    fw.factor(dev(x))
    close(pat, host(fw.projected_inverse()), s)
    t = host(fw.hessian(dev(ys)))
    for r in range(k):
        close(pat, t[r], oracle.hessian(pat, ldl, s, ys[r]))
    fu = mfb.SparseBarrier(pat, wide_j=e["fundamental"]["wide_j"], big_a=e["fundamental"]["big_a"])
    fu.completion(dev(s))
    assert fu.status() == (0, -1)
    close(pat, host(fu.cholesky_product()), x)
    yi = host(fu.inv_hessian(dev(t)))
    for r in range(k):
        close(pat, yi[r], ys[r], 1e-9)


def test_binding_before_torch_uses_one_runtime(tmp_path):
    """Importing the binding before torch (as `python -m` of a module of the
    package does) must leave one HIP runtime in the process.  With the
    system runtime loaded first and torch's beside it, creating a handle of
    the 40^3 relaxed plan after torch had allocated the step's tensors
    failed in the plan upload; the binding now loads torch's runtime first."""
    import pathlib
    import subprocess
    import sys
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    root = str(pathlib.Path(__file__).resolve().parents[1])
    code = (
        f"import sys; sys.path.insert(0, {root!r})\n"
        "from paper_1203_2742_amd import mfb\n"
        "import torch\n"
        "from workloads import get_config, values as V\n"
        "pat = get_config('grid3d_40')\n"
        "x = torch.from_numpy(V.make_x(*pat, seed=0)).cuda()\n"
        "y = torch.from_numpy(V.make_ys(*pat, 16, seed=0)).cuda()\n"
        "t = torch.empty_like(y); y2 = torch.empty_like(y)\n"
        "b = mfb.SparseBarrier(pat, relax=0.05)\n"
        "b.factor(x)\n"
        "print('status', b.status())\n")
    print("[gpu-autotune] binding first, grid3d_40 relaxed handle", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "status (0, -1)" in r.stdout
