"""mfb_hessian_static (no caller arena, no allocation) against mfb_hessian
with a caller arena: the same kernels on the same inputs, so the outputs
are bitwise equal.  Two calls in a row on one GPU, the second on a smaller
input, then a call beyond the static scratch, which is refused."""
import numpy as np
import pytest

from workloads import get_config, patterns as P, values as V

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_static_scratch_hessian_matches_arena_hessian():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_2742_amd import mfb
    cases = [(get_config("grid2d_24"), 3, "grid2d_24, k=3"),
             (P.band(60, 3), 1, "band60, k=1")]
    for pat, k, label in cases:
        print(f"[no-alloc] {label}", flush=True)
        b = mfb.SparseBarrier(pat)
        b.factor(_dev(V.make_x(*pat, seed=0)))
        ys = _dev(V.make_ys(*pat, k, seed=11))
        want = b.hessian(ys)
        got = torch.empty_like(ys)
        mfb.hessian_static(b.f, ys, got, k=k)
        torch.cuda.synchronize()
        assert torch.equal(got, want), label
        assert b.status() == (0, -1)
    # beyond the static scratch: refused before anything is enqueued
    pat = get_config("grid2d_128")
    b = mfb.SparseBarrier(pat)
    b.factor(_dev(V.make_x(*pat, seed=0)))
    k = mfb.STATIC_SCRATCH_BYTES // b.info["rhs_arena_bytes"] + 1
    y = torch.zeros((k, b.nnz), dtype=torch.float64, device="cuda")
    t = torch.empty_like(y)
    with pytest.raises(mfb.MfbError) as e:
        mfb.hessian_static(b.f, y, t, k=k)
    assert e.value.code == mfb.ESCRATCH
