"""GPU parity of the Hessian factor (Algorithms 5.3 and 5.4) and the Gram
matrix of its outputs against the CPU oracle, through the C ABI.

Tolerances and the entry-wise bound are those of test_gpu_parity.  The
oracle's R and R^adj follow the paper's scalar algorithms column by column;
the library's supernodal block form must give the same W = R(Y) entry by
entry, since R is fixed by the choice of R_j upper triangular.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from tests.test_gpu_parity import CASES, TOL, close, dev, host
from workloads import get_config, patterns as P, values as V

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mfb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_2742_amd import mfb as m
    return m


def ip(pat, a, b):
    n, cp, ri = pat
    col = V.column_index(n, cp)
    w = np.where(np.asarray(ri) == col, 1.0, 2.0)
    return float(np.sum(w * np.asarray(a) * np.asarray(b)))


def gram_host(pat, ws):
    n, cp, ri = pat
    col = V.column_index(n, cp)
    wt = np.where(np.asarray(ri) == col, 1.0, 2.0)
    ws = np.asarray(ws)
    return (ws * wt) @ ws.T


@pytest.fixture(scope="module", params=sorted(CASES))
def hcase(request, mfb):
    name = request.param
    pat = CASES[name]()
    n, cp, _ = pat
    print(f"[gpu-hfactor] case {name}: n={n} nnz={cp[-1]}", flush=True)
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, 3, seed=3)
    wp = V.make_ys(*pat, 2, seed=4)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    return dict(name=name, pat=pat, x=x, ys=ys, wp=wp, ldl=ldl, s=s, b=b)


def test_hessian_factor_matches_oracle(hcase):
    pat, ldl, s, ys, b = hcase["pat"], hcase["ldl"], hcase["s"], hcase["ys"], hcase["b"]
    wk = host(b.hessian_factor(dev(ys)))
    for r in range(len(ys)):
        close(pat, wk[r], oracle.hessian_factor(pat, ldl, s, ys[r]))
    # one right-hand side alone gives the bits it has inside the batch
    assert np.array_equal(host(b.hessian_factor(dev(ys[2]))), wk[2])


def test_hessian_factor_adj_matches_oracle(hcase):
    pat, ldl, s, wp, b = hcase["pat"], hcase["ldl"], hcase["s"], hcase["wp"], hcase["b"]
    tk = host(b.hessian_factor_adj(dev(wp)))
    for r in range(len(wp)):
        close(pat, tk[r], oracle.hessian_factor_adj(pat, ldl, s, wp[r]))


def test_factor_composes_to_hessian_and_gram(hcase):
    """R^adj(R(Y)) = H(Y) on the device, and the Gram matrix of R(Y_i) is
    Y_i . H(Y_j) with H from the oracle."""
    pat, ldl, s, ys, b = hcase["pat"], hcase["ldl"], hcase["s"], hcase["ys"], hcase["b"]
    w = b.hessian_factor(dev(ys))
    t = host(b.hessian_factor_adj(w))
    th = host(b.hessian(dev(ys)))
    for r in range(len(ys)):
        close(pat, t[r], th[r])
    g = host(b.gram(w))
    want = np.array([[ip(pat, ys[i], oracle.hessian(pat, ldl, s, ys[j])) for j in range(3)] for i in range(3)])
    assert np.abs(g - want).max() <= TOL * np.abs(want).max(), (g, want)
    assert np.array_equal(g, g.T)


@pytest.mark.parametrize("m", [1, 3, 64, 70, 129])
def test_gram_against_host(m, mfb):
    """Ragged tile counts (m = 64, 70, 129) and a single vector; nnz spans
    several entry chunks and the diagonal chunk has its own tail."""
    pat = get_config("grid2d_128") if m <= 3 else P.random_chordal(400, 0.02, 3)
    rng = np.random.default_rng(m)
    ws = rng.standard_normal((m, pat[1][-1]))
    plan = mfb.plan_symbolic(*pat)
    g = torch.empty((m, m), dtype=torch.float64, device="cuda")
    arena = torch.empty(max(1, mfb.gram_arena_bytes(plan, m)), dtype=torch.uint8, device="cuda")
    mfb.gram(plan, dev(ws), g, arena, m=m)
    got = host(g)
    want = gram_host(pat, ws)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # fixed summation order: a second call gives the same bits
    mfb.gram(plan, dev(ws), g, arena, m=m)
    assert np.array_equal(host(g), got)


WIDE_PATS = {"band400_w200": lambda: P.band(400, 200), "band700_w520": lambda: P.band(700, 520)}


@pytest.mark.parametrize("name", ["arrow_mixed", "grid3d_8", "roots_mixed", "band400_w200", "band700_w520"])
def test_hessian_factor_wide_plans(name, mfb):
    """The step-1 and root-to-leaf sweeps that R and R^adj reuse take the
    wide and fat tile-parallel paths under MFB_PLAN_WIDE_LOW; the bands put
    the per-supernode G and G^-1 on the tile-parallel factorization of the
    reversed S_AA (A = 200 under the lowered threshold, A = 520 at the
    default one)."""
    pat = WIDE_PATS[name]() if name in WIDE_PATS else CASES[name]()
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, 2, seed=6)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    with cf.ThreadPoolExecutor(4) as ex:
        fw = [ex.submit(oracle.hessian_factor, pat, ldl, s, ys[r]) for r in range(2)]
        ft = [ex.submit(oracle.hessian_factor_adj, pat, ldl, s, ys[r]) for r in range(2)]
        want_w = [q.result() for q in fw]
        want_t = [q.result() for q in ft]
    for flags in ((mfb.PLAN_WIDE_LOW, 0) if name == "band700_w520" else (mfb.PLAN_WIDE_LOW,)):
        b = mfb.SparseBarrier(pat, flags=flags)
        b.factor(dev(x))
        w = host(b.hessian_factor(dev(ys)))
        t = host(b.hessian_factor_adj(dev(ys)))
        for r in range(2):
            close(pat, w[r], want_w[r])
            close(pat, t[r], want_t[r])


def test_hessian_factor_after_completion(mfb):
    """After a completion the factor is that of X-hat and the caches are
    rebuilt: R for X-hat equals R for X when P(X^-1) = S."""
    pat = CASES["arrow_small"]()
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    y = V.make_y(*pat, seed=8)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(V.make_x(*pat, seed=1)))
    b.hessian_factor(dev(y))  # caches for another X
    b.completion(dev(s))
    close(pat, host(b.hessian_factor(dev(y))), oracle.hessian_factor(pat, ldl, s, y))


def test_hessian_factor_arguments(mfb):
    pat = P.band(20, 2)
    b = mfb.SparseBarrier(pat)
    y = dev(V.make_y(*pat))
    w = torch.empty_like(y)
    with pytest.raises(mfb.MfbError) as e:
        mfb.hessian_factor(b.f, y, w, b.arena(1), k=1)
    assert e.value.code == mfb.ESTATE
    b.factor(dev(V.make_x(*pat)))
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(mfb.MfbError) as e:
        mfb.hessian_factor_adj(b.f, y, w, small, k=1)
    assert e.value.code == mfb.EINVAL
    mfb.hessian_factor(b.f, y, w, b.arena(1), k=0)  # k = 0 is a no-op
    plan = b.f.plan
    g = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(mfb.MfbError) as e:
        mfb.gram(plan, y, g, small, m=1)
    assert e.value.code == mfb.EINVAL


def _sparse_ys(pat, k, nz, seed):
    """k right-hand sides with nz random nonzero entries each (one of them
    all zero when k > 2): the sparse arguments of Section 5.5."""
    rng = np.random.default_rng(seed)
    nnz = pat[1][-1]
    ys = np.zeros((k, nnz))
    for r in range(k):
        if k > 2 and r == 1:
            continue
        pos = rng.choice(nnz, size=min(nz, nnz), replace=False)
        ys[r, pos] = rng.uniform(-1, 1, pos.size)
    return ys


@pytest.mark.parametrize("name", ["arrow_mixed", "grid3d_8", "chordal150", "grid2d_24", "band400_w200"])
def test_sparse_arguments_pruned(name, mfb):
    """Hessian step 1 skips the fronts whose subtree holds no nonzero of
    the right-hand side (their K and update blocks are zero) and the Hessian
    factor writes W = 0 there: R(Y) and H(Y) for sparse Y (a few nonzeros,
    one right-hand side all zero, one dense beside them) against the oracle,
    on the default plan and with the tile-parallel kernels forced."""
    pat = WIDE_PATS[name]() if name in WIDE_PATS else CASES[name]()
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    ys = _sparse_ys(pat, 4, 3, seed=11)
    ys[3] = V.make_y(*pat, seed=12)
    with cf.ThreadPoolExecutor(4) as ex:
        fw = [ex.submit(oracle.hessian_factor, pat, ldl, s, ys[r]) for r in range(4)]
        ft = [ex.submit(oracle.hessian, pat, ldl, s, ys[r]) for r in range(4)]
        want_w = [q.result() for q in fw]
        want_t = [q.result() for q in ft]
    for flags in (0, mfb.PLAN_WIDE_LOW):
        b = mfb.SparseBarrier(pat, flags=flags)
        b.factor(dev(x))
        w = host(b.hessian_factor(dev(ys)))
        t = host(b.hessian(dev(ys)))
        assert not w[1].any() and not t[1].any()
        for r in (0, 2, 3):
            close(pat, w[r], want_w[r])
            close(pat, t[r], want_t[r])
        # a sparse right-hand side alone gives the bits it has in the batch
        assert np.array_equal(host(b.hessian_factor(dev(ys[0]))), w[0])
