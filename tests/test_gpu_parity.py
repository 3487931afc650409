"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerance: relative error <= 1e-10 in FP64, measured as ||a - b|| / ||b||
with the Frobenius norm of the full symmetric matrix on V (off-diagonal
entries weighted twice); scalars |a - b| / max(1, |b|).  The exported
factor (not a symmetric matrix) uses the plain 2-norm of the values.
"""
import numpy as np
import pytest

import oracle
from tests.golden import load_fig1
from workloads import get_config, patterns as P, values as V

pytestmark = pytest.mark.gpu

TOL = 1e-10

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def mfb():
    _need_gpu()
    from paper_1203_2742_amd import mfb as m
    return m


def wnorm(pat, v):
    n, cp, ri = pat
    col = V.column_index(n, cp)
    w = np.where(np.asarray(ri) == col, 1.0, 2.0)
    return float(np.sqrt(np.sum(w * np.asarray(v) ** 2)))


def relerr(pat, a, b):
    return wnorm(pat, np.asarray(a) - np.asarray(b)) / max(1e-300, wnorm(pat, b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()



def _roots_mixed():
    sizes = [100, 150, 250]
    n = sum(sizes) + 40
    mask = np.zeros((n, n), dtype=bool)
    o = 0
    for b in sizes:
        mask[o:o + b, o:o + b] = True
        o += b
    for j in range(o, n):
        mask[j:min(n, j + 4), j] = True
    return P.pattern_from_dense_mask(mask)


CASES = {
    "fig1": lambda: load_fig1()["pattern"],
    "band200": lambda: get_config("band200"),
    "diag50": lambda: P.band(50, 0),
    "full70": lambda: P.band(70, 69),
    "forest": lambda: P.random_chordal(90, 0.02, 5),
    "chordal150": lambda: P.random_chordal(150, 0.03, 2),
    "tree300": lambda: P.random_tree_pattern(300, 4),
    "arrow_small": lambda: P.block_arrow([5, 70, 1, 33, 97], 40),
    # fronts of order 63, 65, 80, 160 and 210: every register class and the
    # blocked kernels in one tree
    "arrow_mixed": lambda: P.block_arrow([5, 150, 20, 100, 3], 60),
    # one dense front with 528 columns: the blocked kernels read the column
    # offsets from global memory beyond the LDS cache of 512
    "dense528": lambda: P.block_arrow([520], 8),
    # a forest of roots (A = 0) of orders 100, 150 and 250 beside a band:
    # root fronts of several register classes and of the blocked kernels on
    # one level, where the up-sweeps take no congruences
    "roots_mixed": lambda: _roots_mixed(),
    "grid2d_24": lambda: get_config("grid2d_24"),
    "grid3d_8": lambda: get_config("grid3d_8"),
    "grid2d_128": lambda: get_config("grid2d_128"),
}


class Case:
    def __init__(self, name, mfb):
        self.name = name
        self.pat = CASES[name]()
        n, cp, ri = self.pat
        self.x = V.make_x(*self.pat, seed=0)
        self.ys = V.make_ys(*self.pat, 3, seed=0)
        self.ldl = oracle.factor(self.pat, self.x)
        self.s = oracle.projinv(self.pat, self.ldl)
        self.logdet = oracle.logdet(self.pat, self.ldl)
        self.t = [oracle.hessian(self.pat, self.ldl, self.s, y) for y in self.ys]
        self.yi = [oracle.inv_hessian(self.pat, self.ldl, self.s, y) for y in self.ys[:2]]
        print(f"[gpu-parity] case {name}: n={n} nnz={cp[-1]}", flush=True)
        self.b = mfb.SparseBarrier(self.pat)
        self.b.factor(dev(self.x))


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, mfb):
    return Case(request.param, mfb)


def test_factor_export_ldl(case):
    got = host(case.b.export_ldl())
    err = np.linalg.norm(got - case.ldl) / np.linalg.norm(case.ldl)
    assert err <= TOL, err
    assert case.b.status() == (0, -1)


def test_logdet(case):
    got = float(host(case.b.logdet())[0])
    assert abs(got - case.logdet) / max(1.0, abs(case.logdet)) <= TOL


def test_projected_inverse(case):
    got = host(case.b.projected_inverse())
    assert relerr(case.pat, got, case.s) <= TOL


def test_hessian_batched_and_single(case):
    ys = dev(case.ys)
    tk = host(case.b.hessian(ys))
    for r in range(len(case.ys)):
        assert relerr(case.pat, tk[r], case.t[r]) <= TOL, r
    # one right-hand side alone gives the same bits as inside the batch
    t1 = host(case.b.hessian(dev(case.ys[1])))
    assert np.array_equal(t1, tk[1])
    # repeated calls are bitwise reproducible
    assert np.array_equal(host(case.b.hessian(ys)), tk)


def test_inv_hessian(case):
    yi = host(case.b.inv_hessian(dev(case.ys[:2])))
    for r in range(2):
        assert relerr(case.pat, yi[r], case.yi[r]) <= TOL, r
    # H^-1(H(Y)) = Y on the device
    back = host(case.b.inv_hessian(dev(np.stack(case.t[:1]))))
    assert relerr(case.pat, back[0], case.ys[0]) <= 1e-9


def test_cholesky_product(case):
    got = host(case.b.cholesky_product())
    assert relerr(case.pat, got, case.x) <= TOL


def test_completion_recovers_x(case, mfb):
    b2 = mfb.SparseBarrier(case.pat)
    b2.completion(dev(case.s))
    assert b2.status() == (0, -1)
    ldl = host(b2.export_ldl())
    assert np.linalg.norm(ldl - case.ldl) / np.linalg.norm(case.ldl) <= TOL
    xhat = host(b2.cholesky_product())
    assert relerr(case.pat, xhat, case.x) <= TOL
    n = case.pat[0]
    fstar = float(host(b2.logdet())[0]) - n
    want = case.logdet - n
    assert abs(fstar - want) / max(1.0, abs(want)) <= TOL
    # the completion's cached S serves the Hessian directly
    t0 = host(b2.hessian(dev(case.ys[0])))
    assert relerr(case.pat, t0, case.t[0]) <= TOL


@pytest.mark.parametrize("name", ["arrow_small", "grid2d_24"])
def test_level_gathers_match_the_map(name, mfb):
    """The completion and the inverse Hessian read the A_s x A_s blocks of
    their input either through the plan's source map (one launch) or level
    by level from the parents (MFB_PLAN_NO_GATHER_MAP, the path of plans too
    large for the map): the same values land in the same places, so the
    outputs agree bitwise, and both agree with the oracle."""
    pat = CASES[name]()
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    ys = V.make_ys(*pat, 2, seed=5)
    outs = []
    for flags in (0, mfb.PLAN_NO_GATHER_MAP):
        b = mfb.SparseBarrier(pat, flags=flags)
        b.factor(dev(x))
        yy = host(b.inv_hessian(dev(ys)))
        b.completion(dev(s))
        assert b.status() == (0, -1)
        outs.append((yy, host(b.export_ldl())))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    want_ldl = oracle.factor(pat, x)
    assert np.linalg.norm(outs[1][1] - want_ldl) / np.linalg.norm(want_ldl) <= TOL
    for r in range(2):
        want = oracle.inv_hessian(pat, ldl, s, ys[r])
        assert relerr(pat, outs[1][0][r], want) <= TOL


def test_completion_of_general_s(mfb):
    pat = P.random_chordal(60, 0.06, 8)
    s = V.project(*pat, V.make_spd_dense(pat[0], 3))
    want = oracle.completion(pat, s)
    b = mfb.SparseBarrier(pat)
    b.completion(dev(s))
    got = host(b.export_ldl())
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= TOL


def test_not_positive_definite_reported(mfb):
    pat = P.band(40, 3)
    x = V.make_x(*pat, seed=1)
    x[pat[1][17]] = -5.0
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    code, bad = b.status()
    assert code == mfb.ENOTPD and 0 <= bad <= 17
    # a later good factorization clears the status
    b.factor(dev(V.make_x(*pat, seed=1)))
    assert b.status() == (0, -1)


def test_no_completion_reported(mfb):
    pat = P.band(30, 2)
    s = V.project(*pat, V.make_spd_dense(30, 1))
    s[pat[1][12] + 1] *= 50.0
    b = mfb.SparseBarrier(pat)
    b.completion(dev(s))
    code, _ = b.status()
    assert code == mfb.ENOCOMPLETION


def test_call_order_and_arguments(mfb):
    pat = P.band(20, 2)
    b = mfb.SparseBarrier(pat)
    y = dev(V.make_y(*pat))
    t = torch.empty_like(y)
    with pytest.raises(mfb.MfbError) as e:
        mfb.hessian(b.f, y, t, b.arena(1), k=1)
    assert e.value.code == mfb.ESTATE
    b.factor(dev(V.make_x(*pat)))
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(mfb.MfbError) as e:
        mfb.hessian(b.f, y, t, small, k=1)
    assert e.value.code == mfb.EINVAL
    mfb.hessian(b.f, y, t, b.arena(1), k=0)  # k = 0 is a no-op


@pytest.mark.parametrize("name", ["arrow64"])
def test_large_front_workload_sampled(name, mfb):
    """Block-arrow workload (fronts up to 384): factor, gradient and two
    Hessian right-hand sides against the oracle."""
    pat = get_config(name)
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, 2, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    got = host(b.export_ldl())
    assert np.linalg.norm(got - ldl) / np.linalg.norm(ldl) <= TOL
    assert relerr(pat, host(b.projected_inverse()), s) <= TOL
    tk = host(b.hessian(dev(ys)))
    for r in range(2):
        assert relerr(pat, tk[r], oracle.hessian(pat, ldl, s, ys[r])) <= TOL
    back = host(b.inv_hessian(dev(tk[:1])))
    assert relerr(pat, back[0], ys[0]) <= 1e-9
