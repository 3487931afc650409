"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerance (target: relative error <= 1e-10 in FP64), checked two ways on
every array:

* norm-wise: ||a - b|| / ||b|| <= tol, with the Frobenius norm of the full
  symmetric matrix on V (off-diagonal entries weighted twice); the exported
  factor (not a symmetric matrix) uses the plain 2-norm;
* entry-wise: |a_i - b_i| <= tol * (|b_i| + PHI * max_j |b_j|) for every
  stored entry i, so that no single entry, however small, can be wrong
  while the norm still passes.  PHI = 1e-2: rounding errors of an entry
  come from sums over whole fronts, so they scale with the size of the
  array, not of the entry itself; the floor PHI * max|b| at tol = 1e-10 is
  1e-12 * max|b|, three orders above the errors measured on these cases.

Scalars use |a - b| / max(1, |b|).  Ill-conditioned inputs scale tol with
the condition number (see test_ill_conditioned).
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from tests.golden import load_fig1
from workloads import get_config, patterns as P, values as V

pytestmark = pytest.mark.gpu

TOL = 1e-10
PHI = 1e-2

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


def entry_ratio(a, b):
    """max_i |a_i - b_i| / (|b_i| + PHI max|b|): at most tol when every entry
    meets the entry-wise bound."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    floor = PHI * max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b) / (np.abs(b) + floor)))


def close(pat, a, b, tol=TOL):
    """Norm-wise (symmetric weighting when pat is given) and entry-wise check."""
    if pat is None:
        ne = float(np.linalg.norm(np.asarray(a) - b) / max(1e-300, np.linalg.norm(b)))
    else:
        ne = relerr(pat, a, b)
    ee = entry_ratio(a, b)
    assert ne <= tol and ee <= tol, (ne, ee, tol)
    return ne, ee


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
    close(None, got, case.ldl)
    assert case.b.status() == (0, -1)


def test_logdet(case):
    got = float(host(case.b.logdet())[0])
    assert abs(got - case.logdet) / max(1.0, abs(case.logdet)) <= TOL


def test_projected_inverse(case):
    got = host(case.b.projected_inverse())
    close(case.pat, got, case.s)


def test_hessian_batched_and_single(case):
    ys = dev(case.ys)
    tk = host(case.b.hessian(ys))
    for r in range(len(case.ys)):
        close(case.pat, tk[r], case.t[r])
    # one right-hand side alone gives the same bits as inside the batch
    t1 = host(case.b.hessian(dev(case.ys[1])))
    assert np.array_equal(t1, tk[1])
    # repeated calls are bitwise reproducible
    assert np.array_equal(host(case.b.hessian(ys)), tk)


def test_inv_hessian(case):
    yi = host(case.b.inv_hessian(dev(case.ys[:2])))
    for r in range(2):
        close(case.pat, yi[r], case.yi[r])
    # H^-1(H(Y)) = Y on the device
    back = host(case.b.inv_hessian(dev(np.stack(case.t[:1]))))
    close(case.pat, back[0], case.ys[0], 1e-9)


def test_cholesky_product(case):
    got = host(case.b.cholesky_product())
    close(case.pat, got, case.x)


def test_completion_recovers_x(case, mfb):
    b2 = mfb.SparseBarrier(case.pat)
    b2.completion(dev(case.s))
    assert b2.status() == (0, -1)
    ldl = host(b2.export_ldl())
    close(None, ldl, case.ldl)
    xhat = host(b2.cholesky_product())
    close(case.pat, xhat, case.x)
    n = case.pat[0]
    fstar = float(host(b2.logdet())[0]) - n
    want = case.logdet - n
    assert abs(fstar - want) / max(1.0, abs(want)) <= TOL
    # the completion's cached S serves the Hessian directly
    t0 = host(b2.hessian(dev(case.ys[0])))
    close(case.pat, t0, case.t[0])


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
    close(None, outs[1][1], want_ldl)
    for r in range(2):
        want = oracle.inv_hessian(pat, ldl, s, ys[r])
        close(pat, outs[1][0][r], want)


def test_completion_of_general_s(mfb):
    pat = P.random_chordal(60, 0.06, 8)
    s = V.project(*pat, V.make_spd_dense(pat[0], 3))
    want = oracle.completion(pat, s)
    b = mfb.SparseBarrier(pat)
    b.completion(dev(s))
    got = host(b.export_ldl())
    close(None, got, want)


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


def test_batched_workload_k64(mfb):
    """The block-arrow workload (64 diagonal blocks of 32-256 plus a dense
    arrow of 128: fronts up to 384) with k = 64 right-hand sides in one call
    per operation.  Factor, gradient, Hessian and inverse Hessian against
    the oracle entry by entry (Hessian on four of the 64 right-hand sides,
    inverse Hessian on one), batched against single-RHS calls bitwise, and
    the completion of S recovering X."""
    pat = get_config("arrow64")
    k = 64
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, k, seed=0)
    picked = (0, 21, 42, 63)
    print("[gpu-parity] arrow64 k=64: oracle", flush=True)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    with cf.ThreadPoolExecutor(6) as ex:
        fut_t = {r: ex.submit(oracle.hessian, pat, ldl, s, ys[r]) for r in picked}
        want_t = {r: f.result() for r, f in fut_t.items()}
        fut_y = ex.submit(oracle.inv_hessian, pat, ldl, s, want_t[0])
        want_y0 = fut_y.result()
    print("[gpu-parity] arrow64 k=64: device", flush=True)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    close(None, host(b.export_ldl()), ldl)
    close(pat, host(b.projected_inverse()), s)
    tk = host(b.hessian(dev(ys)))
    for r in picked:
        close(pat, tk[r], want_t[r])
    for r in (0, 63):
        assert np.array_equal(host(b.hessian(dev(ys[r]))), tk[r])
    # inverse Hessian of all 64 in one call: H^-1(H(Y_r)) = Y_r for every r,
    # and the oracle's H^-1 of its own T_0 entry by entry
    tin = tk.copy()
    tin[0] = want_t[0]
    yk = host(b.inv_hessian(dev(tin)))
    close(pat, yk[0], want_y0)
    for r in range(1, k):
        close(pat, yk[r], ys[r], 1e-9)
    assert np.array_equal(host(b.inv_hessian(dev(tin[63]))), yk[63])
    c = mfb.SparseBarrier(pat)
    c.completion(dev(s))
    assert c.status() == (0, -1)
    close(None, host(c.export_ldl()), ldl)
    close(pat, host(c.cholesky_product()), x)


ILL = [("chordal150", 1e-2), ("chordal150", 1e-4), ("chordal150", 1e-6),
       ("band200", 1e-4), ("band200", 1e-6), ("arrow_small", 1e-4), ("arrow_small", 1e-6),
       ("arrow_mixed", 1e-5), ("grid2d_24", 1e-6)]


@pytest.mark.parametrize("name,delta", ILL)
def test_ill_conditioned(name, delta, mfb):
    """X = (weighted graph Laplacian) + delta I, condition number kappa up to
    about 1e8.  To first order a result obtained by solving with X loses
    kappa * eps of relative accuracy (the oracle against dense LAPACK loses
    <= 2e-17 kappa on these families), so the factor, the gradient, the
    Hessian and the completion are held to max(1e-10, 10 kappa eps).  The
    inverse Hessian solves with H, whose condition number is at most
    kappa^2: max(1e-10, 10 kappa^2 eps), checked while that stays below
    1e-6.  The factor 10 covers the entry-wise form of the check: on these
    inputs the error concentrates in the few entries tied to the smallest
    eigenvalues (chordal150 at kappa = 5e3: inverse Hessian entry-wise
    1.3 kappa^2 eps against 0.009 kappa^2 eps norm-wise; a numpy model of
    the block algorithm gives the same error with an explicit S_AA^-1, a
    Gauss-Jordan sweep or a Cholesky solve)."""
    pat = CASES[name]()
    n = pat[0]
    x = V.make_x_laplacian(*pat, delta, seed=3)
    ev = np.linalg.eigvalsh(V.to_dense(*pat, x))
    kappa = float(ev[-1] / ev[0])
    eps = np.finfo(np.float64).eps
    tol = max(TOL, 10 * kappa * eps)
    tol_ih = max(TOL, 10 * kappa ** 2 * eps)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    ys = V.make_ys(*pat, 2, seed=4)
    t = [oracle.hessian(pat, ldl, s, y) for y in ys]
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    errs = {"kappa": kappa}
    errs["ldl"] = close(None, host(b.export_ldl()), ldl, tol)
    errs["s"] = close(pat, host(b.projected_inverse()), s, tol)
    tk = host(b.hessian(dev(ys)))
    errs["t"] = max(close(pat, tk[r], t[r], tol) for r in range(2))
    ld = float(host(b.logdet())[0])
    want_ld = oracle.logdet(pat, ldl)
    assert abs(ld - want_ld) / max(1.0, abs(want_ld)) <= tol
    if tol_ih <= 1e-6:
        want_y = oracle.inv_hessian(pat, ldl, s, t[0])
        errs["inv_hessian"] = close(pat, host(b.inv_hessian(dev(t[0]))), want_y, tol_ih)
    c = mfb.SparseBarrier(pat)
    c.completion(dev(s))
    assert c.status() == (0, -1)
    errs["xhat"] = close(pat, host(c.cholesky_product()), x, tol)
    print(f"[gpu-parity] ill-conditioned {name} delta={delta:g} n={n}: {errs}", flush=True)


WIDE_CASES = [
    # name, plan flags: 0 = default wide threshold (front order above 192)
    ("chordal150", "low"),
    # fronts of more than 64 columns ("fat": the panel work tile-parallel
    # too), among them roots and a 528-column dense front
    ("arrow_small", "low"),
    ("arrow_mixed", "low"),
    ("roots_mixed", "low"),
    ("dense528", "default"),
    ("grid3d_8", "low"),
    ("grid3d_12", "low"),
    ("grid2d_128", "low"),
    # chains of single-column supernodes with 200 (520) ancestors, as in the
    # separators of the 3D grid: 4 (9) tiles per side with a ragged tail
    ("band600_w200", "low"),
    ("band1200_w520", "default"),
]


@pytest.mark.parametrize("name,thr", WIDE_CASES)
def test_wide_fronts(name, thr, mfb):
    """The tile-parallel kernels of wide fronts (front order above the
    threshold: those with at most 64 columns in the leaf-to-root sweeps,
    all of them in the root-to-leaf sweeps) and of fat fronts (above the
    threshold with more than 64 columns) against the oracle on every
    operation, with the threshold lowered to front order 65 where the
    pattern has no front above 512."""
    pat = CASES[name]() if name in CASES else get_config(name)
    flags = mfb.PLAN_WIDE_LOW if thr == "low" else 0
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, 2, seed=7)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    with cf.ThreadPoolExecutor(3) as ex:
        ft = [ex.submit(oracle.hessian, pat, ldl, s, y) for y in ys]
        t = [q.result() for q in ft]
        want_y = ex.submit(oracle.inv_hessian, pat, ldl, s, t[0]).result()
    print(f"[gpu-parity] wide fronts {name} ({thr})", flush=True)
    b = mfb.SparseBarrier(pat, flags=flags)
    b.factor(dev(x))
    assert b.status() == (0, -1)
    close(None, host(b.export_ldl()), ldl)
    ld = float(host(b.logdet())[0])
    want_ld = oracle.logdet(pat, ldl)
    assert abs(ld - want_ld) / max(1.0, abs(want_ld)) <= TOL
    close(pat, host(b.projected_inverse()), s)
    tk = host(b.hessian(dev(ys)))
    for r in range(2):
        close(pat, tk[r], t[r])
    assert np.array_equal(host(b.hessian(dev(ys[1]))), tk[1])
    close(pat, host(b.inv_hessian(dev(t[0]))), want_y)
    close(pat, host(b.cholesky_product()), x)
    c = mfb.SparseBarrier(pat, flags=flags)
    c.completion(dev(s))
    assert c.status() == (0, -1)
    close(None, host(c.export_ldl()), ldl)
    close(pat, host(c.cholesky_product()), x)


@pytest.mark.parametrize("shape", ["band300_w100", "band200_w70", "arrow40x3_100", "arrow100x2_100",
                                   "arrow100x2_250", "band400_w200"])
def test_tile_parallel_inverse_hessian_shapes(shape, mfb):
    """Inverse Hessian through the tile-parallel path (MFB_PLAN_WIDE_LOW) on
    fronts whose ancestor blocks span two to four 64-row tiles: explicit
    (S_AA)^-1 for A = 70 and 100 (N = 1, 40, 100), the factored form for
    A = 200 and 250; the default plan beside it; and the Hessian, whose
    root-to-leaf sweep forms V' L from partial products on fronts with at
    most four columns.  A first version of the explicit product was wrong
    here by O(1)."""
    pat = {"band300_w100": lambda: P.band(300, 100), "band200_w70": lambda: P.band(200, 70),
           "arrow40x3_100": lambda: P.block_arrow([40, 40, 40], 100),
           "arrow100x2_100": lambda: P.block_arrow([100, 100], 100),
           "arrow100x2_250": lambda: P.block_arrow([100, 100], 250),
           "band400_w200": lambda: P.band(400, 200)}[shape]()
    x = V.make_x(*pat, seed=0)
    y = V.make_y(*pat, seed=7)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    t0 = oracle.hessian(pat, ldl, s, y)
    want = oracle.inv_hessian(pat, ldl, s, t0)
    # (without the source map the gathers also form the partial products
    # T_AA L of the fronts with at most four columns)
    for flags in (0, mfb.PLAN_WIDE_LOW, mfb.PLAN_WIDE_LOW | mfb.PLAN_NO_GATHER_MAP):
        b = mfb.SparseBarrier(pat, flags=flags)
        b.factor(dev(x))
        close(pat, host(b.inv_hessian(dev(t0))), want)
        close(pat, host(b.hessian(dev(y))), t0)
        c = mfb.SparseBarrier(pat, flags=flags)
        c.completion(dev(s))
        assert c.status() == (0, -1)
        close(None, host(c.export_ldl()), ldl)


def test_large_grid_sampled(mfb):
    """The 3D 7-point grid 40^3 (n = 64000, 42165 supernodes, 298 levels,
    fronts up to 2360, root of 1601 columns), in full.  The oracle needs
    about half an hour for its full arrays, so its values are compared at
    6712 positions stored by tests/golden/make_grid3d_40_samples.py (which
    runs only the oracle): factor, log det, gradient and the Hessian of two
    right-hand sides, entry by entry.  Properties that hold at any size
    cover the whole arrays: S.X = n, H(X) = S, H^-1(H(Y)) = Y and the
    completion of S recovering X."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "grid3d_40_samples.npz"))
    pat = get_config("grid3d_40")
    n, cp, ri = pat
    assert int(g["nnz"]) == int(cp[-1])
    idx = g["idx"]
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, 2, seed=0)
    print("[gpu-parity] grid3d_40: factor", flush=True)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    assert b.status() == (0, -1)
    close(None, host(b.export_ldl())[idx], g["ldl"])
    ld = float(host(b.logdet())[0])
    assert abs(ld - float(g["logdet"])) / abs(float(g["logdet"])) <= TOL
    s = host(b.projected_inverse())
    close(None, s[idx], g["s"])
    w = np.where(np.asarray(ri) == V.column_index(n, cp), 1.0, 2.0)
    assert abs(float(np.sum(w * s * x)) - n) / n <= TOL
    print("[gpu-parity] grid3d_40: hessian", flush=True)
    tk = host(b.hessian(dev(ys)))
    close(None, tk[0][idx], g["t0"])
    close(None, tk[1][idx], g["t1"])
    close(pat, host(b.hessian(dev(x))), s)
    print("[gpu-parity] grid3d_40: inverse hessian", flush=True)
    yk = host(b.inv_hessian(dev(tk)))
    for r in range(2):
        close(pat, yk[r], ys[r], 1e-9)
    del b
    print("[gpu-parity] grid3d_40: completion", flush=True)
    c = mfb.SparseBarrier(pat)
    c.completion(dev(s))
    assert c.status() == (0, -1)
    close(pat, host(c.cholesky_product()), x)
    fstar = float(host(c.logdet())[0]) - n
    assert abs(fstar - (ld - n)) / abs(ld - n) <= TOL


@pytest.mark.parametrize("shape", ["band300_w100", "arrow100x2_250", "grid3d_8"])
def test_wide_inverse_hessian_batched(shape, mfb):
    """The tile-parallel panel part of the inverse Hessian's step 3 (fronts
    x 64-row tiles x right-hand sides in one grid) with k = 3 under
    MFB_PLAN_WIDE_LOW: every right-hand side against the oracle, and each
    one alone bitwise equal to its column of the batch."""
    pat = {"band300_w100": lambda: P.band(300, 100),
           "arrow100x2_250": lambda: P.block_arrow([100, 100], 250),
           "grid3d_8": lambda: get_config("grid3d_8")}[shape]()
    x = V.make_x(*pat, seed=0)
    ys = V.make_ys(*pat, 3, seed=9)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    with cf.ThreadPoolExecutor(3) as ex:
        ts = [q.result() for q in [ex.submit(oracle.hessian, pat, ldl, s, y) for y in ys]]
    print(f"[gpu-parity] batched wide inverse Hessian {shape}", flush=True)
    b = mfb.SparseBarrier(pat, flags=mfb.PLAN_WIDE_LOW)
    b.factor(dev(x))
    yk = host(b.inv_hessian(dev(np.stack(ts))))
    for r in range(3):
        close(pat, yk[r], ys[r], 1e-9)
        assert np.array_equal(host(b.inv_hessian(dev(ts[r]))), yk[r])
    close(pat, host(b.cholesky_product()), x)


def test_update_blocks_beyond_64_row_tiles(mfb):
    """Leaf fronts whose S_AA block has A = 4300 > 64 * 65 rows: the first
    block columns of its tile-parallel Cholesky factor and inverse run on the
    rectangular grid (more row tiles than the packed grid's offsets hold),
    the later ones on the packed grid.  The oracle would take minutes at this
    order, so the check uses identities that hold at any size (Algorithms
    7.2 and 7.3 invert each other; Algorithm 5.2 inverts Algorithm 5.1): the
    completion of the projected inverse of X gives X back, and the inverse
    Hessian at X (cached S_AA factors) and at X-hat (the completion's
    factors) both undo the Hessian."""
    pat = P.block_arrow([1, 1, 1], 4300)
    print("[gpu-parity] block_arrow 3 x 1 + 4300: factor", flush=True)
    x = V.make_x(*pat, seed=0)
    y = V.make_ys(*pat, 1, seed=1)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    s = host(b.projected_inverse())
    t = host(b.hessian(dev(y)))
    back = host(b.inv_hessian(dev(t)))
    assert b.status() == (0, -1)
    close(pat, back[0], y[0], 1e-9)
    print("[gpu-parity] block_arrow 3 x 1 + 4300: completion", flush=True)
    b2 = mfb.SparseBarrier(pat)
    b2.completion(dev(s))
    assert b2.status() == (0, -1)
    close(pat, host(b2.cholesky_product()), x)
    back2 = host(b2.inv_hessian(dev(t)))
    assert b2.status() == (0, -1)
    close(pat, back2[0], y[0], 1e-9)
