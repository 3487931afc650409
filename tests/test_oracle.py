"""Pins for the CPU oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's recursions.  Each op is checked against
its plain definition computed densely with numpy/LAPACK (Section 1:
grad f = -P(X^-1), Hessian P(X^-1 Y X^-1), X-hat with P(X-hat^-1) = S),
against closed forms (diagonal and tridiagonal patterns, full pattern),
against invariants (S.X = n, H(X) = S, H^-1(S) = X, Fenchel equality),
finite differences of f and grad f, and a brute-force solve of the
Hessian as a |V| x |V| matrix.  Inner products on S^n_V are the trace
inner product (off-diagonal entries count twice, Section 1.1).
"""
import numpy as np
import pytest

import oracle
from workloads import patterns as P
from workloads import values as Vv
from tests.golden import load_fig1


def ip(pat, a, b):
    """Trace inner product A.B on S^n_V from CCS lower-triangle values."""
    n, cp, ri = pat
    col = Vv.column_index(n, cp)
    w = np.where(np.asarray(ri) == col, 1.0, 2.0)
    return float(np.sum(w * a * b))


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(1e-300, np.linalg.norm(np.asarray(b)))


def dense_ldl(x_dense):
    """Scalar L D L^T of a dense SPD matrix from LAPACK's Cholesky."""
    g = np.linalg.cholesky(x_dense)
    d = np.diag(g) ** 2
    return g / np.diag(g)[None, :], d


def ldl_values(pat, l, d):
    n, cp, ri = pat
    col = Vv.column_index(n, cp)
    row = np.asarray(ri, dtype=np.int64)
    v = l[row, col].copy()
    v[cp[:-1]] = d
    return v


def ldl_dense(pat, ldl):
    n, cp, ri = pat
    col = Vv.column_index(n, cp)
    row = np.asarray(ri, dtype=np.int64)
    L = np.zeros((n, n))
    L[row, col] = ldl
    d = L[np.arange(n), np.arange(n)].copy()
    L[np.arange(n), np.arange(n)] = 1.0
    return L, d


def dense_hessian(pat, xd, y):
    n = pat[0]
    xi = np.linalg.inv(xd)
    yd = Vv.to_dense(*pat, y)
    return Vv.project(*pat, xi @ yd @ xi)


PATTERNS = {
    "band30_w4": lambda: P.band(30, 4),
    "band12_w1": lambda: P.band(12, 1),
    "diag9": lambda: P.band(9, 0),
    "full12": lambda: P.band(12, 11),
    "arrow": lambda: P.block_arrow([3, 5, 2, 4], 3),
    "chordal35": lambda: P.random_chordal(35, 0.08, 3),
    "chordal28": lambda: P.random_chordal(28, 0.15, 11),
    "forest": lambda: P.random_chordal(25, 0.03, 5),
    "tree20": lambda: P.random_tree_pattern(20, 2),
    "grid5x6": lambda: P.grid_nd((5, 6)),
    "fig1": lambda: load_fig1()["pattern"],
}


@pytest.fixture(params=sorted(PATTERNS), scope="module")
def case(request, oracle_lib):
    pat = PATTERNS[request.param]()
    x = Vv.make_x(*pat, seed=7)
    y = Vv.make_y(*pat, seed=7, r=0)
    return request.param, pat, x, y


def test_factor_matches_lapack_cholesky(case):
    name, pat, x, _ = case
    xd = Vv.to_dense(*pat, x)
    ldl = oracle.factor(pat, x)
    l, d = dense_ldl(xd)
    assert rel(ldl, ldl_values(pat, l, d)) < 1e-13
    # the factor lives on V: LAPACK's L vanishes off the pattern
    mask = P.dense_mask(*pat)
    assert np.abs(np.tril(l, -1)[~mask]).max(initial=0.0) < 1e-13


def test_product_reconstructs_x(case):
    name, pat, x, _ = case
    ldl = oracle.factor(pat, x)
    assert rel(oracle.product(pat, ldl), x) < 1e-13
    # L D L^T formed densely from the oracle's factor
    L, d = ldl_dense(pat, ldl)
    assert rel(Vv.project(*pat, L @ np.diag(d) @ L.T), x) < 1e-13


def test_logdet_matches_slogdet_and_scaling(case):
    name, pat, x, _ = case
    n = pat[0]
    sign, ld = np.linalg.slogdet(Vv.to_dense(*pat, x))
    assert sign > 0
    got = oracle.logdet(pat, oracle.factor(pat, x))
    assert abs(got - ld) <= 1e-12 * max(1.0, abs(ld))
    got2 = oracle.logdet(pat, oracle.factor(pat, 3.0 * x))
    assert abs(got2 - (ld + n * np.log(3.0))) <= 1e-12 * max(1.0, abs(ld))


def test_projinv_is_projected_dense_inverse(case):
    name, pat, x, _ = case
    n = pat[0]
    xd = Vv.to_dense(*pat, x)
    s = oracle.projinv(pat, oracle.factor(pat, x))
    assert rel(s, Vv.project(*pat, np.linalg.inv(xd))) < 1e-12
    # grad f . X = -n  <=>  S . X = n
    assert abs(ip(pat, s, x) - n) < 1e-10 * n


def test_projinv_finite_difference_of_logdet(case):
    name, pat, x, y = case
    h = 1e-5
    s = oracle.projinv(pat, oracle.factor(pat, x))
    fp = oracle.logdet(pat, oracle.factor(pat, x + h * y))
    fm = oracle.logdet(pat, oracle.factor(pat, x - h * y))
    fd = (fp - fm) / (2 * h)
    assert abs(fd - ip(pat, s, y)) < 1e-7 * max(1.0, abs(fd))


def test_hessian_dense_and_invariants(case):
    name, pat, x, y = case
    xd = Vv.to_dense(*pat, x)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    t = oracle.hessian(pat, ldl, s, y)
    assert rel(t, dense_hessian(pat, xd, y)) < 1e-12
    # H(X) = P(X^-1 X X^-1) = S
    assert rel(oracle.hessian(pat, ldl, s, x), s) < 1e-12
    # self-adjoint and positive definite
    z = Vv.make_y(*pat, seed=7, r=5)
    tz = oracle.hessian(pat, ldl, s, z)
    assert abs(ip(pat, y, tz) - ip(pat, z, t)) < 1e-11 * max(1.0, abs(ip(pat, y, tz)))
    assert ip(pat, y, t) > 0
    # H_{aX} = H_X / a^2
    ldl2 = oracle.factor(pat, 2.0 * x)
    t2 = oracle.hessian(pat, ldl2, oracle.projinv(pat, ldl2), y)
    assert rel(t2, t / 4.0) < 1e-12


def test_hessian_finite_difference_of_gradient(case):
    name, pat, x, y = case
    h = 1e-5
    ldl = oracle.factor(pat, x)
    t = oracle.hessian(pat, ldl, oracle.projinv(pat, ldl), y)
    sp = oracle.projinv(pat, oracle.factor(pat, x + h * y))
    sm = oracle.projinv(pat, oracle.factor(pat, x - h * y))
    assert rel(-(sp - sm) / (2 * h), t) < 1e-7


def test_inv_hessian_round_trips(case):
    name, pat, x, y = case
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    t = oracle.hessian(pat, ldl, s, y)
    assert rel(oracle.inv_hessian(pat, ldl, s, t), y) < 1e-10
    yy = oracle.inv_hessian(pat, ldl, s, y)
    assert rel(oracle.hessian(pat, ldl, s, yy), y) < 1e-10
    # H^-1(S) = X
    assert rel(oracle.inv_hessian(pat, ldl, s, s), x) < 1e-10


def test_inv_hessian_brute_force_matrix(case):
    """Assemble the Hessian as an nnz x nnz matrix from the dense formula and
    solve; compare with the oracle's inverse Hessian."""
    name, pat, x, y = case
    nnz = int(pat[1][-1])
    if nnz > 320:
        pytest.skip("brute force limited to |V| <= 320")
    xd = Vv.to_dense(*pat, x)
    H = np.zeros((nnz, nnz))
    for e in range(nnz):
        u = np.zeros(nnz)
        u[e] = 1.0
        H[:, e] = dense_hessian(pat, xd, u)
    want = np.linalg.solve(H, y)
    ldl = oracle.factor(pat, x)
    got = oracle.inv_hessian(pat, ldl, oracle.projinv(pat, ldl), y)
    assert rel(got, want) < 1e-9


def test_completion_recovers_x(case):
    name, pat, x, _ = case
    n = pat[0]
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    ldl_hat = oracle.completion(pat, s)
    assert rel(oracle.product(pat, ldl_hat), x) < 1e-10
    assert rel(ldl_hat, ldl) < 1e-10


def test_completion_of_projected_spd(case):
    """S = P(Z) for a dense SPD Z: X-hat in S^n_V with P(X-hat^-1) = S, the
    Fenchel equality S.X-hat = n, and f_*(S) = log det X-hat - n equal to
    -log det of the max-det completion minus n."""
    name, pat, _, _ = case
    n = pat[0]
    z = Vv.make_spd_dense(n, seed=4)
    s = Vv.project(*pat, z)
    ldl_hat = oracle.completion(pat, s)
    L, d = ldl_dense(pat, ldl_hat)
    xhat = L @ np.diag(d) @ L.T
    mask = P.dense_mask(*pat)
    assert np.abs(xhat[~mask]).max(initial=0.0) < 1e-12 * np.abs(xhat).max()
    assert rel(Vv.project(*pat, np.linalg.inv(xhat)), s) < 1e-10
    assert abs(ip(pat, s, Vv.project(*pat, xhat)) - n) < 1e-9 * n
    # the completion W = X-hat^-1 agrees with S on V and has the larger det
    w = np.linalg.inv(xhat)
    fstar = oracle.logdet(pat, ldl_hat) - n
    assert abs(fstar - (-np.linalg.slogdet(w)[1] - n)) < 1e-9 * max(1, abs(fstar))
    assert np.linalg.slogdet(w)[1] >= np.linalg.slogdet(z)[1] - 1e-9


def test_hessian_factor_composes_to_hessian(case):
    name, pat, x, y = case
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    w = oracle.hessian_factor(pat, ldl, s, y)
    t = oracle.hessian_factor_adj(pat, ldl, s, w)
    assert rel(t, oracle.hessian(pat, ldl, s, y)) < 1e-11
    z = Vv.make_y(*pat, seed=7, r=3)
    wz = oracle.hessian_factor(pat, ldl, s, z)
    lhs = ip(pat, z, oracle.hessian(pat, ldl, s, y))
    assert abs(lhs - ip(pat, wz, w)) < 1e-10 * max(1.0, abs(lhs))
    # R^adj is the adjoint of R: R(Y).W' = Y.R^adj(W')
    wp = Vv.make_y(*pat, seed=9, r=1)
    assert abs(ip(pat, w, wp) - ip(pat, y, oracle.hessian_factor_adj(pat, ldl, s, wp))) < \
        1e-10 * max(1.0, abs(ip(pat, w, wp)))


# ---------------------------------------------------------------- closed forms

def test_diagonal_pattern_closed_forms(oracle_lib):
    pat = P.band(10, 0)
    x = np.linspace(1.0, 3.0, 10)
    y = np.linspace(-1.0, 1.0, 10)
    ldl = oracle.factor(pat, x)
    assert np.allclose(ldl, x, rtol=0, atol=0)
    s = oracle.projinv(pat, ldl)
    assert np.allclose(s, 1.0 / x, rtol=1e-15)
    assert np.allclose(oracle.hessian(pat, ldl, s, y), y / x**2, rtol=1e-15)
    assert np.allclose(oracle.inv_hessian(pat, ldl, s, y), y * x**2, rtol=1e-15)
    assert np.allclose(oracle.completion(pat, s), x, rtol=1e-15)


def test_tridiagonal_pivot_recurrence(oracle_lib):
    """D_j = x_jj - x_{j,j-1}^2 / D_{j-1} for a tridiagonal X."""
    pat = P.band(15, 1)
    x = Vv.make_x(*pat, seed=3)
    ldl = oracle.factor(pat, x)
    cp = pat[1]
    d = np.empty(15)
    d[0] = x[cp[0]]
    for j in range(1, 15):
        off = x[cp[j - 1] + 1]
        d[j] = x[cp[j]] - off * off / d[j - 1]
    assert np.allclose(ldl[cp[:-1]], d, rtol=1e-14)
    for j in range(14):
        assert abs(ldl[cp[j] + 1] - x[cp[j] + 1] / d[j]) < 1e-14


def test_full_pattern_is_dense_inverse(oracle_lib):
    pat = P.band(8, 7)
    x = Vv.make_x(*pat, seed=1)
    xd = Vv.to_dense(*pat, x)
    s = oracle.projinv(pat, oracle.factor(pat, x))
    assert rel(Vv.to_dense(*pat, s), np.linalg.inv(xd)) < 1e-13
    # completion on a full pattern: X-hat = S^-1
    z = Vv.make_spd_dense(8, 2)
    sv = Vv.project(*pat, z)
    L, d = ldl_dense(pat, oracle.completion(pat, sv))
    assert rel(L @ np.diag(d) @ L.T, np.linalg.inv(z)) < 1e-12


# ---------------------------------------------------------------- failures

def test_non_pd_and_no_completion_are_reported(oracle_lib):
    pat = P.band(12, 2)
    x = Vv.make_x(*pat, seed=2)
    x[pat[1][5]] = -1.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.factor(pat, x)
    assert e.value.code == "ENOTPD" and 0 <= e.value.bad <= 5
    s = Vv.project(*pat, Vv.make_spd_dense(12, 1))
    s[pat[1][4] + 1] *= 50.0        # break positive semidefiniteness of a clique block
    with pytest.raises(oracle.OracleError) as e:
        oracle.completion(pat, s)
    assert e.value.code == "ENOCOMPLETION"


def test_unfilled_pattern_rejected(oracle_lib):
    g = load_fig1()
    n, cp, ri = g["pattern"]
    # drop (15, 5): (5,3) and (15,3) force it (Section 2, eq. e-filled)
    col = 4
    rows = list(ri[cp[col]:cp[col + 1]])
    rows.remove(14)
    ri2 = np.concatenate([ri[:cp[col]], np.array(rows, np.int32), ri[cp[col + 1]:]])
    cp2 = cp.copy()
    cp2[col + 1:] -= 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.etree((n, cp2, ri2))
    assert e.value.code == "ENOTCHORDAL"


def test_worked_example_etree_and_degrees(oracle_lib):
    g = load_fig1()
    parent, degree = oracle.etree(g["pattern"])
    assert [p + 1 if p >= 0 else 0 for p in parent] == g["parent"]
    assert list(degree) == g["degree"]
