"""Pins of the oracle's completion with factored update matrices
(Algorithm 4.3, eqs. e-mf-compl-1-factored, e-mfp-compl-3-factored,
e-mf-compl-2-factored) against what the mathematics fixes: the completion
factor is unique, so it must equal Algorithm 4.2's and the factor of the X
whose projected inverse is S; every propagated R_j must be the upper
triangular factor of S_{I_j I_j} with a positive diagonal (unique, and
computed here by numpy's Cholesky of the index-reversed matrix); the dense
inverse of the result must reproduce S on V.  No GPU."""
import numpy as np
import pytest

import oracle
from workloads import get_config, patterns as P, values as V

PATS = {
    "band30_4": lambda: P.band(30, 4),
    "band40_1": lambda: P.band(40, 1),
    "arrow": lambda: P.block_arrow([5, 40, 1, 33, 20], 12),
    "chordal120": lambda: P.random_chordal(120, 0.04, 3),
    "forest": lambda: P.random_chordal(60, 0.03, 5),
    "grid2d_12": lambda: P.grid_nd((12, 12)),
    "dense9": lambda: P.band(9, 8),
    "diag7": lambda: P.band(7, 0),
}


def _dense(pat, v):
    n, cp, ri = pat
    a = np.zeros((n, n))
    for j in range(n):
        for e in range(cp[j], cp[j + 1]):
            a[ri[e], j] = a[j, ri[e]] = v[e]
    return a


def _ldl_dense(pat, ldl):
    n, cp, ri = pat
    L = np.eye(n)
    d = np.zeros(n)
    for j in range(n):
        d[j] = ldl[cp[j]]
        for e in range(cp[j] + 1, cp[j + 1]):
            L[ri[e], j] = ldl[e]
    return L, d


def _case(name):
    pat = PATS[name]()
    x = V.make_x(*pat, seed=1)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    return pat, x, ldl, s


@pytest.mark.parametrize("name", sorted(PATS))
def test_factored_completion_equals_plain_and_original_factor(name):
    pat, x, ldl, s = _case(name)
    got = oracle.completion_factored(pat, s)
    plain = oracle.completion(pat, s)
    scale = np.max(np.abs(ldl))
    assert np.max(np.abs(got - plain)) <= 1e-12 * scale
    assert np.max(np.abs(got - ldl)) <= 1e-11 * scale


@pytest.mark.parametrize("name", sorted(PATS))
def test_every_r_is_the_reverse_cholesky_of_the_clique_block(name):
    pat, x, ldl, s = _case(name)
    n, cp, ri = pat
    sd = _dense(pat, s)
    _, rs = oracle.completion_factored(pat, s, with_r=True)
    for j in range(n):
        idx = np.asarray(ri[cp[j] + 1:cp[j + 1]])
        r = rs[j]
        assert r.shape == (len(idx), len(idx))
        if len(idx) == 0:
            continue
        assert np.array_equal(r, np.triu(r)) and (np.diag(r) > 0).all()
        v = sd[np.ix_(idx, idx)]
        assert np.max(np.abs(r @ r.T - v)) <= 1e-12 * np.max(np.abs(v))
        flip = np.linalg.cholesky(v[::-1, ::-1])[::-1, ::-1]
        assert np.max(np.abs(r - flip)) <= 1e-10 * np.max(np.abs(flip))


@pytest.mark.parametrize("name", ["arrow", "chordal120", "grid2d_12"])
def test_dense_inverse_reproduces_s_on_the_pattern(name):
    pat, x, ldl, s = _case(name)
    n, cp, ri = pat
    L, d = _ldl_dense(pat, oracle.completion_factored(pat, s))
    xinv = np.linalg.inv(L @ np.diag(d) @ L.T)
    sd = _dense(pat, s)
    mask = _dense(pat, np.ones(cp[-1])) != 0
    assert np.max(np.abs(xinv[mask] - sd[mask])) <= 1e-10 * np.max(np.abs(sd))


def test_no_deleted_row_keeps_the_parent_factor():
    """On a dense pattern every child keeps all of its parent's rows
    (E = I): the reduction must leave R_j unchanged, bit for bit."""
    pat, x, ldl, s = _case("dense9")
    n, cp, ri = pat
    _, rs = oracle.completion_factored(pat, s, with_r=True)
    for c in range(n - 1):
        j = c + 1
        assert np.array_equal(rs[c][1:, 1:], rs[j])


def test_band_deletes_one_row_per_step():
    """Band of width w: I_c \\ {j} drops the last row of R_j (c = j - 1 in
    the interior), so R is R_j without its last row, retriangularized; its
    Gram matrix must be the leading block of R_j R_j^T."""
    pat, x, ldl, s = _case("band30_4")
    n, cp, ri = pat
    _, rs = oracle.completion_factored(pat, s, with_r=True)
    for c in range(n - 6):
        j = c + 1
        rj = rs[j]
        lead = (rj @ rj.T)[:-1, :-1]
        r = rs[c][1:, 1:]
        assert np.max(np.abs(r @ r.T - lead)) <= 1e-12 * np.max(np.abs(lead))
        assert not np.allclose(r, rj[:-1, :-1])  # a real reduction took place


def test_not_completable_raises_like_plain():
    pat = P.band(6, 2)
    n, cp, ri = pat
    s = np.zeros(cp[-1])
    for j in range(n):
        s[cp[j]] = 1.0
        for e in range(cp[j] + 1, cp[j + 1]):
            s[e] = 0.99  # every 3 x 3 clique block nearly singular, some not PD
    s[cp[2] + 1] = -0.99
    with pytest.raises(oracle.OracleError) as a:
        oracle.completion(pat, s)
    with pytest.raises(oracle.OracleError) as b:
        oracle.completion_factored(pat, s)
    assert a.value.code == b.value.code == "ENOCOMPLETION"
