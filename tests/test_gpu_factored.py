"""GPU parity of the completion with factored update matrices
(mfb_completion_factored: Algorithm 4.3 in supernodal form) against the
oracle's Algorithm 4.3, through the C ABI, element by element.  The
completion factor is unique, so the result must also agree with
mfb_completion and with the factor of the X whose projected inverse is S;
the handle must serve the operations that follow a completion (log det,
product, Hessian, inverse Hessian)."""
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


PATS = dict(CASES)
PATS["band300_40"] = lambda: P.band(300, 40)
PATS["grid3d_12"] = lambda: get_config("grid3d_12")
NAMES = ["fig1", "band200", "diag50", "full70", "forest", "chordal150", "tree300", "arrow_small",
         "arrow_mixed", "dense528", "roots_mixed", "grid2d_24", "grid3d_8", "band300_40", "grid3d_12"]


@pytest.mark.parametrize("name", NAMES)
def test_factored_completion_matches_oracle(name, mfb):
    pat = PATS[name]()
    print(f"[gpu-factored] {name}", flush=True)
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    want = oracle.completion_factored(pat, s)
    b = mfb.SparseBarrier(pat)
    b.completion_factored(dev(s))
    assert b.status() == (0, -1)
    got = host(b.export_ldl())
    close(None, got, want)
    close(None, got, ldl)
    # the same factor as the completion that factors every S_AA from scratch
    a = mfb.SparseBarrier(pat)
    a.completion(dev(s))
    close(None, got, host(a.export_ldl()))
    n = pat[0]
    ld = float(host(b.logdet())[0])
    want_ld = oracle.logdet(pat, want)
    assert abs(ld - want_ld) / max(1.0, abs(want_ld)) <= TOL
    close(pat, host(b.cholesky_product()), x)


@pytest.mark.parametrize("name", ["arrow_mixed", "grid2d_24", "grid3d_8"])
def test_factored_completion_serves_the_hessians(name, mfb):
    """S cached and V_s gathered: the Hessian and inverse Hessian that
    follow the completion match the oracle at X."""
    pat = PATS[name]()
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    ys = V.make_ys(*pat, 2, seed=3)
    b = mfb.SparseBarrier(pat)
    b.completion_factored(dev(s))
    t = host(b.hessian(dev(ys)))
    for r in range(2):
        close(pat, t[r], oracle.hessian(pat, ldl, s, ys[r]))
    yi = host(b.inv_hessian(dev(ys)))
    for r in range(2):
        close(pat, yi[r], oracle.inv_hessian(pat, ldl, s, ys[r]))


def test_factored_completion_of_general_s(mfb):
    pat = P.random_chordal(60, 0.06, 8)
    s = V.project(*pat, V.make_spd_dense(pat[0], 3))
    want = oracle.completion_factored(pat, s)
    b = mfb.SparseBarrier(pat)
    b.completion_factored(dev(s))
    assert b.status() == (0, -1)
    close(None, host(b.export_ldl()), want)


def test_factored_completion_repeated_and_after_other_ops(mfb):
    """Two calls in a row (the second with another S) and a call after a
    factor and an inverse Hessian (whose cached blocks live where the
    completion keeps its R_s) give the oracle's results."""
    pat = PATS["arrow_mixed"]()
    b = mfb.SparseBarrier(pat)
    for seed in (0, 4):
        x = V.make_x(*pat, seed=seed)
        s = oracle.projinv(pat, oracle.factor(pat, x))
        b.factor(dev(x))
        b.inv_hessian(dev(V.make_ys(*pat, 1, seed=1)))
        b.completion_factored(dev(s))
        assert b.status() == (0, -1)
        close(None, host(b.export_ldl()), oracle.completion_factored(pat, s))


def test_factored_completion_not_completable(mfb):
    pat = P.band(6, 2)
    n, cp, ri = pat
    s = np.zeros(cp[-1])
    for j in range(n):
        s[cp[j]] = 1.0
        for e in range(cp[j] + 1, cp[j + 1]):
            s[e] = 0.99
    s[cp[2] + 1] = -0.99
    with pytest.raises(oracle.OracleError):
        oracle.completion_factored(pat, s)
    b = mfb.SparseBarrier(pat)
    b.completion_factored(dev(s))
    code, _ = b.status()
    assert code == mfb.ENOCOMPLETION


def test_factored_completion_refused_on_relaxed_plan(mfb):
    pat = get_config("grid3d_8")
    b = mfb.SparseBarrier(pat, relax=0.2)
    s = dev(np.ones(pat[1][-1]))
    with pytest.raises(mfb.MfbError) as e:
        mfb.completion_factored(b.f, s)
    assert e.value.code == mfb.EINVAL


@pytest.mark.parametrize("name,flags", [("empty", 0), ("roots_mixed", 0), ("arrow_mixed", 1), ("grid3d_8", 1)])
def test_factored_completion_edge_plans(name, flags, mfb):
    """No supernode at all; a forest of roots beside a band (fronts with
    A = 0 next to fronts whose parent holds every ancestor); plans with the
    tile-parallel classes forced low (the factored completion ignores the
    classes, the plain one does not, and both must agree)."""
    if name == "empty":
        pat = (0, np.zeros(1, np.int64), np.zeros(0, np.int32))
        b = mfb.SparseBarrier(pat)
        b.completion_factored(torch.zeros(1, dtype=torch.float64, device="cuda")[:0])
        assert b.status() == (0, -1)
        return
    pat = PATS[name]()
    x = V.make_x(*pat, seed=2)
    s = oracle.projinv(pat, oracle.factor(pat, x))
    fl = mfb.PLAN_WIDE_LOW if flags else 0
    b = mfb.SparseBarrier(pat, flags=fl)
    b.completion_factored(dev(s))
    assert b.status() == (0, -1)
    got = host(b.export_ldl())
    close(None, got, oracle.completion_factored(pat, s))
    a = mfb.SparseBarrier(pat, flags=fl)
    a.completion(dev(s))
    close(None, got, host(a.export_ldl()))


@pytest.mark.parametrize("name", ["fig1", "band200", "forest", "tree300", "arrow_small", "arrow_mixed", "dense528",
                                  "roots_mixed", "grid2d_24", "grid3d_8", "band300_40"])
def test_factored_inverse_hessian_matches_oracle(name, mfb):
    """mfb_inv_hessian_factored (S_AA through the R_s of the factored
    completion) against the oracle's Algorithm 5.2 at X, and against
    mfb_inv_hessian (S_AA through its cached inverse factors)."""
    pat = PATS[name]()
    print(f"[gpu-factored] inverse Hessian {name}", flush=True)
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    ts = V.make_ys(*pat, 3, seed=7)
    b = mfb.SparseBarrier(pat)
    b.completion_factored(dev(s))
    got = host(b.inv_hessian_factored(dev(ts)))
    for r in range(3):
        close(pat, got[r], oracle.inv_hessian(pat, ldl, s, ts[r]))
    # one right-hand side alone gives its bits inside the batch; the call
    # leaves R_s in place (a second call gives the same bits)
    assert np.array_equal(host(b.inv_hessian_factored(dev(ts[1]))), got[1])
    a = mfb.SparseBarrier(pat)
    a.completion(dev(s))
    plain = host(a.inv_hessian(dev(ts)))
    for r in range(3):
        close(pat, got[r], plain[r])


def test_factored_inverse_hessian_state_rules(mfb):
    """R_s must come from the last factor of the handle: refused after a
    plain factor, after a product or a plain inverse Hessian (both rewrite
    the update arena); allowed after a Hessian, which does not."""
    pat = PATS["arrow_mixed"]()
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    t = dev(V.make_ys(*pat, 1, seed=2))
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    for step in ("factor", "product", "plain", "hessian"):
        if step != "factor":
            b.completion_factored(dev(s))
        if step == "product":
            b.cholesky_product()
        elif step == "plain":
            b.inv_hessian(t)
        elif step == "hessian":
            b.hessian(t)
        if step == "hessian":
            y = host(b.inv_hessian_factored(t))
            close(pat, y[0] if y.ndim == 2 else y, oracle.inv_hessian(pat, ldl, s, host(t)[0]))
        else:
            with pytest.raises(mfb.MfbError) as e:
                b.inv_hessian_factored(t)
            assert e.value.code == mfb.ESTATE, step


def test_factored_completion_large_grid_sampled(mfb):
    """The 40^3 grid at full size: the factored completion of the gradient
    S = P(X^-1) gives the factor of X, checked against the oracle's factor
    values stored at 6712 sampled positions and its log det, and X-hat = X
    on the whole array."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "grid3d_40_samples.npz"))
    pat = get_config("grid3d_40")
    idx = g["idx"]
    x = V.make_x(*pat, seed=0)
    print("[gpu-factored] grid3d_40: factor and gradient", flush=True)
    b = mfb.SparseBarrier(pat)
    b.factor(dev(x))
    s = b.projected_inverse().clone()
    print("[gpu-factored] grid3d_40: factored completion", flush=True)
    b.completion_factored(s)
    assert b.status() == (0, -1)
    close(None, host(b.export_ldl())[idx], g["ldl"])
    ld = float(host(b.logdet())[0])
    assert abs(ld - float(g["logdet"])) / abs(float(g["logdet"])) <= TOL
    close(pat, host(b.cholesky_product()), x)


ILL = [("chordal150", 1e-2), ("chordal150", 1e-4), ("chordal150", 1e-6), ("band200", 1e-4), ("band200", 1e-6),
       ("arrow_small", 1e-6), ("arrow_mixed", 1e-5), ("grid2d_24", 1e-6)]


@pytest.mark.parametrize("name,delta", ILL)
def test_factored_paths_ill_conditioned(name, delta, mfb):
    """X = (weighted graph Laplacian) + delta I, kappa up to about 1e8, with
    the tolerances of test_gpu_parity.test_ill_conditioned: the factored
    completion (Householder row deletion) to max(1e-10, 10 kappa eps), and
    the inverse Hessian through its R_s to max(1e-10, 10 kappa^2 eps) while
    that stays below 1e-6; both against the oracle."""
    from tests.test_gpu_parity import CASES as C
    pat = C[name]()
    x = V.make_x_laplacian(*pat, delta, seed=3)
    ev = np.linalg.eigvalsh(V.to_dense(*pat, x))
    kappa = float(ev[-1] / ev[0])
    eps = np.finfo(np.float64).eps
    tol = max(TOL, 10 * kappa * eps)
    tol_ih = max(TOL, 10 * kappa ** 2 * eps)
    ldl = oracle.factor(pat, x)
    s = oracle.projinv(pat, ldl)
    b = mfb.SparseBarrier(pat)
    b.completion_factored(dev(s))
    assert b.status() == (0, -1)
    errs = {"kappa": kappa}
    errs["ldl"] = close(None, host(b.export_ldl()), oracle.completion_factored(pat, s), tol)
    if tol_ih <= 1e-6:
        t = oracle.hessian(pat, ldl, s, V.make_ys(*pat, 1, seed=4)[0])
        errs["inv_hessian"] = close(pat, host(b.inv_hessian_factored(dev(t))), oracle.inv_hessian(pat, ldl, s, t),
                                    tol_ih)
    errs["xhat"] = close(pat, host(b.cholesky_product()), x, tol)
    print(f"[gpu-factored] ill-conditioned {name} delta={delta:g}: {errs}", flush=True)
