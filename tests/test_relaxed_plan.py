"""Host-side tests of relaxed plans (mfb_plan_symbolic_opts with a zero
budget): the pattern V' they run on contains the caller's V, is filled, is cut into
dense-trapezoid supernodes that each stay within the zero budget, and has
as many supernodes as a separate bottom-up merge computed here from the
fundamental partition.  No GPU."""
import numpy as np
import pytest

from workloads import get_config, patterns as P

mfb = pytest.importorskip("paper_1203_2742_amd.mfb")

PATS = {
    "grid3d_12": lambda: get_config("grid3d_12"),
    "grid2d_48": lambda: get_config("grid2d_48"),
    "chordal300": lambda: P.random_chordal(300, 0.02, 4),
    "arrow": lambda: P.block_arrow([5, 40, 1, 33, 20], 12),
    "band60": lambda: P.band(60, 3),
}


def _cols(cp, ri, j):
    return ri[cp[j]:cp[j + 1]]


def _merge_count(pat, frac):
    """Bottom-up merge from the fundamental partition: each supernode takes
    the child with the fewest added zeros when the merged supernode's zeros
    stay within frac of its N(N+1)/2 + N A entries."""
    n, cp, ri = pat
    plan = mfb.plan_symbolic(n, cp, ri)
    snode_of, sparent, srep = mfb.plan_supernodes(plan)
    ns = len(sparent)
    N = np.bincount(snode_of, minlength=ns)
    J = np.array([cp[r + 1] - cp[r] for r in srep])
    A = J - N
    cols, zeros = N.astype(np.int64).copy(), np.zeros(ns, np.int64)
    kids = [[] for _ in range(ns)]
    for s in range(ns):
        if sparent[s] >= 0:
            kids[sparent[s]].append(s)
    merged = 0
    for s in range(ns):  # postorder numbering: children first
        best, bz = -1, 0
        for c in kids[s]:
            z = zeros[c] + zeros[s] + cols[c] * (J[s] - A[c])
            nm = cols[c] + cols[s]
            if z <= frac * (nm * (nm + 1) / 2 + nm * A[s]) and (best < 0 or z < bz):
                best, bz = c, z
        if best >= 0:
            cols[s] += cols[best]
            zeros[s] = bz
            merged += 1
    return ns - merged


@pytest.mark.parametrize("name", sorted(PATS))
@pytest.mark.parametrize("frac", [0.01, 0.05, 0.2])
def test_relaxed_pattern(name, frac):
    pat = PATS[name]()
    n, cp, ri = pat
    cp, ri = np.asarray(cp), np.asarray(ri)
    plan = mfb.plan_symbolic(n, cp, ri, relax=frac)
    info = plan.info
    cp2, ri2 = mfb.plan_pattern(plan)
    assert info["nnz"] == cp[-1] and info["nnz_relaxed"] == cp2[-1] >= cp[-1]
    # V inside V', column by column
    for j in range(n):
        assert np.isin(_cols(cp, ri, j), _cols(cp2, ri2, j)).all(), j
    # V' is filled (a plan of it builds), and every relaxed supernode is a
    # dense trapezoid of V': each member column holds the later members and
    # the ancestors of the representative's column
    mfb.plan_symbolic(n, cp2, ri2)
    snode_of, sparent, srep = mfb.plan_supernodes(plan)
    ns = info["nsuper"]
    for s in range(ns):
        mem = np.flatnonzero(snode_of == s)
        assert mem[0] == srep[s]
        rows = _cols(cp2, ri2, mem[0])
        assert np.array_equal(rows[:len(mem)], mem)
        for i, v in enumerate(mem):
            assert np.array_equal(_cols(cp2, ri2, v), rows[i:])
        anc = rows[len(mem):]
        if len(anc):  # the ancestors sit in the parent's front
            prow = _cols(cp2, ri2, srep[sparent[s]])
            assert np.isin(anc, prow).all()
        else:
            assert sparent[s] < 0
    # every supernode within the zero budget
    extra = np.zeros(ns, np.int64)
    ent = np.zeros(ns, np.int64)
    for j in range(n):
        ent[snode_of[j]] += cp2[j + 1] - cp2[j]
        extra[snode_of[j]] += (cp2[j + 1] - cp2[j]) - (cp[j + 1] - cp[j])
    assert (extra <= frac * ent + 1e-9).all()
    # the same number of supernodes as the merge computed here
    assert ns == _merge_count(pat, frac)
    # fewer supernodes and update entries than the fundamental plan
    base = mfb.plan_symbolic(n, cp, ri).info
    assert ns <= base["nsuper"] and info["update_doubles"] <= base["update_doubles"]


def test_zero_budget_gives_fundamental_plan():
    pat = get_config("grid3d_12")
    base = mfb.plan_symbolic(*pat)
    plan = mfb.plan_symbolic(*pat, relax=0.0)
    assert plan.info["nsuper"] == base.info["nsuper"]
    assert plan.info["nnz_relaxed"] == plan.info["nnz"]
    cp2, ri2 = mfb.plan_pattern(plan)
    assert np.array_equal(cp2, pat[1]) and np.array_equal(ri2, pat[2])


def test_large_grid_relaxed_statistics():
    """The 40^3 grid: 1% zeros take the update blocks from 11.95 GB to under
    1 GB (31,673 supernodes), with 0.7% more entries."""
    pat = get_config("grid3d_40")
    base = mfb.plan_symbolic(*pat).info
    info = mfb.plan_symbolic(*pat, relax=0.01).info
    assert info["nsuper"] == 31673
    assert info["update_doubles"] * 8 < 1e9 < base["update_doubles"] * 8
    assert info["nnz_relaxed"] < 1.01 * info["nnz"]
    assert info["nlevels_up"] <= base["nlevels_up"]


@pytest.mark.parametrize("frac", [1.0, 1.5, float("nan")])
def test_relaxed_rejects_bad_budget(frac):
    with pytest.raises(mfb.MfbError) as e:
        mfb.plan_symbolic(*P.band(10, 2), relax=frac)
    assert e.value.code == mfb.EINVAL


def test_plan_options_thresholds():
    """A negative budget is the fundamental partition; the front thresholds
    move fronts between kernel classes without changing the plan's
    structure; thresholds below their minimum are refused."""
    pat = get_config("grid3d_12")
    base = mfb.plan_symbolic(*pat).info
    for kw in ({"relax": -1.0}, {"wide_j": 64}, {"big_a": 192}, {"wide_j": 512, "big_a": 1024}):
        info = mfb.plan_symbolic(*pat, **kw).info
        for key in ("nsuper", "nnz", "nnz_relaxed", "update_doubles", "max_front", "flops_hessian"):
            assert info[key] == base[key], (kw, key)
    for kw in ({"wide_j": 63}, {"big_a": 191}, {"wide_j": -5}):
        with pytest.raises(mfb.MfbError) as e:
            mfb.plan_symbolic(*pat, **kw)
        assert e.value.code == mfb.EINVAL


def test_relaxed_rejects_unfilled_pattern():
    # column 0 -> {1, 2}, column 1 -> {1} only: (2, 1) is missing
    cp = np.array([0, 3, 4, 5], np.int64)
    ri = np.array([0, 1, 2, 1, 2], np.int32)
    with pytest.raises(mfb.MfbError) as e:
        mfb.plan_symbolic(3, cp, ri, relax=0.1)
    assert e.value.code == mfb.ENOTCHORDAL


@pytest.mark.parametrize("pat", [(0, np.zeros(1, np.int64), np.zeros(0, np.int32)), P.band(12, 11), P.band(9, 0)],
                         ids=["empty", "dense", "diagonal"])
def test_relaxed_degenerate_patterns(pat):
    """No supernode, one dense supernode (nothing to merge) and a diagonal
    (roots only, nothing to merge) give the fundamental plan."""
    n = pat[0]
    base = mfb.plan_symbolic(*pat).info
    info = mfb.plan_symbolic(*pat, relax=0.5).info
    assert info["nsuper"] == base["nsuper"] and info["nnz_relaxed"] == info["nnz"] == int(pat[1][-1])
    cp2, ri2 = mfb.plan_pattern(mfb.plan_symbolic(*pat, relax=0.5))
    assert np.array_equal(cp2, np.asarray(pat[1])) and np.array_equal(ri2, np.asarray(pat[2]))
    assert n >= 0
