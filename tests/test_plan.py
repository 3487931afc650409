"""Host-side tests of the C ABI: symbolic plan against the paper's worked
example, error paths, and the exported symbol set.  No GPU needed."""
import ctypes
import subprocess

import numpy as np
import pytest

from tests.golden import load_fig1
from workloads import get_config, patterns as P

mfb = pytest.importorskip("paper_1203_2742_amd.mfb")


def _partition(plan):
    snode_of, sparent, srep = mfb.plan_supernodes(plan)
    n = plan.n
    groups = {}
    for v in range(n):
        groups.setdefault(int(snode_of[v]), []).append(v + 1)
    out = {}
    for s, members in groups.items():
        rep = int(srep[s]) + 1
        par = int(sparent[s])
        out[rep] = (members, int(srep[par]) + 1 if par >= 0 else 0)
    return out


@pytest.mark.parametrize("part,flags", [(2, 0), (1, 1)])
def test_worked_example_partitions(part, flags):
    """Supernodes N_k, first-ancestor sets and clique-tree parents of
    Table t-example / Figure f-etree2.  The lowest-label tie-break at vertex 16
    (eligible children 14 and 15) gives the right-hand partition, the
    highest-label one the left-hand partition."""
    g = load_fig1()
    n, cp, ri = g["pattern"]
    plan = mfb.plan_symbolic(n, cp, ri, flags)
    got = _partition(plan)
    want = {rep: (nset, par) for rep, nset, aset, par in g["snodes"][part]}
    assert sorted(got) == sorted(want) == g["representatives"]
    for rep, (nset, par) in want.items():
        assert got[rep][0] == nset, rep
        assert got[rep][1] == par, rep
    # A_k = J_rep \ N_k  (column rep of the filled pattern)
    for rep, nset, aset, _ in g["snodes"][part]:
        rows = [int(r) + 1 for r in ri[cp[rep - 1]:cp[rep]]]
        assert [r for r in rows if r not in nset] == aset
    info = plan.info
    assert info["nsuper"] == 9 and info["n"] == 17 and info["nnz"] == 17 + len(g["entries"])


def test_unfilled_pattern_rejected():
    g = load_fig1()
    n, cp, ri = g["pattern"]
    col = 4  # drop (15, 5), implied by (5, 3) and (15, 3)
    rows = list(ri[cp[col]:cp[col + 1]])
    rows.remove(14)
    ri2 = np.concatenate([ri[:cp[col]], np.array(rows, np.int32), ri[cp[col + 1]:]])
    cp2 = cp.copy()
    cp2[col + 1:] -= 1
    with pytest.raises(mfb.MfbError) as e:
        mfb.plan_symbolic(n, cp2, ri2)
    assert e.value.code == mfb.ENOTCHORDAL


@pytest.mark.parametrize("mutate", ["unsorted", "no_diag", "row_oob", "colptr0"])
def test_malformed_ccs_rejected(mutate):
    n, cp, ri = P.band(10, 2)
    cp = cp.copy()
    ri = ri.copy()
    if mutate == "unsorted":
        ri[cp[3] + 1], ri[cp[3] + 2] = ri[cp[3] + 2], ri[cp[3] + 1]
    elif mutate == "no_diag":
        ri[cp[2]] = 3
    elif mutate == "row_oob":
        ri[cp[8] + 1] = 10
    else:
        cp = cp + 1
    with pytest.raises(mfb.MfbError) as e:
        mfb.plan_symbolic(n, cp, ri)
    assert e.value.code == mfb.EINVAL


@pytest.mark.parametrize("name,nsuper,levels,maxfront", [
    ("band200", 195, 195, 6),
    ("grid2d_128", 10334, 26, 191),
    ("arrow64", 64, 2, 384),
    ("grid3d_40", 42165, 298, 2360),
])
def test_workload_plans(name, nsuper, levels, maxfront):
    plan = mfb.plan_symbolic(*get_config(name))
    info = plan.info
    assert info["nsuper"] == nsuper
    assert info["nlevels_up"] == levels
    assert info["max_front"] == maxfront
    assert info["factor_workspace_bytes"] > 0 and info["rhs_arena_bytes"] > 0


def test_large_grid_plan_statistics():
    """The 3D 7-point grid 40^3 under nested dissection: order, entries, the
    root front (1601 columns, no ancestors) and the largest front."""
    n, cp, ri = get_config("grid3d_40")
    plan = mfb.plan_symbolic(n, cp, ri)
    info = plan.info
    assert (info["n"], info["nnz"]) == (64000, 21288984)
    assert info["max_ncols"] == 1601 and info["max_nanc"] == 2320
    snode_of, sparent, srep = mfb.plan_supernodes(plan)
    roots = np.flatnonzero(sparent < 0)
    assert len(roots) == 1
    root = int(roots[0])
    assert int((snode_of == root).sum()) == 1601
    assert int(cp[srep[root] + 1] - cp[srep[root]]) == 1601


def test_forest_and_diagonal_plans():
    plan = mfb.plan_symbolic(*P.band(7, 0))
    assert plan.info["nsuper"] == 7 and plan.info["nlevels_up"] == 1
    pat = P.random_chordal(40, 0.03, 5)
    plan = mfb.plan_symbolic(*pat)
    _, sparent, _ = mfb.plan_supernodes(plan)
    assert (sparent < 0).sum() >= 2  # several roots
    empty = mfb.plan_symbolic(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert empty.info["nsuper"] == 0


def test_library_exports_every_header_symbol():
    names = mfb.header_symbols()
    assert len(names) == 31
    lib = ctypes.CDLL(mfb.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", mfb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_strerror_and_numeric_entry_points_reject_null():
    assert mfb.strerror(mfb.ENOTCHORDAL).startswith("pattern")
    lib = mfb._lib
    assert lib.mfb_factor(None, None, None) == mfb.EINVAL
    assert lib.mfb_hessian(None, 1, None, None, None, 0, None) == mfb.EINVAL
    assert lib.mfb_get_status(None, None) == mfb.EINVAL
    plan = mfb.plan_symbolic(*P.band(5, 1))
    h = ctypes.c_void_p()
    assert lib.mfb_factor_create(plan.handle, None, 0, ctypes.byref(h)) == mfb.EINVAL


def test_plan_info_canonical_bytes():
    """The plan's canonical byte counts are the per-supernode sums of panel
    entries p = N J - N(N-1)/2 and packed update entries u = A(A+1)/2."""
    pat = P.random_chordal(120, 0.04, 3)
    n, cp, ri = pat
    plan = mfb.plan_symbolic(*pat)
    snode_of, _, srep = mfb.plan_supernodes(plan)
    ns = plan.info["nsuper"]
    Ns = np.bincount(snode_of, minlength=ns).astype(float)
    Js = np.array([cp[r + 1] - cp[r] for r in srep], dtype=float)
    As = Js - Ns
    pe = (Ns * Js - Ns * (Ns - 1) / 2).sum()
    ue = (As * (As + 1) / 2).sum()
    info = plan.info
    assert pe == cp[-1]  # the panels tile the pattern
    assert info["bytes_factor"] == 8 * (2 * pe + 2 * ue)
    assert info["bytes_projinv"] == 8 * (2 * pe + 2 * ue)
    assert info["bytes_hessian"] == 8 * (6 * pe + 5 * ue)
    assert info["bytes_inv_hessian"] == 8 * (7 * pe + 7 * ue)
    assert info["bytes_completion"] == 8 * (4 * pe + 5 * ue)
    assert info["bytes_product"] == 8 * (2 * pe + 2 * ue)
