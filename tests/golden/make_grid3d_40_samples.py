"""Writes grid3d_40_samples.npz: oracle values of the 40^3 grid workload at
sampled CCS positions (the oracle needs about half an hour for the full
arrays, too long for a test run).

    python tests/golden/make_grid3d_40_samples.py

Inputs: X = make_x(seed 0) and Y_r = make_y(seed 0, r) for r = 0, 1 on the
filled 3D 7-point grid 40^3 under nested dissection.  Outputs, at the
sampled positions: the scalar factor (D on the diagonal slots, L below),
S = P(X^-1), T_r = P(X^-1 Y_r X^-1); and the scalars log det X and S.X.
Only the oracle computes values here.
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import get_config, values as V  # noqa: E402

OUT = os.path.join(HERE, "grid3d_40_samples.npz")
NAME = "grid3d_40"


def sample_positions(pat):
    """Seeded uniform positions, every entry of the longest column, and the
    diagonal slots of the last 256 columns (the top of the tree)."""
    n, cp, ri = pat
    nnz = int(cp[-1])
    rng = np.random.default_rng(20260)
    pos = set(rng.choice(nnz, 4096, replace=False).tolist())
    lens = np.diff(cp)
    j = int(np.argmax(lens))
    pos.update(range(int(cp[j]), int(cp[j + 1])))
    pos.update(int(cp[c]) for c in range(n - 256, n))
    return np.array(sorted(pos), dtype=np.int64)


def _hess(args):
    r, ldl, s = args
    pat = get_config(NAME)
    return oracle.hessian(pat, ldl, s, V.make_y(*pat, seed=0, r=r))


def main():
    pat = get_config(NAME)
    n, cp, ri = pat
    idx = sample_positions(pat)
    x = V.make_x(*pat, seed=0)
    ldl = oracle.factor(pat, x)
    print("factor done", flush=True)
    ld = oracle.logdet(pat, ldl)
    s = oracle.projinv(pat, ldl)
    print("projected inverse done", flush=True)
    w = np.where(np.asarray(ri) == V.column_index(n, cp), 1.0, 2.0)
    sx = float(np.sum(w * s * x))
    with Pool(2) as pool:
        ts = pool.map(_hess, [(0, ldl, s), (1, ldl, s)])
    print("hessians done", flush=True)
    np.savez_compressed(OUT, idx=idx, ldl=ldl[idx], s=s[idx], t0=ts[0][idx], t1=ts[1][idx],
                        logdet=np.float64(ld), sx=np.float64(sx), nnz=np.int64(cp[-1]))
    print("wrote", OUT, len(idx), "positions", flush=True)


if __name__ == "__main__":
    main()
