"""Seeded values on a pattern (input generation only).

Recipe (fixed so that every consumer sees identical inputs):

* ``make_x``: the strict-lower entries of V, in CCS order, are drawn
  uniform(-1, 1) from ``numpy.random.default_rng(seed)``; each diagonal entry
  is then the sum of the absolute values of the off-diagonal entries of its
  full symmetric row, plus one.  X is strictly diagonally dominant with a
  positive diagonal, hence positive definite.
* ``make_y(r)``: every entry of V, diagonal included, is drawn
  uniform(-1, 1) from ``default_rng([seed, r + 1])``.
* ``make_x_laplacian(delta)``: an ill-conditioned X.  The strict-lower
  entries are minus the absolute values of uniform(-1, 1) draws from
  ``default_rng(seed)`` (CCS order); each diagonal entry is the absolute
  row sum of its full symmetric row plus ``delta``.  X is then a weighted
  graph Laplacian plus delta I: positive definite, with its smallest
  eigenvalue delta on a connected pattern and condition number about
  (largest eigenvalue) / delta.

Values are returned in the CCS order of the pattern (lower triangle,
diagonal first in each column) as float64 arrays.
"""
from __future__ import annotations

import numpy as np


def column_index(n, colptr):
    """Column of every stored entry (int64, length nnz)."""
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))


def diag_positions(colptr):
    return np.asarray(colptr[:-1], dtype=np.int64)


def make_x(n, colptr, rowind, seed: int = 0) -> np.ndarray:
    nnz = int(colptr[-1])
    col = column_index(n, colptr)
    row = np.asarray(rowind, dtype=np.int64)
    strict = row != col
    x = np.zeros(nnz, dtype=np.float64)
    x[strict] = np.random.default_rng(seed).uniform(-1.0, 1.0, int(strict.sum()))
    a = np.abs(x)
    rowsum = np.zeros(n, dtype=np.float64)
    np.add.at(rowsum, row[strict], a[strict])
    np.add.at(rowsum, col[strict], a[strict])
    x[diag_positions(colptr)] = rowsum + 1.0
    return x


def make_x_laplacian(n, colptr, rowind, delta: float, seed: int = 0) -> np.ndarray:
    nnz = int(colptr[-1])
    col = column_index(n, colptr)
    row = np.asarray(rowind, dtype=np.int64)
    strict = row != col
    x = np.zeros(nnz, dtype=np.float64)
    x[strict] = -np.abs(np.random.default_rng(seed).uniform(-1.0, 1.0, int(strict.sum())))
    rowsum = np.zeros(n, dtype=np.float64)
    np.add.at(rowsum, row[strict], -x[strict])
    np.add.at(rowsum, col[strict], -x[strict])
    x[diag_positions(colptr)] = rowsum + float(delta)
    return x


def make_y(n, colptr, rowind, seed: int = 0, r: int = 0) -> np.ndarray:
    nnz = int(colptr[-1])
    return np.random.default_rng([seed, r + 1]).uniform(-1.0, 1.0, nnz)


def make_ys(n, colptr, rowind, k: int, seed: int = 0) -> np.ndarray:
    """k right-hand sides, shape (k, nnz), row r = make_y(r)."""
    return np.stack([make_y(n, colptr, rowind, seed, r) for r in range(k)]) if k else \
        np.zeros((0, int(colptr[-1])))


def make_spd_dense(n: int, seed: int) -> np.ndarray:
    """Dense SPD matrix (for completion tests: S = P(Z) has a PD completion)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    return g @ g.T / n + np.eye(n)


def project(n, colptr, rowind, dense: np.ndarray) -> np.ndarray:
    """Values of a dense symmetric matrix at the CCS positions of V."""
    col = column_index(n, colptr)
    return np.asarray(dense[np.asarray(rowind, dtype=np.int64), col], dtype=np.float64)


def to_dense(n, colptr, rowind, vals) -> np.ndarray:
    """Dense symmetric matrix from CCS lower-triangle values."""
    col = column_index(n, colptr)
    row = np.asarray(rowind, dtype=np.int64)
    d = np.zeros((n, n), dtype=np.float64)
    d[row, col] = vals
    d[col, row] = vals
    return d
