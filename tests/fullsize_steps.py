"""Float64 checks of large full-size solves on sampled rows and columns (test helpers).

A full-size problem at n = 8192 or 16384 is too large for the float64 oracle to iterate in a
test's time, but every half-step can be checked exactly where it is sampled: the returned row
potential at row I must be the oracle's row update (``sinkhorn.row_update``) of the previous
column potential over all n columns, and the returned column potential at column J the
oracle's column update (``sinkhorn.col_update``) of the returned row potential over all n
rows.  Costs are the problem's as given: squared distances of the float32 coordinates
evaluated in float64, or the dense float32 cost.
"""
from __future__ import annotations

import numpy as np

from oracle import cost, sinkhorn


class FullData:
    """Coordinates (x, y) or a dense [n, n] cost, with the marginals, in float64 views."""

    def __init__(self, a, b, eps, x=None, y=None, C=None):
        self.a = np.asarray(a, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.eps = float(eps)
        self.x = None if x is None else np.asarray(x, dtype=np.float64)
        self.y = None if y is None else np.asarray(y, dtype=np.float64)
        self.C = C  # float32 [n, n] or None
        self.n = self.a.shape[0]

    def rows(self, I):
        if self.C is None:
            return cost.sq_euclidean(self.x[I], self.y)
        return self.C[I].astype(np.float64)

    def cols(self, J):
        if self.C is None:
            return cost.sq_euclidean(self.x, self.y[J])
        return self.C[:, J].astype(np.float64)


def block_circulant_f32(C_row0, K):
    """The full float32 cost whose block-row r is block-row 0 rotated by r blocks, so that
    block (r, c) is C_{(c - r) mod K} (built row-block by row-block, no float64 copy)."""
    m, n = C_row0.shape
    C = np.empty((n, n), dtype=np.float32)
    for r in range(K):
        C[r * m:(r + 1) * m] = np.roll(C_row0, r * m, axis=1)
    return C


def sample(n, count, seed, boundaries=()):
    """`count` distinct indices below n plus the given boundary indices (clipped, unique)."""
    rng = np.random.default_rng(seed)
    idx = set(int(v) for v in rng.choice(n, size=min(count, n), replace=False))
    idx.update(int(v) for v in boundaries if 0 <= v < n)
    return np.array(sorted(idx))


def one_step_errors(data, g_prev, f, g, I, J):
    """max |f_I - row_update(g_prev)_I| / eps over I and max |g_J - col_update(f)_J| / eps over
    J, both in float64 against every partner."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    g_prev = np.asarray(g_prev, dtype=np.float64)
    f_ref = sinkhorn.row_update(g_prev, data.rows(I), data.a[I], data.eps)
    g_ref = sinkhorn.col_update(f, data.cols(J), data.b[J], data.eps)
    return (float(np.abs(f[I] - f_ref).max() / data.eps),
            float(np.abs(g[J] - g_ref).max() / data.eps))


def row_residual(data, f, g, chunk=512):
    """The full-space float64 row-marginal residual ||T 1 - a||_2 over all rows."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    sq = 0.0
    for s in range(0, data.n, chunk):
        I = np.arange(s, min(s + chunk, data.n))
        T = np.exp((f[I, None] + g[None, :] - data.rows(I)) / data.eps)
        sq += float(((T.sum(axis=1) - data.a[I]) ** 2).sum())
    return float(np.sqrt(sq))
