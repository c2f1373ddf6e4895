"""Cost matrices for the oracle (float64).

* ``sq_euclidean``: ``C_IJ = sum_d (x_Id - y_Jd)^2`` -- the Euclidean-type cost of Example 2
  (urban planning) squared, as used by every point-cloud workload.
* Block structure (Assumption 1, Eq. blkstr_cost): block ``(r, c)`` of the full ``n x n`` cost
  is ``C_{(c - r) mod K}``; block-row 0 ``[m, n]`` holds every ``C_k`` side by side:
  ``C_row0[i, k*m + j] = C_k[i, j]``.

Pins: ``block_circulant_from_row0`` is pinned by the shift-invariance identity of Lemma 1's
proof (``P^l C P^l^T = C`` with the block permutation ``P``) and by comparison with
``sq_euclidean`` on exactly rotated clouds; ``median`` by the K-copies identity.
"""
from __future__ import annotations

import numpy as np


def sq_euclidean(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Full squared Euclidean cost matrix ``[len(x), len(y)]`` in float64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = np.zeros((x.shape[0], y.shape[0]))
    for d in range(x.shape[1]):
        C += (x[:, None, d] - y[None, :, d]) ** 2
    return C


def row0_from_points(x: np.ndarray, y: np.ndarray, K: int) -> np.ndarray:
    """Block-row 0 of the cost: the first m points of x against all n points of y."""
    n = np.asarray(y).shape[0]
    m = n // K
    return sq_euclidean(np.asarray(x)[:m], y)


def blocks_from_row0(C_row0: np.ndarray, K: int) -> np.ndarray:
    """``[K, m, m]`` stack of the cost blocks ``C_k`` read from block-row 0."""
    C_row0 = np.asarray(C_row0, dtype=np.float64)
    m = C_row0.shape[0]
    return np.stack([C_row0[:, k * m:(k + 1) * m] for k in range(K)])


def block_circulant_from_blocks(Ck: np.ndarray) -> np.ndarray:
    """Full ``n x n`` block-circulant matrix with block ``(r, c) = C_{(c - r) mod K}``."""
    K, m, _ = Ck.shape
    n = K * m
    C = np.empty((n, n))
    for r in range(K):
        for c in range(K):
            C[r * m:(r + 1) * m, c * m:(c + 1) * m] = Ck[(c - r) % K]
    return C


def block_circulant_from_row0(C_row0: np.ndarray, K: int) -> np.ndarray:
    """The "symmetric by definition" full cost built from block-row 0."""
    return block_circulant_from_blocks(blocks_from_row0(C_row0, K))


def block_shift_permutation(K: int, m: int) -> np.ndarray:
    """The block-circulant permutation matrix ``P`` of Lemma 1's proof (identity blocks on the
    sub-diagonal and in the top-right corner)."""
    n = K * m
    P = np.zeros((n, n))
    for r in range(K):
        c = (r - 1) % K
        P[r * m:(r + 1) * m, c * m:(c + 1) * m] = np.eye(m)
    return P


def median(C: np.ndarray) -> float:
    return float(np.median(np.asarray(C, dtype=np.float64)))
