"""Block-circulant projection of a cost matrix (oracle; test infrastructure only).

For data that is only approximately K-fold symmetric, the reduced method needs cost blocks
``C_k``.  The paper averages the marginals over the K blocks (Alg. 3, stage 1) because its costs
are exactly symmetric; for the cost we use the analogous average over the K block-rows,
``C_k[i, j] = (1/K) sum_r C[r m + i, ((r + k) mod K) m + j]``, which is the same group average
that Lemma 1's proof applies to a plan: ``(1/K) sum_l P^l C (P^l)^T`` (a reading, listed in the
design notes).

Pins: equality with the permutation-matrix average of Lemma 1's proof (a different
computation), idempotence, and exactness on block-circulant input.  The size of the resulting
objective gap on jittered data is a reported number only: parity unpinned.
"""
from __future__ import annotations

import numpy as np

from . import cost as _cost


def project_blocks(C, K):
    """``[K, m, m]`` averaged blocks of an arbitrary ``n x n`` cost."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    m = n // K
    out = np.zeros((K, m, m))
    for k in range(K):
        for r in range(K):
            c = (r + k) % K
            out[k] += C[r * m:(r + 1) * m, c * m:(c + 1) * m]
    return out / K


def group_average(C, K):
    """``(1/K) sum_l P^l C (P^l)^T`` with the block permutation P of Lemma 1's proof."""
    C = np.asarray(C, dtype=np.float64)
    m = C.shape[0] // K
    P = _cost.block_shift_permutation(K, m)
    acc = np.zeros_like(C)
    Pl = np.eye(C.shape[0])
    for _ in range(K):
        acc += Pl @ C @ Pl.T
        Pl = P @ Pl
    return acc / K


def project_rows_from_points(x, y, K, rows):
    """Rows ``rows`` (block-row-0 indices i in [0, m)) of the projected cost, as block-row 0:
    entry ``(i, k m + j) = (1/K) sum_r |x_{r m + i} - y_{((r + k) mod K) m + j}|^2``.  The same
    average as ``project_blocks`` without forming the n x n cost; shape ``[len(rows), n]``."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    m = n // K
    out = np.empty((len(rows), n))
    for t, i in enumerate(rows):
        Ci = _cost.sq_euclidean(x[i::m][:K], y).reshape(K, K, m)   # [r, block c, j]
        for k in range(K):
            out[t, k * m:(k + 1) * m] = np.mean([Ci[r, (r + k) % K] for r in range(K)], axis=0)
    return out
