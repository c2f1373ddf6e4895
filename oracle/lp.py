"""Brute-force linear programs (oracle; test infrastructure only).

* ``lot_value``: the linear OT problem (eq. problem_ROT with the indicator regulariser of eq.
  reg_for_original_OT) solved as a dense LP with SciPy's HiGHS.  Used for the eps -> 0
  bracket of the entropic value: with H(T) <= 2 log n on the transport polytope,
  ``LP - eps - 2 eps log n <= P_eps <= LP - eps`` and ``LP <= <C, T_eps> <= LP + 2 eps log n``.
* ``small_lot_value``: Thm. 1 -- the cyclic LOT equals K times a small LOT on
  ``G_ij = min_k C_ijk`` (eq. definition_G) with marginals alpha, beta.
* ``min_fold``: G and the smallest minimising k (eq. definition_G and the tie rule stated with
  Thm. 1).
* ``lot_plan``: the full plan of Thm. 1 (eq. optimal_solution_problem_CLOT) placed in the
  block-circulant layout of Lemma 1, written out block by block.  Pinned by the brute-force LP:
  the plan is feasible and its cost equals the full problem's optimum.

These solve tiny problems only (n <= 40).  Parity unpinned by themselves: they are the pins.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog


def lot_value(a, b, C):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    n1, n2 = C.shape
    A_eq = []
    for i in range(n1):
        row = np.zeros((n1, n2))
        row[i, :] = 1.0
        A_eq.append(row.ravel())
    for j in range(n2):
        col = np.zeros((n1, n2))
        col[:, j] = 1.0
        A_eq.append(col.ravel())
    b_eq = np.concatenate([a, b])
    # one constraint is redundant when the masses agree; drop the last column constraint
    res = linprog(C.ravel(), A_eq=np.array(A_eq[:-1]), b_eq=b_eq[:-1],
                  bounds=(0, None), method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return float(res.fun), res.x.reshape(n1, n2)


def min_fold(Ck):
    """``G_ij = min_k C_ijk`` and the smallest k attaining it (``[m, m]`` each)."""
    Ck = np.asarray(Ck, dtype=np.float64)
    return Ck.min(axis=0), Ck.argmin(axis=0)  # argmin returns the first of equal minima


def small_lot_value(alpha, beta, Ck):
    """Thm. 1: value of the small LOT on ``G = min_k C_k`` (returns value, S, argmin k)."""
    G, kstar = min_fold(Ck)
    val, S = lot_value(alpha, beta, G)
    return val, S, kstar


def lot_plan(S, kstar, K):
    """Full ``n x n`` plan: block (r, c) holds ``S_ij`` where ``kstar_ij == (c - r) mod K``
    and 0 elsewhere."""
    S = np.asarray(S, dtype=np.float64)
    m = S.shape[0]
    T = np.zeros((K * m, K * m))
    for r in range(K):
        for c in range(K):
            k = (c - r) % K
            T[r * m:(r + 1) * m, c * m:(c + 1) * m] = np.where(kstar == k, S, 0.0)
    return T
