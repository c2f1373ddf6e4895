"""Brute-force linear programs (oracle; test infrastructure only).

* ``lot_value``: the linear OT problem (eq. problem_ROT with the indicator regulariser of eq.
  reg_for_original_OT) solved as a dense LP with SciPy's HiGHS.  Used for the eps -> 0
  bracket of the entropic value: with H(T) <= 2 log n on the transport polytope,
  ``LP - eps - 2 eps log n <= P_eps <= LP - eps`` and ``LP <= <C, T_eps> <= LP + 2 eps log n``.
* ``small_lot_value``: Thm. 1 -- the cyclic LOT equals K times a small LOT on
  ``G_ij = min_k C_ijk`` (eq. definition_G) with marginals alpha, beta.

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


def small_lot_value(alpha, beta, Ck):
    """Thm. 1: value of the small LOT on ``G = min_k C_k`` (returns value, S, argmin k)."""
    Ck = np.asarray(Ck, dtype=np.float64)
    G = Ck.min(axis=0)
    kstar = Ck.argmin(axis=0)  # smallest k among ties, as the theorem prescribes
    val, S = lot_value(alpha, beta, G)
    return val, S, kstar
