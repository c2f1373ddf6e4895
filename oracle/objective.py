"""Objective values of entropy-regularised OT (oracle; test infrastructure only).

* primal (eq. problem_ROT with the entropic regulariser eq. reg_for_entropy_ROT):
  ``P(T) = <C, T> + eps * sum T (log T - 1)``.  For a plan given by potentials,
  ``T = exp(Z)`` with ``Z = (f_I + g_J - C_IJ) / eps`` and ``log T = Z`` exactly, so
  ``P = sum T * (C + eps (Z - 1))`` -- never evaluated through ``log T`` (no 0 log 0).
* dual (eq. dual_problem_cyclic_ROT with ``phi*(y) = eps exp(y / eps)``):
  ``D = <f, a> + <g, b> - eps * sum exp(Z)``.
* reduced problem (eq. problem_CROT): the same sums over ``(i, j, k)`` with alpha, beta; its
  value is exactly 1/K of the full one.

Pins: strong duality at convergence (Thm. 2's proof), the eps -> 0 bracket around the LP value,
and ``P_full = K * P_red``.
"""
from __future__ import annotations

import numpy as np


def primal_of_plan(T, C, eps):
    """``<C, T> + eps * sum T (log T - 1)`` for an arbitrary nonnegative plan (0 log 0 = 0)."""
    T = np.asarray(T, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    pos = T > 0
    ent = np.zeros_like(T)
    ent[pos] = T[pos] * (np.log(T[pos]) - 1.0)
    return float((C * T).sum() + eps * ent.sum())


def full_values(f, g, C, eps, a, b):
    """Dict with primal P, dual D, transport cost <C,T>, total mass and L2 marginal errors of
    the plan given by full potentials."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    Z = (f[:, None] + g[None, :] - C) / eps
    T = np.exp(Z)
    P = float((T * (C + eps * (Z - 1.0))).sum())
    D = float(f @ np.asarray(a, dtype=np.float64) + g @ np.asarray(b, dtype=np.float64)
              - eps * T.sum())
    return {"P": P, "D": D, "CT": float((C * T).sum()), "mass": float(T.sum()),
            "err_row": float(np.linalg.norm(T.sum(axis=1) - a)),
            "err_col": float(np.linalg.norm(T.sum(axis=0) - b))}


def reduced_values(f, g, Ck, eps, alpha, beta):
    """Values of the reduced problem (eq. problem_CROT) and its dual; multiply by K for the
    full problem."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    Ck = np.asarray(Ck, dtype=np.float64)
    Z = (f[None, :, None] + g[None, None, :] - Ck) / eps
    T = np.exp(Z)
    P = float((T * (Ck + eps * (Z - 1.0))).sum())
    D = float(f @ np.asarray(alpha) + g @ np.asarray(beta) - eps * T.sum())
    return {"P": P, "D": D, "CT": float((Ck * T).sum()), "mass": float(T.sum())}
