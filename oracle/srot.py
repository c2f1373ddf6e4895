"""Cyclic strongly convex-regularised OT with a quadratic regulariser (oracle; test
infrastructure only: imported by the tests alone).

The regulariser is phi(x) = (lam / 2) x^2 for x >= 0 and +inf otherwise (strongly convex;
the paper treats a general strongly convex phi, this is the instance built here).  Its
conjugate is phi*(y) = max(0, y)^2 / (2 lam), so (phi*)'(y) = max(0, y) / lam.

* Thm. 2 (eq. dual_problem_cyclic_ROT): maximise over w, z in R^m
      <w, alpha> + <z, beta> - sum_{k,i,j} phi*(w_i + z_j - C_ijk);
  the plan is T_ijk = (phi*)'(w_i + z_j - C_ijk) (eq. optimality_condition).
* Alternating maximisation (the algorithm of the C-SROT section): with z fixed, w_i is the
  root of eq. derivative_of_objective_function, alpha_i - sum_{k,j} max(0, w_i + z_j - C_ijk)
  / lam = 0 -- solved here exactly by sorting ("water filling": the sum is piecewise linear
  in w_i); then z likewise with w fixed.  Start from z = 0, w first.
* The full n x n problem is the same with K = 1 and the full cost.

Pins (tests/test_oracle_pins.py): the cyclic iterates equal the full problem's tiled at every
iteration; the water-filling root against bisection; at convergence both marginals hold and
the primal value equals the dual value; the dual optimum equals that of an independent
L-BFGS maximisation of the concave dual; the expanded plan solves the full primal QP (SLSQP).
"""
from __future__ import annotations

import numpy as np


def waterfill(v, t, lam):
    """The w with sum_k max(0, w - v_k) = lam * t (t > 0): the sum is 0 below min v and
    increases with slope p between the p-th and (p+1)-th smallest v."""
    vs = np.sort(np.asarray(v, dtype=np.float64).ravel())
    cs = np.cumsum(vs)
    target = lam * float(t)
    for p in range(1, vs.size + 1):
        w = (target + cs[p - 1]) / p
        if p == vs.size or w <= vs[p]:
            return w
    raise AssertionError("unreachable")


def plan_blocks(w, z, Ck, lam):
    """T_ijk = max(0, w_i + z_j - C_ijk) / lam, ``[K, m, m]``."""
    return np.maximum(0.0, w[None, :, None] + z[None, None, :] - Ck) / lam


def cyclic_srot(alpha, beta, Ck, lam, K, tol=1e-10, max_iter=10000, record=None):
    """Alternating maximisation on the reduced dual.  Stops when the full-space row residual
    sqrt(K) ||T 1 - alpha|| of the state after an iteration is <= tol (the column marginal is
    exact after the z-step).  Returns dict(w, z, iters, err)."""
    Ck = np.asarray(Ck, dtype=np.float64)
    m = Ck.shape[1]
    w = np.zeros(m)
    z = np.zeros(m)
    err = np.inf
    it = 0
    while it < max_iter:
        it += 1
        for i in range(m):
            w[i] = waterfill(Ck[:, i, :] - z[None, :], alpha[i], lam)
        for j in range(m):
            z[j] = waterfill(Ck[:, :, j] - w[None, :], beta[j], lam)
        if record is not None:
            record.append((w.copy(), z.copy()))
        r = plan_blocks(w, z, Ck, lam).sum(axis=(0, 2)) - alpha
        err = np.sqrt(K) * np.linalg.norm(r)
        if tol > 0 and err <= tol:
            break
    return {"w": w, "z": z, "iters": it, "err": err}


def values(w, z, Ck, lam, alpha, beta):
    """Primal <C,T> + sum phi(T) and dual of the reduced problem (multiply by K for the full
    problem, eq. problem_CROT)."""
    T = plan_blocks(w, z, Ck, lam)
    primal = float((Ck * T).sum() + 0.5 * lam * (T * T).sum())
    y = np.maximum(0.0, w[None, :, None] + z[None, None, :] - Ck)
    dual = float(w @ alpha + z @ beta - (y * y).sum() / (2.0 * lam))
    return {"primal": primal, "dual": dual, "row": T.sum(axis=(0, 2)), "col": T.sum(axis=(0, 1))}
