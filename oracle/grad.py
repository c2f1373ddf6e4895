"""Gradients of the entropic OT value (oracle; test infrastructure only).

The paper does not differentiate the OT value; the formulas below are the envelope theorem
applied to the dual of eq. problem_ROT (Thm. 2 with ``phi*(y) = eps exp(y/eps)``):
``OT(a, b, C) = max_{f,g} <f,a> + <g,b> - eps sum exp((f_I + g_J - C_IJ)/eps)``, hence at the
optimum

* ``dOT/dC_IJ = T_IJ``;
* ``dOT/da = f`` and ``dOT/db = g`` up to a common constant (a and b live on the simplex, so
  only differences along ``e_I - e_J`` are defined); returned mean-centred;
* for the squared Euclidean cost, ``dOT/dx_I = 2 sum_J T_IJ (x_I - y_J)`` and
  ``dOT/dy_J = 2 sum_I T_IJ (y_J - x_I)``.

Pins: central finite differences of the converged oracle value (``fd_*``), which use nothing
but ``sinkhorn.full_sinkhorn`` and ``objective.full_values``.
"""
from __future__ import annotations

import numpy as np

from . import cost as _cost
from . import objective as _obj
from . import sinkhorn as _sk


def envelope_grads(f, g, x, y, eps):
    """Gradients of the full problem with squared Euclidean cost from converged full
    potentials (length n).  Returns dict dC, da, db, dx, dy."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = _cost.sq_euclidean(x, y)
    T = np.exp((f[:, None] + g[None, :] - C) / eps)
    dx = 2.0 * (T.sum(axis=1)[:, None] * x - T @ y)
    dy = 2.0 * (T.sum(axis=0)[:, None] * y - T.T @ x)
    return {"dC": T, "da": f - f.mean(), "db": g - g.mean(), "dx": dx, "dy": dy}


def solve_value(x, y, a, b, eps, tol=1e-11, max_iter=100000, g0=None, domain="scaling"):
    """Converged primal value P of the full problem from coordinates (and the state)."""
    C = _cost.sq_euclidean(x, y)
    out = _sk.full_sinkhorn(a, b, C, eps, tol=tol, max_iter=max_iter, g0=g0, domain=domain)
    vals = _obj.full_values(out["f"], out["g"], C, eps, a, b)
    return vals["P"], out


def fd_coordinate(x, y, a, b, eps, which, index, comp, h=1e-4, g0=None, tol=1e-11,
                  domain="scaling"):
    """Central difference of the converged value w.r.t. one coordinate of x or y."""
    vals = []
    for s in (+1.0, -1.0):
        xx = np.array(x, dtype=np.float64, copy=True)
        yy = np.array(y, dtype=np.float64, copy=True)
        tgt = xx if which == "x" else yy
        tgt[index, comp] += s * h
        P, _ = solve_value(xx, yy, a, b, eps, tol=tol, g0=g0, domain=domain)
        vals.append(P)
    return (vals[0] - vals[1]) / (2.0 * h)


def fd_marginal(x, y, a, b, eps, which, I, J, h=1e-7, g0=None, tol=1e-12, domain="scaling"):
    """Central difference along the mass-preserving direction ``e_I - e_J`` of a or b."""
    vals = []
    for s in (+1.0, -1.0):
        aa = np.array(a, dtype=np.float64, copy=True)
        bb = np.array(b, dtype=np.float64, copy=True)
        tgt = aa if which == "a" else bb
        tgt[I] += s * h
        tgt[J] -= s * h
        P, _ = solve_value(x, y, aa, bb, eps, tol=tol, g0=g0, domain=domain)
        vals.append(P)
    return (vals[0] - vals[1]) / (2.0 * h)
