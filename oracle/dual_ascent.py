"""Independent EROT solver for tiny problems (oracle; test infrastructure only).

Maximises the concave dual of entropic OT (Thm. 2, eq. dual_problem_cyclic_ROT with
``phi*(y) = eps exp(y / eps)``; with K = 1 it is the dual of the plain problem)
``D(f, g) = <f, a> + <g, b> - eps sum_IJ exp((f_I + g_J - C_IJ) / eps)``
with SciPy's L-BFGS-B, and returns the plan through the optimality condition
(eq. optimality_condition).  It shares no step with the Sinkhorn code: no alternating closed-form
updates, only a generic quasi-Newton method on the dual objective and its gradient.
Used only to pin ``sinkhorn.full_sinkhorn`` on n <= 64.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def solve_dual(a, b, C, eps, gtol=1e-13, maxiter=20000):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    n1, n2 = C.shape
    s = 1.0 / eps

    def negD(v):
        f, g = v[:n1], v[n1:]
        E = np.exp((f[:, None] + g[None, :] - C) * s)
        val = f @ a + g @ b - eps * E.sum()
        grad_f = a - E.sum(axis=1)
        grad_g = b - E.sum(axis=0)
        return -val, -np.concatenate([grad_f, grad_g])

    res = minimize(negD, np.zeros(n1 + n2), jac=True, method="L-BFGS-B",
                   options={"gtol": gtol, "ftol": 1e-16, "maxiter": maxiter, "maxcor": 50})
    f, g = res.x[:n1], res.x[n1:]
    T = np.exp((f[:, None] + g[None, :] - C) * s)
    return {"f": f, "g": g, "T": T, "D": -res.fun, "success": res.success}
