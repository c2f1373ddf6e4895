"""Plain Sinkhorn iterations in float64 (oracle; test infrastructure only).

Notation: the paper writes d for the vector length, n for the cyclic order and lambda for the
regulariser; here n is the length, K the order, m = n / K and eps the regulariser.  The dual
potentials are f (the paper's w) and g (the paper's z); ``p = exp(f/eps)``, ``q = exp(g/eps)``.

full_sinkhorn
    Textbook Sinkhorn for entropy-regularised OT (Cuturi's method; Alg. 3, stage 2, of the
    paper) in the log domain.  Starting from g = 0 (q = 1) each iteration sets
        f_I = eps log a_I - eps LSE_J((g_J - C_IJ) / eps)
        g_J = eps log b_J - eps LSE_I((f_I - C_IJ) / eps)
    which are the logarithms of ``p = a / (K q)`` and ``q = b / (K^T p)``.  A scaling-domain
    variant (``domain="scaling"``) runs the same map on ``p, q`` with ``K = exp(-C/eps)``; it is
    identical in exact arithmetic and only usable when ``max C / eps`` stays far from float64
    underflow (checked).

row_update, col_update
    The two half-steps of that iteration on a subset of rows (columns), given those rows'
    (columns') costs to every partner: the loop of ``full_sinkhorn`` is made of them, and large
    problems are checked one step at a time on sampled rows and columns with them.

fold_marginals, fold_kernel, reduced_sinkhorn, expand_plan
    The cyclic Sinkhorn algorithm (Alg. 2, Sec. "Algorithm for C-EROT"):
    * fold of the marginals (Alg. 3, stage 1): alpha_i = (1/K) sum_r a_{r m + i};
    * folded Gibbs kernel (eq. def_Kij): K_ij = sum_k exp(-C_ijk / eps), kept as logK;
    * the closed-form row update (eq. optimal_f_sinkhorn_logdomain) and its column analogue
      (the logarithm of eq. optimal_sinkhorn), g initialised to 0 (q = 1);
    * the plan T_ijk = exp((f_i + g_j - C_ijk) / eps) (eq. optimality_condition with
      phi*(y) = eps exp(y / eps)) laid out block-circulantly (Lemma 1, eq.
      blkstr_optimal_solution).

two_stage_sinkhorn
    Alg. 3 for approximately symmetric data: stage 1 solves the symmetrized (block-averaged)
    problem by the cyclic algorithm, stage 2 runs full_sinkhorn on the data as given from the
    tiled stage-1 column potential.

Stopping rule (a reading: the paper only says "until convergence"): after each full iteration
(row update then column update) the row-marginal residual of the current plan,
``err = ||T 1 - a||_2`` on the full n-vector, is compared with ``tol``; the column marginal is
exact after the column update.  For the reduced problem the same full-space quantity is
``sqrt(K) * ||T_red 1 - alpha||_2`` because every block-row of the expanded plan has the same
row sums.  The returned state is the one after the first iteration whose residual is <= tol
(or after ``max_iter`` iterations).

Pins (tests/test_oracle_pins.py): full_sinkhorn against an independent dual L-BFGS solve, the
LP bounds as eps -> 0, strong duality and marginal feasibility; the reduced loop against
full_sinkhorn on the block-circulant problem at every iteration (tiled iterates), the m = 1
closed form and the K = 1 degeneracy; expand_plan against Lemma 1's shift invariance.
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def _row_residual_full(f, g, C, eps, a):
    T = np.exp((f[:, None] + g[None, :] - C) / eps)
    return float(np.linalg.norm(T.sum(axis=1) - a))


def row_update(g, C_rows, a_rows, eps):
    """One row half-step on the rows given: ``f_I = eps log a_I - eps LSE_J((g_J - C_IJ)/eps)``
    (the logarithm of ``p = a / (K q)``), ``C_rows`` holding those rows' costs to all columns."""
    C_rows = np.asarray(C_rows, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    return eps * np.log(np.asarray(a_rows, dtype=np.float64)) - eps * logsumexp(
        (g[None, :] - C_rows) / eps, axis=1)


def col_update(f, C_cols, b_cols, eps):
    """One column half-step on the columns given: ``g_J = eps log b_J - eps LSE_I((f_I -
    C_IJ)/eps)`` (the logarithm of ``q = b / (K^T p)``), ``C_cols`` holding all rows' costs to
    those columns."""
    C_cols = np.asarray(C_cols, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    return eps * np.log(np.asarray(b_cols, dtype=np.float64)) - eps * logsumexp(
        (f[:, None] - C_cols) / eps, axis=0)


def full_sinkhorn(a, b, C, eps, tol=1e-9, max_iter=100000, g0=None, domain="log",
                  record=None):
    """Plain full-size Sinkhorn.  Returns a dict with f, g, iters, err_row, converged and,
    when ``record`` is a set of iteration numbers, ``history = {it: (f, g)}``."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    eps = float(eps)
    g = np.zeros(C.shape[1]) if g0 is None else np.asarray(g0, dtype=np.float64).copy()
    history = {}
    if domain == "scaling":
        if C.max() / eps > 600.0:
            raise ValueError("scaling-domain oracle needs max C/eps < 600")
        Kmat = np.exp(-C / eps)
        q = np.exp(g / eps)
    f = None
    err = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        if domain == "scaling":
            p = a / (Kmat @ q)
            q = b / (Kmat.T @ p)
            f = eps * np.log(p)
            g = eps * np.log(q)
            err = float(np.linalg.norm(p * (Kmat @ q) - a))
        else:
            f = row_update(g, C, a, eps)
            g = col_update(f, C, b, eps)
            err = _row_residual_full(f, g, C, eps, a)
        if record is not None and it in record:
            history[it] = (f.copy(), g.copy())
        if err <= tol:
            break
    return {"f": f, "g": g, "iters": it, "err_row": err, "converged": err <= tol,
            "history": history}


def fold_marginals(a, K):
    """alpha_i = (1/K) sum_r a_{r m + i} (Alg. 3, stage 1); equals the block for periodic a."""
    a = np.asarray(a, dtype=np.float64)
    m = a.shape[0] // K
    return a.reshape(K, m).mean(axis=0)


def fold_kernel(Ck, eps):
    """logK_ij = log sum_k exp(-C_ijk / eps) (eq. def_Kij) from the ``[K, m, m]`` cost blocks."""
    Ck = np.asarray(Ck, dtype=np.float64)
    return logsumexp(-Ck / float(eps), axis=0)


def _reduced_row_residual(f, g, logK, eps, alpha):
    T = np.exp(logK + (f[:, None] + g[None, :]) / eps)
    return T.sum(axis=1) - alpha


def reduced_sinkhorn(alpha, beta, logK, eps, K, tol=1e-9, max_iter=100000, g0=None,
                     record=None):
    """Cyclic Sinkhorn loop on the folded m x m problem (Alg. 2, lines 2-6, log form)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    logK = np.asarray(logK, dtype=np.float64)
    eps = float(eps)
    g = np.zeros(logK.shape[1]) if g0 is None else np.asarray(g0, dtype=np.float64).copy()
    history = {}
    f = None
    err = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        f = eps * np.log(alpha) - eps * logsumexp(logK + g[None, :] / eps, axis=1)
        g = eps * np.log(beta) - eps * logsumexp(logK + f[:, None] / eps, axis=0)
        err = float(np.sqrt(K) * np.linalg.norm(_reduced_row_residual(f, g, logK, eps, alpha)))
        if record is not None and it in record:
            history[it] = (f.copy(), g.copy())
        if err <= tol:
            break
    return {"f": f, "g": g, "iters": it, "err_row": err, "converged": err <= tol,
            "history": history}


def reduced_marginal_errors(f, g, logK, eps, alpha, beta, K):
    """Full-space L2 row and column residuals of the plan given by reduced potentials."""
    T = np.exp(np.asarray(logK) + (np.asarray(f)[:, None] + np.asarray(g)[None, :]) / eps)
    er = np.sqrt(K) * np.linalg.norm(T.sum(axis=1) - alpha)
    ec = np.sqrt(K) * np.linalg.norm(T.sum(axis=0) - beta)
    return float(er), float(ec)


def reduced_plan_blocks(f, g, Ck, eps):
    """T_ijk = exp((f_i + g_j - C_ijk) / eps), shape ``[K, m, m]`` (eq. optimality_condition)."""
    Ck = np.asarray(Ck, dtype=np.float64)
    return np.exp((np.asarray(f)[None, :, None] + np.asarray(g)[None, None, :] - Ck) / eps)


def expand_plan(f, g, Ck, eps):
    """Full n x n plan with block (r, c) = T_{(c - r) mod K} (Lemma 1; Alg. 2, last steps)."""
    Tk = reduced_plan_blocks(f, g, Ck, eps)
    K, m, _ = Tk.shape
    n = K * m
    T = np.empty((n, n))
    for r in range(K):
        for c in range(K):
            T[r * m:(r + 1) * m, c * m:(c + 1) * m] = Tk[(c - r) % K]
    return T


def full_plan(f, g, C, eps):
    """T_IJ = exp((f_I + g_J - C_IJ) / eps) on the full problem."""
    return np.exp((np.asarray(f)[:, None] + np.asarray(g)[None, :] - np.asarray(C)) / eps)


def cyclic_sinkhorn(a, b, Ck, eps, tol=1e-9, max_iter=100000):
    """Alg. 2 end to end from the full marginals and the cost blocks: fold, iterate, and
    return the reduced state (the caller expands with ``expand_plan`` when it needs T)."""
    K = np.asarray(Ck).shape[0]
    alpha = fold_marginals(a, K)
    beta = fold_marginals(b, K)
    logK = fold_kernel(Ck, eps)
    out = reduced_sinkhorn(alpha, beta, logK, eps, K, tol=tol, max_iter=max_iter)
    out.update(alpha=alpha, beta=beta, logK=logK)
    return out


def two_stage_sinkhorn(a, b, C, K, eps, tol=1e-9, max_iter=100000, tol_stage1=None):
    """Alg. 3 for approximately symmetric data, in the paper's order.  Stage 1: average the
    marginals over the K blocks (``fold_marginals``) and the cost over the K shifts (the
    block-circulant projection ``projection.project_blocks``) and solve that reduced problem
    (Alg. 2).  Stage 2: plain full-size Sinkhorn on the data as given, started from the stage-1
    column potential tiled K times.  Both stages use the stopping rule of this module; stage 1
    may use a looser tolerance."""
    from .projection import project_blocks

    C = np.asarray(C, dtype=np.float64)
    stage1 = cyclic_sinkhorn(a, b, project_blocks(C, K), eps,
                             tol=tol if tol_stage1 is None else tol_stage1, max_iter=max_iter)
    stage2 = full_sinkhorn(a, b, C, eps, tol=tol, max_iter=max_iter,
                           g0=np.tile(stage1["g"], K))
    return {"f": stage2["f"], "g": stage2["g"], "stage1": stage1, "stage2": stage2}
