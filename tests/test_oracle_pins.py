"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the piece of mathematics) that fixes the value.
None of these tests touch the GPU library.
"""
import math

import numpy as np
import pytest
from scipy.special import softmax

from oracle import cost, dual_ascent, grad, lp, objective, projection, sinkhorn, srot
import workloads


def _rand_problem(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, scale, size=(n, n))
    a = rng.uniform(0.2, 1.0, size=n)
    b = rng.uniform(0.2, 1.0, size=n)
    return a / a.sum(), b / b.sum(), C


def _exact_cloud(m, K, dim, seed):
    """Exactly rotated float64 clouds (no float32 rounding), periodic marginals."""
    x = workloads.annulus_cloud(m, K, dim, np.random.default_rng(seed))
    y = workloads.annulus_cloud(m, K, dim, np.random.default_rng(seed + 1))
    rng = np.random.default_rng(seed + 2)
    al = rng.dirichlet(np.ones(m))
    be = rng.dirichlet(np.ones(m))
    a = np.tile(al / K, K)
    b = np.tile(be / K, K)
    return x, y, a, b


# ---------------------------------------------------------------- full Sinkhorn ----------

@pytest.mark.parametrize("eps", [0.05, 0.2])
def test_full_sinkhorn_equals_independent_dual_solver(eps):
    """The EROT optimum is unique (strict convexity); a generic L-BFGS ascent on the dual of
    Thm. 2 (K = 1) must reach the same plan as the closed-form alternating updates."""
    a, b, C = _rand_problem(20, seed=3)
    sk = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-14, max_iter=200000)
    ref = dual_ascent.solve_dual(a, b, C, eps)
    T = sinkhorn.full_plan(sk["f"], sk["g"], C, eps)
    assert np.abs(T - ref["T"]).max() < 1e-8
    vals = objective.full_values(sk["f"], sk["g"], C, eps, a, b)
    assert abs(vals["D"] - ref["D"]) < 1e-10


def test_full_sinkhorn_feasible_and_strong_duality():
    """Marginal feasibility and zero duality gap at convergence (Thm. 2 proof: strong
    duality holds by Slater's condition)."""
    x, y, a, b = _exact_cloud(8, 4, 2, seed=11)
    C = cost.sq_euclidean(x, y)
    eps = 0.05 * cost.median(C)
    out = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-13)
    assert out["converged"]
    v = objective.full_values(out["f"], out["g"], C, eps, a, b)
    assert v["err_row"] <= 1e-13 and v["err_col"] <= 1e-13
    assert abs(v["P"] - v["D"]) <= 1e-12 * max(1.0, abs(v["CT"]))
    assert abs(v["mass"] - 1.0) < 1e-12


@pytest.mark.parametrize("eps", [0.1, 0.01, 0.002])
def test_lp_bracket_as_eps_goes_to_zero(eps):
    """With H(T) <= 2 log n on the transport polytope:
    LP <= <C,T_eps> <= LP + 2 eps log n  and  LP - eps - 2 eps log n <= P_eps <= LP - eps."""
    a, b, C = _rand_problem(16, seed=5)
    n = C.shape[0]
    LP, _ = lp.lot_value(a, b, C)
    out = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-13, max_iter=500000)
    v = objective.full_values(out["f"], out["g"], C, eps, a, b)
    slack = 1e-10
    assert LP - slack <= v["CT"] <= LP + 2 * eps * math.log(n) + slack
    assert LP - eps - 2 * eps * math.log(n) - slack <= v["P"] <= LP - eps + slack


def test_primal_via_Z_equals_primal_of_plan():
    """P = <C,T> + eps sum T(log T - 1) evaluated on the plan equals the Z form."""
    a, b, C = _rand_problem(12, seed=8)
    eps = 0.1
    out = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-12)
    T = sinkhorn.full_plan(out["f"], out["g"], C, eps)
    v = objective.full_values(out["f"], out["g"], C, eps, a, b)
    assert abs(objective.primal_of_plan(T, C, eps) - v["P"]) < 1e-13


def test_scaling_domain_matches_log_domain():
    a, b, C = _rand_problem(30, seed=9)
    o1 = sinkhorn.full_sinkhorn(a, b, C, 0.1, tol=1e-12)
    o2 = sinkhorn.full_sinkhorn(a, b, C, 0.1, tol=1e-12, domain="scaling")
    assert o1["iters"] == o2["iters"]
    assert np.abs(o1["f"] - o2["f"]).max() < 1e-12


# ---------------------------------------------------------------- cost structure ---------

def test_rotated_cloud_cost_is_block_circulant():
    """Assumption 1 (eq. blkstr_cost): with point r*m+i = R^r x_i, the cost of the rotated
    clouds has block (r, c) = C_{(c - r) mod K}, built here from block-row 0 only."""
    for K, m, dim in [(4, 5, 2), (6, 3, 3)]:
        x, y, _, _ = _exact_cloud(m, K, dim, seed=21)
        C = cost.sq_euclidean(x, y)
        Csym = cost.block_circulant_from_row0(cost.row0_from_points(x, y, K), K)
        assert np.abs(C - Csym).max() < 1e-14


def test_block_permutation_invariance():
    """Lemma 1's proof: P^l C (P^l)^T = C for a block-circulant C and P^K = I."""
    K, m = 5, 3
    rng = np.random.default_rng(1)
    C = cost.block_circulant_from_blocks(rng.uniform(size=(K, m, m)))
    P = cost.block_shift_permutation(K, m)
    Pl = np.eye(K * m)
    for _ in range(K):
        Pl = P @ Pl
        assert np.abs(Pl @ C @ Pl.T - C).max() == 0.0
    assert np.abs(Pl - np.eye(K * m)).max() == 0.0


def test_median_of_full_cost_equals_block_row0():
    """The full n x n multiset is K copies of block-row 0, so the medians agree."""
    p = workloads.symmetric_problem(96, 8, seed=3)
    row0 = cost.row0_from_points(p.x, p.y, p.K)
    full = cost.block_circulant_from_row0(row0, p.K)
    assert cost.median(full) == cost.median(row0)
    assert abs(p.eps - 0.05 * cost.median(row0)) < 1e-15


# ---------------------------------------------------------------- cyclic Sinkhorn --------

@pytest.mark.parametrize("K,m,dim,fac", [(4, 8, 2, 0.05), (8, 4, 3, 0.01), (3, 7, 2, 0.1)])
def test_reduced_iterates_equal_tiled_full_iterates(K, m, dim, fac):
    """Full Sinkhorn from g = 0 on a cyclic problem stays block-periodic, and its iterates
    equal the tiled iterates of Alg. 2 at every iteration (eq. def_Kij substituted into the
    full updates).  The full run uses the cost computed directly from all n points."""
    x, y, a, b = _exact_cloud(m, K, dim, seed=31)
    C = cost.sq_euclidean(x, y)
    eps = fac * cost.median(C)
    rec = {1, 2, 5, 17}
    full = sinkhorn.full_sinkhorn(a, b, C, eps, tol=0.0, max_iter=17, record=rec)
    Ck = cost.blocks_from_row0(cost.row0_from_points(x, y, K), K)
    alpha, beta = sinkhorn.fold_marginals(a, K), sinkhorn.fold_marginals(b, K)
    logK = sinkhorn.fold_kernel(Ck, eps)
    red = sinkhorn.reduced_sinkhorn(alpha, beta, logK, eps, K, tol=0.0, max_iter=17, record=rec)
    for it in rec:
        ff, gf = full["history"][it]
        fr, gr = red["history"][it]
        assert np.abs(ff - np.tile(fr, K)).max() < 1e-12 * (1 + np.abs(ff).max())
        assert np.abs(gf - np.tile(gr, K)).max() < 1e-12 * (1 + np.abs(gf).max())
    assert abs(full["err_row"] - red["err_row"]) < 1e-13


def test_reduced_and_full_stop_at_the_same_iteration():
    x, y, a, b = _exact_cloud(6, 5, 2, seed=41)
    C = cost.sq_euclidean(x, y)
    eps = 0.02 * cost.median(C)
    full = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-10)
    Ck = cost.blocks_from_row0(cost.row0_from_points(x, y, 5), 5)
    red = sinkhorn.cyclic_sinkhorn(a, b, Ck, eps, tol=1e-10)
    assert full["converged"] and red["converged"]
    assert full["iters"] == red["iters"]


def test_reduced_on_dense_appendix_d_workload():
    """The dense-cost synthetic workload (App. D) through the block-circulant full matrix."""
    p = workloads.dense_appd_problem(40, 5, seed=0)
    Ck = cost.blocks_from_row0(p.C_row0, p.K)
    C = cost.block_circulant_from_blocks(Ck)
    a, b = p.a.astype(np.float64), p.b.astype(np.float64)
    full = sinkhorn.full_sinkhorn(a, b, C, p.eps, tol=1e-11)
    red = sinkhorn.cyclic_sinkhorn(a, b, Ck, p.eps, tol=1e-11)
    assert full["iters"] == red["iters"]
    assert np.abs(full["f"] - np.tile(red["f"], p.K)).max() < 1e-10


def test_m_equals_one_closed_form():
    """m = 1, alpha = beta = 1/K: the reduced problem has a single row and column, so one
    iteration is exact and T[r, c] = (1/K) softmax_k(-c_k/eps)[(c - r) mod K]."""
    K, eps = 7, 0.3
    rng = np.random.default_rng(2)
    ck = rng.uniform(0, 2, size=K)
    Ck = ck.reshape(K, 1, 1)
    a = np.full(K, 1.0 / K)
    out = sinkhorn.cyclic_sinkhorn(a, a, Ck, eps, tol=1e-15, max_iter=5)
    T = sinkhorn.expand_plan(out["f"], out["g"], Ck, eps)
    sm = softmax(-ck / eps)
    ref = np.array([[sm[(c - r) % K] / K for c in range(K)] for r in range(K)])
    assert np.abs(T - ref).max() < 1e-15


def test_K_equals_one_is_plain_sinkhorn():
    """K = 1: the folded kernel is exp(-C/eps) and Alg. 2 is Sinkhorn."""
    a, b, C = _rand_problem(15, seed=4)
    eps = 0.07
    assert np.abs(sinkhorn.fold_kernel(C[None], eps) + C / eps).max() < 1e-13
    full = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-12)
    red = sinkhorn.cyclic_sinkhorn(a, b, C[None], eps, tol=1e-12)
    assert full["iters"] == red["iters"]
    assert np.abs(full["f"] - red["f"]).max() < 1e-12


def test_fold_of_identical_blocks():
    """K identical blocks: K_ij = K exp(-C_ij/eps), i.e. logK = log K - C/eps."""
    rng = np.random.default_rng(6)
    C0 = rng.uniform(0, 3, size=(4, 4))
    for K in (2, 16, 64):
        logK = sinkhorn.fold_kernel(np.repeat(C0[None], K, axis=0), 0.01)
        assert np.abs(logK - (math.log(K) - C0 / 0.01)).max() < 1e-11


def test_expanded_plan_is_shift_invariant_and_equals_full_plan():
    """Lemma 1: the optimal plan is block-circulant, P^l T (P^l)^T = T; it also equals the
    plan of plain Sinkhorn on the full problem."""
    K, m = 4, 6
    x, y, a, b = _exact_cloud(m, K, 2, seed=51)
    C = cost.sq_euclidean(x, y)
    eps = 0.05 * cost.median(C)
    Ck = cost.blocks_from_row0(cost.row0_from_points(x, y, K), K)
    red = sinkhorn.cyclic_sinkhorn(a, b, Ck, eps, tol=1e-13)
    T = sinkhorn.expand_plan(red["f"], red["g"], Ck, eps)
    P = cost.block_shift_permutation(K, m)
    Pl = np.eye(K * m)
    for _ in range(K):
        Pl = P @ Pl
        assert np.abs(Pl @ T @ Pl.T - T).max() < 1e-16
    full = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-13)
    Tf = sinkhorn.full_plan(full["f"], full["g"], C, eps)
    assert np.abs(T - Tf).max() < 1e-13


def test_reduced_objective_is_one_over_K_of_full():
    """eq. problem_CROT: the reduced objective is exactly 1/K of the full one (primal and
    dual)."""
    K, m = 5, 4
    x, y, a, b = _exact_cloud(m, K, 2, seed=61)
    C = cost.sq_euclidean(x, y)
    eps = 0.05 * cost.median(C)
    Ck = cost.blocks_from_row0(cost.row0_from_points(x, y, K), K)
    red = sinkhorn.cyclic_sinkhorn(a, b, Ck, eps, tol=1e-13)
    vr = objective.reduced_values(red["f"], red["g"], Ck, eps, red["alpha"], red["beta"])
    vf = objective.full_values(np.tile(red["f"], K), np.tile(red["g"], K), C, eps, a, b)
    for key in ("P", "D", "CT", "mass"):
        assert abs(K * vr[key] - vf[key]) < 1e-14 * max(1.0, abs(vf[key]))
    er, ec = sinkhorn.reduced_marginal_errors(red["f"], red["g"], red["logK"], eps,
                                              red["alpha"], red["beta"], K)
    assert abs(er - vf["err_row"]) < 1e-15 and abs(ec - vf["err_col"]) < 1e-15


def test_theorem1_small_lp():
    """Thm. 1: the cyclic LOT value equals K times the small LOT on G = min_k C_k."""
    K, m = 3, 5
    rng = np.random.default_rng(71)
    Ck = rng.uniform(0, 1, size=(K, m, m))
    al = rng.dirichlet(np.ones(m)) / K
    be = rng.dirichlet(np.ones(m)) / K
    C = cost.block_circulant_from_blocks(Ck)
    full, _ = lp.lot_value(np.tile(al, K), np.tile(be, K), C)
    small, S, kstar = lp.small_lot_value(al, be, Ck)
    assert abs(full - K * small) < 1e-12


def test_lot_plan_is_feasible_and_optimal():
    """Thm. 1 with Lemma 1: the plan built from the small LP's solution meets the full
    marginals and its cost is the optimum of the full LP (brute force)."""
    K, m = 4, 4
    rng = np.random.default_rng(73)
    Ck = rng.uniform(0, 1, size=(K, m, m))
    al = rng.dirichlet(np.ones(m)) / K
    be = rng.dirichlet(np.ones(m)) / K
    C = cost.block_circulant_from_blocks(Ck)
    full, _ = lp.lot_value(np.tile(al, K), np.tile(be, K), C)
    small, S, kstar = lp.small_lot_value(al, be, Ck)
    T = lp.lot_plan(S, kstar, K)
    assert np.abs(T.sum(1) - np.tile(al, K)).max() < 1e-12
    assert np.abs(T.sum(0) - np.tile(be, K)).max() < 1e-12
    assert T.min() >= 0.0
    assert abs((C * T).sum() - full) < 1e-12


def test_min_fold_takes_the_smallest_k_among_ties():
    Ck = np.array([[[2.0, 1.0]], [[1.0, 1.0]], [[1.0, 3.0]]])  # K = 3, m = 1 x 2 entries
    G, kstar = lp.min_fold(Ck.reshape(3, 1, 2))
    assert np.array_equal(G, [[1.0, 1.0]])
    assert np.array_equal(kstar, [[1, 0]])


def test_srot_waterfill_root_against_bisection():
    rng = np.random.default_rng(91)
    v = rng.uniform(-1, 3, size=37)
    for t, lam in ((0.3, 0.5), (1e-4, 2.0), (5.0, 0.1)):
        w = srot.waterfill(v, t, lam)
        lo, hi = v.min(), v.max() + lam * t
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if np.maximum(0.0, mid - v).sum() < lam * t:
                lo = mid
            else:
                hi = mid
        assert abs(w - 0.5 * (lo + hi)) < 1e-12
        assert abs(np.maximum(0.0, w - v).sum() - lam * t) < 1e-12


def test_srot_cyclic_iterates_equal_tiled_full_iterates():
    """The reduced alternating maximisation equals the full one on the block-circulant cost
    (K = 1 with the n x n matrix), tiled, at every iteration."""
    K, m = 3, 5
    rng = np.random.default_rng(93)
    Ck = rng.uniform(0, 1, size=(K, m, m))
    al = rng.dirichlet(np.ones(m)) / K
    be = rng.dirichlet(np.ones(m)) / K
    C = cost.block_circulant_from_blocks(Ck)
    rec_c, rec_f = [], []
    srot.cyclic_srot(al, be, Ck, 0.2, K, tol=0.0, max_iter=12, record=rec_c)
    srot.cyclic_srot(np.tile(al, K), np.tile(be, K), C[None], 0.2, 1, tol=0.0, max_iter=12,
                     record=rec_f)
    for (wc, zc), (wf, zf) in zip(rec_c, rec_f):
        assert np.abs(np.tile(wc, K) - wf).max() < 1e-12
        assert np.abs(np.tile(zc, K) - zf).max() < 1e-12


def test_srot_converges_to_the_dual_optimum():
    """At convergence both marginals hold, primal = dual, and the dual value equals that of an
    independent L-BFGS maximisation of the concave dual."""
    from scipy.optimize import minimize
    K, m, lam = 2, 6, 0.3
    rng = np.random.default_rng(95)
    Ck = rng.uniform(0, 1, size=(K, m, m))
    al = rng.dirichlet(np.ones(m)) / K
    be = rng.dirichlet(np.ones(m)) / K
    out = srot.cyclic_srot(al, be, Ck, lam, K, tol=1e-12, max_iter=20000)
    v = srot.values(out["w"], out["z"], Ck, lam, al, be)
    assert np.abs(v["row"] - al).max() < 1e-11 and np.abs(v["col"] - be).max() < 1e-13
    assert abs(v["primal"] - v["dual"]) < 1e-10

    def neg_dual(u):
        w, z = u[:m], u[m:]
        y = np.maximum(0.0, w[None, :, None] + z[None, None, :] - Ck)
        val = w @ al + z @ be - (y * y).sum() / (2 * lam)
        gw = al - y.sum(axis=(0, 2)) / lam
        gz = be - y.sum(axis=(0, 1)) / lam
        return -val, -np.concatenate([gw, gz])

    res = minimize(neg_dual, np.zeros(2 * m), jac=True, method="L-BFGS-B",
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 10000})
    assert abs(-res.fun - v["dual"]) < 1e-9


def test_srot_full_plan_solves_the_primal_qp():
    """The expanded quadratic-regularised plan (Lemma 1 with eq. optimality_condition) solves
    the full primal QP min <C,T> + lam/2 ||T||^2 over the transport polytope: checked against
    SciPy's SLSQP on the n x n problem (n = 8), and its value is K times the reduced one."""
    from scipy.optimize import minimize
    K, m, lam = 2, 4, 0.5
    rng = np.random.default_rng(97)
    Ck = rng.uniform(0, 1, size=(K, m, m))
    al = rng.dirichlet(np.ones(m)) / K
    be = rng.dirichlet(np.ones(m)) / K
    out = srot.cyclic_srot(al, be, Ck, lam, K, tol=1e-13, max_iter=20000)
    Tk = srot.plan_blocks(out["w"], out["z"], Ck, lam)
    C = cost.block_circulant_from_blocks(Ck)
    T = cost.block_circulant_from_blocks(Tk)
    n = K * m
    a, b = np.tile(al, K), np.tile(be, K)
    obj = lambda t: float((C.ravel() * t).sum() + 0.5 * lam * (t * t).sum())
    cons = [{"type": "eq", "fun": lambda t, i=i: t.reshape(n, n)[i].sum() - a[i]} for i in range(n)]
    cons += [{"type": "eq", "fun": lambda t, j=j: t.reshape(n, n)[:, j].sum() - b[j]}
             for j in range(n - 1)]
    res = minimize(obj, np.full(n * n, 1.0 / (n * n)), method="SLSQP", constraints=cons,
                   bounds=[(0, None)] * (n * n), options={"ftol": 1e-14, "maxiter": 1000})
    assert res.success
    v = srot.values(out["w"], out["z"], Ck, lam, al, be)
    assert abs(obj(T.ravel()) - K * v["primal"]) < 1e-12
    assert abs(obj(T.ravel()) - res.fun) < 1e-8
    assert np.abs(T.ravel() - res.x).max() < 1e-5


def test_counter_example_single_block_is_not_the_answer():
    """App. A: solving OT on one symmetric block alone and tiling it is wrong in general;
    the cyclic solution differs from the block-diagonal tiling."""
    K, m = 4, 5
    x, y, a, b = _exact_cloud(m, K, 2, seed=81)
    C = cost.sq_euclidean(x, y)
    eps = 0.05 * cost.median(C)
    full = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-12)
    vf = objective.full_values(full["f"], full["g"], C, eps, a, b)
    blk = sinkhorn.full_sinkhorn(a[:m] * K, b[:m] * K, C[:m, :m], eps, tol=1e-12)
    vb = objective.full_values(blk["f"], blk["g"], C[:m, :m], eps, a[:m] * K, b[:m] * K)
    assert vf["P"] < vb["P"] - 1e-6


# ---------------------------------------------------------------- gradients --------------

def test_envelope_gradients_match_finite_differences():
    """dOT/dx, dOT/dy by central differences of the converged value (FP64, h = 1e-4), and
    dOT/da, dOT/db along mass-preserving directions e_I - e_J."""
    p = workloads.symmetric_problem(24, 3, seed=7)
    x, y = p.x.astype(np.float64), p.y.astype(np.float64)
    a, b = p.a.astype(np.float64), p.b.astype(np.float64)
    P0, out = grad.solve_value(x, y, a, b, p.eps, tol=1e-13)
    G = grad.envelope_grads(out["f"], out["g"], x, y, p.eps)
    rng = np.random.default_rng(0)
    for _ in range(6):
        I, d = int(rng.integers(24)), int(rng.integers(2))
        fdx = grad.fd_coordinate(x, y, a, b, p.eps, "x", I, d, h=1e-4, g0=out["g"])
        fdy = grad.fd_coordinate(x, y, a, b, p.eps, "y", I, d, h=1e-4, g0=out["g"])
        assert abs(fdx - G["dx"][I, d]) < 1e-7
        assert abs(fdy - G["dy"][I, d]) < 1e-7
    for I, J in [(0, 5), (7, 20)]:
        fda = grad.fd_marginal(x, y, a, b, p.eps, "a", I, J, g0=out["g"])
        fdb = grad.fd_marginal(x, y, a, b, p.eps, "b", I, J, g0=out["g"])
        assert abs(fda - (G["da"][I] - G["da"][J])) < 1e-6
        assert abs(fdb - (G["db"][I] - G["db"][J])) < 1e-6


def test_cost_gradient_is_the_plan():
    """dOT/dC_IJ = T_IJ: central difference on a single cost entry."""
    a, b, C = _rand_problem(10, seed=12)
    eps, h = 0.1, 1e-5
    base = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-14)
    T = sinkhorn.full_plan(base["f"], base["g"], C, eps)
    for (I, J) in [(0, 0), (3, 7), (9, 2)]:
        vals = []
        for s in (1, -1):
            C2 = C.copy()
            C2[I, J] += s * h
            o = sinkhorn.full_sinkhorn(a, b, C2, eps, tol=1e-14, g0=base["g"])
            vals.append(objective.full_values(o["f"], o["g"], C2, eps, a, b)["P"])
        assert abs((vals[0] - vals[1]) / (2 * h) - T[I, J]) < 1e-8


# ---------------------------------------------------------------- projection -------------

def test_projection_equals_group_average_and_is_idempotent():
    K, m = 4, 3
    rng = np.random.default_rng(91)
    C = rng.uniform(size=(K * m, K * m))
    blocks = projection.project_blocks(C, K)
    avg = projection.group_average(C, K)
    assert np.abs(cost.block_circulant_from_blocks(blocks) - avg).max() < 1e-15
    again = projection.project_blocks(cost.block_circulant_from_blocks(blocks), K)
    assert np.abs(again - blocks).max() < 1e-15


def test_projection_is_exact_on_symmetric_input():
    """sigma = 0 and no marginal noise: the projected problem is the problem itself, so the
    objective gap is exactly zero."""
    p = workloads.jittered_problem(48, 4, sigma=0.0, noise=0.0, seed=5)
    q = workloads.symmetric_problem(48, 4, seed=5)
    assert np.array_equal(p.x, q.x) and np.array_equal(p.y, q.y)
    x, y = p.x.astype(np.float64), p.y.astype(np.float64)
    C = cost.sq_euclidean(x, y)
    blocks = projection.project_blocks(C, p.K)
    Cp = cost.block_circulant_from_blocks(blocks)
    assert np.abs(Cp - C).max() < 1e-6  # float32 coordinates: symmetric up to rounding


def test_projection_rows_from_points_equal_group_average():
    """The row-wise projection from coordinates (used at sizes where the n x n cost is not
    formed) equals block-row 0 of Lemma 1's permutation average of the full cost."""
    p = workloads.jittered_problem(60, 5, sigma=0.05, noise=0.1, dim=3, seed=13)
    x, y = p.x.astype(np.float64), p.y.astype(np.float64)
    avg = projection.group_average(cost.sq_euclidean(x, y), p.K)
    rows = [0, 4, 11]
    got = projection.project_rows_from_points(x, y, p.K, rows)
    assert np.abs(got - avg[rows]).max() < 1e-13


def test_envelope_gradients_match_stored_asymmetric_differences():
    """The envelope gradients of the converged float64 full solution at n = 4096, K = 8 against
    the central differences stored by tests/golden/make_fd_grad.py (each from two further
    float64 solves with one coordinate or one e_I - e_J marginal direction perturbed)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_grad_n4096_K8.json")
    with open(path) as fh:
        gold = json.load(fh)
    wl = gold["workload"]
    p = workloads.symmetric_problem(wl["n"], wl["K"], wl["dim"], wl["eps_factor"], seed=wl["seed"])
    x, y, a, b = (v.astype(np.float64) for v in (p.x, p.y, p.a, p.b))
    P, out = grad.solve_value(x, y, a, b, p.eps, tol=1e-12)
    assert abs(P - gold["value_P"]) <= 1e-12 * abs(P)
    g = grad.envelope_grads(out["f"], out["g"], x, y, p.eps)
    for c in gold["coords"]:
        got = g["dx" if c["which"] == "x" else "dy"][c["index"], c["comp"]]
        assert abs(got - c["fd"]) <= 1e-6 * abs(c["fd"]) + 1e-9, c
    for c in gold["marginals"]:
        v = g["da" if c["which"] == "a" else "db"]
        # the value's curvature in a marginal entry grows like 1 / entry, so h = 1e-7 leaves a
        # truncation error up to ~1e-4 relative where b_J or a_J is small (most agree to 1e-7)
        assert abs((v[c["I"]] - v[c["J"]]) - c["fd"]) <= 1e-4 * abs(c["fd"]) + 1e-9, c


# ---------------------------------------------------------------- two-stage (Alg. 3) -------

def _plan(f, g, C, eps):
    return np.exp((f[:, None] + g[None, :] - C) / eps)


def test_two_stage_on_exact_symmetry_needs_one_full_iteration():
    """On exactly block-circulant data the stage-1 solution tiled is already the full solution
    (Lemma 1 with iterate equivalence), so stage 2 stops after its first iteration, at the plan
    of a cold full-size solve (the EROT solution is unique)."""
    m, K, eps = 12, 4, 0.15
    x, y, a, b = _exact_cloud(m, K, 2, seed=31)
    C = cost.sq_euclidean(x, y)
    out = sinkhorn.two_stage_sinkhorn(a, b, C, K, eps, tol=1e-10)
    assert out["stage1"]["converged"] and out["stage2"]["iters"] == 1
    cold = sinkhorn.full_sinkhorn(a, b, C, eps, tol=1e-10)
    T2, Tc = _plan(out["f"], out["g"], C, eps), _plan(cold["f"], cold["g"], C, eps)
    assert np.abs(T2 - Tc).sum() / Tc.sum() < 1e-8


def test_two_stage_reaches_the_unique_solution_on_jittered_data():
    """Jittered copies and perturbed marginals: stage 2 starts from the symmetrized solution and
    ends at the unique EROT plan of the given data (equal to a cold solve's, marginals met,
    primal = dual), in no more full-size iterations than the cold start.  (The saving is small:
    the slow modes of the full iteration come from the symmetry breaking itself, and a cold
    start from g = 0, which is block-periodic too, carries them with the same amplitude.)"""
    p = workloads.jittered_problem(96, 4, sigma=1e-2, noise=0.05, seed=41)
    x, y, a, b = (v.astype(np.float64) for v in (p.x, p.y, p.a, p.b))
    C = cost.sq_euclidean(x, y)
    out = sinkhorn.two_stage_sinkhorn(a, b, C, 4, p.eps, tol=1e-11)
    cold = sinkhorn.full_sinkhorn(a, b, C, p.eps, tol=1e-11)
    assert out["stage2"]["converged"] and cold["converged"]
    T2, Tc = _plan(out["f"], out["g"], C, p.eps), _plan(cold["f"], cold["g"], C, p.eps)
    assert np.abs(T2 - Tc).sum() / Tc.sum() < 1e-8
    assert np.abs(T2.sum(axis=0) - b).max() < 1e-12
    v = objective.full_values(out["f"], out["g"], C, p.eps, a, b)
    assert abs(v["P"] - v["D"]) <= 1e-9 * max(abs(v["P"]), v["CT"])
    assert out["stage2"]["iters"] <= cold["iters"]
