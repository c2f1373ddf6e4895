"""GPU parity: every call of the C ABI against the float64 CPU oracle on the same seeded
inputs (float32 arrays on the GPU, float64 copies of the same values in the oracle).

Tolerance (the stated target for float32 results): relative error 1e-5 on the objective and
on the plan (L1), which for an entry T = exp(Z) means |dZ| = |d(f + g - C)| / eps <= 1e-5;
potentials are therefore compared as max |df| / eps and the fold as max |d logK|.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import cost, grad, objective, projection, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
REL = 1e-5


def T_(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _problem(lib, p):
    if p.dim == 0:
        return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, C=T_(p.C_row0))
    return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))


def _blocks(p):
    if p.dim == 0:
        return cost.blocks_from_row0(p.C_row0, p.K)
    return cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)


def _f64(v):
    return np.asarray(v, dtype=np.float64)


CASES = [
    ("sym_n512_K8_d2", lambda: workloads.symmetric_problem(512, 8, 2, 0.05, seed=0)),
    ("sym_n600_K8_d3_ragged", lambda: workloads.symmetric_problem(600, 8, 3, 0.05, seed=7)),
    ("sym_n390_K6_d2_ragged", lambda: workloads.symmetric_problem(390, 6, 2, 0.01, seed=9)),
    ("appd_n700_K7_dense", lambda: workloads.dense_appd_problem(700, 7, seed=0)),
    # the method's degenerate orders: K = 1 (the reduced problem is the full one) and m = 1
    # (one point per block: logK is a scalar and one iteration reaches the fixed point)
    ("sym_n300_K1_d2_order1", lambda: workloads.symmetric_problem(300, 1, 2, 0.05, seed=41)),
    ("sym_n64_K64_d2_m1", lambda: workloads.symmetric_problem(64, 64, 2, 0.05, seed=43)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fp64", [0, 1])
def test_fold_parity(lib, name, mk, fp64):
    p = mk()
    print(f"[fold] {name} fp64={fp64}", flush=True)
    prob = _problem(lib, p)
    logK, alpha, beta = lib.ot_fold_kernel(prob, lib.make_opts(fold_fp64=fp64))
    torch.cuda.synchronize()
    ref = sinkhorn.fold_kernel(_blocks(p), p.eps)
    err = np.abs(logK.cpu().numpy() - ref)
    # float32 rounding of |logK| (<= ~400) plus float32 cost rounding in float32 mode
    scale = np.abs(ref) + 1.0
    assert (err / scale).max() < (2e-7 if fp64 else 2e-6)
    assert np.abs(alpha.cpu().numpy() - sinkhorn.fold_marginals(_f64(p.a), p.K)).max() < 1e-9
    assert np.abs(beta.cpu().numpy() - sinkhorn.fold_marginals(_f64(p.b), p.K)).max() < 1e-9


def _reduced_ref(p, tol, max_iter, record=None):
    Ck = _blocks(p)
    alpha = sinkhorn.fold_marginals(_f64(p.a), p.K)
    beta = sinkhorn.fold_marginals(_f64(p.b), p.K)
    logK = sinkhorn.fold_kernel(Ck, p.eps)
    out = sinkhorn.reduced_sinkhorn(alpha, beta, logK, p.eps, p.K, tol=tol, max_iter=max_iter,
                                    record=record)
    out.update(Ck=Ck, alpha=alpha, beta=beta, logK=logK)
    return out


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_reduced_fixed_iterations(lib, name, mk):
    """Potentials after exactly 1, 3 and 25 iterations (tol = 0) match the oracle's."""
    p = mk()
    prob = _problem(lib, p)
    for its in (1, 3, 25):
        print(f"[reduced fixed] {name} iters={its}", flush=True)
        opts = lib.make_opts(tol=0.0, max_iter=its, fold_fp64=1)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
        ref = _reduced_ref(p, 0.0, its)
        assert st["iters"] == its
        df = np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps
        dg = np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps
        assert df < 2e-5 and dg < 2e-5, (df, dg)


@pytest.mark.parametrize("name,mk", CASES[:2] + CASES[4:5], ids=[c[0] for c in CASES[:2] + CASES[4:5]])
def test_reduced_warm_start(lib, name, mk):
    """warm_start = 1: the solve starts from the g it is given (Alg. 2 with q = exp(g/eps) in
    place of 1).  From the oracle's g after 7 cold iterations, 1 and 4 further iterations
    match the oracle started from the same g, and a tolerance solve from it stops earlier than
    the cold one with the same marginal error."""
    p = mk()
    prob = _problem(lib, p)
    ref0 = _reduced_ref(p, 0.0, 7)
    g0 = ref0["g"].astype(np.float32)
    opts = lib.make_opts(tol=0.0, max_iter=1, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    for its in (1, 4):
        print(f"[reduced warm] {name} iters={its}", flush=True)
        o = lib.make_opts(tol=0.0, max_iter=its, fold_fp64=1)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, o, g0=T_(g0))
        ref = sinkhorn.reduced_sinkhorn(ref0["alpha"], ref0["beta"], ref0["logK"], p.eps, p.K,
                                        tol=0.0, max_iter=its, g0=_f64(g0))
        assert st["iters"] == its
        df = np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps
        dg = np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps
        assert df < 2e-5 and dg < 2e-5, (its, df, dg)
    o = lib.make_opts(tol=1e-6, max_iter=5000, fold_fp64=1)
    _, _, cold = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, o)
    _, _, warm = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta,
                                         lib.make_opts(tol=1e-6, max_iter=5000, fold_fp64=1),
                                         g0=T_(g0))
    assert warm["converged"] and cold["converged"]
    assert warm["iters"] <= cold["iters"], (warm["iters"], cold["iters"])
    assert warm["err_row"] <= 1.05e-6


def test_reduced_more_workgroups_than_one_xcd(lib):
    """m = 1000 needs 63 workgroups, more than one XCD holds: the solver is launched without
    the one-XCD placement and publishes with agent-scope stores (dstats[7] = 0); fixed
    iterations and the tolerance solve still match the oracle."""
    p = workloads.symmetric_problem(2000, 2, 2, 0.05, seed=29)
    print("[reduced many WGs] n2000 K2 m1000", flush=True)
    prob = _problem(lib, p)
    for its in (3, 12):
        opts = lib.make_opts(tol=0.0, max_iter=its, fold_fp64=1)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, ds = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts, host_stats=False)
        dsh = ds.cpu().numpy()
        ref = _reduced_ref(p, 0.0, its)
        assert dsh[0] == its and dsh[7] == 0.0, dsh
        assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
        assert np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps < 2e-5
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    ref = _reduced_ref(p, 1e-6, 20000)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1


def test_reduced_too_large_is_unsupported(lib):
    """m = 19968: even with the slabs left in device memory, the staged potentials of one
    workgroup per CU exceed LDS; the call returns OT_ERR_UNSUPPORTED before any launch (the
    planner's searches end).  Inputs are placeholders: nothing is read."""
    m, K = 19968, 2
    n = m * K
    rng = np.random.default_rng(3)
    xy = T_(rng.uniform(-1, 1, size=(n, 2)).astype(np.float32))
    a = T_(np.full(n, 1.0 / n, dtype=np.float32))
    prob = lib.Problem(a, a, 0.05, K, x=xy, y=xy)
    logK = torch.empty((m, m), dtype=torch.float32, device=DEV)
    alpha = torch.full((m,), 1.0 / n, dtype=torch.float32, device=DEV)
    with pytest.raises(lib.CsotError) as ei:
        lib.ot_sinkhorn_reduced(prob, logK, alpha, alpha, lib.make_opts(tol=1e-6))
    assert ei.value.code == 8  # OT_ERR_UNSUPPORTED


@pytest.mark.parametrize("n,its", [(4608, (1, 5)), (8192, (2,))])
def test_reduced_large_m_reads_slabs_from_device_memory(lib, n, its):
    """m = 2304 and m = 4096 (K = 2): the slabs no longer fit in LDS, so the solver reads padded
    copies of logK from device memory every half-step; fixed iterations against the float64
    oracle, and (m = 2304) the tolerance solve with its float64 check."""
    p = workloads.symmetric_problem(n, 2, 2, 0.05, seed=37)
    prob = _problem(lib, p)
    ref0 = _reduced_ref(p, 0.0, 1)
    for k in its:
        print(f"[reduced large m] m={p.m} iters={k}", flush=True)
        opts = lib.make_opts(tol=0.0, max_iter=k, fold_fp64=1)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
        ref = sinkhorn.reduced_sinkhorn(ref0["alpha"], ref0["beta"], ref0["logK"], p.eps, p.K,
                                        tol=0.0, max_iter=k)
        assert st["iters"] == k
        assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
        assert np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps < 2e-5
    if p.m <= 2304:
        print(f"[reduced large m] m={p.m} tol=1e-6", flush=True)
        opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
        ref = sinkhorn.reduced_sinkhorn(ref0["alpha"], ref0["beta"], ref0["logK"], p.eps, p.K,
                                        tol=1e-6, max_iter=20000)
        assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1
        er, ec = sinkhorn.reduced_marginal_errors(_f64(f.cpu()), _f64(g.cpu()), ref0["logK"],
                                                  p.eps, ref0["alpha"], ref0["beta"], p.K)
        assert abs(st["err_row"] - er) <= 1e-3 * er + 1e-12


def test_reduced_near_empty_rows_take_the_exact_path(lib):
    """Block position 5 carries a marginal of 1e-25 in every block: that row's plan sum, which
    is the shifted sum the row update starts from, stays near 1e-25 (below 2^-60), so the row
    is recomputed with a running maximum every iteration; potentials still match the oracle."""
    p = workloads.symmetric_problem(256, 4, 2, 0.05, seed=23)
    a = p.a.astype(np.float64).copy()
    a.reshape(p.K, p.m)[:, 5] = 1e-25
    a = (a / a.sum()).astype(np.float32)
    print("[reduced tiny row] n256 K4", flush=True)
    prob = lib.Problem(T_(a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))
    q = workloads.Problem(n=p.n, K=p.K, dim=p.dim, x=p.x, y=p.y, a=a, b=p.b, eps=p.eps,
                          seed=p.seed, name="tiny")
    for its in (2, 10):
        opts = lib.make_opts(tol=0.0, max_iter=its, fold_fp64=1)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
        ref = _reduced_ref(q, 0.0, its)
        assert st["iters"] == its
        assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
        assert np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps < 2e-5


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_reduced_to_tolerance(lib, name, mk):
    p = mk()
    print(f"[reduced tol] {name}", flush=True)
    prob = _problem(lib, p)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    ref = _reduced_ref(p, 1e-6, 20000)
    assert st["converged"] and ref["converged"]
    assert abs(st["iters"] - ref["iters"]) <= 1, (st["iters"], ref["iters"])
    # the float64 check kernel: same norms as the oracle evaluates on the very same stored
    # (float32) logK and potentials -- isolates the check's own arithmetic
    er, ec = sinkhorn.reduced_marginal_errors(_f64(f.cpu()), _f64(g.cpu()), _f64(logK.cpu()),
                                              p.eps, _f64(alpha.cpu()), _f64(beta.cpu()), p.K)
    assert st["err_row"] <= 1e-6 * 1.05
    assert abs(st["err_row"] - er) <= 1e-6 * er + 1e-13
    assert abs(st["err_col"] - ec) <= 1e-6 * ec + 1e-13
    # against the float64 fold, the residuals agree up to float32 rounding of logK
    er64, _ = sinkhorn.reduced_marginal_errors(_f64(f.cpu()), _f64(g.cpu()), ref["logK"], p.eps,
                                               ref["alpha"], ref["beta"], p.K)
    assert abs(st["err_row"] - er64) <= 2e-6 * np.linalg.norm(_f64(p.a))
    # objective and plan
    vg = objective.reduced_values(_f64(f.cpu()), _f64(g.cpu()), ref["Ck"], p.eps,
                                  ref["alpha"], ref["beta"])
    vr = objective.reduced_values(ref["f"], ref["g"], ref["Ck"], p.eps, ref["alpha"], ref["beta"])
    assert abs(vg["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_expand_parity(lib, name, mk):
    p = mk()
    print(f"[expand] {name}", flush=True)
    prob = _problem(lib, p)
    ref = _reduced_ref(p, 1e-6, 20000)
    f, g = T_(ref["f"].astype(np.float32)), T_(ref["g"].astype(np.float32))
    T = lib.ot_expand_plan(prob, f, g).cpu().numpy().astype(np.float64)
    Tref = sinkhorn.expand_plan(ref["f"].astype(np.float32), ref["g"].astype(np.float32),
                                ref["Ck"], p.eps)
    assert np.abs(T - Tref).sum() / Tref.sum() < REL
    big = Tref > 1e-3 * Tref.max()
    assert (np.abs(T - Tref)[big] / Tref[big]).max() < 2e-5
    # Lemma 1: block-circulant (shift invariance), exactly, as every copy is the same value
    m = p.m
    assert np.array_equal(T[m:, m:], T[:-m, :-m])


GRAD_CASES = CASES + [
    # the cyclic orders the adjoint kernel is specialised for, beyond K = 8 above
    ("sym_n1024_K16_d2", lambda: workloads.symmetric_problem(1024, 16, 2, 0.05, seed=51)),
    ("sym_n600_K2_d2_ragged", lambda: workloads.symmetric_problem(600, 2, 2, 0.05, seed=52)),
    ("sym_n1040_K4_d3_ragged", lambda: workloads.symmetric_problem(1040, 4, 3, 0.01, seed=53)),
    ("sym_n2048_K16_d3", lambda: workloads.symmetric_problem(2048, 16, 3, 0.05, seed=54)),
]


@pytest.mark.parametrize("name,mk", GRAD_CASES, ids=[c[0] for c in GRAD_CASES])
def test_cost_and_grad_reduced(lib, name, mk):
    p = mk()
    print(f"[costgrad reduced] {name}", flush=True)
    prob = _problem(lib, p)
    ref = _reduced_ref(p, 1e-9, 50000)
    f32, g32 = ref["f"].astype(np.float32), ref["g"].astype(np.float32)
    res = lib.ot_cost_and_grad(prob, T_(f32), T_(g32), reduced=True, want_dC=True,
                               want_dxy=p.dim > 0, want_dab=True)
    v = lib.values_dict(res["values"])
    vr = objective.reduced_values(_f64(f32), _f64(g32), ref["Ck"], p.eps, ref["alpha"],
                                  ref["beta"])
    scale = max(abs(vr["P"]), vr["CT"]) * p.K
    assert abs(v["P"] - p.K * vr["P"]) / scale < REL
    assert abs(v["D"] - p.K * vr["D"]) / scale < REL
    assert abs(v["CT"] - p.K * vr["CT"]) / (p.K * vr["CT"]) < REL
    assert abs(v["mass"] - p.K * vr["mass"]) < 1e-5
    Tk = sinkhorn.reduced_plan_blocks(_f64(f32), _f64(g32), ref["Ck"], p.eps)
    # block-row 0 layout [m, K m]: dP/dC[i, k m + j] = K T_ijk (eq. problem_CROT)
    want = p.K * np.concatenate(list(Tk), axis=1)
    dC = res["dC"].cpu().numpy()
    assert dC.shape == (p.m, p.n)
    assert np.abs(dC - want).sum() / want.sum() < REL
    n = p.n
    fa = np.tile(_f64(f32), p.K)
    assert np.abs(res["da"].cpu().numpy() - (fa - fa.mean())).max() < 1e-5 * (1 + np.abs(fa).max())
    if p.dim > 0:
        # error model: each plan entry carries a float32 relative error, so a gradient
        # component may be off by that error times 2 sum_J T_IJ |x_I - y_J| (per component)
        Tfull = sinkhorn.expand_plan(_f64(f32), _f64(g32), ref["Ck"], p.eps)
        x, y = _f64(p.x), _f64(p.y)
        dx = 2 * (Tfull.sum(1)[:, None] * x - Tfull @ y)
        dy = 2 * (Tfull.sum(0)[:, None] * y - Tfull.T @ x)
        bx = 2 * np.stack([(Tfull * np.abs(x[:, d:d + 1] - y[None, :, d])).sum(1)
                           for d in range(p.dim)], axis=1)
        by = 2 * np.stack([(Tfull * np.abs(y[None, :, d] - x[:, d:d + 1])).sum(0)
                           for d in range(p.dim)], axis=1)
        for key, want, scale in (("dx", dx, bx), ("dy", dy, by)):
            got = res[key].cpu().numpy()
            ratio = (np.abs(got - want) / scale).max()
            print(f"[costgrad reduced] {name} {key}: max |d| / scale = {ratio:.2e}, "
                  f"max |d| / max |grad| = {np.abs(got - want).max() / np.abs(want).max():.2e}",
                  flush=True)
            assert ratio < 2e-5, ratio


FULL_CASES = [
    ("sym_n512_K8_d2", lambda: workloads.symmetric_problem(512, 8, 2, 0.05, seed=0)),
    ("sym_n1100_K4_d3_ragged", lambda: workloads.symmetric_problem(1100, 4, 3, 0.05, seed=3)),
    ("jit_n768_K8", lambda: workloads.jittered_problem(768, 8, seed=200)),
]


def _full_ref(p, tol, max_iter):
    C = cost.sq_euclidean(p.x, p.y)
    out = sinkhorn.full_sinkhorn(_f64(p.a), _f64(p.b), C, p.eps, tol=tol, max_iter=max_iter)
    out["C"] = C
    return out


@pytest.mark.parametrize("name,mk", FULL_CASES, ids=[c[0] for c in FULL_CASES])
def test_full_fixed_and_tolerance(lib, name, mk):
    p = mk()
    prob = _problem(lib, p)
    for its in (1, 4, 30):
        print(f"[full fixed] {name} iters={its}", flush=True)
        f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=its))
        ref = _full_ref(p, 0.0, its)
        assert st["iters"] == its
        assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
        assert np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps < 2e-5
    print(f"[full tol] {name}", flush=True)
    f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=1e-6, max_iter=20000))
    ref = _full_ref(p, 1e-6, 20000)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1
    v = objective.full_values(_f64(f.cpu()), _f64(g.cpu()), ref["C"], p.eps, _f64(p.a), _f64(p.b))
    assert abs(st["err_row"] - v["err_row"]) <= 1e-3 * v["err_row"] + 1e-12
    assert abs(st["err_col"] - v["err_col"]) <= 1e-3 * v["err_col"] + 1e-11
    vr = objective.full_values(ref["f"], ref["g"], ref["C"], p.eps, _f64(p.a), _f64(p.b))
    assert abs(v["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL
    # values and gradients of the full path
    res = lib.ot_cost_and_grad(prob, f, g, reduced=False, want_dC=True, want_dxy=True,
                               want_dab=True)
    gv = lib.values_dict(res["values"])
    assert abs(gv["P"] - v["P"]) / max(abs(v["P"]), v["CT"]) < REL
    assert abs(gv["D"] - v["D"]) / max(abs(v["P"]), v["CT"]) < REL
    G = grad.envelope_grads(_f64(f.cpu()), _f64(g.cpu()), p.x, p.y, p.eps)
    dC = res["dC"].cpu().numpy()
    assert np.abs(dC - G["dC"]).sum() / G["dC"].sum() < REL
    for key in ("dx", "dy"):
        got = res[key].cpu().numpy()
        assert np.abs(got - G[key]).max() / np.abs(G[key]).max() < 1e-4


def test_full_multi_block_workgroups(lib):
    """n = 20000 > 64 rows x 256 workgroups: every workgroup owns two row blocks (the last one
    a ragged 32-row block).  K = 4 rotates by exact quarter turns, so the float32 problem is
    exactly block-circulant and the tiled float64 reduced iterates are the reference (iterate
    equivalence); the oracle never forms the 20000 x 20000 cost."""
    p = workloads.symmetric_problem(20000, 4, 2, 0.05, seed=13)
    m = p.n // p.K
    x0 = p.x[:m].astype(np.float64)
    for r in range(1, p.K):  # the copies are exact quarter turns of block 0
        rot = x0 @ np.linalg.matrix_power(np.array([[0.0, 1.0], [-1.0, 0.0]]), r)
        assert np.array_equal(np.abs(rot), np.abs(p.x[r * m:(r + 1) * m].astype(np.float64)))
    prob = _problem(lib, p)
    for its in (1, 4):
        print(f"[full multi-block] n20000 K4 iters={its}", flush=True)
        f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=its))
        ref = _reduced_ref(p, 0.0, its)
        assert st["iters"] == its
        assert np.abs(f.cpu().numpy() - np.tile(ref["f"], p.K)).max() / p.eps < 2e-5
        assert np.abs(g.cpu().numpy() - np.tile(ref["g"], p.K)).max() / p.eps < 2e-5
    print("[full multi-block] n20000 K4 tol=1e-6", flush=True)
    f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=1e-6, max_iter=20000))
    ref = _reduced_ref(p, 1e-6, 20000)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1, (st["iters"], ref["iters"])
    fh, gh = _f64(f.cpu()), _f64(g.cpu())
    vg = objective.reduced_values(fh[:m], gh[:m], ref["Ck"], p.eps, ref["alpha"], ref["beta"])
    vr = objective.reduced_values(ref["f"], ref["g"], ref["Ck"], p.eps, ref["alpha"], ref["beta"])
    assert abs(vg["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL
    # block-circulance of the full-size solution (shift invariance)
    assert np.abs(fh.reshape(p.K, m) - fh[:m]).max() / p.eps < 2e-5


def test_two_stage_parity(lib):
    """Alg. 3 on jittered data: stage 1 (projection, fold, reduced solve) and stage 2 (full-size
    solve warm-started from the tiled stage-1 g, tiled on the device) against the float64
    two-stage oracle: iteration counts, objective, and the gauge-free f_I + g_J."""
    p = workloads.jittered_problem(768, 8, seed=200)
    print("[two-stage] jit n768 K8", flush=True)
    prob = _problem(lib, p)
    out = lib.two_stage_sinkhorn(prob, tol=1e-6)
    C = cost.sq_euclidean(p.x, p.y)
    ref = sinkhorn.two_stage_sinkhorn(_f64(p.a), _f64(p.b), C, p.K, p.eps, tol=1e-6)
    s1, s2 = out["stage1"], out["stage2"]
    assert s1["converged"] and abs(s1["iters"] - ref["stage1"]["iters"]) <= 1
    assert s2["converged"] and abs(s2["iters"] - ref["stage2"]["iters"]) <= 1
    f, g = _f64(out["f"].cpu()), _f64(out["g"].cpu())
    v = objective.full_values(f, g, C, p.eps, _f64(p.a), _f64(p.b))
    vr = objective.full_values(ref["f"], ref["g"], C, p.eps, _f64(p.a), _f64(p.b))
    assert abs(v["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL
    assert v["err_row"] <= 1e-6 * 1.05
    rng = np.random.default_rng(5)
    I, J = rng.integers(0, p.n, 256), rng.integers(0, p.n, 256)
    assert np.abs((f[I] + g[J]) - (ref["f"][I] + ref["g"][J])).max() / p.eps < 2e-5


def test_full_shift_overflow_redoes_in_exact_mode(lib):
    """Rows whose costs carry offsets of 0 or 100 eps alternate, so the previous potentials of
    a workgroup's rows spread by ~144 (base 2): the common shift of the shifted phase would
    overflow float32, the phase is redone in exact mode (counted in dstats[6]) and the result
    still matches the float64 oracle."""
    n = 2048
    rng = np.random.default_rng(17)
    eps = 0.05
    C = rng.uniform(0.0, 1.0, size=(n, n)) + (np.arange(n) % 2)[:, None] * (100.0 * eps)
    C = C.astype(np.float32)
    a = rng.uniform(0.5, 1.5, size=n)
    b = rng.uniform(0.5, 1.5, size=n)
    a, b = workloads.equal_mass_pair(a / a.sum(), b / b.sum())
    print("[full redo] dense n2048 row offsets", flush=True)
    prob = lib.Problem(T_(a), T_(b), eps, 1, C=T_(C))
    f, g, ds = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=6), host_stats=False)
    dsh = ds.cpu().numpy()
    assert dsh[0] == 6 and dsh[5] == 0 and dsh[6] > 0, dsh
    ref = sinkhorn.full_sinkhorn(_f64(a), _f64(b), _f64(C), eps, tol=0.0, max_iter=6)
    assert np.abs(f.cpu().numpy() - ref["f"]).max() / eps < 2e-5
    assert np.abs(g.cpu().numpy() - ref["g"]).max() / eps < 2e-5


def test_full_wide_potentials_shift_per_row_group(lib):
    """Groups of 4 consecutive rows carry cost offsets of 0 or 100 eps in turn: a workgroup's
    previous potentials spread by ~144 (base 2), but each wave's 4 rows share one offset, so the
    shifted phase shifts every row group by its own potential and nothing is redone in exact
    mode (dstats[6] = 0); the result matches the float64 oracle."""
    n = 2048
    rng = np.random.default_rng(19)
    eps = 0.05
    C = rng.uniform(0.0, 1.0, size=(n, n)) + ((np.arange(n) // 4) % 2)[:, None] * (100.0 * eps)
    C = C.astype(np.float32)
    a = rng.uniform(0.5, 1.5, size=n)
    b = rng.uniform(0.5, 1.5, size=n)
    a, b = workloads.equal_mass_pair(a / a.sum(), b / b.sum())
    print("[full wide] dense n2048 row-group offsets", flush=True)
    prob = lib.Problem(T_(a), T_(b), eps, 1, C=T_(C))
    f, g, ds = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=6), host_stats=False)
    dsh = ds.cpu().numpy()
    assert dsh[0] == 6 and dsh[5] == 0 and dsh[6] == 0, dsh
    ref = sinkhorn.full_sinkhorn(_f64(a), _f64(b), _f64(C), eps, tol=0.0, max_iter=6)
    assert np.abs(f.cpu().numpy() - ref["f"]).max() / eps < 2e-5
    assert np.abs(g.cpu().numpy() - ref["g"]).max() / eps < 2e-5


def test_validate_option_reports_bad_inputs(lib):
    """validate = 1: the host-side checks reject a non-positive marginal, unequal masses and
    (for the reduced path) data that is not block-circulant, and accept valid inputs."""
    p = workloads.symmetric_problem(512, 8, 2, 0.05, seed=0)
    opts = lib.make_opts(validate=1)
    print("[validate] n512 K8", flush=True)
    lib.ot_fold_kernel(_problem(lib, p), opts)                       # valid: no error

    def code_of(fn):
        with pytest.raises(lib.CsotError) as ei:
            fn()
        return ei.value.code

    a_neg = p.a.copy()
    a_neg[3] = -a_neg[3]
    pn = lib.Problem(T_(a_neg), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))
    assert code_of(lambda: lib.ot_fold_kernel(pn, opts)) == 2          # OT_ERR_MASS
    a_more = (p.a * np.float32(1.01)).astype(np.float32)
    pm = lib.Problem(T_(a_more), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))
    assert code_of(lambda: lib.ot_fold_kernel(pm, opts)) == 2
    j = workloads.jittered_problem(512, 8, sigma=1e-3, noise=0.0, seed=200)
    pj = _problem(lib, j)
    assert code_of(lambda: lib.ot_fold_kernel(pj, opts)) == 3          # OT_ERR_NOT_SYMMETRIC
    # the full-size solver needs no symmetry
    f, g, st = lib.ot_sinkhorn_full(pj, lib.make_opts(validate=1, tol=1e-6))
    assert st["converged"]


def test_full_dense(lib):
    p = workloads.dense_appd_problem(600, 6, seed=1)
    print("[full dense] appd n600", flush=True)
    Cfull = cost.block_circulant_from_row0(p.C_row0, p.K).astype(np.float32)
    prob = lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, C=T_(Cfull))
    f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=20))
    ref = sinkhorn.full_sinkhorn(_f64(p.a), _f64(p.b), _f64(Cfull), p.eps, tol=0.0, max_iter=20)
    assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
    assert np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps < 2e-5


def test_symmetrize_parity(lib):
    p = workloads.jittered_problem(640, 8, seed=201)
    print("[symmetrize] jit n640", flush=True)
    prob = _problem(lib, p)
    Cs = lib.ot_symmetrize_cost(prob).cpu().numpy()
    ref = projection.project_blocks(cost.sq_euclidean(p.x, p.y), p.K)
    got = cost.blocks_from_row0(Cs, p.K)
    assert np.abs(got - ref).max() / ref.max() < 1e-6


def test_reduced_matches_full_on_symmetric_data(lib):
    """Iterate equivalence on the GPU: the reduced solve and the full solve stop at the same
    iteration with the same objective (cost recomputed from float32 coordinates, so only
    equal up to the float32 asymmetry of the rotated copies)."""
    p = workloads.symmetric_problem(1024, 8, 2, 0.05, seed=11)
    print("[reduced vs full] n1024 K8", flush=True)
    prob = _problem(lib, p)
    opts = lib.make_opts(tol=1e-6, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    ff, gf, stf = lib.ot_sinkhorn_full(prob, opts)
    assert abs(st["iters"] - stf["iters"]) <= 1
    vr = lib.values_dict(lib.ot_cost_and_grad(prob, f, g, reduced=True)["values"])
    vf = lib.values_dict(lib.ot_cost_and_grad(prob, ff, gf, reduced=False)["values"])
    assert abs(vr["P"] - vf["P"]) / max(abs(vf["P"]), vf["CT"]) < 1e-4


def test_padded_leading_dimensions(lib):
    """Dense costs with a leading dimension beyond n (ldc = n + 13, the extra columns holding a
    huge sentinel that must never be read) and plans written with ldt = n + 7 (the rows'
    padding must stay untouched): fold, reduced solve, expand, the linear OT steps and the
    dense full-size solve against the oracle."""
    from oracle import lp
    p = workloads.dense_appd_problem(600, 6, seed=3)
    n, m, K = p.n, p.m, p.K
    print("[padded strides] appd n600 K6", flush=True)
    Cp = np.full((m, n + 13), 1.0e6, dtype=np.float32)
    Cp[:, :n] = p.C_row0
    prob = lib.Problem(T_(p.a), T_(p.b), p.eps, K, C=T_(Cp))
    opts = lib.make_opts(tol=0.0, max_iter=5, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    ref = _reduced_ref(p, 0.0, 5)
    assert (np.abs(logK.cpu().numpy() - ref["logK"]) / (np.abs(ref["logK"]) + 1.0)).max() < 2e-7
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    assert st["iters"] == 5
    assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
    # expand into rows of stride n + 7: the plan in the first n columns, the padding untouched
    Tbuf = torch.full((n, n + 7), -7.0, dtype=torch.float32, device=DEV)
    lib.ot_expand_plan(prob, f, g, out=Tbuf[:, :n])
    Tb = Tbuf.cpu().numpy()
    Tref = sinkhorn.expand_plan(_f64(f.cpu()), _f64(g.cpu()), ref["Ck"], p.eps)
    assert np.abs(Tb[:, :n] - Tref).sum() / Tref.sum() < REL
    assert (Tb[:, n:] == -7.0).all()
    # linear OT steps on the padded cost
    G, kmin, _, _ = lib.ot_lot_fold(prob)
    Gref, kref = lp.min_fold(ref["Ck"])
    assert np.array_equal(kmin.cpu().numpy(), kref)
    assert np.array_equal(G.cpu().numpy(), Gref.astype(np.float32))
    S = np.random.default_rng(4).uniform(0, 1, size=(m, m)).astype(np.float32)
    Tbuf.fill_(-7.0)
    lib.ot_lot_expand(prob, T_(S), kmin, out=Tbuf[:, :n])
    Tb = Tbuf.cpu().numpy()
    assert np.array_equal(Tb[:, :n].astype(np.float64), lp.lot_plan(S, kref, K))
    assert (Tb[:, n:] == -7.0).all()
    # the dense full-size solver on a padded n x (n + 13) cost
    Cf = np.full((n, n + 13), 1.0e6, dtype=np.float32)
    Cf[:, :n] = cost.block_circulant_from_row0(p.C_row0, K).astype(np.float32)
    fprob = lib.Problem(T_(p.a), T_(p.b), p.eps, K, C=T_(Cf))
    ff, gf, stf = lib.ot_sinkhorn_full(fprob, lib.make_opts(tol=0.0, max_iter=5))
    fref = sinkhorn.full_sinkhorn(_f64(p.a), _f64(p.b), _f64(Cf[:, :n]), p.eps, tol=0.0,
                                  max_iter=5)
    assert stf["iters"] == 5
    assert np.abs(ff.cpu().numpy() - fref["f"]).max() / p.eps < 2e-5
    assert np.abs(gf.cpu().numpy() - fref["g"]).max() / p.eps < 2e-5
