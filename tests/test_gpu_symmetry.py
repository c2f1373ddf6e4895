"""Approximately symmetric data (n = 16384, K = 32, m = 512): block-circulant projection of
the cost and averaging of the marginals, then the reduced solve, beside plain full-size
Sinkhorn on the exact jittered data.

Parity: the projected cost on sampled rows and the projected problem's reduced solution
against the float64 oracle; the full-size solution through a property checked at sampled
columns (g is the column update of the returned f).  The objective gap between the two is a
reported number (no pin exists for its size beyond the exact-symmetry case, where it is 0)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, objective, projection, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N, K = 16384, 32


def _t(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _solve_both(lib, p):
    prob = lib.Problem(_t(p.a), _t(p.b), p.eps, K, x=_t(p.x), y=_t(p.y))
    Csym = lib.ot_symmetrize_cost(prob)                                  # [m, n]
    sprob = lib.Problem(_t(p.a), _t(p.b), p.eps, K, C=Csym)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    logK, al, be = lib.ot_fold_kernel(sprob, opts)
    fr, gr, sr = lib.ot_sinkhorn_reduced(sprob, logK, al, be, opts)
    vr = lib.values_dict(lib.ot_cost_and_grad(sprob, fr, gr, reduced=True)["values"])
    ff, gf, sf = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=1e-6, max_iter=20000))
    vf = lib.values_dict(lib.ot_cost_and_grad(prob, ff, gf, reduced=False)["values"])
    torch.cuda.synchronize()
    return dict(Csym=Csym, fr=fr, gr=gr, sr=sr, vr=vr, ff=ff, gf=gf, sf=sf, vf=vf)


def test_projected_reduced_vs_full_on_jittered_data(lib):
    p = workloads.jittered_problem(N, K, sigma=1e-3, noise=0.01, seed=200)
    m = p.m
    print(f"[symmetry] jittered n={N} K={K}", flush=True)
    r = _solve_both(lib, p)
    x, y = p.x.astype(np.float64), p.y.astype(np.float64)
    a, b = p.a.astype(np.float64), p.b.astype(np.float64)
    # projected cost: all rows from the oracle (row-wise, float64)
    ref_rows = projection.project_rows_from_points(x, y, K, range(m))
    Cs = r["Csym"].cpu().numpy()
    assert np.abs(Cs - ref_rows).max() / ref_rows.max() < 1e-6
    # reduced solve of the projected problem against the float64 oracle
    Ck = cost.blocks_from_row0(ref_rows, K)
    ref = sinkhorn.cyclic_sinkhorn(a, b, Ck, p.eps, tol=1e-6)
    vo = objective.reduced_values(ref["f"], ref["g"], Ck, p.eps, ref["alpha"], ref["beta"])
    assert r["sr"]["converged"] and abs(r["sr"]["iters"] - ref["iters"]) <= 1
    Pr = r["vr"]["P"]
    assert abs(Pr - K * vo["P"]) / max(abs(K * vo["P"]), K * vo["CT"]) < 1e-5
    # full-size solve on the jittered data: converged, and g is the column update of f at
    # sampled columns (float64 log-sum-exp over all n rows)
    assert r["sf"]["converged"] and r["vf"]["err_row"] <= 1e-6
    f = r["ff"].cpu().numpy().astype(np.float64)
    g = r["gf"].cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(3)
    J = rng.choice(N, size=64, replace=False)
    CJ = cost.sq_euclidean(x, y[J])                                      # [n, 64]
    z = (f[:, None] - CJ) / p.eps
    zmax = z.max(axis=0)
    lse = zmax + np.log(np.exp(z - zmax).sum(axis=0))
    g_ref = p.eps * np.log(b[J]) - p.eps * lse
    assert np.abs(g[J] - g_ref).max() / p.eps < 2e-5
    Pf = r["vf"]["P"]
    gap = abs(Pf - Pr) / abs(Pf)
    print(f"[symmetry] P_full={Pf:.9g} K*P_red={Pr:.9g} gap={gap:.3e} "
          f"iters full/reduced = {r['sf']['iters']}/{r['sr']['iters']}", flush=True)
    assert gap < 1e-3


def test_exact_symmetry_gives_zero_gap(lib):
    """sigma = 0 and no marginal noise: projection changes nothing, so both paths solve the
    same problem (equal to float32 rounding) and stop at the same iteration."""
    p = workloads.jittered_problem(N, K, sigma=0.0, noise=0.0, seed=200)
    print(f"[symmetry] exact n={N} K={K}", flush=True)
    r = _solve_both(lib, p)
    Pf, Pr = r["vf"]["P"], r["vr"]["P"]
    assert abs(Pf - Pr) / max(abs(Pf), r["vf"]["CT"]) < 1e-5
    assert abs(r["sf"]["iters"] - r["sr"]["iters"]) <= 1


def test_two_stage_on_jittered_data(lib):
    """Alg. 3 at n = 16384, K = 32: the two-stage result solves the given (jittered) problem --
    converged under the float64 check, at the objective of a cold full-size solve, g the column
    update of f at sampled columns -- and stage 2 needs no more iterations than the cold start."""
    p = workloads.jittered_problem(N, K, sigma=1e-3, noise=0.01, seed=200)
    print(f"[two-stage] jittered n={N} K={K}", flush=True)
    prob = lib.Problem(_t(p.a), _t(p.b), p.eps, K, x=_t(p.x), y=_t(p.y))
    out = lib.two_stage_sinkhorn(prob, tol=1e-6)
    s1, s2 = out["stage1"], out["stage2"]
    ff, gf, sf = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=1e-6, max_iter=20000))
    v2 = lib.values_dict(lib.ot_cost_and_grad(prob, out["f"], out["g"], reduced=False)["values"])
    vf = lib.values_dict(lib.ot_cost_and_grad(prob, ff, gf, reduced=False)["values"])
    print(f"[two-stage] stage1 {s1['iters']} + stage2 {s2['iters']} iterations; cold full "
          f"{sf['iters']}; P {v2['P']:.9g} vs cold {vf['P']:.9g}", flush=True)
    assert s1["converged"] and s2["converged"] and s2["err_row"] <= 1e-6 * 1.05
    assert s2["iters"] <= sf["iters"]
    assert abs(v2["P"] - vf["P"]) / max(abs(vf["P"]), vf["CT"]) < 1e-5
    f = out["f"].cpu().numpy().astype(np.float64)
    x, y, b = p.x.astype(np.float64), p.y.astype(np.float64), p.b.astype(np.float64)
    g = out["g"].cpu().numpy().astype(np.float64)
    J = np.random.default_rng(4).choice(N, size=64, replace=False)
    z = (f[:, None] - cost.sq_euclidean(x, y[J])) / p.eps
    zmax = z.max(axis=0)
    g_ref = p.eps * np.log(b[J]) - p.eps * (zmax + np.log(np.exp(z - zmax).sum(axis=0)))
    assert np.abs(g[J] - g_ref).max() / p.eps < 2e-5
