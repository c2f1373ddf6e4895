"""Differentiable reduced EROT (n = 4096, K = 8, m = 512): the autograd wrapper's forward value
and the hand-written adjoint kernels against the float64 oracle -- its envelope gradient at the
same potentials, and central finite differences (h = 1e-4) of its converged value."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, grad, objective, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cfg4():
    return workloads.symmetric_problem(4096, 8, 2, 0.05, seed=300)


def _t(v, rg=False):
    t = torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
    return t.requires_grad_(rg)


def test_autograd_forward_backward(lib, cfg4):
    p = cfg4
    print("[grad] CyclicOT forward/backward n=4096 K=8", flush=True)
    x, y, a, b = _t(p.x, True), _t(p.y, True), _t(p.a, True), _t(p.b, True)
    P = lib.CyclicOT.apply(x, y, a, b, p.eps, p.K, 2e-8, 100000, 1)
    P.backward()
    torch.cuda.synchronize()
    # oracle: converged float64 reduced solution, value and expanded plan
    Ck = cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)
    ref = sinkhorn.cyclic_sinkhorn(p.a.astype(np.float64), p.b.astype(np.float64), Ck, p.eps,
                                   tol=1e-13)
    v = objective.reduced_values(ref["f"], ref["g"], Ck, p.eps, ref["alpha"], ref["beta"])
    assert abs(P.item() - p.K * v["P"]) / max(abs(p.K * v["P"]), p.K * v["CT"]) < 1e-5
    T = sinkhorn.expand_plan(ref["f"], ref["g"], Ck, p.eps)
    X, Y = p.x.astype(np.float64), p.y.astype(np.float64)
    dx = 2 * (T.sum(1)[:, None] * X - T @ Y)
    dy = 2 * (T.sum(0)[:, None] * Y - T.T @ X)
    fa = np.tile(ref["f"], p.K)
    gb = np.tile(ref["g"], p.K)
    for got, want in ((x.grad, dx), (y.grad, dy)):
        err = np.abs(got.cpu().numpy() - want).max() / np.abs(want).max()
        assert err < 2e-4, err
    # da, db up to the simplex gauge: compare differences along e_I - e_J
    for got, want in ((a.grad, fa), (b.grad, gb)):
        gd = got.cpu().numpy().astype(np.float64)
        rng = np.random.default_rng(1)
        I, J = rng.integers(0, p.n, 64), rng.integers(0, p.n, 64)
        assert np.abs((gd[I] - gd[J]) - (want[I] - want[J])).max() < 2e-5 * (1 + np.abs(want).max())


def test_adjoint_matches_finite_differences(lib, cfg4):
    """32 random coordinates of the first block: moving x_i in block-row 0 of the cyclic cost
    moves it in all K block-rows, so d(K P_red)/dx_i = K dx_i (the GPU's full-space gradient
    of the first block's point).  Central differences of the float64 reduced oracle, h = 1e-4."""
    p = cfg4
    print("[grad] 32 central differences (float64 reduced oracle)", flush=True)
    prob = lib.Problem(_t(p.a), _t(p.b), p.eps, p.K, x=_t(p.x), y=_t(p.y))
    opts = lib.make_opts(tol=2e-8, max_iter=100000, fold_fp64=1)
    logK, al, be = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, al, be, opts)
    res = lib.ot_cost_and_grad(prob, f, g, reduced=True, want_dxy=True)
    dx = res["dx"].cpu().numpy().astype(np.float64)
    a, b = p.a.astype(np.float64), p.b.astype(np.float64)
    y = p.y.astype(np.float64)
    x0 = p.x.astype(np.float64)

    def value(xb):
        Ck = cost.blocks_from_row0(cost.sq_euclidean(xb[:p.m], y), p.K)
        r = sinkhorn.cyclic_sinkhorn(a, b, Ck, p.eps, tol=1e-12)
        v = objective.reduced_values(r["f"], r["g"], Ck, p.eps, r["alpha"], r["beta"])
        return p.K * v["P"]

    rng = np.random.default_rng(7)
    h = 1e-4
    for _ in range(32):
        i, d = int(rng.integers(p.m)), int(rng.integers(2))
        xp, xm = x0.copy(), x0.copy()
        xp[i, d] += h
        xm[i, d] -= h
        fd = (value(xp) - value(xm)) / (2 * h)
        assert abs(fd - p.K * dx[i, d]) <= 1e-6 + 2e-4 * abs(fd), (i, d, fd, p.K * dx[i, d])


def test_full_autograd_matches_cyclic(lib):
    """On exactly symmetric data the full problem's solution is the expanded reduced one
    (Thm. 1), so the plain full-size path's value and gradients equal the cyclic path's."""
    p = workloads.symmetric_problem(2048, 8, 3, 0.05, seed=301)
    print("[grad] FullOT vs CyclicOT n=2048 K=8 dim=3", flush=True)
    outs = []
    for fn, extra in ((lib.CyclicOT, (p.K, 1e-7, 100000, 1)), (lib.FullOT, (p.K, 1e-7, 100000))):
        x, y = _t(p.x, True), _t(p.y, True)
        a, b = _t(p.a, True), _t(p.b, True)
        P = fn.apply(x, y, a, b, p.eps, *extra)
        P.backward()
        outs.append((P.item(), x.grad.cpu().numpy(), y.grad.cpu().numpy(),
                     a.grad.cpu().numpy(), b.grad.cpu().numpy()))
    (Pc, dxc, dyc, dac, dbc), (Pf, dxf, dyf, daf, dbf) = outs
    assert abs(Pc - Pf) / abs(Pf) < 1e-5
    for u, v in ((dxc, dxf), (dyc, dyf)):
        assert np.abs(u - v).max() / np.abs(v).max() < 2e-4
    for u, v in ((dac, daf), (dbc, dbf)):     # both mean-centred
        assert np.abs(u - v).max() < 2e-5 * (1 + np.abs(v).max())


def test_dense_cost_autograd(lib):
    """Dense block-circulant cost (App. D workload): dOT/dC_row0[i, k m + j] = K T_ijk."""
    p = workloads.dense_appd_problem(600, 6, seed=2)
    print("[grad] CyclicOTCost n=600 K=6 dense", flush=True)
    C = _t(p.C_row0, True)
    a, b = _t(p.a, True), _t(p.b, True)
    P = lib.CyclicOTCost.apply(C, a, b, p.eps, p.K, 1e-8, 100000, 1)
    P.backward()
    Ck = cost.blocks_from_row0(p.C_row0.astype(np.float64), p.K)
    r = sinkhorn.cyclic_sinkhorn(p.a.astype(np.float64), p.b.astype(np.float64), Ck, p.eps,
                                 tol=1e-13)
    v = objective.reduced_values(r["f"], r["g"], Ck, p.eps, r["alpha"], r["beta"])
    assert abs(P.item() - p.K * v["P"]) / (p.K * v["CT"]) < 1e-5
    Tk = sinkhorn.reduced_plan_blocks(r["f"], r["g"], Ck, p.eps)          # [K, m, m]
    want = p.K * np.concatenate(list(Tk), axis=1)                        # [m, K m]
    got = C.grad.cpu().numpy().astype(np.float64)
    assert np.abs(got - want).max() / want.max() < 1e-4
    assert abs(got.sum() - 1.0) < 1e-4          # K times the reduced mass 1/K


def _fd_golden():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "fd_grad_n4096_K8.json")
    with open(path) as fh:
        return json.load(fh)


@pytest.mark.parametrize("path", ["cyclic", "full"])
def test_gradients_match_asymmetric_finite_differences(lib, path):
    """Single-coordinate perturbations of the full problem (they break the symmetry): central
    differences of the float64 full-size solver, stored by tests/golden/make_fd_grad.py, at
    32 point coordinates and 16 e_I - e_J marginal directions, against the GPU gradients of
    both paths (the cyclic path's dx, dy cover all n points)."""
    g = _fd_golden()
    wl = g["workload"]
    p = workloads.symmetric_problem(wl["n"], wl["K"], wl["dim"], wl["eps_factor"], seed=wl["seed"])
    assert abs(p.eps - wl["eps"]) <= 1e-12 * wl["eps"]
    print(f"[grad] {path} vs stored central differences", flush=True)
    x, y, a, b = _t(p.x, True), _t(p.y, True), _t(p.a, True), _t(p.b, True)
    if path == "cyclic":
        P = lib.CyclicOT.apply(x, y, a, b, p.eps, p.K, 1e-7, 100000, 1)
    else:
        P = lib.FullOT.apply(x, y, a, b, p.eps, p.K, 1e-7, 100000)
    P.backward()
    assert abs(P.item() - g["value_P"]) <= 1e-5 * abs(g["value_P"])
    grads = {"x": x.grad.cpu().numpy(), "y": y.grad.cpu().numpy(),
             "a": a.grad.cpu().numpy().astype(np.float64),
             "b": b.grad.cpu().numpy().astype(np.float64)}
    scale = max(abs(c["fd"]) for c in g["coords"])
    for c in g["coords"]:
        got = float(grads[c["which"]][c["index"], c["comp"]])
        assert abs(got - c["fd"]) <= 2e-4 * abs(c["fd"]) + 1e-5 * scale, (c, got)
    for c in g["marginals"]:
        v = grads[c["which"]]
        got = v[c["I"]] - v[c["J"]]
        assert abs(got - c["fd"]) <= 1e-4 * abs(c["fd"]) + 1e-6, (c, got)
