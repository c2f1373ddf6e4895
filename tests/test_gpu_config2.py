"""Parity at the benchmark's own workload: n = 8192, K = 16 (m = 512), a 2-D cloud with 16-fold
rotational symmetry (seed 100), eps = 0.1 and 0.01 times the median cost, in the launch
configuration the benchmark times (default options: the full-size solver's (RT, CQ) = (4, 2)
variant on 256 workgroups, the reduced solver's 32 workgroups on one XCD).

Every step of the path against the float64 oracle on the same inputs:
* fold (eq. def_Kij) and marginal fold (Alg. 3, stage 1): all m x m entries;
* reduced iterations (Alg. 2): potentials after 1, 3 and 26 iterations, and the solve to the
  1e-6 row residual (iteration count, float64 check values, objective);
* full-size iterations (Alg. 3, stage 2): after 1 and 4 iterations and at tolerance, (a)
  against the tiled float64 reduced iterates (iterate equivalence: on this workload the float64
  full-size iterates on the as-given float32 coordinates differ from them by 5e-7 eps, far below
  the 2e-5 tolerance), and (b) exactly, step by step, at 64+ sampled rows and columns: the
  returned f at row I is the float64 row update of the previous g over all 8192 columns, the
  returned g at column J the column update of the returned f over all 8192 rows;
* expand (Lemma 1): the plan from the oracle's potentials on 3 block rows x 64 rows, and the
  end-to-end plan from the GPU's own solution against the oracle's plan on the same rows;
  exact shift invariance over the whole n x n plan.
"""
import numpy as np
import pytest
import torch

import workloads
from fullsize_steps import FullData, one_step_errors, row_residual, sample
from oracle import cost, objective, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N, K, SEED = 8192, 16, 100
REL = 1e-5
POT = 2e-5   # potentials: max |df| / eps (the exponent error of a plan entry)


def _t(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _f64(v):
    if isinstance(v, torch.Tensor):
        v = v.cpu().numpy()
    return np.asarray(v, dtype=np.float64)


class Cfg:
    def __init__(self, factor):
        p = workloads.symmetric_problem(N, K, 2, factor, seed=SEED)
        self.p = p
        self.m = p.m
        self.Ck = cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, K), K)
        self.alpha = sinkhorn.fold_marginals(_f64(p.a), K)
        self.beta = sinkhorn.fold_marginals(_f64(p.b), K)
        self.logK = sinkhorn.fold_kernel(self.Ck, p.eps)
        self.data = FullData(p.a, p.b, p.eps, x=p.x, y=p.y)
        self._traj = {}

    def reduced(self, its):
        """float64 reduced iterates after `its` iterations (tol = 0)."""
        if its not in self._traj:
            r = sinkhorn.reduced_sinkhorn(self.alpha, self.beta, self.logK, self.p.eps, K,
                                          tol=0.0, max_iter=its)
            self._traj[its] = (r["f"], r["g"])
        return self._traj[its]


@pytest.fixture(scope="module", params=[0.1, 0.01], ids=["eps0.1med", "eps0.01med"])
def cfg(request):
    return Cfg(request.param)


def _prob(lib, p):
    return lib.Problem(_t(p.a), _t(p.b), p.eps, K, x=_t(p.x), y=_t(p.y))


def test_launch_configuration_is_the_benchmarked_one(lib, cfg):
    prob = _prob(lib, cfg.p)
    fi = lib.ot_full_plan_info(prob)
    ri = lib.ot_reduced_plan_info(prob)
    print(f"[config2] full plan {fi}, reduced plan {ri}", flush=True)
    if torch.cuda.get_device_properties(0).multi_processor_count == 256:
        assert (fi["RT"], fi["CQ"]) == (4, 2)
        assert fi["workgroups"] == 256 and fi["rows"] == 32 and fi["blocks"] == 1
        assert ri["workgroups"] == 32 and ri["stride"] == 8 and ri["gslab"] == 0


def test_fold(lib, cfg):
    p = cfg.p
    print(f"[config2 fold] eps={p.eps:.5g}", flush=True)
    logK, alpha, beta = lib.ot_fold_kernel(_prob(lib, p), lib.make_opts())
    # float32 error model of the fold: each of the K exponentials of the (non-positive) shifted
    # exponents carries about one float32 rounding u = 2^-24, the K-term sum K - 1 more, the
    # final log and the shift-back a few u of |logK|
    u = 2.0 ** -24
    err = np.abs(_f64(logK) - cfg.logK)
    bound = (K + 2) * u + 4 * u * np.abs(cfg.logK)
    print(f"[config2 fold] max |d logK| = {err.max():.3e}, max ratio to the bound "
          f"{(err / bound).max():.3f}", flush=True)
    assert (err <= bound).all(), (err / bound).max()
    assert np.abs(_f64(alpha) - cfg.alpha).max() < 1e-9
    assert np.abs(_f64(beta) - cfg.beta).max() < 1e-9


def test_reduced_fixed_iterations(lib, cfg):
    p = cfg.p
    prob = _prob(lib, p)
    for its in (1, 3, 26):
        print(f"[config2 reduced fixed] eps={p.eps:.5g} iters={its}", flush=True)
        opts = lib.make_opts(tol=0.0, max_iter=its)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
        fr, gr = cfg.reduced(its)
        assert st["iters"] == its
        df = np.abs(_f64(f) - fr).max() / p.eps
        dg = np.abs(_f64(g) - gr).max() / p.eps
        assert df < POT and dg < POT, (df, dg)


def test_reduced_to_tolerance(lib, cfg):
    p = cfg.p
    print(f"[config2 reduced tol] eps={p.eps:.5g}", flush=True)
    prob = _prob(lib, p)
    opts = lib.make_opts(tol=1e-6, max_iter=20000)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    ref = sinkhorn.reduced_sinkhorn(cfg.alpha, cfg.beta, cfg.logK, p.eps, K, tol=1e-6)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1, (st, ref["iters"])
    fh, gh = _f64(f), _f64(g)
    er, ec = sinkhorn.reduced_marginal_errors(fh, gh, cfg.logK, p.eps, cfg.alpha, cfg.beta, K)
    assert st["err_row"] <= 1e-6 * 1.05
    assert abs(st["err_row"] - er) <= 2e-6 * np.linalg.norm(_f64(p.a))
    assert abs(st["err_col"] - ec) <= 2e-6 * np.linalg.norm(_f64(p.b))
    vg = objective.reduced_values(fh, gh, cfg.Ck, p.eps, cfg.alpha, cfg.beta)
    vr = objective.reduced_values(ref["f"], ref["g"], cfg.Ck, p.eps, cfg.alpha, cfg.beta)
    assert abs(vg["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL
    # the library's objective of the full problem (K times the reduced one, eq. problem_CROT)
    v = lib.values_dict(lib.ot_cost_and_grad(prob, f, g, reduced=True)["values"])
    assert abs(v["P"] - K * vr["P"]) / (K * max(abs(vr["P"]), vr["CT"])) < REL


def _rows_cols(seed):
    # boundaries of the (4, 2) variant's 32-row workgroups and of the 2048-column chunks
    bounds = (0, 31, 32, 2047, 2048, 4095, 4096, N - 33, N - 32, N - 1)
    return sample(N, 64, seed, bounds), sample(N, 64, seed + 1, bounds)


def test_full_fixed_iterations(lib, cfg):
    p = cfg.p
    prob = _prob(lib, p)
    I, J = _rows_cols(11)
    g_prev = np.zeros(N)
    done = 0
    for its in (1, 4):
        if its - 1 > done:
            _, gp, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=its - 1))
            assert st["iters"] == its - 1
            g_prev = _f64(gp)
        print(f"[config2 full fixed] eps={p.eps:.5g} iters={its}", flush=True)
        f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=its))
        assert st["iters"] == its
        fh, gh = _f64(f), _f64(g)
        fr, gr = cfg.reduced(its)
        assert np.abs(fh - np.tile(fr, K)).max() / p.eps < POT
        assert np.abs(gh - np.tile(gr, K)).max() / p.eps < POT
        ef, eg = one_step_errors(cfg.data, g_prev, fh, gh, I, J)
        assert ef < POT and eg < POT, (ef, eg)
        g_prev, done = gh, its


def test_full_to_tolerance(lib, cfg):
    p = cfg.p
    prob = _prob(lib, p)
    print(f"[config2 full tol] eps={p.eps:.5g}", flush=True)
    f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=1e-6, max_iter=20000))
    ref = sinkhorn.reduced_sinkhorn(cfg.alpha, cfg.beta, cfg.logK, p.eps, K, tol=1e-6)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1, (st, ref["iters"])
    fh, gh = _f64(f), _f64(g)
    # the last step, exactly, at sampled rows and columns
    I, J = _rows_cols(21)
    if st["iters"] > 1:
        _, gp, sp = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=st["iters"] - 1))
        g_prev = _f64(gp)
    else:
        g_prev = np.zeros(N)
    ef, eg = one_step_errors(cfg.data, g_prev, fh, gh, I, J)
    assert ef < POT and eg < POT, (ef, eg)
    # the float64 check value is the row residual of the returned state over all rows
    er = row_residual(cfg.data, fh, gh)
    assert st["err_row"] <= 1e-6 * 1.05
    assert abs(st["err_row"] - er) <= 1e-3 * er + 1e-12, (st["err_row"], er)
    # equal marginal error as the reduced solve, and the same objective (K P_red)
    v = lib.values_dict(lib.ot_cost_and_grad(prob, f, g, reduced=False)["values"])
    vr = objective.reduced_values(ref["f"], ref["g"], cfg.Ck, p.eps, cfg.alpha, cfg.beta)
    assert abs(v["P"] - K * vr["P"]) / (K * max(abs(vr["P"]), vr["CT"])) < REL


def _plan_rows(cfg, f, g, rows):
    """Oracle plan rows T[r m + i, :] of the expanded reduced plan (Lemma 1)."""
    Tk = sinkhorn.reduced_plan_blocks(f, g, cfg.Ck, cfg.p.eps)            # [K, m, m]
    m = cfg.m
    out = np.empty((len(rows), N))
    for t, I in enumerate(rows):
        r, i = divmod(int(I), m)
        for c in range(K):
            out[t, c * m:(c + 1) * m] = Tk[(c - r) % K, i]
    return out


def _compare_plan(T, Tref):
    l1 = np.abs(T - Tref).sum() / Tref.sum()
    big = Tref > 1e-3 * Tref.max()
    ent = (np.abs(T - Tref)[big] / Tref[big]).max()
    return l1, ent


def test_expand(lib, cfg):
    p = cfg.p
    m = cfg.m
    prob = _prob(lib, p)
    ref = sinkhorn.reduced_sinkhorn(cfg.alpha, cfg.beta, cfg.logK, p.eps, K, tol=1e-6)
    f32, g32 = ref["f"].astype(np.float32), ref["g"].astype(np.float32)
    rng = np.random.default_rng(31)
    rows = np.concatenate([r * m + np.sort(rng.choice(m, 64, replace=False)) for r in (0, 7, 15)])
    print(f"[config2 expand] eps={p.eps:.5g}", flush=True)
    # (1) the expand kernel from the oracle's (float32-rounded) potentials
    T = lib.ot_expand_plan(prob, _t(f32), _t(g32))
    torch.cuda.synchronize()
    # Lemma 1: block (r, c) is block (r+1, c+1): exact, as every copy is the same value
    assert torch.equal(T[m:, m:], T[:-m, :-m]) and torch.equal(T[m:, :m], T[:-m, N - m:])
    Tr = T[torch.as_tensor(rows, device=DEV)].cpu().numpy().astype(np.float64)
    l1, ent = _compare_plan(Tr, _plan_rows(cfg, _f64(f32), _f64(g32), rows))
    assert l1 < REL and ent < 2e-5, (l1, ent)
    # (2) end to end: fold, reduced solve and expand on the GPU against the oracle's plan,
    # at the oracle's stopping iteration (one iteration more or less moves the plan by about
    # the 1e-6 residual per row, beyond the 1e-5 L1 bar)
    opts = lib.make_opts(tol=0.0, max_iter=ref["iters"])
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    T = lib.ot_expand_plan(prob, f, g, out=T)
    Tr = T[torch.as_tensor(rows, device=DEV)].cpu().numpy().astype(np.float64)
    l1, ent = _compare_plan(Tr, _plan_rows(cfg, ref["f"], ref["g"], rows))
    print(f"[config2 expand] end-to-end plan L1 {l1:.2e}, entry-wise {ent:.2e}", flush=True)
    assert l1 < REL, l1


def _grad_ref(cfg, T, X, Y):
    """Oracle gradient rows 2 sum_J T_IJ (x_I - y_J) of sampled points and their error scale
    2 sum_J T_IJ |x_I - y_J| (per component), T given row by row ([rows, N]), X [rows, 2] the
    sampled points, Y [N, 2] their partners."""
    D = X[:, None, :] - Y[None, :, :]
    return 2.0 * np.einsum("ij,ijd->id", T, D), 2.0 * np.einsum("ij,ijd->id", T, np.abs(D))


def _full_plan_rows(cfg, f, g, rows):
    """Oracle rows of the full plan T_IJ = exp((f_I + g_J - C_IJ) / eps) on the given float32
    coordinates (float64 costs)."""
    C = cost.sq_euclidean(_f64(cfg.p.x)[rows], _f64(cfg.p.y))
    return np.exp((f[rows, None] + g[None, :] - C) / cfg.p.eps)


def test_gradients(lib, cfg):
    """Adjoint kernels at the benchmark's shape, both paths, on the oracle's converged
    potentials rounded to float32: dx at 3 x 64 sampled rows and dy at 3 x 64 sampled columns
    against the oracle's envelope gradient (2 sum_J T_IJ (x_I - y_J)) over all 8192 partners,
    dC (reduced: block-row 0, K T_ijk) and the mean-centred da, db.  Error model: every plan
    entry carries a float32 relative error (exponent and cost rounding), so a gradient
    component may be off by that relative error times 2 sum_J T_IJ |x_I - y_J|; the bar is
    2e-5 of that scale (twice the 1e-5 plan bar)."""
    p = cfg.p
    m = cfg.m
    prob = _prob(lib, p)
    ref = sinkhorn.reduced_sinkhorn(cfg.alpha, cfg.beta, cfg.logK, p.eps, K, tol=1e-6)
    f32, g32 = ref["f"].astype(np.float32), ref["g"].astype(np.float32)
    fh, gh = _f64(f32), _f64(g32)
    rng = np.random.default_rng(41)
    rows = np.concatenate([r * m + np.sort(rng.choice(m, 64, replace=False)) for r in (0, 5, 15)])
    cols = np.concatenate([c * m + np.sort(rng.choice(m, 64, replace=False)) for c in (0, 9, 15)])
    X, Y = _f64(p.x), _f64(p.y)
    for path in ("reduced", "full"):
        print(f"[config2 grad] eps={p.eps:.5g} {path}", flush=True)
        if path == "reduced":
            res = lib.ot_cost_and_grad(prob, _t(f32), _t(g32), True, want_dC=True, want_dxy=True,
                                       want_dab=True)
            Tr = _plan_rows(cfg, fh, gh, rows)
            # columns of the expanded plan are rows of its transpose: T[r m + i, c m + j] =
            # T_{ij,(c - r) mod K}, so column c m + j over r, i is Tk[(c - r) mod K][:, j]
            Tk = sinkhorn.reduced_plan_blocks(fh, gh, cfg.Ck, p.eps)
            Tc = np.empty((len(cols), N))
            for t, J in enumerate(cols):
                c, j = divmod(int(J), m)
                for r in range(K):
                    Tc[t, r * m:(r + 1) * m] = Tk[(c - r) % K][:, j]
            fa, gb = np.tile(fh, K), np.tile(gh, K)
        else:
            fa, gb = np.tile(fh, K), np.tile(gh, K)
            res = lib.ot_cost_and_grad(prob, _t(fa.astype(np.float32)), _t(gb.astype(np.float32)),
                                       False, want_dxy=True, want_dab=True)
            Tr = _full_plan_rows(cfg, fa, gb, rows)
            C = cost.sq_euclidean(X, Y[cols])
            Tc = np.exp((fa[:, None] + gb[None, cols] - C) / p.eps).T
        torch.cuda.synchronize()
        dx_want, dx_scale = _grad_ref(cfg, Tr, X[rows], Y)
        dy_want, dy_scale = _grad_ref(cfg, Tc, Y[cols], X)
        worst = 0.0
        for got, want, scale in ((res["dx"].cpu().numpy()[rows], dx_want, dx_scale),
                                 (res["dy"].cpu().numpy()[cols], dy_want, dy_scale)):
            ratio = np.abs(_f64(got) - want) / scale
            worst = max(worst, float(ratio.max()))
        print(f"[config2 grad] {path}: max |d grad| / (2 sum T |x - y|) = {worst:.2e}", flush=True)
        assert worst < 2e-5, worst
        # da, db: the potentials, tiled and mean-centred
        for got, want in ((res["da"], fa), (res["db"], gb)):
            assert np.abs(_f64(got.cpu()) - (want - want.mean())).max() <= 1e-6 * (1 + np.abs(want).max())
        if path == "reduced":
            dC = res["dC"][torch.as_tensor(rows[:64], device=DEV)].cpu().numpy()
            want = K * np.concatenate(list(Tk), axis=1)[rows[:64]]
            assert np.abs(_f64(dC) - want).sum() / want.sum() < REL
