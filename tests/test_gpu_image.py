"""GPU parity on image workloads (Example 1): pixel distances between images with mirror
(K = 2) or quarter-turn (K = 4) symmetry, through the dense-cost and point paths, against the
float64 oracle; and approximately symmetric images through the two-stage method."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, objective, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
REL = 1e-5


def T_(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _f64(v):
    return np.asarray(v, dtype=np.float64)


def _row0_prob(lib, p):
    if p.dim == 0:
        return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, C=T_(p.C_row0))
    return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))


@pytest.mark.parametrize("K,metric", [(2, "euclidean"), (4, "euclidean"), (4, "manhattan"),
                                      (2, "sqeuclidean")])
def test_symmetric_images_reduced_equals_full(lib, K, metric):
    """32 x 32 images (n = 1024): fold, reduced solve to 1e-6 and expand against the oracle;
    the full-size solve on the dense block-circulant cost stops at the same iteration with
    K times the reduced objective."""
    # squared pixel distances need a larger regulariser for a comparable C / eps range
    p = workloads.image_problem(32, K, metric, lam=25.0 if metric == "sqeuclidean" else 0.5)
    print(f"[image] {p.name}", flush=True)
    prob = _row0_prob(lib, p)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    if p.dim == 0:
        Ck = cost.blocks_from_row0(_f64(p.C_row0), K)
    else:
        Ck = cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, K), K)
    ref_logK = sinkhorn.fold_kernel(Ck, p.eps)
    assert (np.abs(logK.cpu().numpy() - ref_logK) / (np.abs(ref_logK) + 1.0)).max() < 2e-7
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    al, be = sinkhorn.fold_marginals(_f64(p.a), K), sinkhorn.fold_marginals(_f64(p.b), K)
    ref = sinkhorn.reduced_sinkhorn(al, be, ref_logK, p.eps, K, tol=1e-6, max_iter=20000)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 1
    vg = objective.reduced_values(_f64(f.cpu()), _f64(g.cpu()), Ck, p.eps, al, be)
    vr = objective.reduced_values(ref["f"], ref["g"], Ck, p.eps, al, be)
    assert abs(vg["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL
    T = lib.ot_expand_plan(prob, f, g).cpu().numpy().astype(np.float64)
    Tref = sinkhorn.expand_plan(_f64(f.cpu()), _f64(g.cpu()), Ck, p.eps)
    assert np.abs(T - Tref).sum() / Tref.sum() < REL
    # the full-size solver on the same problem (dense n x n cost, or the points)
    if p.dim == 0:
        Cfull = cost.block_circulant_from_row0(p.C_row0, K).astype(np.float32)
        fprob = lib.Problem(T_(p.a), T_(p.b), p.eps, K, C=T_(Cfull))
    else:
        fprob = prob
    ff, gf, stf = lib.ot_sinkhorn_full(fprob, lib.make_opts(tol=1e-6, max_iter=20000))
    assert stf["converged"] and abs(stf["iters"] - st["iters"]) <= 1
    C = cost.block_circulant_from_blocks(Ck)
    vf = objective.full_values(_f64(ff.cpu()), _f64(gf.cpu()), C, p.eps, _f64(p.a), _f64(p.b))
    assert abs(vf["P"] - K * vg["P"]) / max(abs(vf["P"]), vf["CT"]) < REL


def test_mirror_image_64_reduced_against_oracle(lib):
    """The 64 x 64 mirror workload (m = 2048: 256 workgroups, beyond one XCD) against the
    float64 reduced oracle at fixed iteration counts; to tolerance, the float64 check of the
    returned state."""
    p = workloads.image_problem(64, 2, "euclidean")
    prob = _row0_prob(lib, p)
    Ck = cost.blocks_from_row0(_f64(p.C_row0), 2)
    ref_logK = sinkhorn.fold_kernel(Ck, p.eps)
    al, be = sinkhorn.fold_marginals(_f64(p.a), 2), sinkhorn.fold_marginals(_f64(p.b), 2)
    for its in (1, 10):
        print(f"[image 64 mirror] iters={its}", flush=True)
        opts = lib.make_opts(tol=0.0, max_iter=its, fold_fp64=1)
        logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
        ref = sinkhorn.reduced_sinkhorn(al, be, ref_logK, p.eps, 2, tol=0.0, max_iter=its)
        assert st["iters"] == its
        assert np.abs(f.cpu().numpy() - ref["f"]).max() / p.eps < 2e-5
        assert np.abs(g.cpu().numpy() - ref["g"]).max() / p.eps < 2e-5
    print("[image 64 mirror] tol=1e-6", flush=True)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    logK, alpha, beta = lib.ot_fold_kernel(prob, opts)
    f, g, st = lib.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    assert st["converged"] and st["err_row"] <= 1e-6 * 1.05
    er, ec = sinkhorn.reduced_marginal_errors(_f64(f.cpu()), _f64(g.cpu()), ref_logK, p.eps,
                                              al, be, 2)
    assert er <= 1.1e-6 and ec <= 1.1e-6


@pytest.mark.parametrize("K,side", [(2, 32), (4, 24)])
def test_noisy_images_two_stage_reaches_the_full_solution(lib, K, side):
    """Approximately symmetric images (pixel noise 5 %): the two-stage method reaches the
    float64 full-size solution; the cyclic stage alone is the solution of the averaged
    problem, whose marginals differ from the given ones by the asymmetry."""
    p = workloads.image_problem(side, K, "euclidean", noise=0.05)
    print(f"[image two-stage] {p.name}", flush=True)
    Cfull = cost.block_circulant_from_row0(p.C_row0, K).astype(np.float32)
    prob = lib.Problem(T_(p.a), T_(p.b), p.eps, K, C=T_(Cfull))
    out = lib.two_stage_sinkhorn(prob, tol=1e-6)
    C = _f64(Cfull)
    ref = sinkhorn.full_sinkhorn(_f64(p.a), _f64(p.b), C, p.eps, tol=1e-6, max_iter=20000)
    assert out["stage1"]["converged"] and out["stage2"]["converged"]
    v = objective.full_values(_f64(out["f"].cpu()), _f64(out["g"].cpu()), C, p.eps, _f64(p.a),
                              _f64(p.b))
    vr = objective.full_values(ref["f"], ref["g"], C, p.eps, _f64(p.a), _f64(p.b))
    assert abs(v["P"] - vr["P"]) / max(abs(vr["P"]), vr["CT"]) < REL
    assert v["err_row"] <= 1e-6 * 1.05
