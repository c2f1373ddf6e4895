"""The allocation-free reduced solve (ot_sinkhorn_reduced_noalloc: the library's fixed device
scratch instead of a workspace argument) against the workspace entry point
ot_sinkhorn_reduced on the same inputs, two calls in a row, the second with a smaller problem
(so it runs on what the first left in the shared scratch), plus the float64 oracle (Alg. 2) on
each, and the host-side rejection of a problem whose plan needs more scratch than the array
holds."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
POT = 2e-5  # potentials: max |df| / eps, the exponent error of a plan entry (rel. 1e-5 bar)


def _t(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _case(lib, n, K, factor, seed):
    p = workloads.symmetric_problem(n, K, 2, factor, seed=seed)
    prob = lib.Problem(_t(p.a), _t(p.b), p.eps, K, x=_t(p.x), y=_t(p.y))
    logK, al, be = lib.ot_fold_kernel(prob, lib.make_opts(fold_fp64=1))
    return p, prob, logK, al, be


def _oracle(p, tol, max_iter):
    Ck = cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)
    alpha = sinkhorn.fold_marginals(p.a.astype(np.float64), p.K)
    beta = sinkhorn.fold_marginals(p.b.astype(np.float64), p.K)
    logK = sinkhorn.fold_kernel(Ck, p.eps)
    return sinkhorn.reduced_sinkhorn(alpha, beta, logK, p.eps, p.K, tol=tol, max_iter=max_iter)


@pytest.mark.parametrize("tol", [1e-6, 0.0], ids=["to_tol", "fixed_40"])
def test_noalloc_matches_workspace_call_twice(lib, tol):
    # first call: the benchmark's shape (m = 512, 32 workgroups); second: a smaller problem
    # (m = 100, ragged) on the same scratch
    for n, K, factor, seed in ((8192, 16, 0.01, 100), (400, 4, 0.05, 3)):
        print(f"[noalloc] n={n} K={K} eps={factor}*median tol={tol}", flush=True)
        p, prob, logK, al, be = _case(lib, n, K, factor, seed)
        m = p.m
        max_iter = 40 if tol == 0.0 else 100000
        opts = lib.make_opts(tol=tol, max_iter=max_iter)
        out_a = (torch.empty(m, device=DEV), torch.empty(m, device=DEV))
        out_b = (torch.empty(m, device=DEV), torch.empty(m, device=DEV))
        ds_a = torch.zeros(lib.OT_DSTATS_LEN, dtype=torch.float64, device=DEV)
        ds_b = torch.zeros(lib.OT_DSTATS_LEN, dtype=torch.float64, device=DEV)
        fa, ga, sa = lib.ot_sinkhorn_reduced(prob, logK, al, be, opts, out=out_a, dstats=ds_a)
        fb, gb, sb = lib.ot_sinkhorn_reduced_noalloc(prob, logK, al, be, opts, out=out_b,
                                                     dstats=ds_b)
        torch.cuda.synchronize()
        assert sb["iters"] == sa["iters"] and sb["converged"] == sa["converged"], (sa, sb)
        fa, ga, fb, gb = (v.cpu().numpy().astype(np.float64) for v in (fa, ga, fb, gb))
        d = max(np.abs(fa - fb).max(), np.abs(ga - gb).max()) / p.eps
        assert d < POT, d
        assert abs(sb["err_row"] - sa["err_row"]) <= 1e-6 * max(sa["err_row"], 1e-12) + 1e-15
        # the float64 oracle at the same iteration count
        ref = _oracle(p, tol, max_iter)
        assert abs(sb["iters"] - ref["iters"]) <= 1, (sb["iters"], ref["iters"])
        if sb["iters"] == ref["iters"]:
            e = max(np.abs(fb - ref["f"]).max(), np.abs(gb - ref["g"]).max()) / p.eps
            assert e < POT, e


def test_noalloc_rejects_a_plan_beyond_its_scratch(lib):
    # m = 4096 keeps its logK slabs in device memory (32 MiB of padded copies): far beyond the
    # fixed scratch, so the call must refuse before launching anything
    p = workloads.symmetric_problem(8192, 2, 2, 0.05, seed=5)
    prob = lib.Problem(_t(p.a), _t(p.b), p.eps, 2, x=_t(p.x), y=_t(p.y))
    m = p.m
    z = torch.zeros((m, m), device=DEV)
    v = torch.full((m,), 1.0 / 8192, device=DEV)
    with pytest.raises(lib.CsotError) as ei:
        lib.ot_sinkhorn_reduced_noalloc(prob, z, v, v, lib.make_opts())
    assert "OT_ERR_UNSUPPORTED" in str(ei.value) and "scratch" in str(ei.value)
