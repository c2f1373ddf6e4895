"""Two-stage Sinkhorn for approximately symmetric data (Alg. 3): marshalling only, every step
runs in the library's kernels.

Stage 1 solves the symmetrized problem -- the block-circulant projection of the cost
(ot_symmetrize_cost, the averaging over the K shifts) with the marginals averaged over the K
blocks by the fold -- on the reduced m x m problem.  Stage 2 runs plain full-size Sinkhorn on the
data as given, started from the stage-1 column potential tiled K times (warm_start = 2: the
reduced solver writes its g straight into the first m entries of the full-size g, and the
full-size solver tiles it on the device).  Both stages stop on the same full-space L2 row
residual; stage 1 may use a looser tolerance, since only stage 2 decides the result.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _binding as B


def two_stage_sinkhorn(prob: B.Problem, tol: float = 1e-6, max_iter: int = 20000,
                       tol_stage1: Optional[float] = None, out=None) -> dict:
    """-> {"f", "g": the stage-2 solution ([n] each), "stage1", "stage2": the host statistics
    of the two solves}.

    prob: a point-cloud (dim 2/3) or dense full-size problem, n = K m."""
    n, m, K = prob.n, prob.m, prob.K
    dev = prob.device
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev))
    f, g = out
    # stage 1: projection, fold (marginals averaged over the blocks), reduced solve
    csym = B.ot_symmetrize_cost(prob)                       # [m, n], block-row 0
    sprob = B.Problem(prob.a, prob.b, prob.eps, K, C=csym)
    o1 = B.make_opts(tol=tol if tol_stage1 is None else tol_stage1, max_iter=max_iter,
                     fold_fp64=1)
    logK, alpha, beta = B.ot_fold_kernel(sprob, o1)
    fr = torch.empty(m, dtype=torch.float32, device=dev)
    _, _, st1 = B.ot_sinkhorn_reduced(sprob, logK, alpha, beta, o1, out=(fr, g[:m]))
    # stage 2: full-size Sinkhorn on the given data from the tiled stage-1 potential
    o2 = B.make_opts(tol=tol, max_iter=max_iter, warm_start=2)
    _, _, st2 = B.ot_sinkhorn_full(prob, o2, out=(f, g))
    return {"f": f, "g": g, "stage1": st1, "stage2": st2}
