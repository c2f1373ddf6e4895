"""torch.autograd.Function wrappers around the C ABI.

CyclicOT.apply(x, y, a, b, eps, K) -> OT_eps (scalar, float64 tensor) of the FULL n x n
problem, solved through the cyclic reduction (fold -> reduced Sinkhorn), i.e. the primal value
<C, T> + eps sum T (log T - 1) of eq. problem_ROT with eq. reg_for_entropy_ROT, which equals K
times the reduced objective (eq. problem_CROT).  backward calls the hand-written adjoint
kernels of ot_cost_and_grad on the saved converged potentials and returns grad_output times
(dx, dy, da, db); the gradients are the envelope theorem applied to the dual (exact at the
optimum; da, db are mean-centred because a, b live on the simplex).

CyclicOTCost.apply(C_row0, a, b, eps, K) is the dense-cost variant: its input is block-row 0
of a block-circulant cost ([m, n], block k = C_k), each entry of which appears once in every
block-row of the full cost, so dOT/dC_row0[i, k m + j] = K T_ijk -- the library's dC output
for reduced potentials.
"""
from __future__ import annotations

import torch

from . import _binding as B


def _solve_reduced(prob, tol, max_iter, fold_fp64):
    opts = B.make_opts(tol=tol, max_iter=max_iter, fold_fp64=fold_fp64)
    logK, alpha, beta = B.ot_fold_kernel(prob, opts)
    f, g, st = B.ot_sinkhorn_reduced(prob, logK, alpha, beta, opts)
    return f, g, st


class CyclicOT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, a, b, eps, K, tol=1e-6, max_iter=10000, fold_fp64=-1):
        x_, y_, a_, b_ = (t.detach().contiguous().float() for t in (x, y, a, b))
        prob = B.Problem(a_, b_, float(eps), int(K), x=x_, y=y_)
        f, g, st = _solve_reduced(prob, tol, max_iter, fold_fp64)
        res = B.ot_cost_and_grad(prob, f, g, reduced=True)
        ctx.save_for_backward(x_, y_, a_, b_, f, g)
        ctx.eps, ctx.K = float(eps), int(K)
        ctx.stats = st
        return res["values"][0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        x_, y_, a_, b_, f, g = ctx.saved_tensors
        prob = B.Problem(a_, b_, ctx.eps, ctx.K, x=x_, y=y_)
        res = B.ot_cost_and_grad(prob, f, g, reduced=True, want_dxy=True, want_dab=True)
        go = grad_out.to(torch.float32)
        return (go * res["dx"], go * res["dy"], go * res["da"], go * res["db"],
                None, None, None, None, None)


class FullOT(torch.autograd.Function):
    """Same value and gradients through plain full-size Sinkhorn (the baseline)."""

    @staticmethod
    def forward(ctx, x, y, a, b, eps, K=1, tol=1e-6, max_iter=10000):
        x_, y_, a_, b_ = (t.detach().contiguous().float() for t in (x, y, a, b))
        prob = B.Problem(a_, b_, float(eps), int(K), x=x_, y=y_)
        f, g, st = B.ot_sinkhorn_full(prob, B.make_opts(tol=tol, max_iter=max_iter))
        res = B.ot_cost_and_grad(prob, f, g, reduced=False)
        ctx.save_for_backward(x_, y_, a_, b_, f, g)
        ctx.eps, ctx.K = float(eps), int(K)
        ctx.stats = st
        return res["values"][0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        x_, y_, a_, b_, f, g = ctx.saved_tensors
        prob = B.Problem(a_, b_, ctx.eps, ctx.K, x=x_, y=y_)
        res = B.ot_cost_and_grad(prob, f, g, reduced=False, want_dxy=True, want_dab=True)
        go = grad_out.to(torch.float32)
        return (go * res["dx"], go * res["dy"], go * res["da"], go * res["db"],
                None, None, None, None)


class CyclicOTCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C_row0, a, b, eps, K, tol=1e-6, max_iter=10000, fold_fp64=-1):
        C_, a_, b_ = (t.detach().contiguous().float() for t in (C_row0, a, b))
        prob = B.Problem(a_, b_, float(eps), int(K), C=C_)
        f, g, st = _solve_reduced(prob, tol, max_iter, fold_fp64)
        res = B.ot_cost_and_grad(prob, f, g, reduced=True)
        ctx.save_for_backward(C_, a_, b_, f, g)
        ctx.eps, ctx.K = float(eps), int(K)
        ctx.stats = st
        return res["values"][0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        C_, a_, b_, f, g = ctx.saved_tensors
        prob = B.Problem(a_, b_, ctx.eps, ctx.K, C=C_)
        res = B.ot_cost_and_grad(prob, f, g, reduced=True, want_dC=True, want_dab=True)
        go = grad_out.to(torch.float32)
        return (go * res["dC"], go * res["da"], go * res["db"], None, None, None, None, None)
