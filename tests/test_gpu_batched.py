"""GPU tests of the batched path (many uneven reduced problems in one launch sequence).

Each problem of a batch must equal its own unbatched solve (same C ABI, same stopping rule)
and the float64 oracle; the batched launch sequence must replay correctly from a HIP graph.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, objective, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problems(shapes):
    out = []
    for m, K, dim, seed in shapes:
        p = workloads.symmetric_problem(m * K, K, dim, 0.05, seed=seed)
        out.append(dict(x=p.x, y=p.y, a=p.a, b=p.b, eps=p.eps, K=p.K, _p=p))
    return out


SMALL = [(8, 4, 2, 1), (33, 3, 3, 2), (64, 8, 2, 3), (100, 2, 2, 4), (150, 4, 3, 5),
         (257, 8, 2, 6), (31, 16, 2, 7), (128, 32, 3, 8), (5, 5, 2, 9), (200, 4, 2, 10),
         (96, 6, 3, 11), (520, 2, 2, 12)]


def _oracle(p):
    Ck = cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)
    r = sinkhorn.cyclic_sinkhorn(p.a.astype(np.float64), p.b.astype(np.float64), Ck, p.eps,
                                 tol=1e-6)
    v = objective.reduced_values(r["f"], r["g"], Ck, p.eps, r["alpha"], r["beta"])
    return r, v, Ck


def test_batched_equals_unbatched_and_oracle(lib):
    probs = _problems(SMALL)
    print(f"[batched small] {len(probs)} problems", flush=True)
    batch = lib.Batch(probs, device=DEV)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    batch.run(opts)
    torch.cuda.synchronize()
    for k, pr in enumerate(probs):
        p = pr["_p"]
        t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
        prob = lib.Problem(t(p.a), t(p.b), p.eps, p.K, x=t(p.x), y=t(p.y))
        logK, al, be = lib.ot_fold_kernel(prob, opts)
        f, g, st = lib.ot_sinkhorn_reduced(prob, logK, al, be, opts)
        res = lib.ot_cost_and_grad(prob, f, g, reduced=True, want_dxy=True)
        vu = lib.values_dict(res["values"])
        vb = batch.values(k)
        assert vb["converged"] and vb["flags"] == 0, (k, vb)
        assert abs(vb["iters"] - st["iters"]) <= 1, (k, vb["iters"], st["iters"])
        scale = max(abs(vu["P"]), vu["CT"])
        assert abs(vb["P"] - vu["P"]) / scale < 1e-5, (k, vb["P"], vu["P"])
        assert abs(vb["D"] - vu["D"]) / scale < 1e-5
        assert vb["err_row"] <= 1.05e-6
        m = p.m
        for got, want in ((batch.dx(k), res["dx"][:m]), (batch.dy(k), res["dy"][:m])):
            got, want = got.cpu().numpy(), want.cpu().numpy()
            assert np.abs(got - want).max() / np.abs(want).max() < 1e-4, k
        # the oracle
        r, v, Ck = _oracle(p)
        assert abs(vb["iters"] - r["iters"]) <= 1
        assert abs(vb["P"] - p.K * v["P"]) / max(abs(p.K * v["P"]), p.K * v["CT"]) < 1e-5
        Tg = sinkhorn.reduced_plan_blocks(batch.f(k).cpu().numpy().astype(np.float64),
                                          batch.g(k).cpu().numpy().astype(np.float64), Ck, p.eps)
        Tr = sinkhorn.reduced_plan_blocks(r["f"], r["g"], Ck, p.eps)
        assert np.abs(Tg - Tr).sum() / Tr.sum() < 1e-5, k


def test_batched_full_workload_sampled(lib):
    """The uneven workload: 1024 problems, m log-uniform in [32, 1024], K in {4, 8, 16, 32},
    2-D or 3-D, eps = 0.05 median(C) each; every problem converges, sampled problems match
    the float64 oracle."""
    items = workloads.batched_problems(1024)
    probs = [dict(x=p.x, y=p.y, a=p.a, b=p.b, eps=p.eps, K=p.K, _p=p)
             for p in (workloads.symmetric_problem(it.m * it.K, it.K, it.dim, 0.05, seed=it.seed)
                       for it in items)]
    print(f"[batched full] {len(probs)} problems, sum m^2 = {sum(p['_p'].m ** 2 for p in probs)}",
          flush=True)
    batch = lib.Batch(probs, device=DEV)
    opts = lib.make_opts(tol=1e-6, max_iter=20000)
    batch.run(opts)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.run(opts)
    e1.record()
    torch.cuda.synchronize()
    out = batch.OUT.cpu().numpy()
    print(f"[batched full] {e0.elapsed_time(e1):.3f} ms for {len(probs)} problems; iterations "
          f"min/median/max = {out[:, 5].min():.0f}/{np.median(out[:, 5]):.0f}/{out[:, 5].max():.0f}",
          flush=True)
    assert (out[:, 6] == 1).all() and (out[:, 7] == 0).all()
    assert (out[:, 3] <= 1.05e-6).all()
    rng = np.random.default_rng(0)
    for k in rng.choice(len(probs), size=6, replace=False):
        p = probs[k]["_p"]
        r, v, Ck = _oracle(p)
        vb = batch.values(int(k))
        assert abs(vb["iters"] - r["iters"]) <= 1, (k, vb["iters"], r["iters"])
        assert abs(vb["P"] - p.K * v["P"]) / max(abs(p.K * v["P"]), p.K * v["CT"]) < 1e-5, k


def test_batched_graph_replay(lib):
    """The batched launch sequence captured once and replayed several times, with eager work
    and synchronisation between replays; every replay reproduces the eager result."""
    probs = _problems(SMALL[:8])
    print("[batched graph] capture + 3 replays", flush=True)
    batch = lib.Batch(probs, device=DEV)
    opts = lib.make_opts(tol=1e-6, max_iter=5000)
    batch.run(opts)
    torch.cuda.synchronize()
    ref_out = batch.OUT.clone()
    ref_f, ref_g, ref_dx = batch.F.clone(), batch.G.clone(), batch.DX.clone()
    graph = batch.capture(opts)
    for rep in range(3):
        batch.OUT.zero_()
        batch.F.fill_(7.0)
        batch.G.zero_()
        batch.DX.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.F, ref_f), rep
        assert torch.equal(batch.G, ref_g), rep
        assert torch.equal(batch.DX, ref_dx), rep
        # float64 sums use atomics (order may differ): compare to rounding
        assert torch.allclose(batch.OUT, ref_out, rtol=1e-12, atol=1e-15), rep
