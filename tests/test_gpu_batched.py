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


def _check_grads(batch, k, p, Ck, rows=None):
    """The batched gradients of problem k against the oracle's envelope gradients of the
    expanded plan (Lemma 1) built from the batch's own potentials: dx, dy of every point (or
    of the sampled `rows` of the expanded plan, and as many sampled columns), da, db.  Error
    model as for the single-problem adjoint: each plan entry carries a float32 relative error,
    so a component may be off by that error times 2 sum_J T_IJ |x_I - y_J|; bar 2e-5 of it."""
    f = batch.f(k).cpu().numpy().astype(np.float64)
    g = batch.g(k).cpu().numpy().astype(np.float64)
    X, Y = p.x.astype(np.float64), p.y.astype(np.float64)
    n, m, K = p.n, p.m, p.K
    Tk = sinkhorn.reduced_plan_blocks(f, g, Ck, p.eps)                   # [K, m, m]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    worst = 0.0
    for key, pts, other in (("dx", X, Y), ("dy", Y, X)):
        got = (batch.dx(k) if key == "dx" else batch.dy(k)).cpu().numpy().astype(np.float64)
        for I in rows:
            r, i = divmod(int(I), m)
            # row I of the plan (dx) or column I (dy): blocks (r, c) hold T_{(c - r) mod K}
            if key == "dx":
                t = np.concatenate([Tk[(c - r) % K][i] for c in range(K)])
            else:
                t = np.concatenate([Tk[(r - c) % K][:, i] for c in range(K)])
            D = pts[I][None, :] - other
            want = 2.0 * (t[:, None] * D).sum(0)
            scale = 2.0 * (t[:, None] * np.abs(D)).sum(0)
            worst = max(worst, float((np.abs(got[I] - want) / scale).max()))
    fa, gb = np.tile(f, K), np.tile(g, K)
    for got, want in ((batch.da(k), fa), (batch.db(k), gb)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.abs(got - (want - want.mean())).max() <= 1e-6 * (1 + np.abs(want).max()), k
    return worst


def _check_plan_at_gpu_iterations(batch, k, p, Ck, r, iters):
    """The reduced plan from the batch's potentials against the oracle's after the same number
    of iterations (a stop one iteration apart moves the plan by about the 1e-6 residual per
    row, which is the size of the 1e-5 L1 bar)."""
    if iters != r["iters"]:
        r = sinkhorn.reduced_sinkhorn(r["alpha"], r["beta"], r["logK"], p.eps, p.K, tol=0.0,
                                      max_iter=iters)
    Tg = sinkhorn.reduced_plan_blocks(batch.f(k).cpu().numpy().astype(np.float64),
                                      batch.g(k).cpu().numpy().astype(np.float64), Ck, p.eps)
    Tr = sinkhorn.reduced_plan_blocks(r["f"], r["g"], Ck, p.eps)
    l1 = np.abs(Tg - Tr).sum() / Tr.sum()
    assert l1 < 1e-5, (k, l1, iters)


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
        res = lib.ot_cost_and_grad(prob, f, g, reduced=True)
        vu = lib.values_dict(res["values"])
        vb = batch.values(k)
        assert vb["converged"] and vb["flags"] == 0, (k, vb)
        assert abs(vb["iters"] - st["iters"]) <= 1, (k, vb["iters"], st["iters"])
        scale = max(abs(vu["P"]), vu["CT"])
        assert abs(vb["P"] - vu["P"]) / scale < 1e-5, (k, vb["P"], vu["P"])
        assert abs(vb["D"] - vu["D"]) / scale < 1e-5
        assert vb["err_row"] <= 1.05e-6
        # the oracle
        r, v, Ck = _oracle(p)
        worst = _check_grads(batch, k, p, Ck)
        print(f"[batched small] problem {k} (m={p.m}, K={p.K}, dim={p.dim}): gradients "
              f"max |d| / scale = {worst:.2e}", flush=True)
        assert worst < 2e-5, (k, worst)
        assert abs(vb["iters"] - r["iters"]) <= 1
        assert abs(vb["P"] - p.K * v["P"]) / max(abs(p.K * v["P"]), p.K * v["CT"]) < 1e-5
        _check_plan_at_gpu_iterations(batch, k, p, Ck, r, vb["iters"])


def test_batched_values_only_equals_with_gradients(lib):
    """A batch that asks for no gradients takes value tiles of 16 points with the column sums
    fused into the row pass (a different kernel path): same potentials, iterations and values
    as the batch with gradients.  The float64 sums differ only in their order, except two:
    the primal value (the gradient path accumulates T (f + g - eps) in float32 partials, the
    values-only path forms the same sum as sum_i (f_i - eps) rowsum_i + sum_j g_j colsum_j
    from the float64 marginal sums) and <C, T> (float32 partials in both, over the K shifts of
    one partner on the matrix-core gradient path, over every chunk and shift of a lane on the
    values-only path): these agree to float32 accumulation (1e-7)."""
    probs = _problems(SMALL)
    print("[batched values only] 12 problems", flush=True)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    bg = lib.Batch(probs, device=DEV)
    bv = lib.Batch(probs, device=DEV, want_grad=False)
    bg.run(opts)
    bv.run(opts)
    torch.cuda.synchronize()
    assert torch.equal(bg.F, bv.F) and torch.equal(bg.G, bv.G)
    og, ov = bg.OUT.cpu().numpy(), bv.OUT.cpu().numpy()
    assert (og[:, 5:] == ov[:, 5:]).all()
    for k in range(len(probs)):
        scale = max(abs(og[k, 0]), og[k, 2])
        assert abs(og[k, 0] - ov[k, 0]) <= 1e-7 * scale, k
        assert abs(og[k, 1] - ov[k, 1]) <= 1e-9 * scale, k
        assert abs(og[k, 2] - ov[k, 2]) <= 1e-7 * og[k, 2], k
        assert abs(og[k, 3] - ov[k, 3]) <= 1e-6 * og[k, 3] + 1e-15, k
        assert abs(og[k, 4] - ov[k, 4]) <= 1e-6 * og[k, 4] + 1e-15, k


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
    # six random problems, plus the largest K = 32 problems in 2-D and 3-D (the adjoint's
    # two-group case)
    pick = list(rng.choice(len(probs), size=6, replace=False))
    for dim in (2, 3):
        cand = [q for q in range(len(probs)) if probs[q]["_p"].K == 32 and probs[q]["_p"].dim == dim]
        pick.append(max(cand, key=lambda q: probs[q]["_p"].m))
    for k in pick:
        k = int(k)
        p = probs[k]["_p"]
        r, v, Ck = _oracle(p)
        vb = batch.values(k)
        assert abs(vb["iters"] - r["iters"]) <= 1, (k, vb["iters"], r["iters"])
        scale = max(abs(p.K * v["P"]), p.K * v["CT"])
        assert abs(vb["P"] - p.K * v["P"]) / scale < 1e-5, k
        assert abs(vb["D"] - p.K * v["D"]) / scale < 1e-5, k
        _check_plan_at_gpu_iterations(batch, k, p, Ck, r, vb["iters"])
        # gradients at 3 x 16 sampled rows / columns of the expanded plan
        rows = np.concatenate([c * p.m + rng.choice(p.m, min(16, p.m), replace=False)
                               for c in (0, p.K // 2, p.K - 1)])
        worst = _check_grads(batch, k, p, Ck, rows)
        print(f"[batched full] problem {k} (m={p.m}, K={p.K}, dim={p.dim}): iterations "
              f"{vb['iters']}, gradients max |d| / scale = {worst:.2e}", flush=True)
        assert worst < 2e-5, (k, worst)


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
    ref_f, ref_g, ref_dx, ref_db = batch.F.clone(), batch.G.clone(), batch.DX.clone(), batch.DB.clone()
    graph = batch.capture(opts)
    for rep in range(3):
        batch.OUT.zero_()
        batch.F.fill_(7.0)
        batch.G.zero_()
        batch.DX.fill_(-1.0)
        batch.DB.fill_(3.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.F, ref_f), rep
        assert torch.equal(batch.G, ref_g), rep
        assert torch.equal(batch.DX, ref_dx), rep
        assert torch.equal(batch.DB, ref_db), rep
        # float64 sums use atomics (order may differ): compare to rounding
        assert torch.allclose(batch.OUT, ref_out, rtol=1e-12, atol=1e-15), rep


def test_batched_launch_knobs(lib):
    """The two tuned launch knobs change only how the work is cut: the fold's columns per
    tile (64, 128, 256, 512) leave every folded entry, hence the potentials and iteration counts,
    bit for bit unchanged; the lanes per row of the solve (16, 32, 64) reorder the log-sum-exp
    sums only, so the potentials agree to float32 rounding and the values to 1e-6."""
    probs = _problems(SMALL + [(600, 4, 2, 13), (1000, 8, 3, 14)])
    print("[batched knobs] fold widths and lanes per row", flush=True)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    b = lib.Batch(probs, device=DEV, want_grad=False, tile_cfg=[32] * len(probs))
    b.run(opts)
    torch.cuda.synchronize()
    F0, G0, O0 = b.F.clone(), b.G.clone(), b.OUT.cpu().numpy()
    for cols in (64, 128, 512):
        b.set_tile_cfg([32 | (cols // 64) << 8] * len(probs))
        b.run(opts)
        torch.cuda.synchronize()
        assert torch.equal(b.F, F0) and torch.equal(b.G, G0), cols
        assert (b.OUT.cpu().numpy()[:, 5:] == O0[:, 5:]).all(), cols
    scale = float(max(F0.abs().max(), G0.abs().max()))
    for lanes in (16, 64):
        b.set_tile_cfg([lanes] * len(probs))
        b.run(opts)
        torch.cuda.synchronize()
        O = b.OUT.cpu().numpy()
        assert np.abs(O[:, 5] - O0[:, 5]).max() <= 1, lanes
        assert float((b.F - F0).abs().max()) <= 2e-5 * scale, lanes
        assert float((b.G - G0).abs().max()) <= 2e-5 * scale, lanes
        rel = np.abs(O[:, 0] - O0[:, 0]) / np.maximum(np.abs(O0[:, 0]), O0[:, 2])
        assert rel.max() <= 1e-6, (lanes, rel.max())


def test_batched_degenerate_sizes(lib):
    """Blocks of one and two points (m = 1: every point its own block, the reduced problem
    1 x 1; m = 2), K = 1 (no symmetry used) and K = 2, with and without gradients, against the
    float64 oracle: potentials, values and the marginal errors the call reports.  The solver
    stops on its float32 view of the row residual (<= 1e-6); the reported float64 residual
    differs from it by the float32 rounding of the folded kernel, which a handful of entries
    does not average out (up to ~1e-6 here), hence the 2e-6 bound."""
    shapes = [(1, 8, 2, 21), (2, 4, 3, 22), (40, 1, 2, 23), (3, 2, 2, 24), (1, 32, 3, 25),
              (130, 1, 3, 26)]
    probs = _problems(shapes)
    print("[batched degenerate] m = 1, 2, 3, 130 and K = 1", flush=True)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    for want_grad in (True, False):
        batch = lib.Batch(probs, device=DEV, want_grad=want_grad)
        batch.run(opts)
        torch.cuda.synchronize()
        out = batch.OUT.cpu().numpy()
        for k, q in enumerate(probs):
            p = q["_p"]
            r, v, Ck = _oracle(p)
            assert out[k, 6] == 1, (k, want_grad)
            assert out[k, 3] <= 2e-6 and out[k, 4] <= 2e-6, (k, out[k, 3:5])
            P, CT = p.K * v["P"], p.K * v["CT"]
            assert abs(out[k, 0] - P) <= 1e-5 * max(abs(P), CT), (k, want_grad)
            f = batch.f(k).cpu().numpy().astype(np.float64)
            g = batch.g(k).cpu().numpy().astype(np.float64)
            # potentials are defined up to f + c, g - c: compare f + g pairs and f - f[0]
            s = max(np.abs(r["f"]).max(), np.abs(r["g"]).max(), p.eps)
            assert np.abs((f[:, None] + g[None, :]) - (r["f"][:, None] + r["g"][None, :])).max() <= 2e-4 * s, k
            if want_grad:
                # every gradient tile shape: one point, a partial tile, K = 1 and 2, three tiles
                # of 64 own points with a ragged tail (m = 130)
                worst = _check_grads(batch, k, p, Ck)
                assert worst < 2e-5, (k, worst)


def test_batched_single_problem_and_large_block(lib):
    """A batch of one problem, and a batch mixing a block of m = 2000 (a gang of 16
    workgroups, logK streamed) with small ones: iterations, potentials' plan and value against
    the float64 oracle."""
    print("[batched one / large] count 1, m = 2000 in a mixed batch", flush=True)
    opts = lib.make_opts(tol=1e-6, max_iter=20000, fold_fp64=1)
    for shapes in ([(300, 4, 2, 41)], [(2000, 2, 2, 42), (20, 4, 3, 43), (70, 8, 2, 44)]):
        probs = _problems(shapes)
        batch = lib.Batch(probs, device=DEV)
        batch.run(opts)
        torch.cuda.synchronize()
        out = batch.OUT.cpu().numpy()
        for k, q in enumerate(probs):
            p = q["_p"]
            r, v, Ck = _oracle(p)
            assert out[k, 6] == 1 and out[k, 3] <= 1.05e-6, (shapes[k], out[k])
            assert abs(out[k, 5] - r["iters"]) <= 1, (shapes[k], out[k, 5], r["iters"])
            P, CT = p.K * v["P"], p.K * v["CT"]
            assert abs(out[k, 0] - P) <= 1e-5 * max(abs(P), CT), shapes[k]
            _check_plan_at_gpu_iterations(batch, k, p, Ck, r, int(out[k, 5]))
