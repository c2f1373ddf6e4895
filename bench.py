"""Benchmark: cyclic (reduced) vs plain full-size entropic-OT Sinkhorn on one MI355X.

Workload: n = 8192 points per side, cyclic order K = 16 (m = 512), 2-D K-fold rotationally
symmetric point clouds (area-uniform annulus r in [0.5, 1]), squared Euclidean cost recomputed
on the fly from float32 coordinates, a and b = Dirichlet(1) blocks tiled K times,
eps = 0.01 * median(C), stopping tolerance 1e-6 on the full-space L2 row-marginal residual.
Synthetic, seeded (seed 100); inputs are resident in HBM before the timed region.

One step = one pass of the whole path on that input:
  reduced : fold (float64 log-sum) -> Sinkhorn to 1e-6 -> expand to the n x n plan ->
            objective + gradients (dx, dy, da, db);
            plus a fixed-count reduced solve (tol = 0, --fixed-reduced iterations);
  full    : plain full-size Sinkhorn to 1e-6 -> objective + gradients;
            plus a fixed-count full solve (tol = 0, --fixed-full iterations);
  eps 0.1 : reduced and full solves to 1e-6 at eps = 0.1 median(C);
  approximate symmetry (n = 16384, K = 32, jittered points, noisy marginals): the plain
            full-size solve from g = 0 and the two-stage method (projection of the cost,
            cyclic solve of the averaged problem, full-size solve from its tiled potential);
  n = 4096, K = 8 : forward + backward (solve to 1e-6, values, all gradients), reduced and
            full, replayed from graphs;
  batched : one call on 1024 uneven cyclic problems (fold, solve, values, gradients).
`value` is the reduced Sinkhorn iteration rate (iterations / second) of the fixed-count legs;
the time-to-tolerance and the full-size rates are reported beside it.  All timing uses HIP
events on the stream the kernels run on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N, K, DIM, SEED, EPS_FACTOR, TOL = 8192, 16, 2, 100, 0.01, 1e-6
EPS_FACTOR_2 = 0.1  # the workload's second regulariser (time to tolerance only)
# Algorithmic work per (I, J) entry of a full-size half-step, counted as the operation count
# of its definition: one exponential plus the flops around it -- dim subtractions, dim
# multiply-adds for the squared distance, the scale by 1/eps, the potential add and the
# accumulation (dim 2: 1 + 7 = 8; dim 3: 1 + 9 = 10).  The published fp32 vector peak of
# MI355X (157.3 TFLOP/s) counts packed FMAs as 4 flops per lane and cycle; the non-packed peak
# (this build emits no packed FP32 instructions) and the measured issue ceiling of this exact
# instruction mix are reported beside it.
OPS_PER_ENTRY = {2: 8, 3: 10}
PUBLISHED_FP32_TFLOPS = 157.3
NON_PACKED_FP32_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = "profiles/sinkhorn_n8192_K16_kernel_stats.md"


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fixed-reduced", type=int, default=1000)
    ap.add_argument("--fixed-full", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batched", action="store_true",
                    help="only time the batched workload (1024 uneven cyclic problems) and exit")
    ap.add_argument("--batched-calls", action="store_true",
                    help="only the batched calls, with and without gradients (no full-size "
                         "comparison): a short program for counter runs")
    ap.add_argument("--two-stage", action="store_true",
                    help="only the approximate-symmetry workload: cold full vs two-stage")
    ap.add_argument("--images", action="store_true",
                    help="only the image workloads (64 x 64 and 96 x 96 pixels, mirror K=2 and quarter-turn "
                         "K=4, pixel Euclidean distance, lambda 0.5): cyclic vs full")
    ap.add_argument("--lot", action="store_true",
                    help="only the cyclic linear OT steps on the GPU (min-fold, plan scatter) at "
                         "n=8192, K=16")
    ap.add_argument("--srot", action="store_true",
                    help="only the quadratically regularised problem (cyclic vs full, n=8192, "
                         "K=16)")
    ap.add_argument("--peaks", action="store_true",
                    help="only run the device micro-benchmarks (issue rates of fp32/fp64 FMA and "
                         "exp2, the full-size entry mix, copy bandwidth, slot latencies) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (the reference kernel "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE) and exit")
    return ap.parse_args()


class BatchedLeg:
    """The batched workload: 1024 cyclic problems, m log-uniform in [32, 1024], K in
    {4, 8, 16, 32}, 2-D or 3-D, eps = 0.05 median each, tol 1e-6.  One call: fold, solve,
    objective values and the gradients (every point, both marginals) of all of them; the same
    call without gradients (forward only) and the plain method -- each problem solved at full
    size, one after another, with values and the same gradients -- are timed beside it."""

    def __init__(self):
        import torch

        import paper_2311_13147_amd as csot
        import workloads

        self.items = workloads.batched_problems(1024)
        self.probs = [dict(x=p.x, y=p.y, a=p.a, b=p.b, eps=p.eps, K=p.K)
                      for p in (workloads.symmetric_problem(it.m * it.K, it.K, it.dim, 0.05,
                                                            seed=it.seed)
                                for it in self.items)]
        self.batch = csot.Batch(self.probs, device="cuda:0")
        self.batch_fwd = csot.Batch(self.probs, device="cuda:0", want_grad=False)
        self.opts = csot.make_opts(tol=1e-6, max_iter=20000)
        self.csot, self.torch = csot, torch

    def run(self):
        self.batch.run(self.opts)

    def report(self, ms_call, steps):
        import numpy as np

        csot, torch = self.csot, self.torch
        E = lambda: torch.cuda.Event(enable_timing=True)
        out = self.batch.OUT.cpu().numpy()
        # the solve kernel alone, timed by events the library records right around its launch
        sev = (E(), E())
        opts_ev = csot.make_opts(tol=1e-6, max_iter=20000, timing_events=sev)
        solve_ms = []
        for _ in range(steps):
            self.batch.run(opts_ev)
            torch.cuda.synchronize()
            solve_ms.append(sev[0].elapsed_time(sev[1]))
        solve_ms = sum(solve_ms) / steps
        # forward only (values, no gradients)
        self.batch_fwd.run(self.opts)
        torch.cuda.synchronize()
        e0, e1 = E(), E()
        e0.record()
        for _ in range(steps):
            self.batch_fwd.run(self.opts)
        e1.record()
        torch.cuda.synchronize()
        fwd_ms = e0.elapsed_time(e1) / steps
        # Algorithmic bytes of the solve: every pass over a problem's folded kernel that is not
        # kept in LDS reads m * mp floats (logK rows in the row pass, its transpose in the
        # column pass).  One workgroup stops at the row pass of iteration iters + 1
        # (2 iters + 1 passes); a gang tests the state two iterations back (2 iters + 3
        # passes); LDS-resident problems read logK and its transpose once.
        lds_floats = 148 * 1024 // 4
        solve_bytes = 0
        for m_, it_ in zip(self.batch.ms, out[:, 5]):
            mp_ = (m_ + 3) // 4 * 4
            it_ = int(it_)
            if m_ > 256:
                passes = 2 * it_ + 3
            elif 6 * mp_ + 2 * m_ * mp_ <= lds_floats:
                passes = 2
            else:
                passes = 2 * it_ + 1
            solve_bytes += passes * m_ * mp_ * 4
        # the float64 multiply-adds of the gradients (on the matrix cores): dx and dy of every
        # point, 2 n^2 dim per problem
        grad_fma = float(sum(2.0 * (it.m * it.K) ** 2 * it.dim for it in self.items))

        # The same problems solved one at a time at full size (n = K m points per side) on the
        # GPU: full-size Sinkhorn to the same tolerance, then values and the gradients of all
        # n points and both marginals -- the plain method the batched reduced call replaces.
        # Outputs preallocated; the loop is timed once with HIP events around it (host
        # dispatch of the calls included).
        dev = "cuda:0"
        T_ = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
        fulls = []
        for q in self.probs:
            n, d = q["x"].shape
            pr = csot.Problem(T_(q["a"]), T_(q["b"]), q["eps"], q["K"], x=T_(q["x"]), y=T_(q["y"]))
            f32 = dict(dtype=torch.float32, device=dev)
            fulls.append((pr, (torch.empty(n, **f32), torch.empty(n, **f32)),
                          torch.zeros(8, dtype=torch.float64, device=dev),
                          {"dx": torch.empty((n, d), **f32), "dy": torch.empty((n, d), **f32),
                           "da": torch.empty(n, **f32), "db": torch.empty(n, **f32)},
                          torch.empty(8, dtype=torch.float64, device=dev)))
        csot.workspace(max(fulls, key=lambda r: r[0].n)[0])  # the largest, allocated once

        def full_pass():
            for pr, fg, ds, gr, vals in fulls:
                f, g, _ = csot.ot_sinkhorn_full(pr, self.opts, host_stats=False, out=fg, dstats=ds)
                csot.ot_cost_and_grad(pr, f, g, False, want_dxy=True, want_dab=True, grads=gr,
                                      out=vals)

        full_pass()
        torch.cuda.synchronize()
        e0.record()
        full_pass()
        e1.record()
        torch.cuda.synchronize()
        full_ms = e0.elapsed_time(e1)
        fout = torch.stack([r[4] for r in fulls]).cpu().numpy()
        fit = torch.stack([r[2] for r in fulls]).cpu().numpy()
        del fulls
        return {"workload": "batched: 1024 cyclic problems, m log-uniform [32, 1024], "
                            "K in {4,8,16,32}, dim 2/3, eps=0.05*median, tol=1e-6",
                "ms_per_call": round(ms_call, 3),
                "problems_per_s": round(1024 / ms_call * 1e3, 1),
                "forward_only_ms_per_call": round(fwd_ms, 3),
                "sum_m2": int(sum(it.m * it.m for it in self.items)),
                "all_converged": bool((out[:, 6] == 1).all()),
                "max_err_row_fp64": float(out[:, 3].max()),
                "max_err_col_fp64": float(out[:, 4].max()),
                "iterations_median_max": [float(np.median(out[:, 5])), float(out[:, 5].max())],
                "solve_kernel_ms": round(solve_ms, 3),
                "solve_roofline": {"bound": "hbm", "unit": "GB/s",
                                   "achieved": round(solve_bytes / (solve_ms * 1e-3) / 1e9, 1),
                                   "peak": HBM_PEAK_GBS,
                                   "frac": round(solve_bytes / (solve_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                   "bytes_per_launch": solve_bytes},
                "gradient_fp64_fma_per_call": grad_fma,
                "full_size_one_by_one": {
                    "ms": round(full_ms, 3),
                    "all_converged": bool((fit[:, 1] == 1).all()),
                    "max_err_row_fp64": float(fout[:, 3].max()),
                    "iterations_median_max": [float(np.median(fit[:, 0])), float(fit[:, 0].max())]},
                "speedup_vs_full_size": round(full_ms / ms_call, 2)}


def batched_only(steps, warmup):
    import torch

    leg = BatchedLeg()
    for _ in range(warmup):
        leg.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        leg.run()
    e1.record()
    torch.cuda.synchronize()
    print(json.dumps(leg.report(e0.elapsed_time(e1) / steps, steps)), flush=True)


def batched_calls_only(steps, warmup):
    """Warm-up + timed batched calls with gradients, then the same without gradients; nothing
    else (hardware-counter runs profile every dispatch, so the program is kept short)."""
    import torch

    leg = BatchedLeg()
    out = {}
    for name, b in (("with_gradients", leg.batch), ("forward_only", leg.batch_fwd)):
        for _ in range(warmup):
            b.run(leg.opts)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            b.run(leg.opts)
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = round(e0.elapsed_time(e1) / steps, 3)
    print(json.dumps({"workload": "batched: 1024 cyclic problems (calls only)", **out}), flush=True)


def two_stage_only(steps, warmup):
    """The approximate-symmetry workload (n=16384, K=32, m=512, jitter 1e-3, marginal noise 1%,
    eps = 0.05 median of the symmetric cloud, tol 1e-6): plain full-size Sinkhorn from g = 0 on
    the given data beside the two-stage method (Alg. 3: reduced solve of the block-averaged
    problem, then the full-size solve from its tiled potential), each timed with HIP events."""
    import numpy as np
    import torch

    import paper_2311_13147_amd as csot
    import workloads

    p = workloads.jittered_problem(16384, 32, sigma=1e-3, noise=0.01, seed=200)
    T_ = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0")
    prob = csot.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))
    opts = csot.make_opts(tol=1e-6, max_iter=20000)
    E = lambda: torch.cuda.Event(enable_timing=True)
    t_cold, t_two = [], []
    for it in range(warmup + steps):
        e = [E() for _ in range(3)]
        e[0].record()
        ff, gf, sf = csot.ot_sinkhorn_full(prob, opts, host_stats=False)
        e[1].record()
        out = csot.two_stage_sinkhorn(prob, tol=1e-6)
        e[2].record()
        torch.cuda.synchronize()
        if it >= warmup:
            t_cold.append(e[0].elapsed_time(e[1]))
            t_two.append(e[1].elapsed_time(e[2]))
    sf = sf.cpu().tolist()
    vf = csot.values_dict(csot.ot_cost_and_grad(prob, ff, gf, reduced=False)["values"])
    v2 = csot.values_dict(csot.ot_cost_and_grad(prob, out["f"], out["g"], reduced=False)["values"])
    print(json.dumps({"workload": "approximate symmetry: n=16384, K=32, m=512, jitter 1e-3, "
                                  "marginal noise 1%, eps=0.05*median, tol=1e-6",
                      "cold_full_ms": round(sum(t_cold) / steps, 3),
                      "two_stage_ms": round(sum(t_two) / steps, 3),
                      "iterations": {"cold_full": int(sf[0]), "stage1": out["stage1"]["iters"],
                                     "stage2": out["stage2"]["iters"]},
                      "err_row_fp64": {"cold_full": sf[2], "two_stage": out["stage2"]["err_row"]},
                      "objective_rel_diff": abs(v2["P"] - vf["P"]) / max(abs(vf["P"]), vf["CT"])}),
          flush=True)


def images_only(steps, warmup):
    """Image workloads (Example 1; synthetic 64 x 64 and 96 x 96 grayscale images stand in for
    the paper's real ones): pixel-wise Euclidean cost between pixel positions, lambda = 0.5, tol 1e-6, the
    dense-cost path.  Exact symmetry (mirror K=2, quarter turn K=4): the cyclic solve (fold +
    reduced solve) against the full-size solve on the dense n x n cost.  Approximate symmetry
    (5 % pixel noise, mirror): the cyclic solve of the averaged problem, the two-stage method
    and the full-size solve, with the objective gap and the marginal error of each against the
    given marginals.  One line of JSON per workload; times from HIP events."""
    import numpy as np
    import torch

    import paper_2311_13147_amd as csot
    import workloads

    T_ = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0")
    E = lambda: torch.cuda.Event(enable_timing=True)

    def full_cost(p):
        m, n, K = p.m, p.n, p.K
        C = np.empty((n, n), dtype=np.float32)
        for r in range(K):  # block (r, c) = C_{(c - r) mod K}
            for c in range(K):
                k = (c - r) % K
                C[r * m:(r + 1) * m, c * m:(c + 1) * m] = p.C_row0[:, k * m:(k + 1) * m]
        return C

    for side, K, noise in ((64, 2, 0.0), (64, 4, 0.0), (64, 2, 0.05), (96, 2, 0.0), (96, 4, 0.0),
                           (96, 2, 0.05)):
        p = workloads.image_problem(side, K, "euclidean", noise=noise)
        rprob = csot.Problem(T_(p.a), T_(p.b), p.eps, K, C=T_(p.C_row0))
        fprob = csot.Problem(T_(p.a), T_(p.b), p.eps, K, C=T_(full_cost(p)))
        opts = csot.make_opts(tol=1e-6, max_iter=20000)
        t_red, t_full, t_two = [], [], []
        for it in range(warmup + steps):
            e = [E() for _ in range(4)]
            e[0].record()
            logK, al, be = csot.ot_fold_kernel(rprob, opts)
            fr, gr, sr = csot.ot_sinkhorn_reduced(rprob, logK, al, be, opts, host_stats=False)
            e[1].record()
            ff, gf, sf = csot.ot_sinkhorn_full(fprob, opts, host_stats=False)
            e[2].record()
            if noise > 0.0:
                two = csot.two_stage_sinkhorn(fprob, tol=1e-6)
            e[3].record()
            torch.cuda.synchronize()
            if it >= warmup:
                t_red.append(e[0].elapsed_time(e[1]))
                t_full.append(e[1].elapsed_time(e[2]))
                t_two.append(e[2].elapsed_time(e[3]))
        sr, sf = sr.cpu().tolist(), sf.cpu().tolist()
        vf = csot.values_dict(csot.ot_cost_and_grad(fprob, ff, gf, reduced=False)["values"])
        # the cyclic solution tiled to full size, measured against the given marginals
        vr = csot.values_dict(csot.ot_cost_and_grad(fprob, fr.repeat(K), gr.repeat(K),
                                                    reduced=False)["values"])
        gap = lambda v: abs(v["P"] - vf["P"]) / max(abs(vf["P"]), vf["CT"])
        rec = {"workload": f"images {side}x{side}, {'mirror' if K == 2 else 'quarter turn'} K={K}, "
                           f"pixel Euclidean cost, lambda=0.5, tol=1e-6"
                           + (f", pixel noise {noise:g} (approximate symmetry)" if noise else ""),
               "n": p.n, "m": p.m,
               "cyclic_ms": round(sum(t_red) / steps, 3),
               "full_ms": round(sum(t_full) / steps, 3),
               "speedup": round(sum(t_full) / sum(t_red), 2),
               "iterations": {"cyclic": int(sr[0]), "full": int(sf[0])},
               # phases the full-size solver redid in exact (running-maximum) mode because its
               # common shift would leave float32 range
               "full_exact_redos": int(sf[6]),
               "err_row_fp64": {"full": sf[2]},
               "cyclic_objective_rel_gap": gap(vr),
               "cyclic_err_vs_given_marginals": {"row": vr["err_row"], "col": vr["err_col"]}}
        if noise > 0.0:
            v2 = csot.values_dict(csot.ot_cost_and_grad(fprob, two["f"], two["g"],
                                                        reduced=False)["values"])
            rec.update(two_stage_ms=round(sum(t_two) / steps, 3),
                       two_stage_iterations={"stage1": two["stage1"]["iters"],
                                             "stage2": two["stage2"]["iters"]},
                       two_stage_objective_rel_gap=gap(v2),
                       two_stage_err_row_fp64=two["stage2"]["err_row"])
        print(json.dumps(rec), flush=True)


def lot_only(steps, warmup):
    """Cyclic linear OT (Thm. 1, Alg. 1) at n=8192, K=16, m=512: the GPU steps around the
    small LP -- the min-fold (G = min_k C_ijk and the minimising k, float64 costs) and the
    scatter of an m x m solution into the n x n plan (HBM-write bound) -- timed with HIP
    events.  The small LP itself (m^2 variables) is the caller's and is not timed here."""
    import numpy as np
    import torch

    import paper_2311_13147_amd as csot
    import workloads

    p = workloads.symmetric_problem(8192, 16, 2, 0.01, seed=100)
    T_ = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0")
    prob = csot.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))
    G, kmin, al, be = csot.ot_lot_fold(prob)
    S = torch.rand((p.m, p.m), device="cuda:0", dtype=torch.float32)
    T = torch.empty((p.n, p.n), device="cuda:0", dtype=torch.float32)
    E = lambda: torch.cuda.Event(enable_timing=True)
    tf, te = [], []
    for it in range(warmup + steps):
        e = [E() for _ in range(3)]
        e[0].record()
        csot.ot_lot_fold(prob, out=(G, kmin, al, be))
        e[1].record()
        csot.ot_lot_expand(prob, S, kmin, out=T)
        e[2].record()
        torch.cuda.synchronize()
        if it >= warmup:
            tf.append(e[0].elapsed_time(e[1]))
            te.append(e[1].elapsed_time(e[2]))
    fold_ms, exp_ms = sum(tf) / steps, sum(te) / steps
    gbps = p.n * p.n * 4 / (exp_ms * 1e-3) / 1e9
    print(json.dumps({"workload": "cyclic linear OT steps, n=8192, K=16, m=512, 2-D clouds",
                      "min_fold_ms": round(fold_ms, 4),
                      "min_fold_cost_evals_per_s": p.K * p.m * p.m / (fold_ms * 1e-3),
                      "plan_scatter_ms": round(exp_ms, 4), "plan_scatter_GBps": round(gbps, 1),
                      "plan_scatter_frac_of_hbm": round(gbps / HBM_PEAK_GBS, 3)}), flush=True)


def srot_only(steps, warmup):
    """Quadratically regularised OT (phi(x) = lam/2 x^2, lam = 10 median(C)) at n=8192, K=16:
    the cyclic alternating maximisation (m = 512) and the full-size problem (the same call
    with K = 1 on all n points), each to tol = 1e-6 and over 50 fixed iterations.  Every call
    is one persistent solver launch with the stop test on the device, then the float64
    residuals and one host synchronisation; host-timed around the call."""
    import time

    import numpy as np
    import torch

    import paper_2311_13147_amd as csot
    import workloads

    p = workloads.symmetric_problem(8192, 16, 2, 0.01, seed=100)
    T_ = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0")
    x, y = T_(p.x), T_(p.y)
    lam = 10.0 * workloads.median_sq_dist_row0(p.x, p.y, p.m)
    red = csot.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=x, y=y)
    full = csot.Problem(T_(p.a), T_(p.b), p.eps, 1, x=x, y=y)

    def timed(prob, opts):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, z, st = csot.ot_srot_reduced(prob, lam, opts)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, st

    fixed = csot.make_opts(tol=0.0, max_iter=50)
    to_tol = csot.make_opts(tol=1e-6, max_iter=5000)
    rows = {k: [] for k in ("red_fixed", "full_fixed", "red_tol", "full_tol")}
    for it in range(warmup + steps):
        got = {"red_fixed": timed(red, fixed), "full_fixed": timed(full, fixed),
               "red_tol": timed(red, to_tol), "full_tol": timed(full, to_tol)}
        if it >= warmup:
            for k, (ms, _) in got.items():
                rows[k].append(ms)
    mean = {k: sum(v) / steps for k, v in rows.items()}
    st_r, st_f = got["red_tol"][1], got["full_tol"][1]
    print(json.dumps({"workload": "quadratically regularised OT, lam=10*median(C), n=8192, K=16, "
                                  "m=512, tol=1e-6",
                      "cyclic_ms_per_iteration": round(mean["red_fixed"] / 50, 4),
                      "full_ms_per_iteration": round(mean["full_fixed"] / 50, 4),
                      "iteration_speedup": round(mean["full_fixed"] / mean["red_fixed"], 1),
                      "cyclic_time_to_tol_ms": round(mean["red_tol"], 3),
                      "full_time_to_tol_ms": round(mean["full_tol"], 3),
                      "time_to_tol_speedup": round(mean["full_tol"] / mean["red_tol"], 1),
                      "cyclic_iterations_to_tol": st_r["iters"],
                      "full_iterations_to_tol": st_f["iters"],
                      "cyclic_err_row_fp64": st_r["err_row"],
                      "full_err_row_fp64": st_f["err_row"]}), flush=True)


def copy_calibration():
    import torch
    src = torch.ones(64 * 1024 * 1024, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)


def _source_hash(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2311_13147_amd", "csrc", nm), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel_file):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 --pmc summary
    (lines `source_hash: ...` and `bytes_per_launch: ...`), or None when it is missing or the
    kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "full_solver_n8192_K16_pmc.md")
    rec = {}
    try:
        with open(path) as fh:
            for line in fh:
                if ":" in line and line.split(":", 1)[0].strip() in ("source_hash", "bytes_per_launch"):
                    k, v = line.split(":", 1)
                    rec[k.strip()] = v.strip().strip("`")
    except OSError:
        return None
    if rec.get("source_hash") != _source_hash(kernel_file, "common.hpp"):
        return None
    try:
        return int(float(rec["bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def peaks_only():
    import paper_2311_13147_amd as csot
    pk = csot.ot_measure_peaks()
    print(json.dumps({"device_peaks": pk,
                      "derived": {"fp32_fma_TFLOPs": 2 * pk["fma32_per_s"] / 1e12,
                                  "fp64_fma_TFLOPs": 2 * pk["fma64_per_s"] / 1e12,
                                  "exp2_T_per_s": pk["exp2_per_s"] / 1e12,
                                  "full_entry_mix_T_per_s": pk["full_entry_mix_per_s"] / 1e12,
                                  "copy_GBps": pk["copy_bytes_per_s"] / 1e9,
                                  "slot_hop_us_same_xcd": pk["slot_hop_s_same_xcd"] * 1e6,
                                  "slot_hop_us_cross_xcd": pk["slot_hop_s_cross_xcd"] * 1e6,
                                  "fp64_matrix_TFLOPs": 2 * pk["mfma64_madd_per_s"] / 1e12}}),
          flush=True)


def main():
    args = _args()
    if args.peaks:
        peaks_only()
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_calls:
        batched_calls_only(args.steps, args.warmup)
        return
    if args.batched:
        batched_only(args.steps, args.warmup)
        return
    if args.two_stage:
        two_stage_only(args.steps, args.warmup)
        return
    if args.images:
        images_only(args.steps, args.warmup)
        return
    if args.lot:
        lot_only(args.steps, args.warmup)
        return
    if args.srot:
        srot_only(args.steps, args.warmup)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2311_13147_amd as csot
    import workloads

    dev = torch.device("cuda:0")
    p = workloads.symmetric_problem(N, K, DIM, EPS_FACTOR, seed=SEED)
    T_ = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    prob = csot.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))
    m = p.m
    o_tol = csot.make_opts(tol=TOL, max_iter=100000, fold_fp64=1)
    # the fixed-count legs also time their solver kernel alone (events recorded by the library
    # right around that launch, on the stream it runs on)
    kev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for k in ("red_fixed", "full_fixed")}
    o_fr = csot.make_opts(tol=0.0, max_iter=args.fixed_reduced, fold_fp64=1,
                          timing_events=kev["red_fixed"])
    o_ff = csot.make_opts(tol=0.0, max_iter=args.fixed_full, timing_events=kev["full_fixed"])
    # preallocated outputs (nothing allocated inside the timed region)
    logK = torch.empty((m, m), device=dev)
    al, be = torch.empty(m, device=dev), torch.empty(m, device=dev)
    fr, gr = torch.empty(m, device=dev), torch.empty(m, device=dev)
    fr2, gr2 = torch.empty(m, device=dev), torch.empty(m, device=dev)
    ff, gf = torch.empty(N, device=dev), torch.empty(N, device=dev)
    ff2, gf2 = torch.empty(N, device=dev), torch.empty(N, device=dev)
    Tplan = torch.empty((N, N), device=dev)
    ds = [torch.zeros(8, dtype=torch.float64, device=dev) for _ in range(4)]
    vals_r = torch.empty(8, dtype=torch.float64, device=dev)
    vals_f = torch.empty(8, dtype=torch.float64, device=dev)
    f32 = dict(dtype=torch.float32, device=dev)
    grads_r = {"dx": torch.empty((N, DIM), **f32), "dy": torch.empty((N, DIM), **f32),
               "da": torch.empty(N, **f32), "db": torch.empty(N, **f32)}
    grads_f = {k: torch.empty_like(v) for k, v in grads_r.items()}
    csot.workspace(prob, o_tol)

    # The time-to-tolerance work also recorded once in graphs (kernels only; the stopping
    # decision is made on the GPU), so that a replay shows the GPU time without the host's
    # per-call dispatch: fold + reduced solve, and the full-size solve.
    fr3, gr3 = torch.empty(m, device=dev), torch.empty(m, device=dev)
    ff3, gf3 = torch.empty(N, device=dev), torch.empty(N, device=dev)
    ds_g = [torch.zeros(8, dtype=torch.float64, device=dev) for _ in range(2)]
    logK3 = torch.empty((m, m), device=dev)
    al3, be3 = torch.empty(m, device=dev), torch.empty(m, device=dev)

    def red_tol():
        csot.ot_fold_kernel(prob, o_tol, out=(logK3, al3, be3))
        csot.ot_sinkhorn_reduced(prob, logK3, al3, be3, o_tol, host_stats=False, out=(fr3, gr3),
                                 dstats=ds_g[0])

    def full_tol():
        csot.ot_sinkhorn_full(prob, o_tol, host_stats=False, out=(ff3, gf3), dstats=ds_g[1])

    # forward + backward: the same solves followed by values and all gradients
    vals_rg = torch.empty(8, dtype=torch.float64, device=dev)
    vals_fg = torch.empty(8, dtype=torch.float64, device=dev)
    grads_rg = {k: torch.empty_like(v) for k, v in grads_r.items()}
    grads_fg = {k: torch.empty_like(v) for k, v in grads_r.items()}

    def red_fb():
        red_tol()
        csot.ot_cost_and_grad(prob, fr3, gr3, True, want_dxy=True, want_dab=True, out=vals_rg,
                              grads=grads_rg)

    def full_fb():
        full_tol()
        csot.ot_cost_and_grad(prob, ff3, gf3, False, want_dxy=True, want_dab=True, out=vals_fg,
                              grads=grads_fg)

    # the workload's second regulariser, eps = 0.1 median(C): time to the same tolerance
    p2 = workloads.symmetric_problem(N, K, DIM, EPS_FACTOR_2, seed=SEED)
    prob2 = csot.Problem(T_(p2.a), T_(p2.b), p2.eps, p2.K, x=T_(p2.x), y=T_(p2.y))
    logK2 = torch.empty((m, m), device=dev)
    al2, be2 = torch.empty(m, device=dev), torch.empty(m, device=dev)
    fr4, gr4 = torch.empty(m, device=dev), torch.empty(m, device=dev)
    ff4, gf4 = torch.empty(N, device=dev), torch.empty(N, device=dev)
    ds2 = [torch.zeros(8, dtype=torch.float64, device=dev) for _ in range(2)]
    csot.workspace(prob2, o_tol)

    # approximate symmetry (config 3, Alg. 3): n=16384, K=32, jitter 1e-3, marginal noise 1%,
    # eps = 0.05 median of the symmetric cloud -- plain full-size Sinkhorn from g = 0 on the
    # given data beside the two-stage method (cyclic solve of the block-averaged problem, then
    # the full-size solve from its tiled potential)
    p3 = workloads.jittered_problem(16384, 32, sigma=1e-3, noise=0.01, seed=200)
    prob3 = csot.Problem(T_(p3.a), T_(p3.b), p3.eps, p3.K, x=T_(p3.x), y=T_(p3.y))
    n3 = p3.n
    ff5, gf5 = torch.empty(n3, device=dev), torch.empty(n3, device=dev)
    two_out = (torch.empty(n3, device=dev), torch.empty(n3, device=dev))
    ds3 = torch.zeros(8, dtype=torch.float64, device=dev)
    csot.workspace(prob3, o_tol)
    two_last = {}

    def cfg3_two_stage():
        two_last["r"] = csot.two_stage_sinkhorn(prob3, tol=TOL, out=two_out)

    # forward + backward at n=4096, K=8 (config 4, eps = 0.05 median): replayed from graphs
    p4 = workloads.symmetric_problem(4096, 8, 2, 0.05, seed=SEED)
    prob4 = csot.Problem(T_(p4.a), T_(p4.b), p4.eps, p4.K, x=T_(p4.x), y=T_(p4.y))
    m4, n4 = p4.m, p4.n
    b4 = {"logK": torch.empty((m4, m4), device=dev), "al": torch.empty(m4, device=dev),
          "be": torch.empty(m4, device=dev), "fr": torch.empty(m4, device=dev),
          "gr": torch.empty(m4, device=dev), "ff": torch.empty(n4, device=dev),
          "gf": torch.empty(n4, device=dev),
          "ds": [torch.zeros(8, dtype=torch.float64, device=dev) for _ in range(2)],
          "vr": torch.empty(8, dtype=torch.float64, device=dev),
          "vf": torch.empty(8, dtype=torch.float64, device=dev)}
    g4r = {"dx": torch.empty((n4, 2), **f32), "dy": torch.empty((n4, 2), **f32),
           "da": torch.empty(n4, **f32), "db": torch.empty(n4, **f32)}
    g4f = {k: torch.empty_like(v) for k, v in g4r.items()}
    csot.workspace(prob4, o_tol)

    def cfg4_red_fb():
        csot.ot_fold_kernel(prob4, o_tol, out=(b4["logK"], b4["al"], b4["be"]))
        csot.ot_sinkhorn_reduced(prob4, b4["logK"], b4["al"], b4["be"], o_tol, host_stats=False,
                                 out=(b4["fr"], b4["gr"]), dstats=b4["ds"][0])
        csot.ot_cost_and_grad(prob4, b4["fr"], b4["gr"], True, want_dxy=True, want_dab=True,
                              out=b4["vr"], grads=g4r)

    def cfg4_full_fb():
        csot.ot_sinkhorn_full(prob4, o_tol, host_stats=False, out=(b4["ff"], b4["gf"]),
                              dstats=b4["ds"][1])
        csot.ot_cost_and_grad(prob4, b4["ff"], b4["gf"], False, want_dxy=True, want_dab=True,
                              out=b4["vf"], grads=g4f)

    # the batched workload (config 5): one batched call per step
    bleg = BatchedLeg()

    graphs = {}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        red_fb()
        full_fb()
        cfg4_red_fb()
        cfg4_full_fb()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for name, fn in (("red_graph", red_tol), ("full_graph", full_tol), ("red_fb_graph", red_fb),
                     ("full_fb_graph", full_fb), ("cfg4_red_fb_graph", cfg4_red_fb),
                     ("cfg4_full_fb_graph", cfg4_full_fb)):
        gr_ = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr_):
            fn()
        graphs[name] = gr_
    torch.cuda.synchronize()

    E = lambda: torch.cuda.Event(enable_timing=True)
    legs = ["fold", "red_solve", "expand", "red_grad", "red_fixed", "full_solve", "full_grad",
            "full_fixed", "red_graph", "full_graph", "red_fb_graph", "full_fb_graph",
            "red_tol_eps2", "full_tol_eps2", "cfg3_cold_full", "cfg3_two_stage",
            "cfg4_red_fb_graph", "cfg4_full_fb_graph", "batched"]

    def step(record):
        ev = {k: (E(), E()) for k in legs}
        def run(name, fn):
            ev[name][0].record()
            out = fn()
            ev[name][1].record()
            return out
        run("fold", lambda: csot.ot_fold_kernel(prob, o_tol, out=(logK, al, be)))
        run("red_solve", lambda: csot.ot_sinkhorn_reduced(prob, logK, al, be, o_tol,
                                                          host_stats=False, out=(fr, gr),
                                                          dstats=ds[0]))
        run("expand", lambda: csot.ot_expand_plan(prob, fr, gr, out=Tplan))
        res_r = run("red_grad", lambda: csot.ot_cost_and_grad(prob, fr, gr, True, want_dxy=True,
                                                              want_dab=True, out=vals_r,
                                                              grads=grads_r))
        run("red_fixed", lambda: csot.ot_sinkhorn_reduced(prob, logK, al, be, o_fr,
                                                          host_stats=False, out=(fr2, gr2),
                                                          dstats=ds[1]))
        run("full_solve", lambda: csot.ot_sinkhorn_full(prob, o_tol, host_stats=False,
                                                        out=(ff, gf), dstats=ds[2]))
        run("full_grad", lambda: csot.ot_cost_and_grad(prob, ff, gf, False, want_dxy=True,
                                                       want_dab=True, out=vals_f,
                                                       grads=grads_f))
        run("full_fixed", lambda: csot.ot_sinkhorn_full(prob, o_ff, host_stats=False,
                                                        out=(ff2, gf2), dstats=ds[3]))
        run("red_graph", graphs["red_graph"].replay)
        run("full_graph", graphs["full_graph"].replay)
        run("red_fb_graph", graphs["red_fb_graph"].replay)
        run("full_fb_graph", graphs["full_fb_graph"].replay)

        def red_eps2():
            csot.ot_fold_kernel(prob2, o_tol, out=(logK2, al2, be2))
            csot.ot_sinkhorn_reduced(prob2, logK2, al2, be2, o_tol, host_stats=False,
                                     out=(fr4, gr4), dstats=ds2[0])
        run("red_tol_eps2", red_eps2)
        run("full_tol_eps2", lambda: csot.ot_sinkhorn_full(prob2, o_tol, host_stats=False,
                                                           out=(ff4, gf4), dstats=ds2[1]))
        run("cfg3_cold_full", lambda: csot.ot_sinkhorn_full(prob3, o_tol, host_stats=False,
                                                            out=(ff5, gf5), dstats=ds3))
        run("cfg3_two_stage", cfg3_two_stage)
        run("cfg4_red_fb_graph", graphs["cfg4_red_fb_graph"].replay)
        run("cfg4_full_fb_graph", graphs["cfg4_full_fb_graph"].replay)
        run("batched", bleg.run)
        return ev

    def kernel_ms():
        torch.cuda.synchronize()
        return {k: e[0].elapsed_time(e[1]) for k, e in kev.items()}

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs, kms = [], []
    for _ in range(args.steps):
        evs.append(step(True))
        kms.append(kernel_ms())   # after the step's last launch: no extra sync inside a step
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = {k: sum(d[k] for d in kms) / args.steps for k in kev}

    ms = {k: sum(e[k][0].elapsed_time(e[k][1]) for e in evs) / args.steps for k in legs}
    st = [d.cpu().tolist() for d in ds]
    it_red, it_full = int(st[0][0]), int(st[2][0])
    stg = [d.cpu().tolist() for d in ds_g]
    st2 = [d.cpu().tolist() for d in ds2]
    # a replay must reproduce the eager solve: same iteration count, converged, same potentials
    graph_ok = (int(stg[0][0]) == it_red and int(stg[1][0]) == it_full and stg[0][1] == 1.0
                and stg[1][1] == 1.0 and torch.equal(fr3, fr) and torch.equal(ff3, ff))
    vr, vf = csot.values_dict(vals_r), csot.values_dict(vals_f)
    red_ips = args.fixed_reduced / (ms["red_fixed"] * 1e-3)
    full_ips = args.fixed_full / (ms["full_fixed"] * 1e-3)
    ttt_red = ms["fold"] + ms["red_solve"]
    ttt_full = ms["full_solve"]
    step_ms = wall * 1e3 / args.steps

    pk = csot.ot_measure_peaks()  # after the timed region
    # roofline of the dominant kernel: the full-size solver (fixed-count leg), in the work
    # units of its definition (OPS_PER_ENTRY per (I, J) entry of a half-step)
    units = 2.0 * N * N * args.fixed_full
    t_full = kern["full_fixed"] * 1e-3
    achieved = units * OPS_PER_ENTRY[DIM] / t_full / 1e12
    roof = {"bound": "alu", "kernel": "full_solver_kernel", "achieved": round(achieved, 3),
            "peak": PUBLISHED_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PUBLISHED_FP32_TFLOPS, 4),
            "traffic": _traffic("full.hip"),
            "ops_per_unit": OPS_PER_ENTRY[DIM],
            "unit_def": "one (I, J) entry of a half-step: 1 exp2 + 7 flops",
            "units_per_launch": units,
            "kernel_ms_per_launch": round(kern["full_fixed"], 4),
            "source": PROFILE_SUMMARY,
            "non_packed_peak": NON_PACKED_FP32_TFLOPS,
            "frac_of_non_packed_peak": round(achieved / NON_PACKED_FP32_TFLOPS, 4),
            # the measured issue rate of the solver's own instruction mix (ot_measure_peaks)
            "mix_ceiling_entries_per_s": pk["full_entry_mix_per_s"],
            "frac_of_mix_ceiling": round(units / t_full / pk["full_entry_mix_per_s"], 4)}
    # the reduced path's kernels, each against what bounds it
    red_iter_s = kern["red_fixed"] * 1e-3 / args.fixed_reduced
    hop = pk["slot_hop_s_same_xcd"]
    plan_bytes = 4.0 * N * N
    adj_fma = 2.0 * N * N * DIM      # float64 FMAs: dx and dy of every point
    fold_units = float(K) * m * m
    roof_red = {
        "solver": {"bound": "latency", "us_per_iter": round(red_iter_s * 1e6, 4),
                   # an iteration holds two dependent exchanges of potentials between
                   # workgroups (row -> column -> row): two slot hops at least
                   "floor_us_per_iter": round(2 * hop * 1e6, 4),
                   "frac": round(2 * hop / red_iter_s, 4),
                   "slot_hop_us": round(hop * 1e6, 4)},
        "expand": {"bound": "hbm", "unit": "GB/s",
                   "achieved": round(plan_bytes / (ms["expand"] * 1e-3) / 1e9, 1),
                   "peak": HBM_PEAK_GBS,
                   "frac": round(plan_bytes / (ms["expand"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "measured_copy_GBps": round(pk["copy_bytes_per_s"] / 1e9, 1)},
        "adjoint": {"bound": "alu", "unit": "fp64 FMA/s",
                    "fp64_fma_per_call": adj_fma, "exp2_per_call": 2.0 * fold_units,
                    "achieved": adj_fma / (ms["red_grad"] * 1e-3),
                    "measured_fp64_fma_per_s": pk["fma64_per_s"],
                    "frac": round(adj_fma / (ms["red_grad"] * 1e-3) / pk["fma64_per_s"], 4),
                    "leg": "adjoint launch + finalize launch"},
        "fold": {"bound": "alu", "unit": "TFLOP/s", "ops_per_unit": 8,
                 "units_per_call": fold_units,
                 "achieved": round(fold_units * 8 / (ms["fold"] * 1e-3) / 1e12, 3),
                 "peak": PUBLISHED_FP32_TFLOPS,
                 "frac": round(fold_units * 8 / (ms["fold"] * 1e-3) / 1e12 / PUBLISHED_FP32_TFLOPS, 4)},
    }
    red_kernel_us = kern["red_fixed"] * 1e3 / args.fixed_reduced

    out = {
        "metric": "Sinkhorn iters/s & time-to-1e-6 marginal err, reduced vs full, n=8192 K=16",
        "value": round(red_ips, 1),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cyclic EROT, 2-D {K}-fold rotational point clouds, n={N}, K={K}, "
                               f"m={m}, eps={EPS_FACTOR}*median(C), tol={TOL}",
                   "n": N, "K": K, "m": m, "dim": DIM, "eps": p.eps, "seed": SEED},
        "reduced_iters_per_s": round(red_ips, 1),
        "reduced_kernel_us_per_iter": round(red_kernel_us, 3),
        "full_kernel_us_per_iter": round(kern["full_fixed"] * 1e3 / args.fixed_full, 3),
        "full_iters_per_s": round(full_ips, 1),
        "iter_speedup": round(red_ips / full_ips, 2),
        "time_to_tol_ms": {"reduced_fold_plus_solve": round(ttt_red, 4),
                           "reduced_end_to_end_with_expand": round(ttt_red + ms["expand"], 4),
                           "full_solve": round(ttt_full, 4),
                           "speedup_solve": round(ttt_full / ttt_red, 2)},
        "time_to_tol_graph_ms": {"reduced_fold_plus_solve": round(ms["red_graph"], 4),
                                 "full_solve": round(ms["full_graph"], 4),
                                 "speedup_solve": round(ms["full_graph"] / ms["red_graph"], 2),
                                 "replays_match_eager": bool(graph_ok)},
        "forward_backward_ms": {"reduced": round(ttt_red + ms["red_grad"], 4),
                                "full": round(ttt_full + ms["full_grad"], 4)},
        "forward_backward_graph_ms": {"reduced": round(ms["red_fb_graph"], 4),
                                      "full": round(ms["full_fb_graph"], 4),
                                      "speedup": round(ms["full_fb_graph"] / ms["red_fb_graph"], 2)},
        "iterations_to_tol": {"reduced": it_red, "full": it_full},
        "reduced_xcd_local_exchange": bool(st[1][7]),
        "marginal_err_fp64": {"reduced_row": st[0][2], "reduced_col": st[0][3],
                              "full_row": st[2][2], "full_col": st[2][3]},
        "objective": {"reduced_P": vr["P"], "full_P": vf["P"],
                      "rel_gap": abs(vr["P"] - vf["P"]) / max(abs(vf["P"]), vf["CT"])},
        "leg_ms": {k: round(v, 4) for k, v in ms.items()},
        "leg_ms_max": {k: round(max(e[k][0].elapsed_time(e[k][1]) for e in evs), 4) for k in legs},
        "time_to_tol_ms_eps0.1": {
            "eps": p2.eps,
            "reduced_fold_plus_solve": round(ms["red_tol_eps2"], 4),
            "full_solve": round(ms["full_tol_eps2"], 4),
            "speedup_solve": round(ms["full_tol_eps2"] / ms["red_tol_eps2"], 2),
            "iterations": {"reduced": int(st2[0][0]), "full": int(st2[1][0])},
            "marginal_err_fp64": {"reduced_row": st2[0][2], "full_row": st2[1][2]}},
        "approximate_symmetry": _cfg3_report(csot, prob3, p3, ms, ds3, ff5, gf5, two_last["r"]),
        "forward_backward_n4096_K8_graph_ms": {
            "reduced": round(ms["cfg4_red_fb_graph"], 4),
            "full": round(ms["cfg4_full_fb_graph"], 4),
            "speedup": round(ms["cfg4_full_fb_graph"] / ms["cfg4_red_fb_graph"], 2),
            "iterations": {"reduced": int(b4["ds"][0][0].item()),
                           "full": int(b4["ds"][1][0].item())},
            "marginal_err_fp64": {"reduced_row": float(b4["ds"][0][2].item()),
                                  "full_row": float(b4["ds"][1][2].item())},
            "objective_rel_gap": _rel_gap(csot.values_dict(b4["vr"]), csot.values_dict(b4["vf"]))},
        "expand_GBps": round(4.0 * N * N / (ms["expand"] * 1e-3) / 1e9, 1),
        "roofline": roof,
        "roofline_reduced_path": roof_red,
        "device_peaks": pk,
        "batched": bleg.report(ms["batched"], args.steps),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, fr, gr, vr, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def _rel_gap(va, vb):
    return abs(va["P"] - vb["P"]) / max(abs(vb["P"]), vb["CT"])


def _cfg3_report(csot, prob3, p3, ms, ds3, ff5, gf5, two):
    """The approximate-symmetry leg: times of the cold full-size solve and of the two-stage
    method, and (evaluated once, after the timed region) Table 2's quantities for the cyclic
    solve of the block-averaged problem alone: its objective against the full-size optimum on
    the given data, and the marginal error of its tiled potentials against the given
    marginals."""
    import torch

    sf = ds3.cpu().tolist()
    o = csot.make_opts(tol=TOL, max_iter=20000, fold_fp64=1)
    csym = csot.ot_symmetrize_cost(prob3)
    sprob = csot.Problem(prob3.a, prob3.b, prob3.eps, prob3.K, C=csym)
    logK, al, be = csot.ot_fold_kernel(sprob, o)
    fr, gr, st1 = csot.ot_sinkhorn_reduced(sprob, logK, al, be, o)
    K = prob3.K
    vf = csot.values_dict(csot.ot_cost_and_grad(prob3, ff5, gf5, reduced=False)["values"])
    vc = csot.values_dict(csot.ot_cost_and_grad(prob3, fr.repeat(K), gr.repeat(K),
                                                reduced=False)["values"])
    v2 = csot.values_dict(csot.ot_cost_and_grad(prob3, two["f"], two["g"],
                                                reduced=False)["values"])
    torch.cuda.synchronize()
    return {"workload": f"n={p3.n}, K={K}, m={p3.m}, jitter 1e-3, marginal noise 1%, "
                        "eps=0.05*median, tol=1e-6",
            "cold_full_ms": round(ms["cfg3_cold_full"], 4),
            "two_stage_ms": round(ms["cfg3_two_stage"], 4),
            "speedup_two_stage": round(ms["cfg3_cold_full"] / ms["cfg3_two_stage"], 3),
            "iterations": {"cold_full": int(sf[0]), "stage1": two["stage1"]["iters"],
                           "stage2": two["stage2"]["iters"]},
            "err_row_fp64": {"cold_full": sf[2], "two_stage": two["stage2"]["err_row"]},
            "two_stage_objective_rel_diff": _rel_gap(v2, vf),
            "cyclic_of_averaged": {"iterations": st1["iters"],
                                   "objective_rel_gap": _rel_gap(vc, vf),
                                   "marginal_err_vs_given": {"row": vc["err_row"],
                                                             "col": vc["err_col"]}}}


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(p, f_gpu, g_gpu, vr, budget_s):
    """The float64 oracle as it stands, timed on the host on bounded samples of the workload:
    * reduced cyclic Sinkhorn (oracle.sinkhorn.reduced_sinkhorn, one thread): iterations/s --
      the reported value;
    * the same iteration on all usable cores (the oracle's own row and column half-steps,
      row_update / col_update, on row / column chunks in a thread pool; NumPy releases the
      GIL inside its array operations);
    * full-size Sinkhorn at n = 8192 (oracle.sinkhorn.full_sinkhorn, one thread, one
      iteration including its residual pass) and its two half-steps on all cores;
    plus the error of the GPU result against the oracle's converged reduced solution."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import cost, objective, sinkhorn

    model, nproc, usable = _host_cpu()
    threads = max(1, min(16, usable))
    Ck = cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)
    a, b = p.a.astype(np.float64), p.b.astype(np.float64)
    alpha, beta = sinkhorn.fold_marginals(a, p.K), sinkhorn.fold_marginals(b, p.K)
    t0 = time.perf_counter()
    logK = sinkhorn.fold_kernel(Ck, p.eps)
    t_fold = time.perf_counter() - t0
    # one timed probe iteration sizes the samples to the time budget
    t0 = time.perf_counter()
    sinkhorn.reduced_sinkhorn(alpha, beta, logK, p.eps, p.K, tol=0.0, max_iter=2)
    per_it = (time.perf_counter() - t0) / 2
    iters = max(5, min(2000, int(0.4 * budget_s / per_it)))
    t0 = time.perf_counter()
    sinkhorn.reduced_sinkhorn(alpha, beta, logK, p.eps, p.K, tol=0.0, max_iter=iters)
    dt = time.perf_counter() - t0

    pool = ThreadPoolExecutor(max_workers=threads)

    def chunks(count):
        step = (count + threads - 1) // threads
        return [slice(s0, min(s0 + step, count)) for s0 in range(0, count, step)]

    # reduced iteration on all cores: the row update with C = -eps logK (exponent logK + g/eps)
    Cred = -p.eps * logK
    mm = p.m
    rch, cch = chunks(mm), chunks(mm)
    g = np.zeros(mm)
    iters_mt = max(5, iters // 2)
    t0 = time.perf_counter()
    for _ in range(iters_mt):
        f = np.concatenate(list(pool.map(
            lambda sl: sinkhorn.row_update(g, Cred[sl], alpha[sl], p.eps), rch)))
        g = np.concatenate(list(pool.map(
            lambda sl: sinkhorn.col_update(f, Cred[:, sl], beta[sl], p.eps), cch)))
    dt_mt = time.perf_counter() - t0

    # full size: the float64 cost of the float32 coordinates, then one iteration on one thread
    # (row and column half-steps and the residual pass) and two half-steps on all cores
    C = cost.sq_euclidean(p.x, p.y)
    t0 = time.perf_counter()
    sinkhorn.full_sinkhorn(a, b, C, p.eps, tol=0.0, max_iter=1)
    full_1t = time.perf_counter() - t0
    n = p.n
    rch, cch = chunks(n), chunks(n)
    gfull = np.zeros(n)
    t0 = time.perf_counter()
    for _ in range(2):
        ffull = np.concatenate(list(pool.map(
            lambda sl: sinkhorn.row_update(gfull, C[sl], a[sl], p.eps), rch)))
        gfull = np.concatenate(list(pool.map(
            lambda sl: sinkhorn.col_update(ffull, C[:, sl], b[sl], p.eps), cch)))
    full_mt = (time.perf_counter() - t0) / 2
    pool.shutdown()
    del C

    # forward + backward at n = 4096, K = 8 (eps = 0.05 median), one thread: the oracle's
    # reduced solve to 1e-6 and its envelope gradients of the tiled potentials, beside the
    # full-size solve to 1e-6 and the same gradients
    from oracle import grad as ograd
    import workloads
    p4 = workloads.symmetric_problem(4096, 8, 2, 0.05, seed=SEED)
    a4, b4 = p4.a.astype(np.float64), p4.b.astype(np.float64)
    x4, y4 = p4.x.astype(np.float64), p4.y.astype(np.float64)
    t0 = time.perf_counter()
    Ck4 = cost.blocks_from_row0(cost.row0_from_points(p4.x, p4.y, p4.K), p4.K)
    al4, be4 = sinkhorn.fold_marginals(a4, p4.K), sinkhorn.fold_marginals(b4, p4.K)
    r4 = sinkhorn.reduced_sinkhorn(al4, be4, sinkhorn.fold_kernel(Ck4, p4.eps), p4.eps, p4.K,
                                   tol=TOL)
    ograd.envelope_grads(np.tile(r4["f"], p4.K), np.tile(r4["g"], p4.K), x4, y4, p4.eps)
    fb_red = time.perf_counter() - t0
    t0 = time.perf_counter()
    rf4 = sinkhorn.full_sinkhorn(a4, b4, cost.sq_euclidean(p4.x, p4.y), p4.eps, tol=TOL)
    ograd.envelope_grads(rf4["f"], rf4["g"], x4, y4, p4.eps)
    fb_full = time.perf_counter() - t0

    ref = sinkhorn.reduced_sinkhorn(alpha, beta, logK, p.eps, p.K, tol=TOL)
    rv = objective.reduced_values(ref["f"], ref["g"], Ck, p.eps, alpha, beta)
    P_ref = p.K * rv["P"]
    f = f_gpu.detach().cpu().numpy().astype(np.float64)
    g = g_gpu.detach().cpu().numpy().astype(np.float64)
    Tg = sinkhorn.reduced_plan_blocks(f, g, Ck, p.eps)
    Tr = sinkhorn.reduced_plan_blocks(ref["f"], ref["g"], Ck, p.eps)
    return {"value": round(iters / dt, 2), "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} float64 reduced Sinkhorn iterations (m={p.m}, NumPy/SciPy "
                      f"logsumexp, one thread) after a {t_fold:.2f} s fold",
            "host": {"cpu_model": model, "nproc": nproc, "usable_cpus": usable},
            "reduced_all_cores": {"value": round(iters_mt / dt_mt, 2), "unit": "iters/s",
                                  "cores": threads,
                                  "sample": f"{iters_mt} iterations of the oracle's row and "
                                            f"column half-steps on {threads} threads"},
            "full_size": {"s_per_iter_one_thread": round(full_1t, 4),
                          "s_per_iter_all_cores": round(full_mt, 4), "cores": threads,
                          "sample": f"n={n}: one full_sinkhorn iteration on one thread (with its "
                                    f"residual pass); two iterations of the half-steps on "
                                    f"{threads} threads"},
            "forward_backward_n4096_K8": {
                "reduced_s": round(fb_red, 4), "full_s": round(fb_full, 4), "cores": 1,
                "sample": "oracle solve to 1e-6 (reduced: fold + cyclic Sinkhorn; full: "
                          "full_sinkhorn on the n x n cost) and the envelope gradients of every "
                          "point and marginal, one thread"},
            "oracle_iters_to_tol": ref["iters"],
            "gpu_vs_fp64": {"objective_rel": abs(vr["P"] - P_ref) / max(abs(P_ref), p.K * rv["CT"]),
                            "plan_l1_rel": float(np.abs(Tg - Tr).sum() / Tr.sum())}}


if __name__ == "__main__":
    main()
