"""Every launch variant of the full-size solver (Alg. 3, stage 2), with coordinates and with a
dense cost, against the float64 oracle.

The planner picks the (RT rows per lane, CQ column split) instance by the problem size: on a
256-CU device n <= 256 -> (1, 16), 512 -> (1, 8), 1024 -> (2, 8), 2048 -> (4, 8), 4096 -> (4, 4),
8192 -> (4, 2), 16384 -> (4, 1).  Each shape below selects one of them (asserted through the
library's plan query).  After 3 iterations from g = 0:
* n <= 2048: f and g against the float64 full-size oracle over all points;
* every n: exactly, step by step, at 64+ sampled rows and columns including the workgroup and
  chunk boundaries (the returned f at row I is the float64 row update of the g after 2
  iterations over all n columns; g at column J the column update of the returned f).
"""
import numpy as np
import pytest
import torch

import workloads
from fullsize_steps import FullData, block_circulant_f32, one_step_errors, sample
from oracle import cost, sinkhorn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
POT = 2e-5

# (n, K, expected (RT, CQ) on 256 CUs)
SHAPES = [(256, 8, (1, 16)), (512, 8, (1, 8)), (1024, 8, (2, 8)), (2048, 16, (4, 8)),
          (4096, 8, (4, 4)), (8192, 16, (4, 2)), (16384, 32, (4, 1))]


def _t(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _f64(v):
    return np.asarray(v.cpu().numpy() if isinstance(v, torch.Tensor) else v, dtype=np.float64)


def _make(n, K, kind):
    if kind == "points":
        dim = 3 if (n // 256) % 3 == 1 else 2
        p = workloads.symmetric_problem(n, K, dim, 0.05, seed=500 + n % 97)
        data = FullData(p.a, p.b, p.eps, x=p.x, y=p.y)
        return p, data, dict(x=_t(p.x), y=_t(p.y))
    p = workloads.dense_appd_problem(n, K, seed=510 + n % 89)
    C = block_circulant_f32(p.C_row0, K)
    return p, FullData(p.a, p.b, p.eps, C=C), dict(C=_t(C))


@pytest.mark.parametrize("kind", ["points", "dense"])
@pytest.mark.parametrize("n,K,variant", SHAPES, ids=[f"n{s[0]}" for s in SHAPES])
def test_full_variant(lib, n, K, variant, kind):
    p, data, dev = _make(n, K, kind)
    prob = lib.Problem(_t(p.a), _t(p.b), p.eps, K, **dev)
    info = lib.ot_full_plan_info(prob)
    print(f"[full variant] n={n} K={K} {kind} plan={info}", flush=True)
    if torch.cuda.get_device_properties(0).multi_processor_count == 256:
        assert (info["RT"], info["CQ"]) == variant
    _, g2, st2 = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=2))
    f, g, st = lib.ot_sinkhorn_full(prob, lib.make_opts(tol=0.0, max_iter=3))
    assert st2["iters"] == 2 and st["iters"] == 3
    fh, gh = _f64(f), _f64(g)
    R = info["rows"]
    bounds = [0, R - 1, R, n - R, n - 1, 2047, 2048, n // 2]
    I = sample(n, 64, 7, bounds)
    J = sample(n, 64, 8, bounds)
    ef, eg = one_step_errors(data, _f64(g2), fh, gh, I, J)
    assert ef < POT and eg < POT, (ef, eg)
    if n <= 2048:
        C = data.rows(np.arange(n))
        ref = sinkhorn.full_sinkhorn(data.a, data.b, C, p.eps, tol=0.0, max_iter=3)
        assert np.abs(fh - ref["f"]).max() / p.eps < POT
        assert np.abs(gh - ref["g"]).max() / p.eps < POT
