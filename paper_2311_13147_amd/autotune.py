"""Autotuner for the batched call: picks, per (power-of-two size bucket, K, dim), two launch
knobs by timing the batched launch (fold, solve and values, without coordinate gradients,
which neither knob touches) on synthetic problems of that class:

* the number of lanes that cooperate on one row of the solve's log-sum-exp (16, 32 or 64),
* the fold's columns per tile (128, 256, 512; fewer, larger tiles or more, smaller ones),

one after the other (the fold knob with the best lane count).  The table, tuning/<arch>.json,
maps "bucket/K/dim" to the packed tile_cfg (lanes | columns / 64 << 8) that `Batch` gives each
descriptor, with every timing beside it.

Run on the GPU:  python -m paper_2311_13147_amd.autotune [--arch gfx950] [--per-bucket 16]
"""
from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np
import torch

from . import _binding as B
from .batched import Batch, _TUNING_DIR, tuning_key

LANES = (16, 32, 64)
FOLD_COLS = (128, 256, 512)
BUCKETS = (32, 64, 128, 256, 512, 1024)
KS = (4, 8, 16, 32)
DIMS = (2, 3)


def _sample_problems(m: int, K: int, dim: int, count: int, rng: np.random.Generator):
    """Tuning inputs: K-fold rotated random clouds in the unit cube, uniform marginals,
    eps = 0.05 median(C)."""
    probs = []
    for _ in range(count):
        base_x = rng.uniform(-1, 1, size=(m, dim))
        base_y = rng.uniform(-1, 1, size=(m, dim))
        xs, ys = [], []
        for k in range(K):
            th = 2 * math.pi * k / K
            R = np.eye(dim)
            R[0, 0], R[0, 1], R[1, 0], R[1, 1] = math.cos(th), -math.sin(th), math.sin(th), math.cos(th)
            xs.append(base_x @ R.T)
            ys.append(base_y @ R.T)
        x = np.concatenate(xs).astype(np.float32)
        y = np.concatenate(ys).astype(np.float32)
        n = K * m
        a = np.full(n, 1.0 / n, np.float32)
        sub = rng.choice(n, size=min(n, 2048), replace=False)  # median over a sample
        c = ((base_x[:256, None, :] - y[None, sub, :]) ** 2).sum(-1)
        probs.append({"x": x, "y": y, "a": a, "b": a.copy(), "eps": 0.05 * float(np.median(c)),
                      "K": K})
    return probs


def _time(batch: Batch, opts, reps: int) -> float:
    batch.run(opts)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.run(opts)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(arch="gfx950", per_bucket=16, buckets=BUCKETS, ks=KS, dims=DIMS, reps=3, seed=0,
         out_dir=None):
    rng = np.random.default_rng(seed)
    table, timings = {}, {}
    opts = B.make_opts(tol=1e-6, max_iter=2000)
    for mb in buckets:
        for K in ks:
            for dim in dims:
                key = tuning_key(mb, K, dim)
                batch = Batch(_sample_problems(mb, K, dim, per_bucket, rng), want_grad=False,
                              tile_cfg=[0] * per_bucket)
                best_l, best_ms = 0, float("inf")
                for lanes in LANES:
                    batch.set_tile_cfg([lanes] * per_bucket)
                    ms = _time(batch, opts, reps)
                    timings[f"{key}/lanes{lanes}"] = round(ms, 4)
                    if ms < best_ms:
                        best_l, best_ms = lanes, ms
                best_c = 0
                if mb > min(FOLD_COLS):  # smaller blocks fit one tile of any width
                    for cols in FOLD_COLS:
                        cfg = best_l | (cols // 64) << 8
                        batch.set_tile_cfg([cfg] * per_bucket)
                        ms = _time(batch, opts, reps)
                        timings[f"{key}/lanes{best_l}/fold{cols}"] = round(ms, 4)
                        if ms < best_ms:
                            best_c, best_ms = cols // 64, ms
                table[key] = best_l | best_c << 8
                print(f"{key:>12s}: lanes {best_l:2d}, fold columns "
                      f"{64 * best_c if best_c else 256:4d}: {best_ms:8.3f} ms", flush=True)
                del batch
    out_dir = out_dir or _TUNING_DIR
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"{arch}.json")
    with open(path, "w") as fh:
        json.dump({"arch": arch, "tile_cfg": table, "timings_ms": timings,
                   "per_bucket": per_bucket, "reps": reps,
                   "key": "size bucket / K / dim", "value": "lanes | fold columns / 64 << 8"},
                  fh, indent=1, sort_keys=True)
    return path, table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--arch", default="gfx950")
    ap.add_argument("--per-bucket", type=int, default=16)
    ap.add_argument("--out-dir", default=None)
    args = ap.parse_args()
    print(tune(args.arch, args.per_bucket, out_dir=args.out_dir))
