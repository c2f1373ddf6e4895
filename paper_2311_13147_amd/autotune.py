"""Autotuner for the batched solver: picks, per power-of-two block-size bucket, the number of
lanes that cooperate on one row of the log-sum-exp (16, 32 or 64) by timing the batched launch
on synthetic problems of that bucket, and writes the table to tuning/<arch>.json, which
`Batch` reads to fill each descriptor's tile_cfg.

Run on the GPU:  python -m paper_2311_13147_amd.autotune [--arch gfx950] [--per-bucket 64]
"""
from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np
import torch

from . import _binding as B
from .batched import Batch, _TUNING_DIR, size_bucket

CANDIDATES = (16, 32, 64)


def _sample_problems(m: int, count: int, rng: np.random.Generator):
    """Tuning inputs: K-fold rotated random clouds in the unit disc, uniform marginals."""
    probs = []
    for _ in range(count):
        K = int(rng.choice([4, 8, 16, 32]))
        dim = int(rng.choice([2, 3]))
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
        probs.append({"x": x, "y": y, "a": a, "b": a.copy(), "eps": 0.1, "K": K})
    return probs


def tune(arch="gfx950", per_bucket=64, buckets=(32, 64, 128, 256, 512, 1024), reps=3, seed=0,
         out_dir=None):
    rng = np.random.default_rng(seed)
    table, timings = {}, {}
    opts = B.make_opts(tol=1e-6, max_iter=200)
    for mb in buckets:
        probs = _sample_problems(mb, per_bucket, rng)
        best, best_ms = 0, float("inf")
        for cfg in CANDIDATES:
            batch = Batch(probs, want_grad=True, tile_cfg=[cfg] * len(probs))
            batch.run(opts)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                batch.run(opts)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            timings[f"{mb}/{cfg}"] = round(ms, 4)
            print(f"bucket m<={mb:5d} lanes/row={cfg:2d}: {ms:8.3f} ms", flush=True)
            if ms < best_ms:
                best, best_ms = cfg, ms
        table[size_bucket(mb)] = best
    out_dir = out_dir or _TUNING_DIR
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"{arch}.json")
    with open(path, "w") as fh:
        json.dump({"arch": arch, "tile_cfg": table, "timings_ms": timings,
                   "per_bucket": per_bucket}, fh, indent=1, sort_keys=True)
    return path, table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--arch", default="gfx950")
    ap.add_argument("--per-bucket", type=int, default=64)
    ap.add_argument("--out-dir", default=None)
    args = ap.parse_args()
    print(tune(args.arch, args.per_bucket, out_dir=args.out_dir))
