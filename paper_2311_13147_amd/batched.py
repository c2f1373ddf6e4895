"""Batched cyclic problems: descriptor packing for ot_sinkhorn_reduced_batched (marshalling
only -- every step runs in the library's kernels).

`Batch` packs many problems into flat device buffers (coordinates, marginals, scratch,
outputs), builds the device descriptor array and the work plan, and launches the batched call
on the current stream.  `Batch.capture()` records the launch in a torch CUDA graph (a HIP graph
on ROCm); the launch sequence contains kernels only.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import _binding as B

_TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


class BatchDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("K", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("tile_cfg", ctypes.c_int32), ("eps", ctypes.c_double),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("a", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("logK", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("g", ctypes.c_void_p), ("dx", ctypes.c_void_p), ("dy", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("da", ctypes.c_void_p), ("db", ctypes.c_void_p)]


def _setup_lib():
    lib = B.raw_lib()
    PD = ctypes.POINTER(BatchDesc)
    lib.ot_batched_plan_len.restype = ctypes.c_size_t
    lib.ot_batched_plan_len.argtypes = [ctypes.c_int32]
    lib.ot_batched_plan.restype = ctypes.c_int
    lib.ot_batched_plan.argtypes = [PD, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.ot_batched_workspace_bytes.restype = ctypes.c_size_t
    lib.ot_batched_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.ot_sinkhorn_reduced_batched.restype = ctypes.c_int
    lib.ot_sinkhorn_reduced_batched.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.POINTER(B.OtOpts),
                                                ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    return lib


_lib = _setup_lib()


def scratch_floats(m: int) -> int:
    """Floats of per-problem scratch that ot_sinkhorn_reduced_batched expects (a multiple
    of 4, so that consecutive scratches stay 16-byte aligned)."""
    mp = (m + 3) // 4 * 4
    return (2 * m * mp + 2 * m + 2 * (2 * mp + 64) + 3) // 4 * 4


def size_bucket(m: int) -> str:
    """Power-of-two bucket of the block size used by the tuning table."""
    b = 1
    while b < m:
        b *= 2
    return str(b)


def tuning_key(m: int, K: int, dim: int) -> str:
    """Key of the tuning table: size bucket / K / dim."""
    return f"{size_bucket(m)}/{K}/{dim}"


def tuned_cfg(tuning: dict, m: int, K: int, dim: int) -> int:
    """tile_cfg for one problem: the (bucket, K, dim) entry, else the bucket's, else 0 (the
    kernels' defaults)."""
    return int(tuning.get(tuning_key(m, K, dim), tuning.get(size_bucket(m), 0)))


def load_tuning(arch: str = "gfx950") -> dict:
    path = os.path.join(_TUNING_DIR, f"{arch}.json")
    try:
        with open(path) as fh:
            return json.load(fh).get("tile_cfg", {})
    except (OSError, ValueError):
        return {}


class Batch:
    """A batch of cyclic problems resident on `device`.

    problems: sequence of dicts with float32 numpy arrays x, y ([n, dim]), a, b ([n]) and
    scalars eps, K.  Outputs after `run()`: f(p), g(p) ([m]), dx(p), dy(p) ([n, dim]: every
    point), da(p), db(p) ([n]), values(p) -> {P, D, CT, err_row, err_col, iters, converged,
    flags}."""

    def __init__(self, problems: Sequence[dict], device="cuda:0", want_grad=True,
                 tile_cfg: Optional[Sequence[int]] = None, tuning: Optional[dict] = None):
        self.count = len(problems)
        if self.count == 0:
            raise ValueError("empty batch")
        dev = torch.device(device)
        self.device = dev
        ns = [int(p["a"].shape[0]) for p in problems]
        Ks = [int(p["K"]) for p in problems]
        dims = [int(p["x"].shape[1]) for p in problems]
        ms = [n // K for n, K in zip(ns, Ks)]
        self.ms, self.ns, self.Ks, self.dims = ms, ns, Ks, dims
        tuning = load_tuning() if tuning is None else tuning
        off = lambda sizes: np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        oxy = off([n * d for n, d in zip(ns, dims)])
        oab = off(ns)
        # scratch per problem: logK and its transpose with rows padded to mp = m rounded up
        # to 4 floats, alpha and beta, then the exchange slots of a gang solve (2 mp + 64
        # 64-bit words); each problem's scratch starts 16-byte aligned
        osc = off([scratch_floats(m) for m in ms])
        ofg = off(ms)
        ogr = off([n * d for n, d in zip(ns, dims)])
        f32 = dict(dtype=torch.float32, device=dev)
        X = np.concatenate([np.ascontiguousarray(p["x"], np.float32).ravel() for p in problems])
        Y = np.concatenate([np.ascontiguousarray(p["y"], np.float32).ravel() for p in problems])
        A = np.concatenate([np.ascontiguousarray(p["a"], np.float32) for p in problems])
        Bm = np.concatenate([np.ascontiguousarray(p["b"], np.float32) for p in problems])
        self.X, self.Y = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
        self.A, self.B = torch.from_numpy(A).to(dev), torch.from_numpy(Bm).to(dev)
        self.S = torch.empty(int(osc[-1]), **f32)
        self.F = torch.zeros(int(ofg[-1]), **f32)
        self.G = torch.zeros(int(ofg[-1]), **f32)
        self.DX = torch.empty(int(ogr[-1]), **f32) if want_grad else None
        self.DY = torch.empty(int(ogr[-1]), **f32) if want_grad else None
        self.DA = torch.empty(int(oab[-1]), **f32) if want_grad else None
        self.DB = torch.empty(int(oab[-1]), **f32) if want_grad else None
        self.OUT = torch.zeros((self.count, 8), dtype=torch.float64, device=dev)
        self._off = dict(xy=oxy, ab=oab, fg=ofg, gr=ogr)
        descs = (BatchDesc * self.count)()
        e4, e8 = 4, 8
        for p in range(self.count):
            d = descs[p]
            d.n, d.K, d.dim = ns[p], Ks[p], dims[p]
            d.tile_cfg = (int(tile_cfg[p]) if tile_cfg is not None
                          else tuned_cfg(tuning, ms[p], Ks[p], dims[p]))
            d.eps = float(problems[p]["eps"])
            d.x = self.X.data_ptr() + e4 * int(oxy[p])
            d.y = self.Y.data_ptr() + e4 * int(oxy[p])
            d.a = self.A.data_ptr() + e4 * int(oab[p])
            d.b = self.B.data_ptr() + e4 * int(oab[p])
            d.logK = self.S.data_ptr() + e4 * int(osc[p])
            d.f = self.F.data_ptr() + e4 * int(ofg[p])
            d.g = self.G.data_ptr() + e4 * int(ofg[p])
            d.dx = (self.DX.data_ptr() + e4 * int(ogr[p])) if want_grad else None
            d.dy = (self.DY.data_ptr() + e4 * int(ogr[p])) if want_grad else None
            d.out = self.OUT.data_ptr() + e8 * 8 * p
            d.da = (self.DA.data_ptr() + e4 * int(oab[p])) if want_grad else None
            d.db = (self.DB.data_ptr() + e4 * int(oab[p])) if want_grad else None
        self.host_descs = descs
        self._upload()
        self.WS = torch.empty(max(int(_lib.ot_batched_workspace_bytes(self.count)), 256),
                              dtype=torch.uint8, device=dev)

    def _upload(self):
        """Device copy of the descriptors and the launch plan made from them."""
        descs = self.host_descs
        self.D = torch.frombuffer(bytearray(bytes(descs)), dtype=torch.uint8).to(self.device)
        plen = int(_lib.ot_batched_plan_len(self.count))
        plan = (ctypes.c_int32 * plen)()
        B._check(_lib.ot_batched_plan(descs, self.count, plan))
        self.plan_host = np.frombuffer(plan, dtype=np.int32).copy()
        self.PLAN = torch.from_numpy(self.plan_host).to(self.device)

    def set_tile_cfg(self, tile_cfg: Sequence[int]):
        """New launch knobs (see ot_batch_desc.tile_cfg) for every problem; re-plans."""
        for p in range(self.count):
            self.host_descs[p].tile_cfg = int(tile_cfg[p])
        self._upload()

    def run(self, opts: Optional[B.OtOpts] = None):
        """Enqueue the batched solve on the current stream (asynchronous)."""
        opts = opts or B.make_opts()
        rc = _lib.ot_sinkhorn_reduced_batched(
            ctypes.c_void_p(self.D.data_ptr()), self.count, ctypes.c_void_p(self.PLAN.data_ptr()),
            ctypes.c_void_p(self.plan_host.ctypes.data), ctypes.byref(opts),
            ctypes.c_void_p(self.WS.data_ptr()), self.WS.numel(),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        B._check(rc)

    def capture(self, opts: Optional[B.OtOpts] = None) -> torch.cuda.CUDAGraph:
        """Record one batched launch sequence in a graph (replay with graph.replay())."""
        self._graph_opts = opts or B.make_opts()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run(self._graph_opts)  # warm-up outside capture (sets kernel attributes)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.run(self._graph_opts)
        return graph

    # -- views of the results -----------------------------------------------------------------
    def f(self, p):
        o = self._off["fg"]
        return self.F[int(o[p]):int(o[p + 1])]

    def g(self, p):
        o = self._off["fg"]
        return self.G[int(o[p]):int(o[p + 1])]

    def dx(self, p):
        o = self._off["gr"]
        return self.DX[int(o[p]):int(o[p + 1])].view(self.ns[p], self.dims[p])

    def dy(self, p):
        o = self._off["gr"]
        return self.DY[int(o[p]):int(o[p + 1])].view(self.ns[p], self.dims[p])

    def da(self, p):
        o = self._off["ab"]
        return self.DA[int(o[p]):int(o[p + 1])]

    def db(self, p):
        o = self._off["ab"]
        return self.DB[int(o[p]):int(o[p + 1])]

    def values(self, p):
        v = self.OUT[p].detach().cpu().tolist()
        return {"P": v[0], "D": v[1], "CT": v[2], "err_row": v[3], "err_col": v[4],
                "iters": int(v[5]), "converged": bool(v[6]), "flags": int(v[7])}
