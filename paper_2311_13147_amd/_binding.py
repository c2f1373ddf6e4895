"""ctypes binding of libcsot.so -- argument marshalling only.

Every function here has the name of the C entry point it calls (include/csot.h) and does
nothing but check tensor shapes/devices, allocate outputs and workspace with PyTorch, and pass
raw device pointers plus the current HIP stream.  All arithmetic runs in the library's HIP
kernels.  There is no CPU fallback: if the library is missing or cannot be loaded, importing
the package raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcsot.so")

OT_OK, OT_ERR_ARG, OT_ERR_MASS, OT_ERR_NOT_SYMMETRIC, OT_ERR_NOCONV = 0, 1, 2, 3, 4
OT_ERR_NONFINITE, OT_ERR_WORKSPACE, OT_ERR_HIP, OT_ERR_UNSUPPORTED = 5, 6, 7, 8
OT_DSTATS_LEN = 8
_CODE_NAMES = {0: "OT_OK", 1: "OT_ERR_ARG", 2: "OT_ERR_MASS", 3: "OT_ERR_NOT_SYMMETRIC",
               4: "OT_ERR_NOCONV", 5: "OT_ERR_NONFINITE", 6: "OT_ERR_WORKSPACE",
               7: "OT_ERR_HIP", 8: "OT_ERR_UNSUPPORTED"}


class CsotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


class OtProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("K", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("ldc", ctypes.c_int64), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("eps", ctypes.c_double)]


class OtOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("fold_fp64", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("timing_events", ctypes.c_void_p)]


class OtStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("err_row", ctypes.c_double), ("err_col", ctypes.c_double),
                ("err_row32", ctypes.c_double), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing; build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, VP, SZ, I32, I64, D = (ctypes.POINTER(OtProblem), ctypes.c_void_p, ctypes.c_size_t,
                              ctypes.c_int32, ctypes.c_int64, ctypes.c_double)
    PO, PS = ctypes.POINTER(OtOpts), ctypes.POINTER(OtStats)
    sig = {
        "ot_workspace_bytes": (SZ, [P, PO]),
        "ot_fold_kernel": (ctypes.c_int, [P, PO, VP, VP, VP, VP, SZ, VP]),
        "ot_symmetrize_cost": (ctypes.c_int, [P, VP, I64, VP]),
        "ot_sinkhorn_reduced": (ctypes.c_int, [P, PO, VP, VP, VP, VP, VP, VP, PS, VP, SZ, VP]),
        "ot_sinkhorn_reduced_noalloc": (ctypes.c_int, [P, PO, VP, VP, VP, VP, VP, VP, PS, VP]),
        "ot_sinkhorn_full": (ctypes.c_int, [P, PO, VP, VP, VP, PS, VP, SZ, VP]),
        "ot_expand_plan": (ctypes.c_int, [P, VP, VP, VP, I64, VP]),
        "ot_full_plan_info": (ctypes.c_int, [P, PO, VP]),
        "ot_reduced_plan_info": (ctypes.c_int, [P, PO, VP]),
        "ot_lot_fold": (ctypes.c_int, [P, VP, VP, VP, VP, VP]),
        "ot_lot_expand": (ctypes.c_int, [P, VP, VP, VP, I64, VP]),
        "ot_srot_workspace_bytes": (SZ, [P]),
        "ot_srot_reduced": (ctypes.c_int, [P, D, PO, VP, VP, PS, VP, SZ, VP]),
        "ot_cost_and_grad": (ctypes.c_int, [P, VP, VP, I32, VP, VP, I64, VP, VP, VP, VP, VP, SZ, VP]),
        "ot_peaks_workspace_bytes": (SZ, []),
        "ot_measure_peaks": (ctypes.c_int, [VP, VP, SZ, VP]),
        "ot_last_error": (ctypes.c_char_p, []),
        "ot_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
LIB_PATH = _LIB_PATH
EXPORTED = ("ot_workspace_bytes", "ot_fold_kernel", "ot_symmetrize_cost", "ot_sinkhorn_reduced",
            "ot_sinkhorn_reduced_noalloc",
            "ot_sinkhorn_full", "ot_expand_plan", "ot_full_plan_info", "ot_reduced_plan_info",
            "ot_lot_fold", "ot_lot_expand",
            "ot_srot_workspace_bytes", "ot_srot_reduced",
            "ot_cost_and_grad", "ot_batched_plan_len",
            "ot_batched_plan", "ot_batched_workspace_bytes", "ot_sinkhorn_reduced_batched",
            "ot_peaks_workspace_bytes", "ot_measure_peaks",
            "ot_last_error", "ot_version")


def raw_lib():
    """The ctypes handle (for tests of the host-side validation)."""
    return _lib


def _check(rc: int, allow=()):
    if rc != OT_OK and rc not in allow:
        raise CsotError(rc, _lib.ot_last_error().decode())
    return rc


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f32(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Problem:
    """Device tensors of one problem.  Coordinates (x, y: [n, dim], dim in {2, 3}) or a dense
    cost C ([rows, ldc], dim = 0); marginals a, b [n]; eps > 0; cyclic order K."""

    def __init__(self, a, b, eps, K, x=None, y=None, C=None):
        self.a = _dev_f32(a, "a")
        self.b = _dev_f32(b, "b")
        self.n = int(a.shape[0])
        self.K = int(K)
        self.eps = float(eps)
        self.x = self.y = self.C = None
        if C is not None:
            self.C = _dev_f32(C, "C")
            self.dim = 0
            self.ldc = int(C.stride(0))
        else:
            self.x = _dev_f32(x, "x")
            self.y = _dev_f32(y, "y")
            self.dim = int(x.shape[1])
            self.ldc = 0
        self.device = a.device
        self._c = OtProblem(self.n, self.K, self.dim, _ptr(self.x), _ptr(self.y), _ptr(self.C),
                            self.ldc, _ptr(self.a), _ptr(self.b), self.eps)
        self._ws_bytes = {}

    @property
    def m(self):
        return self.n // self.K

    def c(self):
        return ctypes.byref(self._c)


def make_opts(tol=1e-6, max_iter=10000, fold_fp64=-1, warm_start=0, validate=0, workgroups=0,
              timing_events=None):
    """Solver options.  timing_events: a pair of torch.cuda.Event(enable_timing=True) that the
    persistent solver calls record right around their solver kernel (elapsed_time between
    them is that kernel alone)."""
    o = OtOpts(float(tol), int(max_iter), int(fold_fp64), int(warm_start), int(validate),
               int(workgroups), 0, None)
    if timing_events is not None:
        e0, e1 = timing_events
        for e in (e0, e1):           # torch creates the native event on first record
            if not e.cuda_event:
                e.record()
        arr = (ctypes.c_void_p * 2)(e0.cuda_event, e1.cuda_event)
        o.timing_events = ctypes.cast(arr, ctypes.c_void_p)
        o._events_keepalive = (arr, e0, e1)
    return o


_ws_cache = {}


def workspace(prob: Problem, opts: Optional[OtOpts] = None,
              stream: Optional[int] = None) -> torch.Tensor:
    """The scratch buffer for calls on `stream` (default: the current stream), grown to what
    `prob` with `opts` needs and kept for later calls on that stream."""
    wg = opts.workgroups if opts else 0
    nbytes = prob._ws_bytes.get(wg)
    if nbytes is None:  # a problem's sizes never change: ask the library once per option set
        nbytes = int(_lib.ot_workspace_bytes(prob.c(), ctypes.byref(opts) if opts else None))
        prob._ws_bytes[wg] = nbytes
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    key = (prob.device, stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=prob.device)
        _ws_cache[key] = ws
    return ws


def ot_workspace_bytes(prob: Problem, opts: Optional[OtOpts] = None) -> int:
    return int(_lib.ot_workspace_bytes(prob.c(), ctypes.byref(opts) if opts else None))


def ot_fold_kernel(prob: Problem, opts: Optional[OtOpts] = None, out=None):
    """-> (logK [m, m], alpha [m], beta [m])"""
    m = prob.m
    if out is None:
        out = (torch.empty((m, m), dtype=torch.float32, device=prob.device),
               torch.empty(m, dtype=torch.float32, device=prob.device),
               torch.empty(m, dtype=torch.float32, device=prob.device))
    logK, alpha, beta = out
    st = torch.cuda.current_stream().cuda_stream
    ws = workspace(prob, opts, st)
    _check(_lib.ot_fold_kernel(prob.c(), ctypes.byref(opts) if opts else None, _ptr(logK),
                               _ptr(alpha), _ptr(beta), _ptr(ws), ws.numel(), ctypes.c_void_p(st)))
    return logK, alpha, beta


def ot_symmetrize_cost(prob: Problem, out=None):
    """-> Csym [m, n]: block-row 0 of the block-circulant projection of the cost."""
    if out is None:
        out = torch.empty((prob.m, prob.n), dtype=torch.float32, device=prob.device)
    _check(_lib.ot_symmetrize_cost(prob.c(), _ptr(out), int(out.stride(0)), _stream()))
    return out


def _stats_dict(st: OtStats):
    return {"iters": st.iters, "converged": bool(st.converged), "err_row": st.err_row,
            "err_col": st.err_col, "err_row32": st.err_row32, "flags": st.flags}


def ot_sinkhorn_reduced(prob: Problem, logK, alpha, beta, opts: Optional[OtOpts] = None,
                        g0=None, host_stats=True, out=None, dstats=None):
    """-> (f [m], g [m], stats).  stats is a dict (host_stats=True, synchronises) or the
    device tensor of OT_DSTATS_LEN doubles."""
    m = prob.m
    _dev_f32(logK, "logK", (m, m))
    _dev_f32(alpha, "alpha", (m,))
    _dev_f32(beta, "beta", (m,))
    opts = opts or make_opts()
    if out is None:
        out = (torch.empty(m, dtype=torch.float32, device=prob.device),
               torch.empty(m, dtype=torch.float32, device=prob.device))
    f, g = out
    if g0 is not None:
        g.copy_(g0)
        opts.warm_start = 1
    if dstats is None:
        dstats = torch.zeros(OT_DSTATS_LEN, dtype=torch.float64, device=prob.device)
    st = torch.cuda.current_stream().cuda_stream
    ws = workspace(prob, opts, st)
    hs = OtStats() if host_stats else None
    _check(_lib.ot_sinkhorn_reduced(prob.c(), ctypes.byref(opts), _ptr(logK), _ptr(alpha),
                                    _ptr(beta), _ptr(f), _ptr(g), _ptr(dstats),
                                    ctypes.byref(hs) if hs is not None else None, _ptr(ws),
                                    ws.numel(), ctypes.c_void_p(st)), allow=(OT_ERR_NOCONV,))
    return f, g, (_stats_dict(hs) if hs is not None else dstats)


def ot_sinkhorn_reduced_noalloc(prob: Problem, logK, alpha, beta, opts: Optional[OtOpts] = None,
                                host_stats=True, out=None, dstats=None):
    """ot_sinkhorn_reduced on the library's fixed device scratch (no workspace) -> (f [m],
    g [m], stats).  Pass `out` and `dstats` to make the call allocate nothing."""
    m = prob.m
    _dev_f32(logK, "logK", (m, m))
    _dev_f32(alpha, "alpha", (m,))
    _dev_f32(beta, "beta", (m,))
    opts = opts or make_opts()
    if out is None:
        out = (torch.empty(m, dtype=torch.float32, device=prob.device),
               torch.empty(m, dtype=torch.float32, device=prob.device))
    f, g = out
    if dstats is None:
        dstats = torch.zeros(OT_DSTATS_LEN, dtype=torch.float64, device=prob.device)
    hs = OtStats() if host_stats else None
    _check(_lib.ot_sinkhorn_reduced_noalloc(prob.c(), ctypes.byref(opts), _ptr(logK), _ptr(alpha),
                                            _ptr(beta), _ptr(f), _ptr(g), _ptr(dstats),
                                            ctypes.byref(hs) if hs is not None else None,
                                            _stream()), allow=(OT_ERR_NOCONV,))
    return f, g, (_stats_dict(hs) if hs is not None else dstats)


def ot_sinkhorn_full(prob: Problem, opts: Optional[OtOpts] = None, g0=None, host_stats=True,
                     out=None, dstats=None):
    """-> (f [n], g [n], stats)"""
    n = prob.n
    opts = opts or make_opts()
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device=prob.device),
               torch.empty(n, dtype=torch.float32, device=prob.device))
    f, g = out
    if g0 is not None:
        g.copy_(g0)
        opts.warm_start = 1
    if dstats is None:
        dstats = torch.zeros(OT_DSTATS_LEN, dtype=torch.float64, device=prob.device)
    st = torch.cuda.current_stream().cuda_stream
    ws = workspace(prob, opts, st)
    hs = OtStats() if host_stats else None
    _check(_lib.ot_sinkhorn_full(prob.c(), ctypes.byref(opts), _ptr(f), _ptr(g), _ptr(dstats),
                                 ctypes.byref(hs) if hs is not None else None, _ptr(ws),
                                 ws.numel(), ctypes.c_void_p(st)), allow=(OT_ERR_NOCONV,))
    return f, g, (_stats_dict(hs) if hs is not None else dstats)


def ot_full_plan_info(prob: Problem, opts: Optional[OtOpts] = None):
    """Launch configuration of ot_sinkhorn_full on the current device -> dict(workgroups,
    rows, blocks, RT, CQ, dense)."""
    info = (ctypes.c_int32 * 6)()
    _check(_lib.ot_full_plan_info(prob.c(), ctypes.byref(opts) if opts else None, info))
    return dict(zip(("workgroups", "rows", "blocks", "RT", "CQ", "dense"), list(info)))


def ot_reduced_plan_info(prob: Problem, opts: Optional[OtOpts] = None):
    """Launch configuration of ot_sinkhorn_reduced on the current device -> dict(workgroups,
    rows, stride, gslab, lds, threads)."""
    info = (ctypes.c_int32 * 6)()
    _check(_lib.ot_reduced_plan_info(prob.c(), ctypes.byref(opts) if opts else None, info))
    return dict(zip(("workgroups", "rows", "stride", "gslab", "lds", "threads"), list(info)))


def ot_expand_plan(prob: Problem, f, g, out=None):
    """-> T [n, n], the block-circulant plan from reduced potentials."""
    if out is None:
        out = torch.empty((prob.n, prob.n), dtype=torch.float32, device=prob.device)
    _check(_lib.ot_expand_plan(prob.c(), _ptr(f), _ptr(g), _ptr(out), int(out.stride(0)),
                               _stream()))
    return out


def ot_lot_fold(prob: Problem, out=None):
    """Cyclic linear OT, first step -> (G [m, m] float32, kmin [m, m] int32, alpha [m],
    beta [m]): G = min_k C_ijk, kmin the smallest minimising k, the folded marginals."""
    m = prob.m
    if out is None:
        out = (torch.empty((m, m), dtype=torch.float32, device=prob.device),
               torch.empty((m, m), dtype=torch.int32, device=prob.device),
               torch.empty(m, dtype=torch.float32, device=prob.device),
               torch.empty(m, dtype=torch.float32, device=prob.device))
    G, kmin, alpha, beta = out
    _dev_f32(G, "G", (m, m))
    if not (kmin.is_cuda and kmin.dtype == torch.int32 and kmin.is_contiguous()
            and tuple(kmin.shape) == (m, m)):
        raise ValueError(f"kmin must be a contiguous int32 CUDA tensor of shape {(m, m)}")
    _check(_lib.ot_lot_fold(prob.c(), _ptr(G), _ptr(kmin), _ptr(alpha), _ptr(beta), _stream()))
    return G, kmin, alpha, beta


def ot_lot_expand(prob: Problem, S, kmin, out=None):
    """Cyclic linear OT, last steps -> T [n, n]: S (the small LP's solution, [m, m] float32)
    placed at k = kmin in every block row (Thm. 1 with Lemma 1)."""
    m = prob.m
    _dev_f32(S, "S", (m, m))
    if not (kmin.is_cuda and kmin.dtype == torch.int32 and kmin.is_contiguous()
            and tuple(kmin.shape) == (m, m)):
        raise ValueError(f"kmin must be a contiguous int32 CUDA tensor of shape {(m, m)}")
    if out is None:
        out = torch.empty((prob.n, prob.n), dtype=torch.float32, device=prob.device)
    _check(_lib.ot_lot_expand(prob.c(), _ptr(S), _ptr(kmin), _ptr(out), int(out.stride(0)),
                              _stream()))
    return out


def ot_srot_reduced(prob: Problem, lam: float, opts: Optional[OtOpts] = None, out=None):
    """Cyclic SROT with the quadratic regulariser (lam/2) x^2 -> (w [m], z [m], stats dict).
    `out` = (w, z) also serves as the warm start when opts.warm_start = 1.  Synchronises."""
    m = prob.m
    opts = opts or make_opts()
    if out is None:
        out = (torch.zeros(m, dtype=torch.float32, device=prob.device),
               torch.zeros(m, dtype=torch.float32, device=prob.device))
    w, z = out
    _dev_f32(w, "w", (m,))
    _dev_f32(z, "z", (m,))
    nbytes = int(_lib.ot_srot_workspace_bytes(prob.c()))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=prob.device)
    hs = OtStats()
    _check(_lib.ot_srot_reduced(prob.c(), float(lam), ctypes.byref(opts), _ptr(w), _ptr(z),
                                ctypes.byref(hs), _ptr(ws), ws.numel(), _stream()),
           allow=(OT_ERR_NOCONV,))
    return w, z, _stats_dict(hs)


def ot_cost_and_grad(prob: Problem, f, g, reduced: bool, want_dC=False, want_dxy=False,
                     want_dab=False, out=None, grads=None):
    """-> dict with 'values' (device double[8]: P, D, <C,T>, err_row, err_col, mass) and the
    requested gradients dC ([m, n] reduced: K T_ijk at [i, k m + j], the derivative with
    respect to block-row 0 of the cost; [n, n] full: T), dx, dy ([n, dim]), da, db
    ([n]).  `grads`: optional dict of preallocated float32 outputs (keys dC, dx, dy, da, db)
    used instead of new tensors."""
    dev = prob.device
    n, m, K = prob.n, prob.m, prob.K
    grads = grads or {}
    vals = out if out is not None else torch.empty(8, dtype=torch.float64, device=dev)

    def buf(key, shape):
        t = grads.get(key)
        if t is None:
            return torch.empty(shape, dtype=torch.float32, device=dev)
        return _dev_f32(t, key, shape)

    dC = buf("dC", (m, n) if reduced else (n, n)) if want_dC else None
    dx = dy = None
    if want_dxy:
        dx = buf("dx", (n, prob.dim))
        dy = buf("dy", (n, prob.dim))
    da = db = None
    if want_dab:
        da = buf("da", (n,))
        db = buf("db", (n,))
    st = torch.cuda.current_stream().cuda_stream
    ws = workspace(prob, None, st)
    lddc = n if dC is not None else 0
    _check(_lib.ot_cost_and_grad(prob.c(), _ptr(f), _ptr(g), 1 if reduced else 0, _ptr(vals),
                                 _ptr(dC), lddc, _ptr(dx), _ptr(dy), _ptr(da), _ptr(db),
                                 _ptr(ws), ws.numel(), ctypes.c_void_p(st)))
    return {"values": vals, "dC": dC, "dx": dx, "dy": dy, "da": da, "db": db}


OT_PEAKS_LEN = 9


def ot_measure_peaks(device="cuda:0"):
    """Micro-benchmarks of the device (synchronises) -> dict of issue rates (lane operations
    per second; the matrix cores in multiply-adds per second), copy bandwidth (bytes/s) and
    slot latencies (s)."""
    nbytes = int(_lib.ot_peaks_workspace_bytes())
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    out = (ctypes.c_double * OT_PEAKS_LEN)()
    _check(_lib.ot_measure_peaks(out, _ptr(ws), nbytes, _stream()))
    del ws
    keys = ("fma32_per_s", "fma64_per_s", "exp2_per_s", "full_entry_mix_per_s", "copy_bytes_per_s",
            "slot_hop_s_same_xcd", "slot_hop_s_cross_xcd", "same_xcd_local_publication",
            "mfma64_madd_per_s")
    return dict(zip(keys, list(out)))


def values_dict(vals: torch.Tensor):
    v = vals.detach().cpu().tolist()
    return {"P": v[0], "D": v[1], "CT": v[2], "err_row": v[3], "err_col": v[4], "mass": v[5]}
