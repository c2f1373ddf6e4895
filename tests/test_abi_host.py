"""Host-side checks of the C ABI: the library loads, exports every symbol the header declares,
and rejects invalid arguments before any device work (these calls never reach HIP, so they
run on a machine without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "csot.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_2311_13147_amd import _binding
    return _binding


def test_library_exports_every_declared_symbol(B):
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _header_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(B.EXPORTED) == set(names)


def test_struct_layouts_match_header(B):
    assert ctypes.sizeof(B.OtProblem) == 72
    assert ctypes.sizeof(B.OtOpts) == 40
    assert ctypes.sizeof(B.OtStats) == 40
    assert B.OtProblem.eps.offset == 64


def _prob(B, n=64, K=4, dim=2, eps=0.1, x=1, y=1, C=None, ldc=0, a=1, b=1):
    return B.OtProblem(n, K, dim, x, y, C, ldc, a, b, eps)


def _call_fold(B, p):
    lib = B.raw_lib()
    return lib.ot_fold_kernel(ctypes.byref(p) if p is not None else None, None, 8, 8, 8, None,
                              0, None)


@pytest.mark.parametrize("kw,code,msg", [
    (dict(n=100, K=7), 1, "multiple of K"),
    (dict(n=0), 1, "n must be positive"),
    (dict(K=0), 1, "K must be positive"),
    (dict(eps=0.0), 1, "eps"),
    (dict(eps=float("nan")), 1, "eps"),
    (dict(dim=4), 1, "dim must be"),
    (dict(x=None), 1, "coordinates"),
    (dict(a=None), 1, "marginals"),
    (dict(dim=0, C=None), 1, "dense cost"),
    (dict(dim=0, C=8, ldc=10), 1, "ldc"),
])
def test_invalid_problem_is_rejected(B, kw, code, msg):
    rc = _call_fold(B, _prob(B, **kw))
    assert rc == code
    assert msg in B.raw_lib().ot_last_error().decode()


def test_null_problem(B):
    assert _call_fold(B, None) == B.OT_ERR_ARG


def test_invalid_options_are_rejected(B):
    lib = B.raw_lib()
    p = _prob(B)
    for opts in (B.make_opts(max_iter=0), B.make_opts(tol=-1.0), B.make_opts(fold_fp64=3),
                 B.make_opts(workgroups=-2)):
        rc = lib.ot_fold_kernel(ctypes.byref(p), ctypes.byref(opts), 8, 8, 8, None, 0, None)
        assert rc == B.OT_ERR_ARG


def test_null_outputs_are_rejected(B):
    lib = B.raw_lib()
    p = _prob(B)
    assert lib.ot_fold_kernel(ctypes.byref(p), None, None, 8, 8, None, 0, None) == B.OT_ERR_ARG
    assert lib.ot_expand_plan(ctypes.byref(p), 8, 8, None, 64, None) == B.OT_ERR_ARG
    assert lib.ot_expand_plan(ctypes.byref(p), 8, 8, 8, 10, None) == B.OT_ERR_ARG
    assert lib.ot_symmetrize_cost(ctypes.byref(p), 8, 3, None) == B.OT_ERR_ARG
    assert lib.ot_sinkhorn_reduced(ctypes.byref(p), None, None, 8, 8, 8, 8, 8, None, None, 0,
                                   None) == B.OT_ERR_ARG
    assert lib.ot_sinkhorn_full(ctypes.byref(p), None, None, 8, 8, None, None, 0,
                                None) == B.OT_ERR_ARG
    # dx/dy make no sense for a dense cost
    pd = _prob(B, dim=0, C=8, ldc=64)
    assert lib.ot_cost_and_grad(ctypes.byref(pd), 8, 8, 1, 8, None, 0, 8, None, None, None,
                                None, 0, None) == B.OT_ERR_ARG
    assert lib.ot_cost_and_grad(ctypes.byref(p), 8, 8, 2, 8, None, 0, None, None, None, None,
                                None, 0, None) == B.OT_ERR_ARG


def test_workspace_is_checked_before_launch(B):
    lib = B.raw_lib()
    p = _prob(B)
    need = lib.ot_workspace_bytes(ctypes.byref(p), None)
    assert need > 0
    rc = lib.ot_cost_and_grad(ctypes.byref(p), 8, 8, 1, 8, None, 0, None, None, None, None,
                              None, 0, None)
    assert rc == B.OT_ERR_WORKSPACE
    rc = lib.ot_cost_and_grad(ctypes.byref(p), 8, 8, 1, 8, None, 0, None, None, None, None,
                              256, 16, None)
    assert rc == B.OT_ERR_WORKSPACE
    assert "too small" in lib.ot_last_error().decode()


def test_workspace_bytes_grows_with_n(B):
    lib = B.raw_lib()
    small = lib.ot_workspace_bytes(ctypes.byref(_prob(B, n=512, K=8)), None)
    big = lib.ot_workspace_bytes(ctypes.byref(_prob(B, n=8192, K=16)), None)
    assert big > small > 0
    assert lib.ot_workspace_bytes(None, None) == 0


def test_workspace_bytes_cover_a_workgroup_hint_above_the_cu_count(B):
    """A workgroups hint beyond the CU count makes the reduced solver keep its logK slabs in
    device memory (padded logK and its transpose, 2 m mp floats); the size query covers that
    with a hint even where m alone would not need it (m = 1024 here)."""
    lib = B.raw_lib()
    p = _prob(B, n=2048, K=2)
    plain = lib.ot_workspace_bytes(ctypes.byref(p), None)
    hinted = lib.ot_workspace_bytes(ctypes.byref(p), ctypes.byref(B.make_opts(workgroups=600)))
    assert hinted > plain and hinted >= 2 * 4 * 1024 * 1024


def test_plan_queries_reject_bad_arguments(B):
    lib = B.raw_lib()
    p = _prob(B)
    info = (ctypes.c_int32 * 6)()
    assert lib.ot_full_plan_info(ctypes.byref(p), None, None) == B.OT_ERR_ARG
    assert lib.ot_reduced_plan_info(ctypes.byref(p), None, None) == B.OT_ERR_ARG
    bad = _prob(B, n=100, K=7)
    assert lib.ot_full_plan_info(ctypes.byref(bad), None, info) == B.OT_ERR_ARG
    assert lib.ot_reduced_plan_info(ctypes.byref(bad), None, info) == B.OT_ERR_ARG
    assert lib.ot_full_plan_info(ctypes.byref(p), ctypes.byref(B.make_opts(max_iter=0)),
                                 info) == B.OT_ERR_ARG


def test_batched_plan_validation_and_order(B):
    from paper_2311_13147_amd.batched import BatchDesc, _lib
    descs = (BatchDesc * 3)()
    for d, (n, K) in zip(descs, [(64, 4), (512, 8), (96, 2)]):
        d.n, d.K, d.dim, d.eps = n, K, 2, 0.1
        d.x = d.y = d.a = d.b = d.logK = d.f = d.g = d.out = 8
    plan = (ctypes.c_int32 * _lib.ot_batched_plan_len(3))()
    # values only (no coordinate gradients): row tiles of 16 block-0 points, ceil(m/16) (the
    # column sums are accumulated in the same pass)
    assert _lib.ot_batched_plan(descs, 3, plan) == 0
    assert plan[1] == 1 + 4 + 3
    assert list(plan[34:38]) == [0, 2, 2, 2]  # values-only kind in the K = 2, 4, 8 classes
    for d in descs:
        d.dx = d.dy = 8
    assert _lib.ot_batched_plan(descs, 3, plan) == 0
    H = 4 + 2 * 15 + 14                    # header: counts, 14 value classes' bounds, kinds
    order = list(plan[H:H + 3])
    assert order == [1, 2, 0]              # m = 16, 64, 48: largest first
    assert list(plan[H + 3:H + 6]) == [0, 2, 4]   # fold tiles in that order: ceil(m/32) = 2, 2, 1
    # value tiles grouped by (dim, K) class -- K = 2 (problem 2), K = 4 (0), K = 8 (1) -- each
    # 2 ceil(m/64) tiles of 64 block-0 points (rows, then columns; matrix-core gradients): 2, 2, 2
    assert list(plan[H + 6:H + 9]) == [2, 0, 1]
    assert list(plan[H + 9:H + 12]) == [0, 2, 4]
    cls_q, cls_tile = list(plan[4:19]), list(plan[19:34])
    assert cls_q[:5] == [0, 0, 1, 2, 3] and cls_q[14] == 3
    assert cls_tile[:5] == [0, 0, 2, 4, 6] and cls_tile[14] == 6
    cls_kind = list(plan[34:48])          # bit 0: gradients, bit 1: values only
    assert cls_kind[:4] == [0, 1, 1, 1] and sum(cls_kind[4:]) == 0
    assert plan[0] == 5 and plan[1] == 6    # fold tiles 1 + 2 + 2
    # a K outside {1, 2, 4, 8, 16, 32} takes the generic gradient path: tiles of 4 points
    descs[2].K = 3                          # n = 96: m = 32, 2 ceil(32 / 4) = 16 tiles
    assert _lib.ot_batched_plan(descs, 3, plan) == 0 and plan[1] == 4 + 16
    descs[2].K = 2
    # within a class the largest problem's tiles come first (they run longest)
    same = (BatchDesc * 3)()
    for d, n in zip(same, (64, 512, 256)):  # K = 4: m = 16, 128, 64
        d.n, d.K, d.dim, d.eps = n, 4, 2, 0.1
        d.x = d.y = d.a = d.b = d.logK = d.f = d.g = d.out = d.dx = d.dy = 8
    assert _lib.ot_batched_plan(same, 3, plan) == 0
    assert list(plan[H + 6:H + 9]) == [1, 2, 0]   # m = 128, 64, 16
    assert list(plan[H + 9:H + 12]) == [0, 4, 6]  # 2 ceil(m / 64) tiles: 4, 2, 2
    descs[1].K = 7                          # 512 % 7 != 0
    assert _lib.ot_batched_plan(descs, 3, plan) == B.OT_ERR_ARG
    descs[1].K, descs[1].tile_cfg = 8, 24
    assert _lib.ot_batched_plan(descs, 3, plan) == B.OT_ERR_ARG
    descs[1].tile_cfg = 32 | 17 << 8        # fold columns above 16 x 64
    assert _lib.ot_batched_plan(descs, 3, plan) == B.OT_ERR_ARG
    descs[1].tile_cfg = 32 | 1 << 8         # 64 fold columns per tile: m = 64 -> 2 x 1 tiles
    assert _lib.ot_batched_plan(descs, 3, plan) == 0
    assert plan[0] == 5
    descs[0].tile_cfg = 16 | 1 << 8         # m = 16: one tile whatever the width
    descs[2].tile_cfg = 1 << 8              # m = 48 (lanes by size)
    assert _lib.ot_batched_plan(descs, 3, plan) == 0 and plan[0] == 5
    descs[0].tile_cfg = descs[2].tile_cfg = 0
    descs[1].n = 4096                       # m = 512: 16 row blocks x (512 / width) columns
    for cols, tiles in ((0, 2), (1, 8), (4, 2), (8, 1)):
        descs[1].tile_cfg = cols << 8
        assert _lib.ot_batched_plan(descs, 3, plan) == 0 and plan[0] == 16 * tiles + 2 + 1
    descs[1].n = 512
    descs[1].tile_cfg = 0                   # m = 8192 is above the supported 4096
    descs[1].K = 2
    descs[1].n = 2 * 8192
    assert _lib.ot_batched_plan(descs, 3, plan) == B.OT_ERR_UNSUPPORTED


def test_binding_requires_device_tensors(B):
    import torch
    with pytest.raises(TypeError):
        B.Problem(torch.ones(8), torch.ones(8), 0.1, 2, x=torch.ones(8, 2), y=torch.ones(8, 2))


def test_reserved_option_must_be_zero_and_events_field_layout(B):
    lib = B.raw_lib()
    p = _prob(B)
    o = B.make_opts()
    assert B.OtOpts.timing_events.offset == 32 and o.timing_events is None
    o.reserved = 1
    assert lib.ot_fold_kernel(ctypes.byref(p), ctypes.byref(o), 8, 8, 8, None, 0, None) == B.OT_ERR_ARG
    assert "reserved" in lib.ot_last_error().decode()


def test_batched_plan_gang_tasks(B):
    """Problems above m = 256 become ceil(m / 128) consecutive tasks (members 0..G-1), the
    largest problem first; smaller ones one task each."""
    import numpy as np
    from paper_2311_13147_amd.batched import BatchDesc, _lib
    shapes = [(64 * 4, 4), (512 * 2, 2), (1000 * 3, 3)]  # m = 64, 512, 1000
    descs = (BatchDesc * 3)()
    for d, (n, K) in zip(descs, shapes):
        d.n, d.K, d.dim, d.eps = n, K, 2, 0.1
        d.x = d.y = d.a = d.b = d.logK = d.f = d.g = d.out = 8
    plan = (ctypes.c_int32 * _lib.ot_batched_plan_len(3))()
    assert _lib.ot_batched_plan(descs, 3, plan) == 0
    nt = plan[3]
    assert nt == 8 + 4 + 1
    H = 4 + 2 * 15 + 14
    tasks = np.frombuffer(plan, dtype=np.uint32)[H + 4 * 3:H + 4 * 3 + nt]
    prob, member, gang = tasks & 0xFFFFF, (tasks >> 20) & 63, (tasks >> 26) + 1
    assert list(prob) == [2] * 8 + [1] * 4 + [0]
    assert list(member) == list(range(8)) + list(range(4)) + [0]
    assert list(gang) == [8] * 8 + [4] * 4 + [1]


def test_linear_ot_and_srot_arguments_are_checked_before_launch(B):
    """The linear OT and quadratic SROT entry points reject bad arguments on the host, before
    any device work: null outputs, a short leading dimension, lam <= 0, a missing host stats
    struct, warm_start = 2, and a too small workspace."""
    lib = B.raw_lib()
    p = _prob(B)
    assert lib.ot_lot_fold(ctypes.byref(p), None, 8, 8, 8, None) == B.OT_ERR_ARG
    assert lib.ot_lot_fold(ctypes.byref(p), 8, None, 8, 8, None) == B.OT_ERR_ARG
    assert lib.ot_lot_expand(ctypes.byref(p), 8, 8, None, 64, None) == B.OT_ERR_ARG
    assert lib.ot_lot_expand(ctypes.byref(p), 8, 8, 8, 63, None) == B.OT_ERR_ARG
    assert "ldt" in lib.ot_last_error().decode()
    st = B.OtStats()
    need = lib.ot_srot_workspace_bytes(ctypes.byref(p))
    assert need > 0
    assert lib.ot_srot_reduced(ctypes.byref(p), 0.0, None, 8, 8, ctypes.byref(st), 8, need,
                               None) == B.OT_ERR_ARG
    assert "lam" in lib.ot_last_error().decode()
    assert lib.ot_srot_reduced(ctypes.byref(p), 1.0, None, 8, 8, None, 8, need,
                               None) == B.OT_ERR_ARG
    assert lib.ot_srot_reduced(ctypes.byref(p), 1.0, None, None, 8, ctypes.byref(st), 8, need,
                               None) == B.OT_ERR_ARG
    o = B.make_opts(warm_start=2)
    assert lib.ot_srot_reduced(ctypes.byref(p), 1.0, ctypes.byref(o), 8, 8, ctypes.byref(st), 8,
                               need, None) == B.OT_ERR_ARG
    assert lib.ot_srot_reduced(ctypes.byref(p), 1.0, None, 8, 8, ctypes.byref(st), 8,
                               need - 1, None) == B.OT_ERR_WORKSPACE
    # the workspace grows with m
    big = _prob(B, n=4096, K=4)
    assert lib.ot_srot_workspace_bytes(ctypes.byref(big)) > need


def test_tuning_table_lookup():
    """The batched tuning table is keyed by size bucket / K / dim; older tables keyed by the
    bucket alone still apply, and a missing entry leaves the kernels' defaults (0)."""
    from paper_2311_13147_amd.batched import size_bucket, tuned_cfg, tuning_key
    assert size_bucket(33) == "64" and size_bucket(64) == "64" and size_bucket(1) == "1"
    assert tuning_key(300, 16, 3) == "512/16/3"
    table = {"512/16/3": 64 | 4 << 8, "512": 32}
    assert tuned_cfg(table, 300, 16, 3) == 64 | 4 << 8
    assert tuned_cfg(table, 300, 8, 3) == 32
    assert tuned_cfg(table, 40, 8, 3) == 0
