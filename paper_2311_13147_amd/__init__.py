"""csot -- cyclic-symmetric entropic optimal transport on AMD MI355X (gfx950).

A HIP implementation of the cyclic Sinkhorn method of "Optimal Transport with Cyclic
Symmetry" (Takeda, Akagi, Marumo, Niwa; AAAI 2024) with plain full-size Sinkhorn beside it.
The compute lives in libcsot.so (C ABI in include/csot.h); this package is a thin ctypes
binding with the same entry-point names plus autograd wrappers.  PyTorch provides device
memory and the stream only.  Importing fails loudly when the library is not built.
"""
from ._binding import (  # noqa: F401
    CsotError,
    EXPORTED,
    LIB_PATH,
    OT_DSTATS_LEN,
    Problem,
    make_opts,
    ot_cost_and_grad,
    ot_expand_plan,
    ot_fold_kernel,
    ot_full_plan_info,
    ot_lot_expand,
    ot_lot_fold,
    ot_measure_peaks,
    ot_reduced_plan_info,
    ot_sinkhorn_full,
    ot_sinkhorn_reduced,
    ot_sinkhorn_reduced_noalloc,
    ot_srot_reduced,
    ot_symmetrize_cost,
    ot_workspace_bytes,
    raw_lib,
    values_dict,
    workspace,
)
from .autograd import CyclicOT, CyclicOTCost, FullOT  # noqa: F401
from .batched import Batch, BatchDesc  # noqa: F401
from .two_stage import two_stage_sinkhorn  # noqa: F401
