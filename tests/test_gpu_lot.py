"""GPU parity of the cyclic linear OT steps (Thm. 1, Alg. 1): the min-fold G = min_k C_ijk
with its smallest minimising k (bit-exact against the float64 oracle, ties included), and the
scatter of the small LP's solution into the full plan, whose cost is the full LP optimum."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, lp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def T_(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _prob(lib, p):
    if p.dim == 0:
        return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, C=T_(p.C_row0))
    return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))


def _blocks(p):
    if p.dim == 0:
        return cost.blocks_from_row0(p.C_row0.astype(np.float64), p.K)
    return cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)


CASES = [
    ("sym_n512_K8_d2", lambda: workloads.symmetric_problem(512, 8, 2, 0.05, seed=0)),
    ("sym_n600_K8_d3", lambda: workloads.symmetric_problem(600, 8, 3, 0.05, seed=7)),
    ("sym_n8192_K16_d2", lambda: workloads.symmetric_problem(8192, 16, 2, 0.01, seed=100)),
    # pixel distances: many exact ties between the K shifts
    ("img32_K4_manhattan", lambda: workloads.image_problem(32, 4, "manhattan")),
    ("img32_K2_chebyshev", lambda: workloads.image_problem(32, 2, "chebyshev")),
    ("img16_K4_sqeuclidean", lambda: workloads.image_problem(16, 4, "sqeuclidean")),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_lot_fold_parity(lib, name, mk):
    p = mk()
    print(f"[lot fold] {name}", flush=True)
    G, kmin, alpha, beta = lib.ot_lot_fold(_prob(lib, p))
    Gref, kref = lp.min_fold(_blocks(p))
    assert np.array_equal(kmin.cpu().numpy(), kref)
    assert np.array_equal(G.cpu().numpy(), Gref.astype(np.float32))
    al = p.a.astype(np.float64).reshape(p.K, p.m).mean(0)
    assert np.abs(alpha.cpu().numpy() - al).max() < 1e-9
    ties = (_blocks(p) == Gref[None]).sum(0) > 1
    print(f"[lot fold] {name}: {int(ties.sum())} entries with tied minima", flush=True)


@pytest.mark.parametrize("K,side", [(4, 8), (2, 8)])
def test_lot_end_to_end_reaches_the_full_lp_optimum(lib, K, side):
    """Alg. 1 on small image problems: G and kmin on the GPU, the small LP on the host (SciPy
    HiGHS, as a caller would), the plan scattered on the GPU; the plan equals the oracle's,
    meets the full marginals and costs the full LP optimum (brute force over n^2 variables)."""
    p = workloads.image_problem(side, K, "euclidean")
    print(f"[lot e2e] {p.name}", flush=True)
    prob = _prob(lib, p)
    G, kmin, alpha, beta = lib.ot_lot_fold(prob)
    al, be = alpha.cpu().numpy().astype(np.float64), beta.cpu().numpy().astype(np.float64)
    val, S = lp.lot_value(al, be, G.cpu().numpy().astype(np.float64))
    S32 = S.astype(np.float32)
    T = lib.ot_lot_expand(prob, T_(S32), kmin).cpu().numpy().astype(np.float64)
    Tref = lp.lot_plan(S32, kmin.cpu().numpy(), K)
    assert np.array_equal(T, Tref)
    C = cost.block_circulant_from_row0(p.C_row0.astype(np.float64), K)
    full, _ = lp.lot_value(np.tile(al, K), np.tile(be, K), C)
    assert abs((C * T).sum() - full) <= 1e-6 * full
    assert abs(K * val - full) <= 1e-9 * full
    assert np.abs(T.sum(1) - np.tile(al, K)).max() < 1e-6


def test_lot_expand_full_size_sampled(lib):
    """n = 8192, K = 16: the scatter of a random S against the oracle's on sampled block rows."""
    p = workloads.symmetric_problem(8192, 16, 2, 0.01, seed=100)
    prob = _prob(lib, p)
    G, kmin, _, _ = lib.ot_lot_fold(prob)
    S = np.random.default_rng(9).uniform(0, 1, size=(p.m, p.m)).astype(np.float32)
    T = lib.ot_lot_expand(prob, T_(S), kmin)
    Tref = lp.lot_plan(S, kmin.cpu().numpy(), p.K)
    for r in (0, 5, 15):
        rows = slice(r * p.m, r * p.m + 64)
        assert np.array_equal(T[rows].cpu().numpy().astype(np.float64), Tref[rows])
