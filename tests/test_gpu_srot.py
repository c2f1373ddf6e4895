"""GPU parity of the cyclic SROT with the quadratic regulariser (Thm. 2 dual, alternating
maximisation) against the float64 oracle: potentials at fixed iteration counts, the
tolerance solve, and the same call with K = 1 on the full block-circulant cost equal to the
reduced solution tiled."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cost, srot

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def T_(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def _f64(v):
    return np.asarray(v, dtype=np.float64)


def _prob(lib, p):
    if p.dim == 0:
        return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, C=T_(p.C_row0))
    return lib.Problem(T_(p.a), T_(p.b), p.eps, p.K, x=T_(p.x), y=T_(p.y))


def _blocks(p):
    if p.dim == 0:
        return cost.blocks_from_row0(_f64(p.C_row0), p.K)
    return cost.blocks_from_row0(cost.row0_from_points(p.x, p.y, p.K), p.K)


CASES = [
    ("sym_n512_K8_d2", lambda: workloads.symmetric_problem(512, 8, 2, 0.05, seed=0)),
    ("sym_n600_K8_d3", lambda: workloads.symmetric_problem(600, 8, 3, 0.05, seed=7)),
    ("appd_n700_K7_dense", lambda: workloads.dense_appd_problem(700, 7, seed=0)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_srot_parity(lib, name, mk):
    p = mk()
    # lam = 10 median(C): ~100 iterations to 1e-6 and a sparse plan (about 1 % of entries)
    Ck = _blocks(p)
    lam = 10.0 * float(np.median(Ck))
    prob = _prob(lib, p)
    al = _f64(p.a).reshape(p.K, p.m).mean(0)
    be = _f64(p.b).reshape(p.K, p.m).mean(0)
    scale = lam * max(al.max(), be.max()) * p.m  # size of a potential step
    for its in (1, 3, 10):
        print(f"[srot fixed] {name} iters={its}", flush=True)
        w, z, st = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=0.0, max_iter=its))
        ref = srot.cyclic_srot(al, be, Ck, lam, p.K, tol=0.0, max_iter=its)
        assert st["iters"] == its
        assert np.abs(w.cpu().numpy() - ref["w"]).max() < 1e-4 * (np.abs(ref["w"]).max() + scale)
        assert np.abs(z.cpu().numpy() - ref["z"]).max() < 1e-4 * (np.abs(ref["z"]).max() + scale)
    print(f"[srot tol] {name}", flush=True)
    w, z, st = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=1e-6, max_iter=5000))
    ref = srot.cyclic_srot(al, be, Ck, lam, p.K, tol=1e-6, max_iter=5000)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 2, (st["iters"], ref["iters"])
    v = srot.values(_f64(w.cpu()), _f64(z.cpu()), Ck, lam, al, be)
    vr = srot.values(ref["w"], ref["z"], Ck, lam, al, be)
    assert abs(v["primal"] - vr["primal"]) <= 1e-5 * abs(vr["primal"])
    assert np.sqrt(p.K) * np.linalg.norm(v["row"] - al) <= 1.1e-6
    assert abs(st["err_row"] - np.sqrt(p.K) * np.linalg.norm(v["row"] - al)) <= 1e-8


def test_srot_full_size_call_equals_tiled_reduced(lib):
    """K = 1 on the dense n x n block-circulant cost is the full-size problem: its potentials
    after a few iterations are the reduced ones tiled."""
    p = workloads.dense_appd_problem(420, 6, seed=2)
    Ck = _blocks(p)
    lam = 10.0 * float(np.median(Ck))
    print("[srot full=tiled] appd n420 K6", flush=True)
    wr, zr, _ = lib.ot_srot_reduced(_prob(lib, p), lam, lib.make_opts(tol=0.0, max_iter=6))
    Cf = cost.block_circulant_from_row0(p.C_row0, p.K).astype(np.float32)
    fprob = lib.Problem(T_(p.a), T_(p.b), p.eps, 1, C=T_(Cf))
    wf, zf, _ = lib.ot_srot_reduced(fprob, lam, lib.make_opts(tol=0.0, max_iter=6))
    scale = np.abs(wr.cpu().numpy()).max() + np.abs(zr.cpu().numpy()).max()
    assert np.abs(wf.cpu().numpy() - np.tile(wr.cpu().numpy(), p.K)).max() < 1e-4 * scale
    assert np.abs(zf.cpu().numpy() - np.tile(zr.cpu().numpy(), p.K)).max() < 1e-4 * scale
