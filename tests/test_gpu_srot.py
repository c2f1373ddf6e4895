"""GPU parity of the cyclic SROT with the quadratic regulariser (Thm. 2 dual, alternating
maximisation) against the float64 oracle: potentials at fixed iteration counts, the
tolerance solve (the stop test runs on the device), the same call with K = 1 on the full
block-circulant cost equal to the reduced solution tiled, and the full-size solve to
tolerance taking the cyclic one's iterations.

Potential tolerance: the solver finds each root in float32, so a potential carries a
rounding error of a few float32 ulps of the largest potential per update; over ten
alternating updates that stays below 2e-5 of max |w| (resp. max |z|)."""
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
    for its in (1, 3, 10):
        print(f"[srot fixed] {name} iters={its}", flush=True)
        w, z, st = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=0.0, max_iter=its))
        ref = srot.cyclic_srot(al, be, Ck, lam, p.K, tol=0.0, max_iter=its)
        assert st["iters"] == its
        ew = np.abs(w.cpu().numpy() - ref["w"]).max() / np.abs(ref["w"]).max()
        ez = np.abs(z.cpu().numpy() - ref["z"]).max() / np.abs(ref["z"]).max()
        print(f"  relative potential error w {ew:.2e} z {ez:.2e}", flush=True)
        assert ew < 2e-5 and ez < 2e-5, (ew, ez)
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


def test_srot_full_size_to_tolerance_matches_cyclic_iterations(lib):
    """The full-size alternating maximisation from zero keeps the tiled reduced iterates
    (Lemma 1 applied to each update), and its row residual is sqrt(K) times the reduced one's
    norm, so the same call with K = 1 meets the same tolerance after the same iterations,
    +-2 for rounding near the threshold."""
    p = workloads.symmetric_problem(512, 8, 2, 0.05, seed=0)
    Ck = _blocks(p)
    lam = 10.0 * float(np.median(Ck))
    print("[srot tol full vs cyclic] n512 K8", flush=True)
    opts = lib.make_opts(tol=1e-6, max_iter=5000)
    wr, zr, sr = lib.ot_srot_reduced(_prob(lib, p), lam, opts)
    fprob = lib.Problem(T_(p.a), T_(p.b), p.eps, 1, x=T_(p.x), y=T_(p.y))
    wf, zf, sf = lib.ot_srot_reduced(fprob, lam, opts)
    assert sr["converged"] and sf["converged"]
    assert abs(sr["iters"] - sf["iters"]) <= 2, (sr["iters"], sf["iters"])
    assert sf["err_row"] <= 1e-6 and sr["err_row"] <= 1e-6
    ref = srot.cyclic_srot(_f64(p.a).reshape(p.K, p.m).mean(0),
                           _f64(p.b).reshape(p.K, p.m).mean(0), Ck, lam, p.K, tol=1e-6,
                           max_iter=5000)
    assert abs(sf["iters"] - ref["iters"]) <= 2


def test_srot_stops_at_max_iter_and_warm_start(lib):
    """max_iter reached before tol: the call reports not converged after exactly max_iter
    iterations (outputs valid); a warm start from the converged potentials meets the
    tolerance after the first iteration."""
    p = workloads.symmetric_problem(600, 8, 3, 0.05, seed=7)
    Ck = _blocks(p)
    lam = 10.0 * float(np.median(Ck))
    prob = _prob(lib, p)
    print("[srot max_iter / warm] n600 K8 d3", flush=True)
    w, z, st = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=1e-12, max_iter=4))
    assert not st["converged"] and st["iters"] == 4
    ref = srot.cyclic_srot(_f64(p.a).reshape(p.K, p.m).mean(0),
                           _f64(p.b).reshape(p.K, p.m).mean(0), Ck, lam, p.K, tol=0.0,
                           max_iter=4)
    assert np.abs(w.cpu().numpy() - ref["w"]).max() < 2e-5 * np.abs(ref["w"]).max()
    w, z, st = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=1e-6, max_iter=5000))
    assert st["converged"]
    w2, z2, st2 = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=1e-6, max_iter=5000,
                                                               warm_start=1), out=(w, z))
    assert st2["converged"] and st2["iters"] == 1


TERM_CASES = [  # K m per point: 8192 (32 cached terms per thread), 12288 (64), 20480 (recomputed)
    ("sym_n8192_K16_m512", lambda: workloads.symmetric_problem(8192, 16, 2, 0.05, seed=3)),
    ("sym_n12288_K16_m768", lambda: workloads.symmetric_problem(12288, 16, 3, 0.05, seed=4)),
    ("sym_n20480_K16_m1280", lambda: workloads.symmetric_problem(20480, 16, 2, 0.05, seed=5)),
]


@pytest.mark.parametrize("name,mk", TERM_CASES, ids=[c[0] for c in TERM_CASES])
def test_srot_term_storage_variants(lib, name, mk):
    """Each way of holding a point's K m terms during the Newton steps (registers at three
    sizes, or recomputation) against the oracle after 1 and 3 iterations."""
    p = mk()
    Ck = _blocks(p)
    lam = 10.0 * float(np.median(Ck))
    prob = _prob(lib, p)
    al = _f64(p.a).reshape(p.K, p.m).mean(0)
    be = _f64(p.b).reshape(p.K, p.m).mean(0)
    rec = []
    srot.cyclic_srot(al, be, Ck, lam, p.K, tol=0.0, max_iter=3, record=rec)
    for its in (1, 3):
        print(f"[srot terms] {name} iters={its}", flush=True)
        w, z, st = lib.ot_srot_reduced(prob, lam, lib.make_opts(tol=0.0, max_iter=its))
        rw, rz = rec[its - 1]
        assert st["iters"] == its
        ew = np.abs(w.cpu().numpy() - rw).max() / np.abs(rw).max()
        ez = np.abs(z.cpu().numpy() - rz).max() / np.abs(rz).max()
        assert ew < 2e-5 and ez < 2e-5, (ew, ez)


@pytest.mark.parametrize("m,K,dim,seed", [(1, 8, 2, 31), (3, 2, 3, 32), (40, 1, 2, 33)])
def test_srot_degenerate_sizes(lib, m, K, dim, seed):
    """One-point blocks (the reduced dual has one w and one z), three-point blocks and K = 1:
    the tolerance solve against the float64 oracle (iterations +-2, primal value, row
    residual)."""
    p = workloads.symmetric_problem(m * K, K, dim, 0.05, seed=seed)
    Ck = _blocks(p)
    lam = 10.0 * float(np.median(Ck))
    al = _f64(p.a).reshape(p.K, p.m).mean(0)
    be = _f64(p.b).reshape(p.K, p.m).mean(0)
    print(f"[srot degenerate] m={m} K={K} dim={dim}", flush=True)
    w, z, st = lib.ot_srot_reduced(_prob(lib, p), lam, lib.make_opts(tol=1e-6, max_iter=5000))
    ref = srot.cyclic_srot(al, be, Ck, lam, p.K, tol=1e-6, max_iter=5000)
    assert st["converged"] and abs(st["iters"] - ref["iters"]) <= 2, (st["iters"], ref["iters"])
    v = srot.values(_f64(w.cpu()), _f64(z.cpu()), Ck, lam, al, be)
    vr = srot.values(ref["w"], ref["z"], Ck, lam, al, be)
    assert abs(v["primal"] - vr["primal"]) <= 1e-5 * abs(vr["primal"])
    assert np.sqrt(p.K) * np.linalg.norm(v["row"] - al) <= 1.1e-6
