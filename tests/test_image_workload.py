"""Images with mirror or quarter-turn symmetry (Example 1): the pixel order, the exact
block-circulance of every pixel distance under it, and the cyclic solution equal to the full
one on such inputs (float64 oracle, CPU)."""
import numpy as np
import pytest

import workloads
from oracle import cost, objective, sinkhorn


def _full_cost(pix, metric):
    d = np.abs(pix[:, None, :].astype(np.float64) - pix[None, :, :].astype(np.float64))
    return {"euclidean": np.sqrt((d ** 2).sum(-1)), "manhattan": d.sum(-1),
            "chebyshev": d.max(-1), "sqeuclidean": (d ** 2).sum(-1)}[metric]


def test_mirror_order_is_the_left_half_then_its_mirror_image():
    h, w = 6, 8
    pix = workloads.image_pixel_order(h, w, 2)
    m = h * w // 2
    # a permutation of the pixels
    assert len({tuple(p) for p in pix}) == h * w
    # block 0: the left half, column by column, rows fastest
    assert np.array_equal(pix[:m, 1], np.repeat(np.arange(w // 2), h))
    assert np.array_equal(pix[:m, 0], np.tile(np.arange(h), w // 2))
    # block 1: the same pixels mirrored about the vertical axis
    assert np.array_equal(pix[m:, 0], pix[:m, 0])
    assert np.array_equal(pix[m:, 1], w - 1 - pix[:m, 1])


def test_quarter_turn_order_rotates_block_0():
    h = 6
    pix = workloads.image_pixel_order(h, h, 4)
    m = h * h // 4
    assert len({tuple(p) for p in pix}) == h * h
    img = np.arange(h * h).reshape(h, h)
    for r in range(4):
        # block r lists the pixels that r quarter turns carry block 0's pixels to
        moved = np.rot90(img, -r)  # moved[i', j'] = img[i, j] for (i', j') = turn^r(i, j)
        got = moved[pix[r * m:(r + 1) * m, 0], pix[r * m:(r + 1) * m, 1]]
        assert np.array_equal(got, img[pix[:m, 0], pix[:m, 1]])


@pytest.mark.parametrize("K", [2, 4])
@pytest.mark.parametrize("metric", ["euclidean", "manhattan", "chebyshev", "sqeuclidean"])
def test_pixel_distances_are_exactly_block_circulant(K, metric):
    side = 8
    pix = workloads.image_pixel_order(side, side, K)
    C = _full_cost(pix, metric)
    n, m = side * side, side * side // K
    for r in range(K):
        for c in range(K):
            k = (c - r) % K
            assert np.array_equal(C[r * m:(r + 1) * m, c * m:(c + 1) * m], C[:m, k * m:(k + 1) * m])
    p = workloads.image_problem(side, K, metric)
    if metric == "sqeuclidean":
        assert np.array_equal(cost.sq_euclidean(p.x, p.y), C)
    else:
        assert np.array_equal(p.C_row0, C[:m].astype(np.float32))


@pytest.mark.parametrize("K", [2, 4])
def test_symmetric_images_give_periodic_marginals_and_noise_breaks_them(K):
    p = workloads.image_problem(16, K, noise=0.0)
    m = p.m
    for r in range(1, K):
        assert np.array_equal(p.a[r * m:(r + 1) * m], p.a[:m])
        assert np.array_equal(p.b[r * m:(r + 1) * m], p.b[:m])
    assert abs(float(p.a.astype(np.float64).sum()) - 1.0) < 1e-6
    q = workloads.image_problem(16, K, noise=0.05)
    assert not np.array_equal(q.a[m:2 * m], q.a[:m])
    assert float(q.a.astype(np.float64).sum()) == float(q.b.astype(np.float64).sum())


@pytest.mark.parametrize("K", [2, 4])
def test_cyclic_solution_equals_full_solution_on_symmetric_images(K):
    """Reduced (cyclic) Sinkhorn on an exactly symmetric image pair stops at the iteration of
    full-size Sinkhorn with its potentials tiled, and K times its objective is the full one."""
    p = workloads.image_problem(12, K, "euclidean", lam=0.5)
    Ck = cost.blocks_from_row0(p.C_row0.astype(np.float64), K)
    C = cost.block_circulant_from_blocks(Ck)
    a, b = p.a.astype(np.float64), p.b.astype(np.float64)
    full = sinkhorn.full_sinkhorn(a, b, C, p.eps, tol=1e-11)
    red = sinkhorn.cyclic_sinkhorn(a, b, Ck, p.eps, tol=1e-11)
    assert full["iters"] == red["iters"]
    assert np.abs(full["f"] - np.tile(red["f"], K)).max() < 1e-9
    vf = objective.full_values(full["f"], full["g"], C, p.eps, a, b)
    al, be = sinkhorn.fold_marginals(a, K), sinkhorn.fold_marginals(b, K)
    vr = objective.reduced_values(red["f"], red["g"], Ck, p.eps, al, be)
    assert abs(vf["P"] - K * vr["P"]) < 1e-12 * max(1.0, abs(vf["P"]))
