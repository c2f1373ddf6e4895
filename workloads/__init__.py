"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs: point clouds with K-fold rotational symmetry, periodic
marginals, dense block-circulant cost blocks and the noise used for the approximate-symmetry
workload.  It holds none of the transport arithmetic (no Gibbs kernel, no Sinkhorn step, no
plan); both the CPU oracle and the GPU path consume what it returns.

Layout conventions (the same everywhere in the project):

* a problem has ``n = K * m`` points per side, stored block-major: point ``I = r*m + i`` is the
  ``i``-th point of block ``r`` (Assumption 1 of the paper: ``a = (alpha; ...; alpha)``).
* coordinates are float32 ``[n, dim]``; marginals are float32 ``[n]``.  The float32 arrays are
  what the GPU receives; the oracle receives float64 copies of the very same values.

Readings of the paper's workload descriptions (all listed in the design notes):

* "uniform in the annulus r in [0.5, 1]" is read as area-uniform: ``r = sqrt(U(0.25, 1))``,
  ``theta ~ U[0, 2 pi)``; block ``r`` is block 0 rotated counter-clockwise by ``2 pi r / K``.
  In 3-D the extra coordinate is ``U(-0.5, 0.5)`` and the rotation is about the z axis.
* "a and b = one random Dirichlet(1) vector tiled K times, divided by K" is read as two
  independent Dirichlet draws, one for a and one for b.
* ``eps = factor * median(C)`` uses the median of the squared Euclidean distances between the
  float32 coordinates (evaluated in float64).  For an exactly symmetric cloud the multiset of
  all ``n*n`` costs is K copies of block-row 0, so the median over block-row 0 is used.  For
  the jittered workload the median of the un-jittered symmetric cloud is used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Problem",
    "annulus_cloud",
    "equal_mass_pair",
    "dirichlet_periodic_pair",
    "median_sq_dist_row0",
    "symmetric_problem",
    "jittered_problem",
    "dense_appd_problem",
    "batched_problems",
    "BatchItem",
    "image_pixel_order",
    "synthetic_image",
    "image_problem",
]


@dataclasses.dataclass
class Problem:
    """One synthetic transport problem (float32 arrays, block-major order)."""

    n: int
    K: int
    dim: int
    x: Optional[np.ndarray]  # [n, dim] float32, or None for a dense-cost problem
    y: Optional[np.ndarray]
    a: np.ndarray  # [n] float32
    b: np.ndarray  # [n] float32
    eps: float
    C_row0: Optional[np.ndarray] = None  # [m, n] float32 dense block-row 0 (dense problems)
    seed: int = 0
    name: str = ""

    @property
    def m(self) -> int:
        return self.n // self.K


def _rotation(theta: float, dim: int) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    R = np.eye(dim)
    R[0, 0], R[0, 1], R[1, 0], R[1, 1] = c, -s, s, c
    return R


def annulus_cloud(m: int, K: int, dim: int, rng: np.random.Generator) -> np.ndarray:
    """K-fold rotationally symmetric cloud, float64 ``[K*m, dim]``, block-major."""
    r = np.sqrt(rng.uniform(0.25, 1.0, size=m))
    th = rng.uniform(0.0, 2.0 * math.pi, size=m)
    base = np.zeros((m, dim))
    base[:, 0] = r * np.cos(th)
    base[:, 1] = r * np.sin(th)
    if dim == 3:
        base[:, 2] = rng.uniform(-0.5, 0.5, size=m)
    blocks = [base @ _rotation(2.0 * math.pi * k / K, dim).T for k in range(K)]
    return np.concatenate(blocks, axis=0)


def equal_mass_pair(a: np.ndarray, b: np.ndarray):
    """Round two nonnegative vectors to float32 values on one common grid ``2^e`` chosen so
    that every entry is an integer multiple below ``2^23`` (hence exact in float32), then move
    the rounding difference onto the largest entry of b.  The two float32 vectors then have
    exactly equal sums (the float64 sums of their values are exact), so a Sinkhorn residual can
    reach any tolerance instead of stalling at the float32 mass mismatch."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mx = max(a.max(), b.max())
    step = 2.0 ** (math.floor(math.log2(mx)) - 22)
    ka = np.rint(a / step)
    kb = np.rint(b / step)
    kb[np.argmax(kb)] += ka.sum() - kb.sum()
    return (ka * step).astype(np.float32), (kb * step).astype(np.float32)


def dirichlet_periodic_pair(m: int, K: int, rng_a: np.random.Generator,
                            rng_b: np.random.Generator):
    """Two independent Dirichlet(1) vectors of length m, divided by K, made equal-mass on a
    common float32 grid and tiled K times (so a and b are periodic, Assumption 1)."""
    al = rng_a.dirichlet(np.ones(m)) / K
    be = rng_b.dirichlet(np.ones(m)) / K
    al, be = equal_mass_pair(al, be)
    return np.tile(al, K), np.tile(be, K)


def median_sq_dist_row0(x: np.ndarray, y: np.ndarray, m: int) -> float:
    """Median of the squared distances between the first m points of x and all of y."""
    x0 = x[:m].astype(np.float64)
    yy = y.astype(np.float64)
    d = np.zeros((m, yy.shape[0]))
    for c in range(x0.shape[1]):
        d += (x0[:, None, c] - yy[None, :, c]) ** 2
    return float(np.median(d))


def symmetric_problem(n: int, K: int, dim: int = 2, eps_factor: float = 0.05,
                      seed: int = 0, name: str = "") -> Problem:
    """Strictly K-fold symmetric point-cloud problem (the n=512/K=8, n=8192/K=16 and
    n=4096/K=8 workloads).  Sub-seeds: x=seed, y=seed+1, a=seed+2, b=seed+3."""
    if n % K:
        raise ValueError("n must be a multiple of K")
    m = n // K
    x = annulus_cloud(m, K, dim, np.random.default_rng(seed)).astype(np.float32)
    y = annulus_cloud(m, K, dim, np.random.default_rng(seed + 1)).astype(np.float32)
    a, b = dirichlet_periodic_pair(m, K, np.random.default_rng(seed + 2),
                                   np.random.default_rng(seed + 3))
    eps = eps_factor * median_sq_dist_row0(x, y, m)
    return Problem(n=n, K=K, dim=dim, x=x, y=y, a=a, b=b, eps=eps, seed=seed,
                   name=name or f"sym_n{n}_K{K}_d{dim}")


def jittered_problem(n: int, K: int, sigma: float = 1e-3, noise: float = 0.01,
                     dim: int = 2, eps_factor: float = 0.05, seed: int = 200,
                     name: str = "") -> Problem:
    """Approximately symmetric problem: every replicated point gets N(0, sigma^2) jitter and
    each marginal entry is multiplied by exp(noise * xi), xi ~ N(0,1), then renormalised.
    The jitter/noise stream uses sub-seed seed+4.  With sigma = noise = 0 this returns the
    strictly symmetric problem of the same seed."""
    base = symmetric_problem(n, K, dim, eps_factor, seed)
    rng = np.random.default_rng(seed + 4)
    x = base.x.astype(np.float64) + sigma * rng.standard_normal(base.x.shape)
    y = base.y.astype(np.float64) + sigma * rng.standard_normal(base.y.shape)
    a = base.a.astype(np.float64) * np.exp(noise * rng.standard_normal(n))
    b = base.b.astype(np.float64) * np.exp(noise * rng.standard_normal(n))
    a, b = equal_mass_pair(a / a.sum(), b / b.sum())
    return Problem(n=n, K=K, dim=dim, x=x.astype(np.float32), y=y.astype(np.float32),
                   a=a, b=b, eps=base.eps, seed=seed,
                   name=name or f"jit_n{n}_K{K}_s{sigma:g}")


def dense_appd_problem(n: int, K: int, seed: int = 0, lam: float = 0.5,
                       name: str = "") -> Problem:
    """Dense-cost workload of the paper's synthetic experiment (App. D): alpha, beta ~
    U[0,1)^m tiled and normalised to sum 1; C_k ~ N(3, 5^2)^{m x m} shifted by the absolute
    value of the overall minimum; lambda = 0.5.  Returns block-row 0 as ``C_row0[i, k*m+j]
    = C_k[i, j]`` (float32)."""
    if n % K:
        raise ValueError("n must be a multiple of K")
    m = n // K
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(0.0, 1.0, size=m)
    beta = rng.uniform(0.0, 1.0, size=m)
    al, be = equal_mass_pair(alpha / (K * alpha.sum()), beta / (K * beta.sum()))
    a, b = np.tile(al, K), np.tile(be, K)
    Ck = rng.normal(3.0, 5.0, size=(K, m, m))
    Ck = Ck + abs(Ck.min())
    C_row0 = np.concatenate(list(Ck), axis=1).astype(np.float32)  # [m, K*m]
    return Problem(n=n, K=K, dim=0, x=None, y=None, a=a, b=b, eps=lam, C_row0=C_row0,
                   seed=seed, name=name or f"appd_n{n}_K{K}")


@dataclasses.dataclass
class BatchItem:
    m: int
    K: int
    dim: int
    seed: int


def batched_problems(count: int = 1024, m_lo: int = 32, m_hi: int = 1024,
                     Ks=(4, 8, 16, 32), seed: int = 400) -> list:
    """Shapes of the uneven batched workload: m = round(exp U[ln m_lo, ln m_hi]),
    K uniform in Ks, dim uniform in {2, 3}; problem p uses base seed ``seed + 10*p``."""
    rng = np.random.default_rng(seed)
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), size=count))).astype(int)
    ks = rng.choice(np.asarray(Ks), size=count)
    dims = rng.choice(np.asarray([2, 3]), size=count)
    return [BatchItem(int(ms[p]), int(ks[p]), int(dims[p]), seed + 10 * p) for p in range(count)]


# ---- images with mirror or 90-degree rotational symmetry (Example 1 of the paper) ----------
#
# Readings (listed in the design notes): the paper orders the pixels of an h x w image with
# mirror symmetry about the vertical axis column by column over the left half, then the
# mirrored columns in the same order (its eq. vectorization_mirror); for 90-degree rotational
# symmetry it only says "appropriately ordering", read here as the top-left quadrant column by
# column, then its images under one, two and three quarter turns about the image centre.  The
# cost is a distance between pixel positions (row, column) in pixel units -- the paper names
# Manhattan, Euclidean and Chebyshev; its real-data experiment uses Euclidean and lambda = 0.5.
# The paper's images (a public symmetry database, resized to 64 x 64 and 96 x 96, normalised to
# unit mass) are not available; seeded synthetic grayscale images stand in for them.


def image_pixel_order(h: int, w: int, K: int) -> np.ndarray:
    """Pixel (row, col) of every position I = r*m + i, int64 ``[h*w, 2]``: K = 2 is the mirror
    order (block 1 = block 0 mirrored about the vertical axis), K = 4 the quarter-turn order
    (block r = block 0 turned r quarter turns; needs h == w)."""
    if K == 2:
        if w % 2:
            raise ValueError("mirror symmetry needs an even width")
        k = np.arange(h * w)
        half = h * w // 2
        col = np.where(k < half, k // h, (3 * w) // 2 - k // h - 1)
        return np.stack([k % h, col], axis=1).astype(np.int64)
    if K == 4:
        if h != w or h % 2:
            raise ValueError("quarter-turn symmetry needs an even square image")
        q = h // 2
        k = np.arange(q * q)
        base = np.stack([k % q, k // q], axis=1)  # top-left quadrant, column by column
        blocks = [base]
        for _ in range(3):
            i, j = blocks[-1][:, 0], blocks[-1][:, 1]
            blocks.append(np.stack([j, h - 1 - i], axis=1))  # a quarter turn about the centre
        return np.concatenate(blocks, axis=0).astype(np.int64)
    raise ValueError("image symmetry: K must be 2 (mirror) or 4 (quarter turn)")


def synthetic_image(h: int, w: int, rng: np.random.Generator, blobs: int = 6) -> np.ndarray:
    """A smooth nonnegative grayscale image: a faint background plus Gaussian blobs of random
    position, width and brightness (float64 ``[h, w]``)."""
    ii, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    img = np.full((h, w), 0.05)
    for _ in range(blobs):
        ci, cj = rng.uniform(0, h), rng.uniform(0, w)
        sd = rng.uniform(0.05, 0.2) * min(h, w)
        img += rng.uniform(0.3, 1.0) * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2 * sd * sd))
    return img


def _symmetrise_image(img: np.ndarray, K: int) -> np.ndarray:
    if K == 2:
        return 0.5 * (img + img[:, ::-1])
    return 0.25 * sum(np.rot90(img, r) for r in range(4))


def image_problem(side: int, K: int, metric: str = "euclidean", noise: float = 0.0,
                  lam: float = 0.5, seed: int = 600, name: str = "") -> Problem:
    """Transport between two side x side grayscale images with mirror (K = 2) or quarter-turn
    (K = 4) symmetry, pixels in the block order of ``image_pixel_order``.  Both images are
    exactly symmetric when ``noise = 0``; otherwise every pixel is multiplied by
    ``exp(noise * xi)``, xi ~ N(0, 1), so the symmetry holds only approximately.  Images are
    normalised to unit mass.

    ``metric`` "euclidean", "manhattan" or "chebyshev" gives a dense-cost problem (block-row 0
    ``C_row0[i, k*m + j]`` = the distance between pixels i and k*m + j, in pixel units);
    "sqeuclidean" gives a point problem (x = y = the pixel positions, float32), whose cost is
    the squared distance.  The cost is exactly block-circulant in every case: the mirror and
    the quarter turns permute pixel positions and preserve all four distances.  Sub-seeds: image
    a = seed, image b = seed + 1, noise = seed + 2."""
    pix = image_pixel_order(side, side, K)
    n = side * side
    m = n // K
    imgs = []
    for t in range(2):
        img = _symmetrise_image(synthetic_image(side, side, np.random.default_rng(seed + t)), K)
        imgs.append(img)
    if noise > 0.0:
        rng = np.random.default_rng(seed + 2)
        imgs = [img * np.exp(noise * rng.standard_normal(img.shape)) for img in imgs]
        a = imgs[0][pix[:, 0], pix[:, 1]]
        b = imgs[1][pix[:, 0], pix[:, 1]]
        a, b = equal_mass_pair(a / a.sum(), b / b.sum())
    else:
        # exactly periodic: block 0's pixels, equal-mass on a common grid, tiled K times
        a0 = imgs[0][pix[:m, 0], pix[:m, 1]]
        b0 = imgs[1][pix[:m, 0], pix[:m, 1]]
        a0, b0 = equal_mass_pair(a0 / (K * a0.sum()), b0 / (K * b0.sum()))
        a, b = np.tile(a0, K), np.tile(b0, K)
    pos = pix.astype(np.float64)
    tag = f"img{side}_K{K}_{metric}" + (f"_noise{noise:g}" if noise > 0.0 else "")
    if metric == "sqeuclidean":
        xy = pos.astype(np.float32)
        return Problem(n=n, K=K, dim=2, x=xy, y=xy.copy(), a=a, b=b, eps=lam, seed=seed,
                       name=name or tag)
    d = np.abs(pos[:m, None, :] - pos[None, :, :])  # [m, n, 2] coordinate differences
    if metric == "euclidean":
        C = np.sqrt((d ** 2).sum(-1))
    elif metric == "manhattan":
        C = d.sum(-1)
    elif metric == "chebyshev":
        C = d.max(-1)
    else:
        raise ValueError(f"unknown metric {metric!r}")
    return Problem(n=n, K=K, dim=0, x=None, y=None, a=a, b=b, eps=lam,
                   C_row0=C.astype(np.float32), seed=seed, name=name or tag)
