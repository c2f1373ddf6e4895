"""CPU oracle for cyclic entropic optimal transport -- TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 NumPy/SciPy code written from the paper "Optimal Transport with Cyclic
Symmetry" (Takeda, Akagi, Marumo, Niwa; AAAI 2024).  It is the yardstick the GPU library is
checked against and shares no code with it: it does not import the package, its kernels, its
headers or its binding, and the package never imports it.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import or run anything here.

Modules
-------
cost        squared Euclidean costs, block-row-0 <-> block-circulant conversions, median.
sinkhorn    plain full-size log-domain Sinkhorn; the cyclic (reduced) Sinkhorn of Alg. 2
            (fold of the Gibbs kernel, reduced loop, expansion of the plan).
objective   primal / dual objective values, transport cost, marginal errors.
grad        envelope-theorem gradients and central finite differences.
lp          brute-force linear programs (LOT and the small LOT of Thm. 1) via SciPy HiGHS.
projection  block-circulant projection of a cost matrix (approximate-symmetry workload).
dual_ascent an independent EROT solver (L-BFGS on the concave dual) used only to pin sinkhorn.
srot        cyclic SROT with a quadratic regulariser: alternating exact dual maximisation.

Pinning status of every function is listed in each module header.  Functions whose result is
only a reported number and has no independent pin say "parity unpinned".
"""
from . import cost, sinkhorn, objective, grad, lp, projection, dual_ascent  # noqa: F401
