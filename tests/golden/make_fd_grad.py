"""Writes fd_grad_n4096_K8.json: central finite differences of the converged float64 value
of the FULL n x n entropic problem (eq. problem_ROT with the entropy of eq.
reg_for_entropy_ROT) at the n = 4096, K = 8 symmetric workload (seed 300, eps = 0.05
median C), one coordinate at a time.  Perturbing one point breaks the cyclic symmetry, so
these differences come from plain full-size Sinkhorn only.

    32 point coordinates (x or y, index, component), h = 1e-4, each side solved to an L2 row
    residual of 1e-12 from the unperturbed g (scaling domain; max C/eps is about 70);
    8 + 8 directions e_I - e_J of a and of b, h = 1e-7.

Calls only oracle/ and workloads/.  Run: python tests/golden/make_fd_grad.py (minutes).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import grad  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fd_grad_n4096_K8.json")


def main():
    p = workloads.symmetric_problem(4096, 8, 2, 0.05, seed=300)
    x, y, a, b = (v.astype(np.float64) for v in (p.x, p.y, p.a, p.b))
    P0, out = grad.solve_value(x, y, a, b, p.eps, tol=1e-12)
    g0 = out["g"]
    rng = np.random.default_rng(11)
    coords = []
    for _ in range(32):
        which = "x" if rng.integers(2) == 0 else "y"
        I, d = int(rng.integers(p.n)), int(rng.integers(2))
        fd = grad.fd_coordinate(x, y, a, b, p.eps, which, I, d, h=1e-4, g0=g0, tol=1e-12)
        coords.append({"which": which, "index": I, "comp": d, "fd": fd})
        print(which, I, d, fd, flush=True)
    marg = []
    for which in ("a", "b"):
        for _ in range(8):
            I, J = (int(v) for v in rng.choice(p.n, size=2, replace=False))
            fd = grad.fd_marginal(x, y, a, b, p.eps, which, I, J, h=1e-7, g0=g0, tol=1e-12)
            marg.append({"which": which, "I": I, "J": J, "fd": fd})
            print(which, I, J, fd, flush=True)
    doc = {"script": "tests/golden/make_fd_grad.py",
           "workload": {"n": 4096, "K": 8, "dim": 2, "eps_factor": 0.05, "seed": 300,
                        "eps": p.eps},
           "value_P": P0, "coords": coords, "marginals": marg}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
