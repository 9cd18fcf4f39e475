"""Write tests/golden/oracle_fixtures.npz: seeded small problems of eq. 2.19
(workloads.make_case, the configuration of the small parity case) with the
oracle's dense LU solution and the condition number of the system: the
2-norm one from the singular values up to n = 16, LAPACK's 1-norm estimate
(zgecon) at n = 20 (P = 8000, the size of the paper's Table 6 run).
Calls only oracle/ and workloads; nothing here comes from the GPU path.

    python tests/golden/make_oracle_fixtures.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads  # noqa: E402

# (n, k, seed): k spans the smooth, medium and oscillatory regimes
FIXTURES = [(1, 1.0, 11), (2, 3.0, 12), (3, 5.0, 13), (4, 1.0, 14), (8, 5.0, 15), (12, 10.0, 16),
            (16, 5.0, 17), (20, 1.0, 18)]
# sizes whose condition number is LAPACK's 1-norm estimate (an SVD of the
# 8000 x 8000 matrix takes minutes)
GECON_FROM = 20


def kappa_method(n):
    return "gecon" if n >= GECON_FROM else "svd"


def compute(n, k, seed):
    case = workloads.make_case(n, k, seed)
    pts = O.cell_points(n)
    A = O.system_matrix(pts, k, O.coupling(case["h"], case["N"], n))
    u = O.solve_direct(A, case["u0"])
    kappa = O.condition_number(A, kappa_method(n))
    return case, u, kappa


def main():
    out = {}
    for n, k, seed in FIXTURES:
        case, u, kappa = compute(n, k, seed)
        tag = f"n{n}"
        out[f"{tag}_params"] = np.array([n, k, seed], dtype=np.float64)
        out[f"{tag}_u"] = u
        name = "kappa1" if kappa_method(n) == "gecon" else "kappa"
        out[f"{tag}_{name}"] = np.array(kappa)
        print(f"{tag}: k={k} seed={seed} {name}={kappa:.4f} |u|={np.linalg.norm(u):.6f}")
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_fixtures.npz"), **out)


if __name__ == "__main__":
    main()
