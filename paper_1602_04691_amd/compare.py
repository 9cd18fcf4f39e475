"""Section 4's comparison of (ORI), (RED) and (IE) on one GPU (Table 4).

    python -m paper_1602_04691_amd.compare [--ori 512] [--red 20] [--ie 40]
                                           [--tol 1e-8] [--precision fp64|mixed]

The three systems differ only in resolution.  (ORI) is eq. 2.15 for M
particles; with M = a^{-(2-kappa)} particles in the unit cube (eq. 4.3, N = 1),
its coefficient c_S h a^{2-kappa} equals c_S h N |Delta| on the M-point
lattice, i.e. eq. 2.19 with n = M^{1/3}.  (RED) is eq. 2.19 on P = red^3
sub-cubes and (IE) the collocation of eq. 2.20 on C = ie^3 points.  All three
use the lattice of eq. 3.3.5 (points at the corners, i / n).  The parameters
are Section 4's: k, h, alpha = e1, N = 1, n0 = 1.  Each solution is compared
with a coarser one by the procedure of Table 4 (ori_interpolation_difference).
Prints one JSON line.
"""

import argparse
import json
import time

import paper_1602_04691_amd as ori

K = 0.182651                          # Section 4
H = 2.65481e-09 + 5.30961e-06j        # Section 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ori", type=int, default=512)
    ap.add_argument("--red", type=int, default=20)
    ap.add_argument("--ie", type=int, default=40)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    a = ap.parse_args()
    import torch
    prec = ori.ORI_FP64 if a.precision == "fp64" else ori.ORI_MIXED
    dev = torch.device("cuda")
    sols, info = {}, {}
    for name, n in (("ORI", a.ori), ("RED", a.red), ("IE", a.ie)):
        P = n ** 3
        x = torch.arange(n, dtype=torch.float64, device=dev) / n          # corner lattice, eq. 3.3.5
        u0 = torch.exp(1j * K * x.to(torch.complex128)).repeat_interleave(n * n)  # e^{ik x1}, alpha = e1
        h = torch.full((P,), H, dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with ori.ori_setup(n, K, h, None, u0, cell_offset=0.0) as ctx:
            u = torch.empty(P, dtype=torch.complex128, device=dev)
            _, i = ori.ori_solve(ctx, u, tol=a.tol, precision=prec)
        torch.cuda.synchronize()
        sols[name] = (n, u)
        info[name] = {"n": n, "unknowns": P, "iterations": i["iterations"], "rel_res_true": i["rel_res_true"],
                      "seconds": round(time.perf_counter() - t0, 4)}
        del h, u0
    diff = {}
    for fine, coarse in (("ORI", "RED"), ("IE", "RED"), ("ORI", "IE")):
        nf, xf = sols[fine]
        nc, yc = sols[coarse]
        with ori.ori_create(nc, cell_offset=0.0) as ctx:
            diff[f"{fine} vs {coarse}"] = ori.ori_interpolation_difference(ctx, yc, xf, nf, 0.0)
    print(json.dumps({"k": K, "h": [H.real, H.imag], "precision": a.precision, "tol": a.tol,
                      "solves": info, "differences": diff}))


if __name__ == "__main__":
    main()
