"""Adjoint gradient dJ/dh of J = sum |u - t|^2 through the C ABI, against
the oracle's dense adjoint and against central finite differences."""

import sys

import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_04691_amd as ori  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def small_case(n, k, seed):
    rng = np.random.default_rng(seed)
    P = n ** 3
    h = (-1.0 + 0.5j) * (1.0 + 0.3 * rng.uniform(-1, 1, P))
    N = 0.5 + rng.uniform(0, 1, P)
    u0 = workloads.plane_wave(n, k, (0.6, 0.0, 0.8))
    t = u0 * (1.0 + 0.2 * rng.standard_normal(P))
    return h, N, u0, t


@pytest.mark.parametrize("n,k,prec", [(4, 3.0, ori.ORI_FP64), (8, 5.0, ori.ORI_FP64), (8, 5.0, ori.ORI_MIXED)])
def test_gradient_vs_dense_adjoint(n, k, prec):
    say(f"[gradient] n={n} k={k} prec={prec}")
    h, N, u0, t = small_case(n, k, seed=n)
    pts = O.cell_points(n)
    J_ref, g_ref, u_ref = O.adjoint_gradient_dense(pts, k, h, N, u0, t, n)
    with ori.ori_setup(n, k, gpu(h), gpu(N), gpu(u0)) as ctx:
        u = torch.empty(n ** 3, dtype=torch.complex128, device="cuda")
        g = torch.empty_like(u)
        tol = 1e-13 if prec == ori.ORI_FP64 else 1e-10
        _, J, info = ori.ori_gradient(ctx, gpu(t), u, g, tol=tol, precision=prec)
        err_g = rel(g.cpu().numpy(), g_ref)
        say(f"   J={J:.6e} ref={J_ref:.6e} grad err={err_g:.2e} iters={info['iterations']}")
        bar = 1e-9 if prec == ori.ORI_FP64 else 1e-7
        assert abs(J - J_ref) <= bar * J_ref
        assert rel(u.cpu().numpy(), u_ref) <= bar
        assert err_g <= bar


def test_adjoint_lambda_vs_dense():
    n, k = 6, 4.0
    say("[adjoint lam]")
    h, N, u0, t = small_case(n, k, seed=1)
    rng = np.random.default_rng(2)
    f = rng.standard_normal(n ** 3) + 1j * rng.standard_normal(n ** 3)
    pts = O.cell_points(n)
    D = O.coupling(h, N, n)
    A = O.system_matrix(pts, k, D)
    u_ref = O.solve_direct(A, u0)
    lam_ref = O.solve_direct(A.T, f)
    c = O.coupling(np.ones(n ** 3), N, n).real
    g_ref = -c * u_ref * (O.green_matrix(pts, k) @ lam_ref)
    with ori.ori_setup(n, k, gpu(h), gpu(N), gpu(u0)) as ctx:
        u = torch.empty(n ** 3, dtype=torch.complex128, device="cuda")
        ori.ori_solve(ctx, u, tol=1e-13)
        g = torch.empty_like(u)
        lam = torch.empty_like(u)
        ori.ori_adjoint(ctx, u, gpu(f), g=g, lam=lam, tol=1e-13)
        assert rel(lam.cpu().numpy(), lam_ref) <= 1e-10
        assert rel(g.cpu().numpy(), g_ref) <= 1e-10


def test_autograd_function_matches_adjoint():
    n, k = 6, 4.0
    say("[autograd]")
    h, N, u0, t = small_case(n, k, seed=3)
    hg = gpu(h).requires_grad_(True)
    u0g = gpu(u0).requires_grad_(True)
    tg = gpu(t)
    u = ori.OriSolve(hg, u0g, n, k, N=gpu(N), tol=1e-13)
    J = torch.sum(torch.abs(u - tg) ** 2)
    J.backward()
    pts = O.cell_points(n)
    J_ref, g_ref, u_ref = O.adjoint_gradient_dense(pts, k, h, N, u0, t, n)
    assert abs(J.item() - J_ref) <= 1e-9 * J_ref
    # torch's complex gradient is dJ/dRe h + i dJ/dIm h = conj(g)
    assert rel(hg.grad.cpu().numpy(), np.conj(g_ref)) <= 1e-9
    # and for u0: dJ = Re sum lam du0 with A^T lam = 2 conj(u - t): grad = conj(lam)
    D = O.coupling(h, N, n)
    lam = O.solve_direct(O.system_matrix(pts, k, D).T, 2 * np.conj(u_ref - t))
    assert rel(u0g.grad.cpu().numpy(), np.conj(lam)) <= 1e-9


def test_config3_finite_differences_n128():
    # n = 128, k = 5, target from the same system with h scaled by 1.2;
    # central differences at step 1e-6 on 16 random cells, real and imaginary
    # parts.  J+ - J- is formed as sum Re[(u+ - u-) conj(u+ + u- - 2t)], and
    # both solves run the same fixed number of COCG iterations from x0 = 0
    # (tol = 0), so that u+ - u- is a smooth function of the step and their
    # solver errors cancel instead of adding ~1e-13 noise per entry.
    case = workloads.make_case(128, 5.0, seed=3)
    n, k = case["n"], case["k"]
    P = n ** 3
    say("[config3 FD] n=128")
    h = gpu(case["h"])
    N = gpu(case["N"])
    u0 = gpu(case["u0"])
    tol = 1e-13
    fixed = 40  # iterations: beyond the ~19 needed for 1e-13
    with ori.ori_create(n) as ctx:
        t = torch.empty(P, dtype=torch.complex128, device="cuda")
        ori.ori_load(ctx, k, 1.2 * h, N, u0)
        ori.ori_solve(ctx, t, tol=tol)
        ori.ori_load(ctx, k, h, N, u0)
        u = torch.empty_like(t)
        g = torch.empty_like(t)
        _, J, info = ori.ori_gradient(ctx, t, u, g, tol=tol)
        say(f"   J={J:.6e} iterations={info['iterations']}")
        g = g.cpu().numpy()
        rng = np.random.default_rng(33)
        cells = rng.choice(P, 16, replace=False)
        eps = 1e-6
        up = torch.empty_like(t)
        um = torch.empty_like(t)
        errs = []
        for p in cells:
            for direction, want in ((1.0, g[p].real), (1j, -g[p].imag)):
                hp = h.clone()
                hp[p] += eps * direction
                ori.ori_load(ctx, k, hp, N, u0)
                st, _ = ori.ori_solve(ctx, up, tol=0.0, max_iter=fixed, true_residual=False, raise_on_error=False)
                assert st == ori.ORI_ERR_NOT_CONVERGED  # ran exactly `fixed` iterations
                hm = h.clone()
                hm[p] -= eps * direction
                ori.ori_load(ctx, k, hm, N, u0)
                st, _ = ori.ori_solve(ctx, um, tol=0.0, max_iter=fixed, true_residual=False, raise_on_error=False)
                assert st == ori.ORI_ERR_NOT_CONVERGED
                dJ = torch.sum(torch.real((up - um) * torch.conj(up + um - 2 * t))).item()
                fd = dJ / (2 * eps)
                errs.append(abs(fd - want) / max(abs(want), 1e-3 * np.max(np.abs(g))))
        say(f"   FD vs adjoint: max rel err {max(errs):.2e}, median {np.median(errs):.2e}")
        assert max(errs) <= 1e-3
