"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test is chosen so that a plausible mistake in the oracle (a dropped
factor, a wrong sign, the diagonal factor on the wrong side, a transposed
axis, a wrong padding) fails at least one of them.  CPU only.
"""

import math
import os

import numpy as np
import pytest

import oracle as O
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _varied_case(n, k, seed, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5):
    rng = np.random.default_rng(seed)
    P = n ** 3
    h = (-1.0 + 0.5j) * (1.0 + 0.3 * rng.uniform(-1, 1, P)) + 0.2j * rng.uniform(-1, 1, P)
    N = 0.5 + rng.uniform(0, 1, P)
    u0 = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    pts = O.cell_points(n, side, origin, offset)
    return pts, h, N, u0


# --- exact special cases -----------------------------------------------------
def test_single_cube_is_incident_field():
    # n = 1: P = 1, the sum of eq. 2.19 is empty, so u = u0 exactly.
    pts = O.cell_points(1)
    D = O.coupling(np.array([-1 + 0.5j]), None, 1)
    A = O.system_matrix(pts, 3.0, D)
    u = O.solve_direct(A, np.array([0.3 - 0.7j]))
    assert u[0] == 0.3 - 0.7j


@pytest.mark.parametrize("side,k,h,N", [(1.0, 1.0, -1 + 0.5j, 1.0),
                                        (1.3, 4.0, 0.7 - 2.0j, 2.5),
                                        (0.2, 11.0, -30 + 1j, 0.25)])
def test_two_per_side_closed_form(side, k, h, N):
    # n = 2, constant h, N and u0 = 1: by the cube's symmetry all 8 unknowns are
    # equal, each cube sees 3 neighbours at distance a = side/2, 3 at a*sqrt(2)
    # and 1 at a*sqrt(3):  u (1 + c_S h N (side/2)^3 * sum G) = 1.
    a = side / 2.0

    def G(r):
        return complex(math.cos(k * r), math.sin(k * r)) / (4 * math.pi * r)

    Dc = 4 * math.pi * h * N * a ** 3
    u_exact = 1.0 / (1.0 + Dc * (3 * G(a) + 3 * G(a * math.sqrt(2)) + G(a * math.sqrt(3))))
    pts = O.cell_points(2, side=side, origin=(0.4, -1.0, 2.0))
    D = O.coupling(np.full(8, h), np.full(8, N), 2, side)
    u = O.solve_direct(O.system_matrix(pts, k, D), np.ones(8, complex))
    assert np.max(np.abs(u - u_exact)) <= 1e-15 * 4


@pytest.mark.parametrize("n", [1, 2, 3])
def test_brute_force_matches_vectorised_lapack(n):
    # Pure-Python assembly (term by term from eq. 2.19) + own Gaussian
    # elimination against the NumPy assembly + LAPACK zgesv.
    k = 2.7
    pts, h, N, u0 = _varied_case(n, k, seed=10 + n, side=1.7, origin=(0.1, 0.2, -0.3))
    A_bf = O.brute_force_system(n, k, h, N, side=1.7, origin=(0.1, 0.2, -0.3))
    u_bf = np.array(O.gauss_solve(A_bf, u0))
    D = O.coupling(h, N, n, 1.7)
    A = O.system_matrix(pts, k, D)
    assert np.max(np.abs(A - np.array(A_bf))) <= 1e-15
    assert _rel(O.solve_direct(A, u0), u_bf) <= 1e-13


def test_green_matrix_symmetric_and_zero_diagonal():
    pts = O.cell_points(4, side=1.1, origin=(0.3, 0.0, 0.0))
    G0 = O.green_matrix(pts, 5.0)
    assert np.all(np.diag(G0) == 0)
    assert np.max(np.abs(G0 - G0.T)) == 0.0


def test_born_limit_sign_and_scale():
    # h = eps*h1: u = u0 - G0 D u0 + O(eps^2).  The first-order field is written
    # out here as the explicit sum of eq. 2.19 over p != q (Python loops).
    n, k = 3, 4.0
    pts, h1, N, u0 = _varied_case(n, k, seed=3)
    P = n ** 3
    vol = 1.0 / P
    born1 = np.zeros(P, complex)
    for q in range(P):
        s = 0j
        for p in range(P):
            if p != q:
                r = math.dist(pts[q], pts[p])
                s += (complex(math.cos(k * r), math.sin(k * r)) / (4 * math.pi * r)) * h1[p] * N[p] * u0[p] * vol
        born1[q] = -4 * math.pi * s
    errs = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        D = O.coupling(eps * h1, N, n)
        u = O.solve_direct(O.system_matrix(pts, k, D), u0)
        errs.append(np.linalg.norm(u - (u0 + eps * born1)))
    assert abs(errs[0] / errs[1] - 4.0) < 0.05 and abs(errs[1] / errs[2] - 4.0) < 0.03


def test_reciprocity_fixes_diagonal_side():
    # D (I + G0 D)^{-1} = (D^{-1} + G0)^{-1} is symmetric, so
    # F_ij = u0_j^T D u_i is symmetric in (i, j) for varying h and N.
    n, k = 3, 3.0
    pts, h, N, _ = _varied_case(n, k, seed=5)
    D = O.coupling(h, N, n)
    A = O.system_matrix(pts, k, D)
    rng = np.random.default_rng(0)
    U0 = rng.standard_normal((O.cell_points(n).shape[0], 4)) + 1j * rng.standard_normal((n ** 3, 4))
    U = O.solve_direct(A, U0)
    F = U0.T @ (D[:, None] * U)
    assert np.max(np.abs(F - F.T)) <= 1e-13 * np.max(np.abs(F))
    # the wrong placement (I + D G0) breaks it
    Aw = O.green_matrix(pts, k) * D[:, None]
    Aw[np.diag_indices_from(Aw)] += 1
    Uw = O.solve_direct(Aw, U0)
    Fw = U0.T @ (D[:, None] * Uw)
    assert np.max(np.abs(Fw - Fw.T)) > 1e-6 * np.max(np.abs(Fw))


def test_mirror_symmetry_per_axis():
    # Data symmetric under i_a -> n-1-i_a gives a symmetric solution; checked
    # for each axis separately (an axis mix-up breaks one of them).
    n, k = 4, 6.0
    rng = np.random.default_rng(7)
    for axis in range(3):
        base_h = (-1 + 0.5j) * (1 + 0.2 * rng.uniform(-1, 1, (n, n, n)))
        base_u = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        h = base_h + np.flip(base_h, axis)
        u0 = base_u + np.flip(base_u, axis)
        pts = O.cell_points(n)
        D = O.coupling(h.reshape(-1), None, n)
        u = O.solve_direct(O.system_matrix(pts, k, D), u0.reshape(-1)).reshape(n, n, n)
        assert np.max(np.abs(u - np.flip(u, axis))) <= 1e-13
        # a field symmetric on another axis only does not give this symmetry
        u_other = O.solve_direct(O.system_matrix(pts, k, D), base_u.reshape(-1)).reshape(n, n, n)
        assert np.max(np.abs(u_other - np.flip(u_other, axis))) > 1e-3


def test_origin_shift_is_a_phase():
    # G depends on x_q - x_p only: moving the cube by t multiplies the
    # plane-wave solution by exp(i k alpha . t).
    n, k = 3, 2.0
    alpha = np.array([0.6, 0.0, 0.8])
    h = np.full(n ** 3, -1 + 0.5j) * (1 + 0.1 * np.linspace(-1, 1, n ** 3))
    t = np.array([0.3, -1.1, 0.7])
    sol = []
    for org in ((0.0, 0.0, 0.0), tuple(t)):
        pts = O.cell_points(n, origin=org)
        u0 = workloads.plane_wave(n, k, alpha, origin=org)
        D = O.coupling(h, None, n)
        sol.append(O.solve_direct(O.system_matrix(pts, k, D), u0))
    assert _rel(sol[1], np.exp(1j * k * alpha @ t) * sol[0]) <= 1e-13


# --- symmetrisation, COCG ------------------------------------------------------
def test_symmetrised_system_gives_the_same_solution():
    n, k = 4, 5.0
    pts, h, N, u0 = _varied_case(n, k, seed=8)
    D = O.coupling(h, N, n)
    u_ref = O.solve_direct(O.system_matrix(pts, k, D), u0)
    S = O.symmetric_scale(D)
    As = O.symmetric_system_matrix(pts, k, S)
    assert np.max(np.abs(As - As.T)) <= 1e-15 * np.max(np.abs(As))
    w = O.solve_direct(As, S * u0)
    assert _rel(w / S, u_ref) <= 1e-13
    u_rec = u0 - O.green_matrix(pts, k) @ (S * w)
    assert _rel(u_rec, u_ref) <= 1e-13
    # the other branch of the square root gives the same u
    w2 = O.solve_direct(O.symmetric_system_matrix(pts, k, -S), -S * u0)
    assert _rel(u0 - O.green_matrix(pts, k) @ (-S * w2), u_ref) <= 1e-13


def test_cocg_real_spd_is_cg_and_terminates():
    # On a real SPD matrix the bilinear form is the Euclidean one, so COCG is
    # textbook CG: exact in at most P steps (here P = 12, well conditioned).
    rng = np.random.default_rng(1)
    M = rng.standard_normal((12, 12))
    A = M @ M.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    x, hist = O.cocg(lambda v: A @ v, b, tol=1e-14, maxiter=12)
    assert _rel(x, np.linalg.solve(A, b)) <= 1e-12
    # the first step is the steepest-descent step x1 = (b^T b / b^T A b) b
    x1, _ = O.cocg(lambda v: A @ v, b, tol=0, maxiter=1)
    alpha = (b @ b) / (b @ A @ b)
    assert _rel(x1, alpha * b) <= 1e-15


def test_cocg_complex_symmetric_matches_lu():
    n, k = 4, 5.0
    pts, h, N, u0 = _varied_case(n, k, seed=9)
    D = O.coupling(h, N, n)
    u_ref = O.solve_direct(O.system_matrix(pts, k, D), u0)
    u, hist = O.solve_symmetrized_cocg(pts, k, D, u0, tol=1e-13)
    assert hist[-1] < 1e-13
    assert _rel(u, u_ref) <= 1e-11


# --- the Section 3 route, the padding example and Table 6 ------------------------
def _read_blocks(path):
    blocks, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            blocks[cur] = []
        else:
            blocks[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def test_section3_padding_example():
    g = _read_blocks(os.path.join(GOLDEN, "section3_padding_example.txt"))
    assert np.array_equal(O.mirror_pad_axis(g["G"], 1), g["G_padded"])
    assert np.array_equal(O.zero_pad_axis(g["G"], 1, 6), g["u_padded"])


@pytest.mark.parametrize("n,k,side", [(1, 1.0, 1.0), (2, 3.0, 1.0), (3, 5.0, 0.7), (5, 2.0, 1.0), (8, 9.0, 2.0)])
def test_section3_route_equals_dense_sum(n, k, side):
    pts, h, N, v = _varied_case(n, k, seed=n, side=side)
    D = O.coupling(h, N, n, side)
    y_dense = O.scatter_dense(pts, k, D, v)
    y_fft = O.scatter_section3(n, k, D, v, side=side)
    if n == 1:
        assert np.all(y_dense == 0) and np.all(y_fft == 0)
    else:
        assert _rel(y_fft, y_dense) <= 1e-13


@pytest.mark.parametrize("n,k,side", [(1, 1.0, 1.0), (2, 3.0, 1.0), (3, 5.0, 0.7), (5, 2.0, 1.0), (8, 9.0, 2.0)])
def test_same_method_baseline_equals_dense_sum(n, k, side):
    # the (2n)^3 cyclic convolution of the CPU baseline (eq. 3.3.8) gives the
    # dense sums of eq. 2.19: a table with g(0) kept, or with the negative
    # offsets of the upper half taken as positive, fails
    pts, h, N, v = _varied_case(n, k, seed=10 + n, side=side)
    D = O.coupling(h, N, n, side)
    y_dense = O.scatter_dense(pts, k, D, v)
    y = O.scatter_fft(n, k, D, v, side=side, workers=2)
    if n == 1:
        assert np.all(y == 0) and np.all(y_dense == 0)
    else:
        assert _rel(y, y_dense) <= 1e-13


def test_same_method_baseline_solve_matches_lu():
    # COCG with the convolution product on the symmetrised system reaches the
    # LU solution of eq. 2.19 (varied h, so the symmetrisation matters)
    n, k = 6, 5.0
    pts, h, N, u0 = _varied_case(n, k, seed=61)
    D = O.coupling(h, N, n)
    u_lu = O.solve_direct(O.system_matrix(pts, k, D), u0)
    u, hist = O.solve_symmetrized_fft(n, k, D, u0, tol=1e-12, workers=2)
    assert hist[-1] < 1e-12 and len(hist) < 60
    assert _rel(u, u_lu) <= 1e-10


def test_row_sampler_equals_dense_rows():
    n, k = 6, 4.0
    pts, h, N, v = _varied_case(n, k, seed=2)
    D = O.coupling(h, N, n)
    rows = np.array([0, 7, 100, 215])
    y = O.sample_scatter_rows(pts, k, D, v, rows, chunk=50)
    y_dense = O.scatter_dense(pts, k, D, v)[rows]
    assert np.max(np.abs(y - y_dense)) <= 1e-14 * np.max(np.abs(y_dense))


def test_paper_table6_first_iterate():
    # Weak pin at the paper's own scale (b = 20, P = 8000, Section 4 values):
    # the printed digits are those of the first COCG iterate of the
    # sign-flipped system on the corner lattice (see the fixture header).
    rows = np.loadtxt(os.path.join(GOLDEN, "table6_red_b20.txt"))
    b, k = 20, 0.182651
    h = np.full(b ** 3, 2.65481e-09 + 5.30961e-06j)
    D = -O.coupling(h, None, b)                       # h -> -h
    u0 = workloads.plane_wave(b, k, (1.0, 0.0, 0.0), offset=0.0)

    def apply(v):
        return v + O.scatter_section3(b, k, D, v)

    x1, _ = O.cocg(apply, u0, tol=0.0, maxiter=1)
    got = x1.reshape(b, b, b)
    for i1, re, im in rows:
        plane = got[int(i1)]
        # all entries of the printed 5x5 block are equal; check the lattice
        # points i2, i3 in {0, 4, 8, 12, 16}
        sub = plane[::4, ::4]
        assert np.all(np.abs(sub.real - re) <= 0.5e-6 + 1e-12)
        assert np.all(np.abs(sub.imag - im) <= 0.5e-6 + 1e-12)
    # and the printed sign of eq. 2.19 does not reproduce the first block
    x1p, _ = O.cocg(lambda v: v + O.scatter_section3(b, k, -D, v), u0, tol=0.0, maxiter=1)
    assert abs(x1p[0].imag - rows[0, 2]) > 1e-5


def test_workload_generator_is_seeded():
    a = workloads.make_case(4, 5.0, 3)
    b = workloads.make_case(4, 5.0, 3)
    assert np.array_equal(a["h"], b["h"]) and np.array_equal(a["u0"], b["u0"])
    assert abs(np.linalg.norm(a["alpha"]) - 1) < 1e-15
    pts = O.cell_points(4)
    assert _rel(a["u0"], np.exp(1j * 5.0 * pts @ a["alpha"])) <= 1e-14
    d = workloads.fibonacci_directions(32)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)


# --- adjoint gradient ------------------------------------------------------------
def test_adjoint_gradient_matches_central_differences():
    # the definition of the derivative: central differences of J computed by
    # dense LU, for the real and the imaginary part of h_p
    n, k = 3, 4.0
    pts, h, N, u0 = _varied_case(n, k, seed=21)
    rng = np.random.default_rng(3)
    t = u0 * (1 + 0.2 * rng.standard_normal(n ** 3))
    J, g, _ = O.adjoint_gradient_dense(pts, k, h, N, u0, t, n)

    def Jof(hh):
        D = O.coupling(hh, N, n)
        return O.objective(O.solve_direct(O.system_matrix(pts, k, D), u0), t)

    assert abs(Jof(h) - J) <= 1e-13 * J
    eps = 1e-6
    for p in (0, 5, 13, 26):
        for direction, part in ((1.0, g[p].real), (1j, -g[p].imag)):
            hp, hm = h.copy(), h.copy()
            hp[p] += eps * direction
            hm[p] -= eps * direction
            fd = (Jof(hp) - Jof(hm)) / (2 * eps)
            assert abs(fd - part) <= 1e-6 * (abs(part) + 1e-3 * np.max(np.abs(g)))
    # a wrong adjoint (A instead of A^T) gives a different gradient
    D = O.coupling(h, N, n)
    A = O.system_matrix(pts, k, D)
    u = O.solve_direct(A, u0)
    lam_wrong = O.solve_direct(A, np.conj(u - t))
    c = O.coupling(np.ones(n ** 3), N, n).real
    g_wrong = -2 * c * u * (O.green_matrix(pts, k) @ lam_wrong)
    assert np.linalg.norm(g_wrong - g) > 1e-3 * np.linalg.norm(g)


def test_frozen_oracle_fixtures_reproduce():
    # the oracle still gives the LU solutions and condition numbers it wrote
    # to tests/golden/oracle_fixtures.npz (make_oracle_fixtures.py)
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(GOLDEN, "make_oracle_fixtures.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    z = np.load(os.path.join(GOLDEN, "oracle_fixtures.npz"))
    for n, k, seed in mk.FIXTURES:
        _, u, kappa = mk.compute(n, k, seed)
        ref = z[f"n{n}_u"]
        assert np.linalg.norm(u - ref) <= 1e-13 * np.linalg.norm(ref), n
        name = "kappa1" if mk.kappa_method(n) == "gecon" else "kappa"
        assert abs(kappa - float(z[f"n{n}_{name}"])) <= 1e-10 * kappa, n


# --- the residual sampler used at every size the dense LU cannot reach -------
@pytest.mark.parametrize("n", [2, 3, 5, 6])
def test_residual_sampler_equals_dense_residual(n, monkeypatch):
    # r_q = u0_q - u_q - (G0 D u)_q is row q of u0 - A u with A = I + G0 D
    # (eq. 2.19), for any u (here not a solution), on random rows; chunks
    # smaller than P put the excluded self term in every position of a chunk
    k = 3.1
    pts, h, N, u0 = _varied_case(n, k, seed=40 + n, side=1.2, origin=(0.1, -0.3, 0.2))
    D = O.coupling(h, N, n, 1.2)
    A = O.system_matrix(pts, k, D)
    rng = np.random.default_rng(50 + n)
    P = n ** 3
    u = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    rows = np.unique(np.concatenate([[0, P - 1], rng.integers(0, P, 6)]))
    r_dense = (u0 - A @ u)[rows]
    scale = np.max(np.abs(r_dense))
    for chunk in (1 << 20, 7, 1):
        r = O.sample_residual_rows(pts, k, D, u, u0, rows, chunk=chunk)
        assert np.max(np.abs(r - r_dense)) <= 1e-13 * scale, chunk
    # planted mistakes in the oracle, each of which this comparison must catch:
    # the sign of the sum flipped, and u left out of the residual
    real = O.ori_oracle.sample_scatter_rows
    monkeypatch.setattr(O.ori_oracle, "sample_scatter_rows", lambda *a, **kw: -real(*a, **kw))
    r_bad = O.sample_residual_rows(pts, k, D, u, u0, rows)
    assert np.max(np.abs(r_bad - r_dense)) > 1e-3 * scale
    # (the sum returned with u_q subtracted gives u0_q - (G0 D u)_q)
    monkeypatch.setattr(O.ori_oracle, "sample_scatter_rows",
                        lambda *a, **kw: real(*a, **kw) - np.asarray(a[3])[np.asarray(a[4])])
    r_bad = O.sample_residual_rows(pts, k, D, u, u0, rows)
    assert np.max(np.abs(r_bad - (u0 - (A - np.eye(P)) @ u)[rows])) <= 1e-13 * scale
    assert np.max(np.abs(r_bad - r_dense)) > 1e-3 * scale


def test_residual_sampler_vanishes_at_the_lu_solution():
    # at the LU solution of eq. 2.19 every sampled residual row is at rounding level
    n, k = 5, 4.4
    pts, h, N, u0 = _varied_case(n, k, seed=61)
    D = O.coupling(h, N, n)
    u = O.solve_direct(O.system_matrix(pts, k, D), u0)
    rows = np.arange(0, n ** 3, 9)
    r = O.sample_residual_rows(pts, k, D, u, u0, rows, chunk=33)
    assert np.max(np.abs(r)) <= 1e-13 * np.max(np.abs(u0))


def test_parallel_rows_equal_serial_rows_bitwise():
    # the multi-process mapper splits the rows only: each row's arithmetic is
    # the single-process function's, so the results are bit for bit the same
    n, k = 8, 2.2
    pts, h, N, u0 = _varied_case(n, k, seed=62)
    D = O.coupling(h, N, n)
    rng = np.random.default_rng(63)
    v = rng.standard_normal(n ** 3) + 1j * rng.standard_normal(n ** 3)
    rows = rng.integers(0, n ** 3, 23)
    s = O.sample_scatter_rows(pts, k, D, v, rows, chunk=100)
    sp, w = O.sample_rows_parallel(pts, k, D, v, rows, workers=4, chunk=100)
    assert w == 4 and np.array_equal(s, sp)
    r = O.sample_residual_rows(pts, k, D, v, u0, rows, chunk=100)
    rp, _ = O.sample_rows_parallel(pts, k, D, v, rows, u0=u0, workers=3, chunk=100)
    assert np.array_equal(r, rp)


# --- the condition number of the system ---------------------------------------
def _two_per_side_spectrum(side, k, h, N):
    # n = 2 with constant h and N: the 8 points are the corners of a cube of
    # edge a = side/2 and G0 = sum_v g(a |v|) T_v over the 7 nonzero v in
    # {0,1}^3, T_v the permutation x -> x xor v.  These commute and share the
    # real orthogonal eigenvectors chi_s(x) = (-1)^(s.x); so A = I + D G0 is
    # normal with eigenvalues mu_s = 1 + D sum_v g(a |v|) (-1)^(s.v), its
    # singular values are |mu_s|, and A^-1 = sum_v b_v T_v with
    # b_v = (1/8) sum_s (-1)^(s.v) / mu_s.
    a = side / 2.0

    def g(r):
        return complex(math.cos(k * r), math.sin(k * r)) / (4 * math.pi * r)

    Dc = 4 * math.pi * h * N * a ** 3
    bits = lambda x: bin(x).count("1")
    mu = [1.0 + Dc * sum(g(a * math.sqrt(bits(v))) * (-1) ** bits(s & v) for v in range(1, 8)) for s in range(8)]
    a_v = [1.0] + [Dc * g(a * math.sqrt(bits(v))) for v in range(1, 8)]
    b_v = [sum((-1) ** bits(s & v) / mu[s] for s in range(8)) / 8 for v in range(8)]
    return mu, a_v, b_v


@pytest.mark.parametrize("side,k,h,N", [(1.0, 1.0, -1 + 0.5j, 1.0), (1.3, 4.0, 0.7 - 2.0j, 2.5),
                                        (0.2, 11.0, -30 + 1j, 0.25), (1.0, 2.0, -40 + 3j, 1.0)])
def test_condition_number_closed_form_two_per_side(side, k, h, N):
    mu, a_v, b_v = _two_per_side_spectrum(side, k, h, N)
    pts = O.cell_points(2, side=side, origin=(0.4, -1.0, 2.0))
    A = O.system_matrix(pts, k, O.coupling(np.full(8, h), np.full(8, N), 2, side))
    kappa2 = max(abs(m) for m in mu) / min(abs(m) for m in mu)
    assert abs(O.condition_number(A) - kappa2) <= 1e-12 * kappa2
    # the 1-norm: every column of A (of A^-1) holds the values a_v (b_v), so
    # kappa_1 = sum |a_v| * sum |b_v|; LAPACK's estimate is a lower bound of it
    # that is exact or close on such small matrices
    kappa1 = sum(abs(x) for x in a_v) * sum(abs(x) for x in b_v)
    est = O.condition_number(A, "gecon")
    assert kappa1 / 3.0 <= est <= kappa1 * (1 + 1e-12)
    # a transposed or dropped coupling would change the spectrum: the
    # identity (no particles) has condition number 1
    assert abs(O.condition_number(np.eye(8, dtype=complex)) - 1.0) <= 1e-15


def test_condition_number_single_cube_and_scaling():
    # n = 1 gives A = [1]; a scaled identity and a diagonal matrix have the
    # obvious condition numbers
    A = O.system_matrix(O.cell_points(1), 2.0, O.coupling(np.array([-1 + 0.5j]), None, 1))
    assert O.condition_number(A) == 1.0
    d = np.array([3.0, -0.5j, 2.0 + 2.0j, 0.25])
    assert abs(O.condition_number(np.diag(d)) - 3.0 / 0.25) <= 1e-13 * 12
    assert abs(O.condition_number(np.diag(d), "gecon") - 3.0 / 0.25) <= 1e-13 * 12
