"""CPU pins of the physics oracle (oracle/physics.py).

Refraction recipe (Section 2, eqs. 2.24-2.26; Section 4, eqs. 4.1-4.2),
charges (eqs. 2.13, 2.18) and the field (eq. 2.10) with its far-field
amplitude.  Each pin fixes the function against something other than its
own formula: the paper's printed worked example, closed forms of the
square-root branch, the solved system eq. 2.19 itself, the large-r limit of
the field, and reciprocity.
"""

import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_refraction_recipe_worked_example():
    v, f, k_pr, n0r, n0i, nr, ni, N, hr, hi = np.loadtxt(os.path.join(GOLDEN, "section4_refraction_example.txt"))
    k = 2.0 * math.pi * f / v
    assert abs(k - k_pr) < 0.5e-6                      # the printed k is 2 pi f / v rounded
    n0, n = complex(n0r, n0i), complex(nr, ni)
    h = O.h_for_refraction(k, n0, n, N)
    # the printed six significant digits of h
    assert abs(h.real - hr) <= 0.5e-5 * abs(hr) and abs(h.imag - hi) <= 0.5e-5 * abs(hi)
    # and the printed h gives back the desired n through eq. 4.1 with the
    # branch of eq. 4.2 (Re n < 0: negative refraction)
    nn = O.refraction_from_h(k, n0, complex(hr, hi), N)
    assert abs(nn - n) <= 2e-6
    # the principal square root would give the opposite sign
    principal = np.sqrt(n0 * n0 - 4 * math.pi * complex(hr, hi) * N / k ** 2)
    assert abs(principal + n) <= 2e-6


@pytest.mark.parametrize("phi", np.linspace(0.0, 2 * math.pi, 17)[:-1].tolist() + [math.pi - 1e-9, 2 * math.pi - 1e-9])
def test_branch_0_2pi_closed_form(phi):
    # z = R e^{i phi}, phi in [0, 2 pi): z^{1/2} = sqrt(R) e^{i phi / 2}
    R = 2.25
    z = R * complex(math.cos(phi), math.sin(phi))
    s = O.sqrt_branch_0_2pi(z)
    expect = math.sqrt(R) * complex(math.cos(phi / 2), math.sin(phi / 2))
    assert abs(s - expect) <= 1e-12
    assert s.imag >= -1e-15 and abs(s * s - z) <= 1e-12


def test_branch_special_values():
    assert O.sqrt_branch_0_2pi(4.0 + 0j) == 2.0                  # on the cut: phi = 0
    assert abs(O.sqrt_branch_0_2pi(-4.0 + 0j) - 2j) <= 1e-15      # phi = pi
    assert O.sqrt_branch_0_2pi(0j) == 0


def test_recipe_round_trip():
    rng = np.random.default_rng(7)
    k = 3.0
    n0 = 1.0 + 0.3 * rng.standard_normal(50) + 0.05j * rng.random(50)
    n = rng.standard_normal(50) + 1j * rng.random(50)            # Im n > 0: inside the branch's range
    N = 0.5 + rng.random(50)
    h = O.h_for_refraction(k, n0, n, N)
    assert np.max(np.abs(O.refraction_from_h(k, n0, h, N) - n)) <= 1e-12
    # n = n0 needs no particles
    assert np.max(np.abs(O.h_for_refraction(k, n0, n0, N))) == 0.0


def test_field_at_cells_is_the_system():
    # u0 + v(x_q) with Q = cell charges of the LU solution reproduces the
    # solution at every cell (eq. 2.10 evaluated at the points of eq. 2.19):
    # a wrong sign or scale of the charges, or a self term in v, fails
    n, k = 5, 4.0
    rng = np.random.default_rng(8)
    pts = O.cell_points(n)
    h = (-1 + 0.5j) * (1 + 0.3 * rng.uniform(-1, 1, n ** 3))
    N = 0.5 + rng.random(n ** 3)
    u0 = np.exp(1j * k * pts @ np.array([0.6, 0.0, 0.8]))
    u = O.solve_direct(O.system_matrix(pts, k, O.coupling(h, N, n)), u0)
    Q = O.cell_charges(h, N, n, u)
    v = O.scattered_field(pts, k, Q, pts)
    assert np.linalg.norm(u0 + v - u) <= 1e-12 * np.linalg.norm(u)


def test_particle_charges_add_up_to_the_cell_charge():
    # a cell holding a^{-(2-kappa)} N |Delta| particles (eq. 2.18), each with
    # the charge of eq. 2.13 and the same effective field
    n, kappa = 4, 0.5
    vol = 1.0 / n ** 3
    count = 1000
    a = (vol / count) ** (1.0 / (2.0 - kappa))       # N = 1
    h, u = np.array([0.3 - 1.1j]), np.array([0.7 + 0.2j])
    q_particles = count * O.particle_charge(h, u, a, kappa)
    assert abs(q_particles[0] - O.cell_charges(h, np.ones(1), n, u)[0]) <= 1e-14


def test_far_field_is_the_limit_of_the_field():
    n, k = 4, 3.0
    rng = np.random.default_rng(9)
    pts = O.cell_points(n)
    Q = rng.standard_normal(n ** 3) + 1j * rng.standard_normal(n ** 3)
    beta = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0], [-0.48, 0.6, -0.64]])
    A = O.far_field(pts, k, Q, beta)
    errs = []
    for r in (1e2, 1e3, 1e4):
        v = O.scattered_field(pts, k, Q, r * beta)
        errs.append(np.max(np.abs(r * np.exp(-1j * k * r) * v - A)))
    # O(1/r) approach
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5 and errs[2] < 1e-3 * np.max(np.abs(A))


def test_far_field_reciprocity():
    # A_alpha(beta) = A_{-beta}(-alpha): D (I + G0 D)^{-1} is symmetric
    n, k = 4, 5.0
    rng = np.random.default_rng(10)
    pts = O.cell_points(n)
    h = (-1 + 0.5j) * (1 + 0.3 * rng.uniform(-1, 1, n ** 3))
    N = 0.5 + rng.random(n ** 3)
    D = O.coupling(h, N, n)
    A = O.system_matrix(pts, k, D)
    alpha = np.array([0.0, 0.6, 0.8])
    beta = np.array([0.48, -0.6, 0.64])

    def amp(inc, out):
        u = O.solve_direct(A, np.exp(1j * k * pts @ inc))
        return O.far_field(pts, k, O.cell_charges(h, N, n, u), out[None, :])[0]

    a1, a2 = amp(alpha, beta), amp(-beta, -alpha)
    assert abs(a1 - a2) <= 1e-12 * abs(a1)
    # and it is not a trivial symmetry: swapping without the sign changes differs
    assert abs(amp(beta, alpha) - a1) > 1e-6 * abs(a1)


def _difference_brute(x, nf, y, nc, off):
    # pure-Python loops over the coarse cells and the fine points inside each
    worst = 0.0
    for q1 in range(nc):
        for q2 in range(nc):
            for q3 in range(nc):
                tot, cnt = 0.0, 0
                for i1 in range(nf):
                    if not (q1 / nc <= (i1 + off) / nf < (q1 + 1) / nc):
                        continue
                    for i2 in range(nf):
                        if not (q2 / nc <= (i2 + off) / nf < (q2 + 1) / nc):
                            continue
                        for i3 in range(nf):
                            if not (q3 / nc <= (i3 + off) / nf < (q3 + 1) / nc):
                                continue
                            tot += abs(x[(i1 * nf + i2) * nf + i3] - y[(q1 * nc + q2) * nc + q3])
                            cnt += 1
                if cnt:
                    worst = max(worst, tot / cnt)
    return worst


@pytest.mark.parametrize("nf,nc,off", [(6, 2, 0.5), (7, 3, 0.5), (5, 5, 0.0), (4, 6, 0.5), (9, 4, 0.0)])
def test_interpolation_difference_vs_brute_force(nf, nc, off):
    rng = np.random.default_rng(nf * 10 + nc)
    x = rng.standard_normal(nf ** 3) + 1j * rng.standard_normal(nf ** 3)
    y = rng.standard_normal(nc ** 3) + 1j * rng.standard_normal(nc ** 3)
    assert abs(O.interpolation_difference(x, nf, y, nc, off) - _difference_brute(x, nf, y, nc, off)) <= 1e-13


def test_interpolation_difference_closed_forms():
    # constants: |c1 - c2|; same grid: max |x - y|
    assert abs(O.interpolation_difference(np.full(64, 1 + 2j), 4, np.full(8, -2 + 6j), 2) - 5.0) <= 1e-14
    rng = np.random.default_rng(3)
    x = rng.standard_normal(27) + 0j
    y = rng.standard_normal(27) + 0j
    assert O.interpolation_difference(x, 3, y, 3) == np.max(np.abs(x - y))
    # a field linear along x1, fine = 2 x coarse, y = the cell mean: each coarse
    # cell holds fine rows 2q and 2q + 1, so the mean |x - y| is 1/2
    nf, nc = 8, 4
    x = np.repeat(np.arange(nf, dtype=float), nf * nf) + 0j
    y = np.repeat(2.0 * np.arange(nc) + 0.5, nc * nc) + 0j
    assert abs(O.interpolation_difference(x, nf, y, nc) - 0.5) <= 1e-14
