"""Property tests of the oracle (CPU): invariants of eq. 2.19 on random small
problems drawn by hypothesis (derandomized, so every run draws the same
cases).  Each property holds for any admissible k, h, N, geometry and
incident direction, not only for the fixed cases of test_oracle_pins.py."""

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle as O  # noqa: E402
import workloads  # noqa: E402

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True, database=None)


@st.composite
def problems(draw, nmax=3):
    n = draw(st.integers(1, nmax))
    k = draw(st.floats(0.1, 12.0))
    side = draw(st.floats(0.3, 3.0))
    origin = tuple(draw(st.floats(-2.0, 2.0)) for _ in range(3))
    # nonzero h (S_p != 0): the division u = w / S needs it
    h0 = draw(st.floats(0.05, 2.0)) * np.exp(1j * draw(st.floats(0.0, 2 * np.pi)))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    P = n ** 3
    h = h0 * (1.0 + 0.2 * rng.uniform(-1, 1, P))
    N = 0.5 + rng.random(P)
    alpha = workloads.random_direction(rng)
    return n, k, side, origin, h, N, alpha


@SETTINGS
@given(problems())
def test_brute_force_equals_lapack(p):
    # the loop assembly with hand-written elimination and the NumPy assembly
    # with LAPACK agree on any small problem
    n, k, side, origin, h, N, alpha = p
    pts = O.cell_points(n, side, origin)
    u0 = np.exp(1j * k * pts @ alpha)
    A_bf = O.brute_force_system(n, k, h, N, side, origin)
    A = O.system_matrix(pts, k, O.coupling(h, N, n, side))
    assert np.allclose(A_bf, A, rtol=1e-13, atol=1e-15)
    u_bf = np.array(O.gauss_solve(A_bf, list(u0)))
    u = O.solve_direct(A, u0)
    assert np.linalg.norm(u_bf - u) <= 1e-14 * np.linalg.cond(A) * np.linalg.norm(u)


@SETTINGS
@given(problems())
def test_symmetrised_system_same_solution(p):
    # (I + S G0 S) w = S u0 and u = w / S solve eq. 2.19 whatever branch of
    # the square root S takes (the sign of each S_p may flip)
    n, k, side, origin, h, N, alpha = p
    pts = O.cell_points(n, side, origin)
    u0 = np.exp(1j * k * pts @ alpha)
    D = O.coupling(h, N, n, side)
    u = O.solve_direct(O.system_matrix(pts, k, D), u0)
    rng = np.random.default_rng(n)
    S = np.sqrt(D) * rng.choice([-1.0, 1.0], n ** 3)
    As = O.symmetric_system_matrix(pts, k, S)
    w = O.solve_direct(As, S * u0)
    kappa = np.linalg.cond(As) * np.abs(S).max() / np.abs(S).min()
    assert np.linalg.norm(w / S - u) <= 1e-14 * kappa * np.linalg.norm(u)


@SETTINGS
@given(problems(), st.tuples(st.floats(-1, 1), st.floats(-1, 1), st.floats(-1, 1)))
def test_translation_is_a_phase(p, t):
    # moving the body by t multiplies the solution for a plane wave by e^{ik alpha.t}
    n, k, side, origin, h, N, alpha = p
    t = np.array(t)
    out = []
    for o in (np.array(origin), np.array(origin) + t):
        pts = O.cell_points(n, side, tuple(o))
        u0 = np.exp(1j * k * pts @ alpha)
        A = O.system_matrix(pts, k, O.coupling(h, N, n, side))
        out.append(O.solve_direct(A, u0))
    err = np.linalg.norm(out[1] - np.exp(1j * k * alpha @ t) * out[0])
    assert err <= 1e-14 * np.linalg.cond(A) * np.linalg.norm(out[0])


@SETTINGS
@given(problems(nmax=2), st.integers(0, 2 ** 31 - 1))
def test_reciprocity_any_pair_of_directions(p, seed):
    # u0^(j)T D u^(i) is symmetric in (i, j): D (I + G0 D)^-1 is symmetric
    n, k, side, origin, h, N, a = p
    b = workloads.random_direction(np.random.default_rng(seed))
    pts = O.cell_points(n, side, origin)
    D = O.coupling(h, N, n, side)
    A = O.system_matrix(pts, k, D)
    ua, ub = (np.exp(1j * k * pts @ d) for d in (a, b))
    xa, xb = O.solve_direct(A, ua), O.solve_direct(A, ub)
    f_ab, f_ba = ub @ (D * xa), ua @ (D * xb)
    scale = np.abs(ub) @ np.abs(D * xa) + np.abs(ua) @ np.abs(D * xb)
    assert abs(f_ab - f_ba) <= 1e-14 * np.linalg.cond(A) * scale


@SETTINGS
@given(problems(nmax=3))
def test_cocg_matches_lu(p):
    # COCG on the symmetrised system reaches the LU solution
    n, k, side, origin, h, N, alpha = p
    pts = O.cell_points(n, side, origin)
    u0 = np.exp(1j * k * pts @ alpha)
    D = O.coupling(h, N, n, side)
    u = O.solve_direct(O.system_matrix(pts, k, D), u0)
    uc, _ = O.solve_symmetrized_cocg(pts, k, D, u0, tol=1e-13)
    S = O.symmetric_scale(D)
    kappa = np.linalg.cond(O.symmetric_system_matrix(pts, k, S)) * np.abs(S).max() / np.abs(S).min()
    assert np.linalg.norm(uc - u) <= 1e-12 * kappa * np.linalg.norm(u)
