"""Properties of the solution of eq. 2.19 checked on the HIP path.

Each test fixes a part of the result that a plausible mistake would break
(sign or scale of the scattering term, geometry, axis handling, linearity,
the COCG recursion) against the mathematics or against the printed numbers
of the paper, through the C ABI.
"""

import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_04691_amd as ori  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_solve(n, k, h, N, u0, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5, **opts):
    with ori.ori_setup(n, k, gpu(h), None if N is None else gpu(N), gpu(u0), side=side, origin=origin,
                       cell_offset=offset) as ctx:
        u = torch.empty(n ** 3, dtype=torch.complex128, device="cuda")
        st, info = ori.ori_solve(ctx, u, raise_on_error=False, **opts)
        return st, info, u.cpu().numpy()


def test_born_limit_on_gpu():
    # h = eps h~: u = u0 - G0 D u0 + O(eps^2) (eq. 2.19 expanded once), so the
    # remainder falls by 4 when eps halves; a wrong sign or scale of the sum
    # leaves an O(eps) remainder (ratio 2)
    n, k = 8, 3.0
    case = workloads.make_case(n, k, seed=51)
    pts = O.cell_points(n)
    errs = []
    for eps in (0.4, 0.2, 0.1, 0.05):
        h = eps * case["h"]
        _, _, u = gpu_solve(n, k, h, None, case["u0"], tol=1e-14)
        D = O.coupling(h, None, n)
        born = case["u0"] - O.scatter_dense(pts, k, D, case["u0"])
        errs.append(np.linalg.norm(u - born))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    say(f"[born] remainders {errs} ratios {ratios}")
    assert 3.5 < ratios[-1] < 4.5 and 3.0 < ratios[-2] < 5.0


def test_origin_shift_is_a_phase_on_gpu():
    # translating the domain by t multiplies u0 = exp(ik alpha.x), hence u, by exp(ik alpha.t)
    n, k = 12, 5.0
    case = workloads.make_case(n, k, seed=52)
    alpha = case["alpha"]
    t = np.array([0.3, -1.7, 2.2])
    _, _, u1 = gpu_solve(n, k, case["h"], None, case["u0"], tol=1e-13)
    u0s = workloads.plane_wave(n, k, alpha, origin=tuple(t))
    _, _, u2 = gpu_solve(n, k, case["h"], None, u0s, origin=tuple(t), tol=1e-13)
    phase = np.exp(1j * k * alpha @ t)
    say(f"[phase] {rel(u2, phase * u1):.2e}")
    assert rel(u2, phase * u1) <= 1e-11


def test_superposition_in_u0_batch():
    # linear in u0: three right-hand sides of one batch, the third a
    # combination of the first two
    n, k = 12, 4.0
    case = workloads.make_case(n, k, seed=53)
    a = workloads.plane_wave(n, k, (1.0, 0.0, 0.0))
    b = workloads.plane_wave(n, k, (0.0, 0.6, 0.8))
    c1, c2 = 0.7 - 0.2j, -1.3 + 0.5j
    u0 = np.concatenate([a, b, c1 * a + c2 * b])
    P = n ** 3
    with ori.ori_create(n, nrhs=3) as ctx:
        ori.ori_load(ctx, k, gpu(case["h"]), gpu(case["N"]), gpu(u0))
        u = torch.empty(3 * P, dtype=torch.complex128, device="cuda")
        ori.ori_solve(ctx, u, tol=1e-13)
        u = u.cpu().numpy().reshape(3, P)
    say(f"[superposition] {rel(u[2], c1 * u[0] + c2 * u[1]):.2e}")
    assert rel(u[2], c1 * u[0] + c2 * u[1]) <= 1e-11


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_per_axis_on_gpu(axis):
    # h, N and u0 even under i_axis -> n-1-i_axis make u even too
    n, k = 10, 4.0
    rng = np.random.default_rng(54 + axis)
    h = ((-1 + 0.5j) * (1 + 0.2 * rng.uniform(-1, 1, n ** 3))).reshape(n, n, n)
    N = (1 + 0.5 * rng.uniform(0, 1, n ** 3)).reshape(n, n, n)
    h = 0.5 * (h + np.flip(h, axis))
    N = 0.5 * (N + np.flip(N, axis))
    dirn = np.array([0.6, 0.0, 0.8]) if axis == 1 else np.array([0.0, 0.6, 0.8]) if axis == 0 else \
        np.array([0.6, 0.8, 0.0])
    u0 = workloads.plane_wave(n, k, dirn).reshape(n, n, n)
    assert np.allclose(u0, np.flip(u0, axis), atol=1e-14)
    _, _, u = gpu_solve(n, k, h.ravel(), N.ravel(), u0.ravel(), tol=1e-13)
    u = u.reshape(n, n, n)
    say(f"[mirror {axis}] {rel(np.flip(u, axis), u):.2e}")
    assert rel(np.flip(u, axis), u) <= 1e-12
    # and a broken symmetry is seen: N not mirrored
    N2 = N.copy()
    N2.reshape(-1)[0] *= 3.0
    _, _, u2 = gpu_solve(n, k, h.ravel(), N2.ravel(), u0.ravel(), tol=1e-13)
    u2 = u2.reshape(n, n, n)
    assert rel(np.flip(u2, axis), u2) > 1e-6


def test_paper_table6_first_iterate_on_gpu():
    # Section 4, Table 6 (b = 20, corner lattice, constant h): the printed
    # digits are the first COCG iterate of the sign-flipped system.  With
    # constant S the symmetric form is a multiple of A, so the library's first
    # iterate (max_iter = 1) is that iterate.
    rows = np.loadtxt(os.path.join(GOLDEN, "table6_red_b20.txt"))
    b, k = 20, 0.182651
    h = np.full(b ** 3, -(2.65481e-09 + 5.30961e-06j))  # h -> -h
    u0 = workloads.plane_wave(b, k, (1.0, 0.0, 0.0), offset=0.0)
    st, info, u = gpu_solve(b, k, h, None, u0, offset=0.0, tol=1e-30, max_iter=1)
    assert st == ori.ORI_ERR_NOT_CONVERGED and info["iterations"] == 1
    got = u.reshape(b, b, b)
    for i1, re, im in rows:
        sub = got[int(i1)][::4, ::4]
        assert np.all(np.abs(sub.real - re) <= 0.5e-6 + 1e-12), (i1, sub.real.min(), sub.real.max(), re)
        assert np.all(np.abs(sub.imag - im) <= 0.5e-6 + 1e-12), (i1, sub.imag.min(), sub.imag.max(), im)


@pytest.mark.parametrize("k", [1.0, 5.0, 10.0])
def test_iteration_counts_match_oracle_cocg(k):
    # the same COCG recursion on the same symmetric system: the oracle's
    # (Section 3 FFT route, dense-free) and the library's iteration counts to
    # 1e-10 agree within one (rounding at the threshold), at every n
    counts = []
    for n in (16, 32, 64):
        case = workloads.make_case(n, k, seed=0, alpha=(1.0, 0.0, 0.0))
        D = O.coupling(case["h"], case["N"], n)
        S = O.symmetric_scale(D)

        def apply(w):
            return w + S * O.scatter_section3(n, k, S, w)

        w, hist = O.cocg(apply, S * case["u0"], tol=1e-10)
        u_or = case["u0"] - O.scatter_section3(n, k, S, w)
        st, info, u = gpu_solve(n, k, case["h"], case["N"], case["u0"], tol=1e-10)
        say(f"[iterations] k={k} n={n} gpu={info['iterations']} oracle={len(hist) - 1} diff={rel(u, u_or):.2e}")
        assert st == ori.ORI_OK
        assert abs(info["iterations"] - (len(hist) - 1)) <= 1
        assert rel(u, u_or) <= 1e-8
        counts.append(info["iterations"])
    # mesh-independent convergence of the discretised integral equation
    assert max(counts) - min(counts) <= 3
