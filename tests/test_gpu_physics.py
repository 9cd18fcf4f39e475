"""GPU parity of the physics entry points with the oracle (oracle/physics.py).

Charges (eqs. 2.13, 2.18), the scattered field (eq. 2.10) and its far-field
amplitude, and the refraction recipe (eqs. 2.24-2.26, 4.1-4.2), through the
C ABI.  Direct sums in FP64 on both sides in different orders: 1e-12.
"""

import math
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


def varied(n, k, seed):
    rng = np.random.default_rng(seed)
    P = n ** 3
    h = (-1 + 0.5j) * (1 + 0.3 * rng.uniform(-1, 1, P))
    N = 0.5 + rng.random(P)
    return h, N


def solved(n, k, h, N, u0, nrhs=1, side=1.0, origin=(0.0, 0.0, 0.0)):
    ctx = ori.ori_create(n, side=side, origin=origin, nrhs=nrhs)
    ori.ori_load(ctx, k, gpu(h), gpu(N), gpu(u0))
    u = torch.empty(nrhs * n ** 3, dtype=torch.complex128, device="cuda")
    ori.ori_solve(ctx, u, tol=1e-13)
    return ctx, u


def test_charges_and_field_vs_oracle():
    n, k = 8, 4.0
    say(f"[field] n={n}")
    h, N = varied(n, k, 61)
    pts = O.cell_points(n, side=1.3, origin=(0.2, -0.1, 0.4))
    u0 = np.exp(1j * k * pts @ np.array([0.0, 0.6, 0.8]))
    ctx, ug = solved(n, k, h, N, u0, side=1.3, origin=(0.2, -0.1, 0.4))
    with ctx:
        u = ug.cpu().numpy()
        q = ori.ori_charges(ctx, ug).cpu().numpy()
        Qo = O.cell_charges(h, N, n, u, side=1.3)
        assert rel(q, Qo) <= 1e-15
        # points inside, outside and exactly at cells (left out of the sum)
        rng = np.random.default_rng(62)
        x = np.concatenate([rng.uniform(-1, 3, (40, 3)), pts[[0, 77, 511]]])
        v = ori.ori_scattered_field(ctx, ug, gpu(x)).cpu().numpy()
        vo = O.scattered_field(pts, k, Qo, x)
        say(f"   charges ok; field err {rel(v, vo):.2e}")
        assert rel(v, vo) <= 1e-12
        # at every cell point, u0 + v is the solution of eq. 2.19
        vc = ori.ori_scattered_field(ctx, ug, gpu(pts)).cpu().numpy()
        assert rel(u0 + vc, u) <= 1e-11
        # far field
        beta = rng.standard_normal((30, 3))
        beta /= np.linalg.norm(beta, axis=1, keepdims=True)
        A = ori.ori_far_field(ctx, ug, gpu(beta)).cpu().numpy()
        Ao = O.far_field(pts, k, Qo, beta)
        assert rel(A, Ao) <= 1e-12


def test_field_many_chunks_and_batch():
    # P = 64^3 spans several chunks of cells; two right-hand sides
    n, k = 64, 5.0
    say(f"[field] n={n} nrhs=2")
    case = workloads.make_case(n, k, seed=63)
    pts = O.cell_points(n)
    u0 = np.concatenate([workloads.plane_wave(n, k, (1.0, 0.0, 0.0)), workloads.plane_wave(n, k, (0.0, 0.0, -1.0))])
    ctx, ug = solved(n, k, case["h"], case["N"], u0, nrhs=2)
    with ctx:
        u = ug.cpu().numpy().reshape(2, -1)
        x = np.array([[0.5, 0.5, 2.0], [-1.0, 0.3, 0.3], [0.25, 0.75, 0.5], [10.0, 10.0, 10.0]])
        v = ori.ori_scattered_field(ctx, ug, gpu(x)).cpu().numpy().reshape(2, -1)
        beta = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [-1.0, 0.0, 0.0]])
        A = ori.ori_far_field(ctx, ug, gpu(beta)).cpu().numpy().reshape(2, -1)
    D = O.coupling(case["h"], case["N"], n)
    for r in range(2):
        Q = -D * u[r]
        assert rel(v[r], O.scattered_field(pts, k, Q, x)) <= 1e-12
        assert rel(A[r], O.far_field(pts, k, Q, beta)) <= 1e-12
    # reciprocity of the far field: A_{e1}(-e3 direction reversed) ... A_a(b) = A_{-b}(-a)
    # with a = e1 (rhs 0) and -b = -e3 (rhs 1): A_0(e3) = A_1(-e1)
    say(f"   reciprocity {abs(A[0, 1] - A[1, 2]) / abs(A[0, 1]):.2e}")
    assert abs(A[0, 1] - A[1, 2]) <= 1e-9 * abs(A[0, 1])


def test_refraction_recipe_worked_example_on_gpu():
    v, f, k_pr, n0r, n0i, nr, ni, Nv, hr, hi = np.loadtxt(os.path.join(GOLDEN, "section4_refraction_example.txt"))
    k = 2 * math.pi * f / v
    n = 4
    P = n ** 3
    with ori.ori_create(n) as ctx:
        n0 = gpu(np.full(P, complex(n0r, n0i)))
        h = ori.ori_design_impedance(ctx, k, n0, gpu(np.full(P, complex(nr, ni))), gpu(np.full(P, Nv))).cpu().numpy()
        assert np.all(np.abs(h.real - hr) <= 0.5e-5 * abs(hr)) and np.all(np.abs(h.imag - hi) <= 0.5e-5 * abs(hi))
        nn = ori.ori_refraction_index(ctx, k, n0, gpu(np.full(P, complex(hr, hi)))).cpu().numpy()
        assert np.all(np.abs(nn - complex(nr, ni)) <= 2e-6)


def test_refraction_recipe_vs_oracle_and_bad_input():
    n, k = 6, 2.5
    P = n ** 3
    rng = np.random.default_rng(64)
    n0 = 1.0 + 0.3 * rng.standard_normal(P) + 0.05j * rng.random(P)
    nt = rng.standard_normal(P) + 1j * rng.random(P)
    N = 0.5 + rng.random(P)
    hh = (rng.standard_normal(P) + 1j * rng.standard_normal(P)) * 0.3
    with ori.ori_create(n) as ctx:
        h = ori.ori_design_impedance(ctx, k, gpu(n0), gpu(nt), gpu(N), c_S=3.0).cpu().numpy()
        assert rel(h, O.h_for_refraction(k, n0, nt, N, c_S=3.0)) <= 1e-14
        nn = ori.ori_refraction_index(ctx, k, gpu(n0), gpu(hh), gpu(N)).cpu().numpy()
        no = O.refraction_from_h(k, n0, hh, N)
        assert rel(nn, no) <= 1e-14
        assert np.all(nn.imag >= 0.0)
        # round trip through the branch
        back = ori.ori_refraction_index(ctx, k, gpu(n0), gpu(h), gpu(N), c_S=3.0).cpu().numpy()
        assert rel(back, nt) <= 1e-12
        # N = 0 cannot host the particles a design needs; NaN is refused
        N0 = N.copy()
        N0[5] = 0.0
        with pytest.raises(ori.OriError) as e:
            ori.ori_design_impedance(ctx, k, gpu(n0), gpu(nt), gpu(N0))
        assert e.value.status == ori.ORI_ERR_INVALID_ARG
        hb = hh.copy()
        hb[3] = np.nan
        with pytest.raises(ori.OriError):
            ori.ori_refraction_index(ctx, k, gpu(n0), gpu(hb), gpu(N))


@pytest.mark.parametrize("nf,nc,off", [(24, 5, 0.0), (24, 8, 0.5), (16, 16, 0.5), (10, 12, 0.0), (40, 20, 0.0)])
def test_interpolation_difference_vs_oracle(nf, nc, off):
    rng = np.random.default_rng(nf + nc)
    x = rng.standard_normal(nf ** 3) + 1j * rng.standard_normal(nf ** 3)
    y = rng.standard_normal(nc ** 3) + 1j * rng.standard_normal(nc ** 3)
    with ori.ori_create(nc) as ctx:
        d = ori.ori_interpolation_difference(ctx, gpu(y), gpu(x), nf, off)
    do = O.interpolation_difference(x, nf, y, nc, off)
    assert abs(d - do) <= 1e-13 * do


def test_ori_red_ie_comparison_in_miniature():
    # Section 4's study on nested corner lattices (eq. 3.3.5): the ORI system
    # of M particles is eq. 2.19 on the M-point lattice (a^{2-kappa} = 1/M,
    # N = 1), RED and IE are the same system on P- and C-point lattices
    k, hval = 0.182651 * 40, 2.65481e-09 + 5.30961e-06j   # a larger k makes the cells matter
    sols = {}
    for name, n in (("ORI", 48), ("RED", 8), ("IE", 16)):
        u0 = workloads.plane_wave(n, k, (1.0, 0.0, 0.0), offset=0.0)
        with ori.ori_setup(n, k, gpu(np.full(n ** 3, hval)), None, gpu(u0), cell_offset=0.0) as ctx:
            u = torch.empty(n ** 3, dtype=torch.complex128, device="cuda")
            ori.ori_solve(ctx, u, tol=1e-12)
            sols[name] = (n, u)
    out = {}
    for fine, coarse in (("ORI", "RED"), ("IE", "RED"), ("ORI", "IE")):
        nf, xf = sols[fine]
        nc, yc = sols[coarse]
        with ori.ori_create(nc, cell_offset=0.0) as ctx:
            d = ori.ori_interpolation_difference(ctx, yc, xf, nf, 0.0)
        do = O.interpolation_difference(xf.cpu().numpy(), nf, yc.cpu().numpy(), nc, 0.0)
        assert abs(d - do) <= 1e-13 * do
        out[(fine, coarse)] = d
    say(f"   ORI-RED {out[('ORI', 'RED')]:.4f}  RED-IE {out[('IE', 'RED')]:.4f}  ORI-IE {out[('ORI', 'IE')]:.4f}")
    # the difference is set by how much u varies inside a coarse cell
    assert out[("ORI", "IE")] < out[("ORI", "RED")]
