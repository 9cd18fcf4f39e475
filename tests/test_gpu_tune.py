"""Layout autotuner (ori_tune) and the layouts it chooses from.

Every layout computes the same product: the row blocking and the prefetch
only move data, so they must be bitwise neutral; narrow tiles regroup the
butterflies over threads and the radix plan of the Z pass factors its
transforms differently, so both may differ at rounding level.
"""

import ctypes
import itertools
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


# the padded lengths (the smallest L >= 2n - 1 of these) and those with a
# second radix plan for the Z pass, as the header states them
LENGTHS = (2, 4, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 192, 256, 384, 512, 1024)
ZPLAN_LENGTHS = (32, 48, 80, 96, 128, 192, 256, 384, 512, 1024)


def padded(n):
    return min(L for L in LENGTHS if L >= 2 * n - 1)


def layouts(n):
    plans = (0, 1) if padded(n) in ZPLAN_LENGTHS else (0,)
    for lg, nar, pf, znar, zp in itertools.product(range(7), (0, 1), (0, 1), (0, 1), plans):
        if n % (1 << lg) == 0:
            yield dict(blk_lg=lg, narrow=nar, prefetch=pf, znarrow=znar, zplan=zp)


@pytest.mark.parametrize("n,R", [(24, 1), (16, 3), (14, 2)])
def test_every_layout_same_product(n, R):
    say(f"[layouts] n={n} nrhs={R}")
    k = 5.0
    case = workloads.make_case(n, k, seed=41)
    rng = np.random.default_rng(42)
    x = gpu(rng.standard_normal(R * n ** 3) + 1j * rng.standard_normal(R * n ** 3))
    with ori.ori_create(n, nrhs=R) as ctx:
        ori.ori_load(ctx, k, gpu(case["h"]), gpu(case["N"]), gpu(np.tile(case["u0"], R)))
        for prec in (ori.ORI_FP64, ori.ORI_MIXED):
            ref = None
            for lay in layouts(n):
                ori.ori_set_layout(ctx, prec, **lay)
                assert ori.ori_get_layout(ctx, prec) == lay
                y = torch.empty_like(x)
                ori.ori_matvec(ctx, x, y, op=ori.ORI_OP_SYMMETRIC, precision=prec)
                y = y.cpu().numpy()
                tiles = (lay["narrow"], lay["znarrow"], lay["zplan"])
                if ref is None:
                    ref = {(0, 0, 0): y}
                if tiles not in ref:
                    ref[tiles] = y
                # blocking and prefetch: bitwise; narrow vs wide tiles and the
                # radix plan: rounding
                assert np.array_equal(y, ref[tiles]), lay
                d = np.linalg.norm(y - ref[(0, 0, 0)]) / np.linalg.norm(ref[(0, 0, 0)])
                assert d <= (1e-14 if prec == ori.ORI_FP64 else 1e-6), (lay, d)


def test_invalid_layout_rejected():
    n = 12
    case = workloads.make_case(n, 2.0, seed=1)
    with ori.ori_setup(n, 2.0, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"])) as ctx:
        before = ori.ori_get_layout(ctx)
        # n = 12 pads to L = 24, which has one radix plan
        for bad in (dict(blk_lg=3), dict(blk_lg=-1), dict(blk_lg=7), dict(narrow=2), dict(prefetch=-1),
                    dict(znarrow=2), dict(zplan=1), dict(zplan=2), dict(zplan=-1)):
            lay = ori.Layout(bad.get("blk_lg", 0), bad.get("narrow", 0), bad.get("prefetch", 0), bad.get("znarrow", 0),
                             bad.get("zplan", 0))
            st = ori.lib().ori_set_layout(ctx.handle, ori.ORI_FP64, ctypes.byref(lay))
            assert st == ori.ORI_ERR_INVALID_ARG, bad
            assert ori.ori_get_layout(ctx) == before
        assert ori.lib().ori_set_layout(ctx.handle, 7, ctypes.byref(ori.Layout(0, 0, 0, 0, 0))) == ori.ORI_ERR_INVALID_ARG


def test_tune_picks_layout_and_records_it():
    n, k, R = 16, 5.0, 2
    say(f"[tune] n={n} nrhs={R}")
    case = workloads.make_case(n, k, seed=43)
    dirs = workloads.fibonacci_directions(R)
    u0 = np.concatenate([workloads.plane_wave(n, k, d) for d in dirs])
    with ori.ori_create(n, nrhs=R) as ctx:
        ori.ori_load(ctx, k, gpu(case["h"]), gpu(case["N"]), gpu(u0))
        u_before = torch.empty(R * n ** 3, dtype=torch.complex128, device="cuda")
        ori.ori_solve(ctx, u_before, tol=1e-12)  # also caches a graph for the old layout
        res = ori.ori_tune(ctx, reps=2)
        say(f"   {res}")
        for key, prec in (("fp64", ori.ORI_FP64), ("c64", ori.ORI_MIXED)):
            lay, ms = res[key]
            assert ms > 0
            assert lay in list(layouts(n))
            assert ori.ori_get_layout(ctx, prec) == lay
        # tuning kept the loaded data: the solve still matches LU
        u = torch.empty(R * n ** 3, dtype=torch.complex128, device="cuda")
        ori.ori_solve(ctx, u, tol=1e-12)
        ue = torch.empty_like(u)
        ori.ori_solve(ctx, ue, tol=1e-12, graph=False)
        assert np.array_equal(u.cpu().numpy(), ue.cpu().numpy())  # the graph follows the new layout
        ub = u_before.cpu().numpy()
        # both solves stop at a relative residual below 1e-12 of the
        # symmetric system (I + S G0 S) w = S u0, so each w is within
        # kappa * 1e-12 of the exact one and u = w / S within spread(|S|) times
        # that: kappa_2 = 3.41 and max|S| / min|S| = 1.11 here (oracle, CPU),
        # so the two differ by at most 2 * 1.11 * 3.41e-12 = 7.5e-12
        assert np.linalg.norm(u.cpu().numpy() - ub) <= 1e-11 * np.linalg.norm(ub)
    # a new context on the same (n, nrhs) starts from the tuned layouts
    with ori.ori_create(n, nrhs=R) as ctx2:
        assert ori.ori_get_layout(ctx2, ori.ORI_FP64) == res["fp64"][0]
        assert ori.ori_get_layout(ctx2, ori.ORI_MIXED) == res["c64"][0]
    # the first right-hand side against the oracle's dense solve
    pts = O.cell_points(n)
    D = O.coupling(case["h"], case["N"], n)
    u_ref = O.solve_direct(O.system_matrix(pts, k, D), u0[: n ** 3])
    got = u.cpu().numpy()[: n ** 3]
    assert np.linalg.norm(got - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_tune_fp64_only_provision():
    n = 8
    case = workloads.make_case(n, 3.0, seed=44)
    with ori.ori_create(n, provision=ori.ORI_PROVISION_FP64) as ctx:
        ori.ori_load(ctx, 3.0, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"]))
        res = ori.ori_tune(ctx, reps=1)
        assert res["fp64"][1] > 0 and res["c64"][1] == -1.0


@pytest.mark.parametrize("n,z128,z64,p128", [(16, 0, 1, 0), (128, 0, 1, 0), (256, 1, 1, 0), (512, 1, 1, 1)])
def test_default_z_tile_width(n, z128, z64, p128):
    # narrow Z tiles by default where they measured faster: complex64 at every
    # length, complex128 from L = 512 on; the alternative radix plan only for
    # the complex128 Z pass at L = 1024
    with ori.ori_create(n) as ctx:
        assert ori.ori_get_layout(ctx, ori.ORI_FP64)["znarrow"] == z128
        assert ori.ori_get_layout(ctx, ori.ORI_MIXED)["znarrow"] == z64
        assert ori.ori_get_layout(ctx, ori.ORI_FP64)["zplan"] == p128
        assert ori.ori_get_layout(ctx, ori.ORI_MIXED)["zplan"] == 0


@pytest.mark.parametrize("n", [40, 48, 64, 96, 128, 192, 256, 512])
def test_zplan_variants_agree(n):
    # the two radix plans of the Z pass (L = 80, 96, 128, 192, 256, 384, 512,
    # 1024 here) give the same product to rounding, in both precisions; the
    # default plans are held to the oracle by the parity tests
    say(f"[zplan] n={n} L={padded(n)}")
    assert padded(n) in ZPLAN_LENGTHS
    k = 5.0
    case = workloads.make_case(n, k, seed=45)
    rng = np.random.default_rng(46)
    x = gpu(rng.standard_normal(n ** 3) + 1j * rng.standard_normal(n ** 3))
    with ori.ori_create(n) as ctx:
        ori.ori_load(ctx, k, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"]))
        for prec, bar in ((ori.ORI_FP64, 1e-13), (ori.ORI_MIXED, 2e-6)):
            base = ori.ori_get_layout(ctx, prec)
            ys = []
            for zp in (0, 1):
                ori.ori_set_layout(ctx, prec, **dict(base, zplan=zp))
                y = torch.empty_like(x)
                ori.ori_matvec(ctx, x, y, op=ori.ORI_OP_SYMMETRIC, precision=prec)
                ys.append(y)
            d = (torch.linalg.vector_norm(ys[1] - ys[0]) / torch.linalg.vector_norm(ys[0])).item()
            say(f"   precision {prec}: plans differ by {d:.2e}")
            assert 0 < d <= bar, (prec, d)  # 0 would mean the knob changed nothing
