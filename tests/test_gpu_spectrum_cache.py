"""Reuse of the kernel spectrum by ori_load (it depends on the grid and k
only): results bitwise equal to a fresh computation, recomputed when k
changes, and a load that keeps k skips the three spectrum passes."""

import sys
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_04691_amd as ori  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [12, 64])
def test_spectrum_reuse_is_bitwise(n):
    k1, k2 = 3.0, 4.5
    a = workloads.make_case(n, k1, seed=500 + n)
    b = workloads.make_case(n, k1, seed=600 + n)
    P = n ** 3
    u = torch.empty(P, dtype=torch.complex128, device="cuda")

    def fresh(k, c):
        with ori.ori_create(n) as c1:
            ori.ori_spectrum_cache(c1, False)
            ori.ori_load(c1, k, gpu(c["h"]), gpu(c["N"]), gpu(c["u0"]))
            v = torch.empty_like(u)
            ori.ori_solve(c1, v, tol=1e-11)
            ori.ori_profile_enable(c1, True)
            ori.ori_load(c1, k, gpu(c["h"]), gpu(c["N"]), gpu(c["u0"]))
            assert ori.ori_profile_read(c1)["spectrum"][1] == 3  # cache off: every load
            ori.ori_profile_enable(c1, False)
            return v

    with ori.ori_create(n) as ctx:
        ori.ori_load(ctx, k1, gpu(a["h"]), gpu(a["N"]), gpu(a["u0"]))
        ori.ori_profile_enable(ctx, True)
        ori.ori_load(ctx, k1, gpu(b["h"]), gpu(b["N"]), gpu(b["u0"]))  # same k: spectrum kept
        assert "spectrum" not in ori.ori_profile_read(ctx)
        ori.ori_solve(ctx, u, tol=1e-11)
        assert torch.equal(u, fresh(k1, b))
        ori.ori_load(ctx, k2, gpu(b["h"]), gpu(b["N"]), gpu(b["u0"]))  # new k: recomputed
        assert ori.ori_profile_read(ctx)["spectrum"][1] == 3
        ori.ori_profile_enable(ctx, False)
        ori.ori_solve(ctx, u, tol=1e-11)
        assert torch.equal(u, fresh(k2, b))


def test_spectrum_reuse_speeds_up_reloads():
    # a design loop at n = 128 that changes h only: reloads with the spectrum
    # kept against reloads that compute it again
    n, k = 128, 5.0
    c = workloads.make_case(n, k, seed=3)
    h, N, u0 = gpu(c["h"]), gpu(c["N"]), gpu(c["u0"])
    times = {}
    with ori.ori_create(n) as ctx:
        for cache in (False, True):
            ori.ori_spectrum_cache(ctx, cache)
            ori.ori_load(ctx, k, h, N, u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(20):
                ori.ori_load(ctx, k, h * (1.0 + 1e-3 * i), N, u0)
            torch.cuda.synchronize()
            times[cache] = (time.perf_counter() - t0) / 20
    say(f"[spectrum cache] n=128 ori_load {times[False] * 1e3:.3f} ms computed, {times[True] * 1e3:.3f} ms kept")
    assert times[True] < times[False]
