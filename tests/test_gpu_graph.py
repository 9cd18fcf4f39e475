"""HIP-graph replay of COCG iteration blocks against eager launches.

A graph block holds the same kernels with the same arguments as the eager
iterations, so every replay must reproduce the eager iterate bit for bit.
Replays are interleaved with the library's own eager work (the first block,
scalar reads, recovery, true residual) and with reloads of new data into
the same context; each replay count is checked against an eager run.
"""

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


def solve_pair(ctx, P, **opts):
    out = []
    for graph in (False, True):
        u = torch.empty(P, dtype=torch.complex128, device="cuda")
        st, info = ori.ori_solve(ctx, u, graph=graph, raise_on_error=False, **opts)
        out.append((st, info, u.cpu().numpy()))
    return out


@pytest.mark.parametrize("precision", [ori.ORI_FP64, ori.ORI_MIXED])
@pytest.mark.parametrize("check_every", [1, 3])
def test_graph_bitwise_every_replay_count(precision, check_every):
    n, k = 16, 5.0
    say(f"[graph] n={n} precision={precision} check_every={check_every}")
    case = workloads.make_case(n, k, seed=31)
    with ori.ori_setup(n, k, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"])) as ctx:
        # max_iter sweeps the number of replays (0 .. several) of the cached graph
        for max_iter in range(1, 4 * check_every + 2):
            (s0, i0, u0), (s1, i1, u1) = solve_pair(ctx, n ** 3, tol=1e-12, max_iter=max_iter, precision=precision,
                                                    check_every=check_every)
            assert s0 == s1 and i0["iterations"] == i1["iterations"] and i0["matvecs"] == i1["matvecs"]
            assert np.array_equal(u0, u1), f"max_iter={max_iter}"
        # to convergence, then again after a reload into the same context
        (s0, i0, u0), (s1, i1, u1) = solve_pair(ctx, n ** 3, tol=1e-10, precision=precision, check_every=check_every)
        assert s0 == s1 == ori.ORI_OK and np.array_equal(u0, u1)
        case2 = workloads.make_case(n, k, seed=32)
        ori.ori_load(ctx, k, gpu(case2["h"]), gpu(case2["N"]), gpu(case2["u0"]))
        (s0, i0, u2), (s1, i1, u3) = solve_pair(ctx, n ** 3, tol=1e-10, precision=precision, check_every=check_every)
        assert s0 == s1 == ori.ORI_OK and np.array_equal(u2, u3)
        say(f"   iters={i1['iterations']}")
    # and the graph result is the solution of eq. 2.19
    pts = O.cell_points(n)
    D = O.coupling(case2["h"], case2["N"], n)
    u_ref = O.solve_direct(O.system_matrix(pts, k, D), case2["u0"])
    err = np.linalg.norm(u3 - u_ref) / np.linalg.norm(u_ref)
    assert err <= (1e-8 if precision == ori.ORI_FP64 else 1e-6)


def test_graph_batch_and_adjoint():
    n, k, R = 12, 4.0, 4
    say(f"[graph batch] n={n} nrhs={R}")
    case = workloads.make_case(n, k, seed=33)
    dirs = workloads.fibonacci_directions(R)
    u0 = np.concatenate([workloads.plane_wave(n, k, d) for d in dirs])
    with ori.ori_create(n, nrhs=R) as ctx:
        ori.ori_load(ctx, k, gpu(case["h"]), gpu(case["N"]), gpu(u0))
        (s0, i0, ua), (s1, i1, ub) = solve_pair(ctx, R * n ** 3, tol=1e-10, check_every=2)
        assert s0 == s1 == ori.ORI_OK and np.array_equal(ua, ub)
        (s0, i0, ua), (s1, i1, ub) = solve_pair(ctx, R * n ** 3, tol=1e-8, precision=ori.ORI_MIXED, check_every=2)
        assert s0 == s1 == ori.ORI_OK and np.array_equal(ua, ub)
    # the adjoint solve runs the same iteration blocks
    with ori.ori_setup(n, k, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"])) as ctx:
        u = torch.empty(n ** 3, dtype=torch.complex128, device="cuda")
        ori.ori_solve(ctx, u, tol=1e-12)
        f = gpu(np.random.default_rng(5).standard_normal(n ** 3) + 0j)
        g = []
        for graph in (False, True):
            gg = torch.empty(n ** 3, dtype=torch.complex128, device="cuda")
            ori.ori_adjoint(ctx, u, f, gg, tol=1e-12, graph=graph)
            g.append(gg.cpu().numpy())
        assert np.array_equal(g[0], g[1])


def test_graph_replay_in_concurrent_contexts():
    # contexts driven from four threads at once (each its own stream), each
    # building and replaying its own iteration graphs (graph replay on, the
    # default), while a fifth thread allocates and frees device memory through
    # torch: every result equals the same problem solved with eager launches
    # in one thread, bit for bit, over three rounds
    import random
    import threading

    say("[graph, threads] n in {12, 16, 20, 24}")
    probs = []
    for j, n in enumerate((12, 16, 20, 24)):
        c = workloads.make_case(n, 4.0, seed=90 + j)
        probs.append(dict(n=n, k=4.0, h=gpu(c["h"]), N=gpu(c["N"]), u0=gpu(c["u0"])))
    ref = [ori.solve(p["n"], p["k"], p["h"], p["N"], p["u0"], tol=1e-10, graph=False)[0] for p in probs]
    torch.cuda.synchronize()
    stop = threading.Event()
    errors = []

    def churn():
        rng = random.Random(5)
        while not stop.is_set():
            t = torch.empty(rng.randint(1, 64) << 18, dtype=torch.float32, device="cuda")
            t.fill_(1.0)
            del t
            torch.cuda.empty_cache()

    def worker(p, r, rnd):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                u, info = ori.solve(p["n"], p["k"], p["h"], p["N"], p["u0"], tol=1e-10, graph=True)
            s.synchronize()
            if not torch.equal(u, r) or not info["rel_res_true"] < 1e-9:
                errors.append((rnd, p["n"]))
        except BaseException as e:  # reported below
            errors.append((rnd, p["n"], repr(e)))

    th = threading.Thread(target=churn)
    th.start()
    try:
        for rnd in range(3):
            ws = [threading.Thread(target=worker, args=(p, r, rnd)) for p, r in zip(probs, ref)]
            for w in ws:
                w.start()
            for w in ws:
                w.join()
    finally:
        stop.set()
        th.join()
    assert not errors, errors
