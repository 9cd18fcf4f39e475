"""Memory safety of the kernels on the library's own workspaces: every
workspace is followed by a guard band of a fixed byte pattern
(ori_check_guards).  Every operation of the library leaves all bands intact;
in the debug mode ORI_CHECK_GUARDS=1 the bands are checked after every kernel
launch."""

import os
import subprocess
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_04691_amd as ori  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# every kind of operation, on small problems of several padded lengths
# (radix 2, 3, 5 stages), in both precisions, batched and single
def exercise(ori, torch, workloads, np, check):
    def g(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for n in (5, 12, 24):
        k = 4.0
        c = workloads.make_case(n, k, seed=n)
        P = n ** 3
        with ori.ori_setup(n, k, g(c["h"]), g(c["N"]), g(c["u0"])) as ctx:
            u = torch.empty(P, dtype=torch.complex128, device="cuda")
            for prec in (ori.ORI_FP64, ori.ORI_MIXED):
                ori.ori_solve(ctx, u, tol=1e-10, precision=prec)
            y = torch.empty_like(u)
            for op in (ori.ORI_OP_SYSTEM, ori.ORI_OP_SYMMETRIC):
                ori.ori_matvec(ctx, u, y, op, ori.ORI_FP64)
            ori.ori_charges(ctx, u)
            pts = g(np.array([[0.5, 0.5, 2.0], [0.1, 0.2, 0.3]]))
            ori.ori_scattered_field(ctx, u, pts)
            ori.ori_far_field(ctx, u, g(np.array([[0.0, 0.0, 1.0]])))
            t = g(c["u0"] * 1.1)
            ori.ori_gradient(ctx, t, u, torch.empty_like(u), tol=1e-10)
            n0 = g(np.full(P, 1.0 + 0.0j))
            hh = ori.ori_design_impedance(ctx, k, n0, g(np.full(P, 1.1 + 0.01j)), g(c["N"]))
            ori.ori_refraction_index(ctx, k, n0, hh, g(c["N"]))
            ori.ori_tune(ctx, reps=1)
            check(ctx)
        with ori.ori_create(n, nrhs=3) as ctx:
            u0 = np.concatenate([workloads.plane_wave(n, k, d) for d in workloads.fibonacci_directions(3)])
            ori.ori_load(ctx, k, g(c["h"]), g(c["N"]), g(u0))
            u = torch.empty(3 * P, dtype=torch.complex128, device="cuda")
            ori.ori_solve(ctx, u, tol=1e-10, precision=ori.ORI_MIXED)
            check(ctx)
    with ori.ori_create(6) as ctx:
        y = g(np.ones(6 ** 3, dtype=np.complex128))
        ori.ori_interpolation_difference(ctx, y, g(np.ones(12 ** 3, dtype=np.complex128)), 12)
        check(ctx)


def test_guards_intact_after_every_operation():
    seen = []

    def check(ctx):
        seen.append(ori.ori_check_guards(ctx))

    exercise(ori, torch, workloads, np, check)
    assert len(seen) == 7 and all(d == 0 for d in seen), seen


def test_guards_checked_after_every_launch():
    # the same operations with the per-launch check switched on, in a fresh
    # process (the switch is read when a context is created)
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "import numpy as np, torch, workloads, paper_1602_04691_amd as ori\n"
        "from test_gpu_guards import exercise\n"
        "exercise(ori, torch, workloads, np, lambda ctx: None)\n"
        "print('OK')\n"
    ) % (ROOT, os.path.join(ROOT, "tests"))
    env = dict(os.environ, ORI_CHECK_GUARDS="1")
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0 and p.stdout.strip().endswith("OK"), p.stdout[-2000:] + p.stderr[-4000:]
