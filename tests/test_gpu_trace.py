"""ORI_TRACE=1: the residual trace of a solve on stderr, one line per
right-hand side after every check (COCG) and per refinement (mixed)."""
import re

import numpy as np
import pytest
import torch

import paper_1602_04691_amd as ori
import workloads

pytestmark = pytest.mark.gpu


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def traced_solve(monkeypatch, capfd, precision):
    case = workloads.make_case(16, 1.0, seed=0, alpha=(1.0, 0.0, 0.0))
    monkeypatch.setenv("ORI_TRACE", "1")  # read when the context is created
    ctx = ori.ori_create(16)
    monkeypatch.delenv("ORI_TRACE")
    with ctx:
        ori.ori_load(ctx, 1.0, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"]))
        u = torch.empty(16 ** 3, dtype=torch.complex128, device="cuda")
        _, info = ori.ori_solve(ctx, u, tol=1e-10 if precision == ori.ORI_FP64 else 1e-8, precision=precision)
    torch.cuda.synchronize()
    return capfd.readouterr().err.splitlines(), info


def test_trace_follows_the_fp64_iterations(monkeypatch, capfd):
    lines, info = traced_solve(monkeypatch, capfd, ori.ORI_FP64)
    cocg = [ln for ln in lines if ln.startswith("[ori] cocg c128 rhs 0 ")]
    # the check before the first iteration, then one per iteration (check_every = 1)
    assert len(cocg) == info["iterations"] + 1
    iters = [int(re.search(r" iter (\d+) ", ln).group(1)) for ln in cocg]
    assert iters == list(range(info["iterations"] + 1))
    rel = [float(re.search(r" rel (\S+)", ln).group(1)) for ln in cocg]
    assert rel[0] == 1.0  # x0 = 0: the run starts from r0 = b
    assert cocg[-1].endswith(" done") and not any(ln.endswith(" done") for ln in cocg[:-1])
    assert rel[-1] <= 1e-10
    assert rel[-1] == pytest.approx(info["rel_res_recursive"], rel=1e-6)


def test_trace_shows_every_refinement(monkeypatch, capfd):
    lines, info = traced_solve(monkeypatch, capfd, ori.ORI_MIXED)
    refine = [ln for ln in lines if ln.startswith("[ori] refine ")]
    assert info["refinements"] >= 1
    assert len(refine) == info["refinements"] + 1
    assert [int(ln.split()[2]) for ln in refine] == list(range(info["refinements"] + 1))
    rel = [float(ln.split()[-1]) for ln in refine]
    assert rel[0] == pytest.approx(1.0, rel=1e-12)
    assert rel[-1] <= 1e-8 and rel[-1] == pytest.approx(info["rel_res_recursive"], rel=1e-12)
    assert any(ln.startswith("[ori] cocg c64 rhs 0 ") for ln in lines)


def test_no_trace_without_the_flag(capfd):
    case = workloads.make_case(8, 1.0, seed=0, alpha=(1.0, 0.0, 0.0))
    u = ori.solve(8, 1.0, gpu(case["h"]), gpu(case["N"]), gpu(case["u0"]), tol=1e-10)[0]
    torch.cuda.synchronize()
    assert u.isfinite().all()
    assert "[ori]" not in capfd.readouterr().err
