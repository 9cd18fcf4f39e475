"""Sampled rows of eq. 2.19 on several host cores.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The rows of the Green's sum are independent of each other, so a list of rows
is split into consecutive groups and each group is handed to
``ori_oracle.sample_scatter_rows`` (or ``sample_residual_rows``) in a worker
process.  The arithmetic of a row is that of the single-process function, so
the result equals it bit for bit (pinned in tests/test_oracle_pins.py).

Workers are forked: the arrays (points, D, the vector) are inherited without
copies and without pickling.  The workers only run NumPy.
"""

import multiprocessing as mp
import os

import numpy as np

from . import ori_oracle

_ARGS = None


def _init(args):
    global _ARGS
    _ARGS = args


def _work(rows):
    points, k, D, v, u0, chunk = _ARGS
    if u0 is None:
        return ori_oracle.sample_scatter_rows(points, k, D, v, rows, chunk=chunk)
    return ori_oracle.sample_residual_rows(points, k, D, v, u0, rows, chunk=chunk)


def default_workers():
    """Host cores to use: the process's CPU affinity, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def sample_rows_parallel(points, k, D, v, rows, u0=None, workers=None, chunk=1 << 20):
    """(G0 (D v))_q for the listed rows q (u0 None), or the residual rows
    u0_q - v_q - (G0 (D v))_q of eq. 2.19 (u0 given), on ``workers`` forked
    processes.  Returns (values, workers used)."""
    rows = np.asarray(rows, dtype=np.int64)
    workers = default_workers() if workers is None else max(1, int(workers))
    workers = min(workers, max(1, len(rows)))
    if workers == 1 or len(rows) <= 1:
        _init((points, k, D, v, u0, chunk))
        try:
            return _work(rows), 1
        finally:
            _init(None)
    groups = [g for g in np.array_split(rows, workers) if len(g)]
    ctx = mp.get_context("fork")
    with ctx.Pool(len(groups), initializer=_init, initargs=((points, k, D, v, u0, chunk),)) as pool:
        parts = pool.map(_work, groups)
    return np.concatenate(parts), len(groups)
