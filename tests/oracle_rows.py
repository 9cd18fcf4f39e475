"""Sampled rows of eq. 2.19 from the oracle, for the GPU tests at sizes the
dense LU cannot reach.  Rows are spread over the grid's corners, edge
midpoints and face centres (where the Green's sums are most one-sided) and
random interior cells; the oracle evaluates them on several host cores."""

import numpy as np

import oracle as O


def boundary_rows(n, n_random=6, seed=0):
    """Flat indices of the 8 corners, 12 edge midpoints, 6 face centres and
    n_random random cells of an n^3 grid (p = (i1 n + i2) n + i3)."""
    lo, mid, hi = 0, n // 2, n - 1
    pts = set()
    for a in (lo, hi):
        for b in (lo, hi):
            for c in (lo, hi):
                pts.add((a, b, c))
    for a in (lo, hi):
        for b in (lo, hi):
            pts.update({(mid, a, b), (a, mid, b), (a, b, mid)})
    for a in (lo, hi):
        pts.update({(a, mid, mid), (mid, a, mid), (mid, mid, a)})
    rows = sorted((i1 * n + i2) * n + i3 for i1, i2, i3 in pts)
    rng = np.random.default_rng(seed)
    extra = rng.integers(0, n ** 3, n_random) if n_random else np.zeros(0, np.int64)
    return np.unique(np.concatenate([np.asarray(rows, np.int64), extra]))


def sampled_relative_residual(n, k, h, N, u, u0, rows, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5):
    """||(u0 - A u)[rows]|| / ||u0[rows]|| with A = I + G0 D of eq. 2.19
    (D from h and N), the rows evaluated by the oracle."""
    pts = O.cell_points(n, side, origin, offset)
    D = O.coupling(h, N, n, side)
    r, _ = O.sample_rows_parallel(pts, k, D, np.asarray(u), rows, u0=np.asarray(u0))
    return float(np.linalg.norm(r) / np.linalg.norm(np.asarray(u0)[rows]))
