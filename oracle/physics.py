"""Physics around the solve of eq. 2.19: what the paper does with u (oracle).

Test infrastructure only (see oracle/__init__.py).  Plain NumPy, complex128,
direct sums; every function cites the passage it follows.

* Refraction recipe (Section 2, eqs. 2.24-2.26; Section 4, eqs. 4.1-4.2):
  the refraction coefficient n of the medium created by the particles, and
  the boundary impedance h that creates a desired n.
* Charges (eq. 2.13 with the distribution law eqs. 2.17-2.18): the total
  Q over the particles of cell p is -c_S h_p N_p |Delta_p| u_p = -D_p u_p.
* Field (eq. 2.10 with the particles of each cell at x_p): the scattered
  field v(x) = sum_p G(x, x_p) Q_p, and its far-field amplitude A(beta)
  with v(r beta) ~ A(beta) e^{ikr} / r as r -> infinity (from eq. 2.6a:
  |r beta - y| = r - beta.y + O(1/r)).
* The solution difference of Section 4 (Table 4): solutions on a fine and a
  coarse grid compared by the mean over the fine points of each coarse cell.
"""

import numpy as np

from .ori_oracle import cell_points, coupling, green


def sqrt_branch_0_2pi(z):
    """z^{1/2} = |z|^{1/2} exp(i phi / 2) with phi = arg z taken in [0, 2 pi)
    (eq. 4.2: the branch with the cut [0, +inf))."""
    z = np.asarray(z, dtype=np.complex128)
    phi = np.angle(z)
    phi = np.where(phi < 0.0, phi + 2.0 * np.pi, phi)
    return np.sqrt(np.abs(z)) * np.exp(0.5j * phi)


def refraction_from_h(k, n0, h, N, c_S=4.0 * np.pi):
    """n = [n0^2 - k^-2 c_S h N]^{1/2} (eq. 4.1, i.e. eqs. 2.20a and 2.24),
    with the square root of eq. 4.2."""
    n0 = np.asarray(n0, dtype=np.complex128)
    p = c_S * np.asarray(N, dtype=np.float64) * np.asarray(h, dtype=np.complex128)  # eq. 2.20a
    return sqrt_branch_0_2pi(n0 * n0 - p / (k * k))                                # eq. 2.24


def h_for_refraction(k, n0, n, N, c_S=4.0 * np.pi):
    """h = p / (c_S N) with p = k^2 (n0^2 - n^2) (eqs. 2.25, 2.26)."""
    n0 = np.asarray(n0, dtype=np.complex128)
    n = np.asarray(n, dtype=np.complex128)
    p = k * k * (n0 * n0 - n * n)                                                  # eq. 2.25
    return p / (c_S * np.asarray(N, dtype=np.float64))                             # eq. 2.26


def cell_charges(h, N, n, u, side=1.0):
    """Q_p = -c_S h_p N_p |Delta_p| u_p = -D_p u_p: eq. 2.13 summed over the
    a^{-(2-kappa)} N_p |Delta_p| particles of cell p (eq. 2.18), each with
    the effective field u_p."""
    return -coupling(h, N, n, side) * np.asarray(u, dtype=np.complex128)


def particle_charge(h, u, a, kappa, c_S=4.0 * np.pi):
    """Q_m = -c_S a^{2-kappa} h(x_m) u_e(x_m) (eq. 2.13, leading order)."""
    return -c_S * a ** (2.0 - kappa) * np.asarray(h) * np.asarray(u)


def scattered_field(points, k, Q, x, block=256):
    """v(x) = sum_p G(x, x_p) Q_p (eq. 2.10, the sum term), for each row of
    x (shape (M, 3)); a source at distance exactly 0 is left out (the p != q
    of eq. 2.19 when x is a cell point)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    Q = np.asarray(Q, dtype=np.complex128)
    out = np.empty(x.shape[0], dtype=np.complex128)
    for s in range(0, x.shape[0], block):
        d = x[s:s + block, None, :] - points[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        zero = r == 0.0
        g = green(np.where(zero, 1.0, r), k)
        g[zero] = 0.0
        out[s:s + block] = g @ Q
    return out


def far_field(points, k, Q, beta):
    """A(beta) = (1 / 4 pi) sum_p exp(-i k beta . x_p) Q_p, so that
    v(r beta) = A(beta) e^{ikr} / r + O(1/r^2) (eq. 2.6a expanded for large
    r; unit vectors beta, rows of shape (M, 3))."""
    beta = np.atleast_2d(np.asarray(beta, dtype=np.float64))
    Q = np.asarray(Q, dtype=np.complex128)
    ph = np.exp(-1j * k * (beta @ points.T))
    return (ph @ Q) / (4.0 * np.pi)




def coarse_cell_of(n_fine, n_coarse, offset=0.5):
    """Coarse cell, along one axis, of each fine point: the fine point
    (i + offset) / n_fine (units of the side) lies in the coarse cell
    [q / n_coarse, (q + 1) / n_coarse) with q = floor((i + offset) n_coarse /
    n_fine)."""
    i = np.arange(n_fine, dtype=np.float64)
    return np.floor((i + offset) * n_coarse / n_fine).astype(np.int64)


def interpolation_difference(x_fine, n_fine, y_coarse, n_coarse, offset_fine=0.5):
    """Section 4, the procedure of Table 4: for each coarse cell Delta_q, the
    mean of |x_i - y_q| over the fine points x_i in Delta_q, and the sup of
    that mean over the cells that hold fine points."""
    q1 = coarse_cell_of(n_fine, n_coarse, offset_fine)
    x = np.asarray(x_fine, dtype=np.complex128).reshape(n_fine, n_fine, n_fine)
    y = np.asarray(y_coarse, dtype=np.complex128).reshape(n_coarse, n_coarse, n_coarse)
    yq = y[q1[:, None, None], q1[None, :, None], q1[None, None, :]]   # y of the cell of each fine point
    cell = (q1[:, None, None] * n_coarse + q1[None, :, None]) * n_coarse + q1[None, None, :]
    d = np.abs(x - yq).ravel()
    P = n_coarse ** 3
    sums = np.bincount(cell.ravel(), weights=d, minlength=P)
    counts = np.bincount(cell.ravel(), minlength=P)
    held = counts > 0
    return float(np.max(sums[held] / counts[held]))
