"""Same-method CPU baseline: the product of Section 3 on the host.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This module does not
define the result (the dense sums of ``ori_oracle`` do).  It runs the
paper's own method on the CPU: the Green's sum of eq. 3.3.4 as a cyclic
convolution evaluated with the convolution theorem (eq. 3.3.8), with
``scipy.fft`` on all host cores, and COCG on the symmetrised system.  Its
purpose is timing: ``bench.py`` sets a CPU running the same algorithm beside
the GPU, next to the dense-row oracle.  A CPU test pins it against the dense
sum and against LU.

Embedding: each axis is padded to L = 2n (the GPU path's length; the
paper's (2b - 2) mirror padding gives the same sums).  The Green's table holds
g(m) = G(d|m|) at the cyclic index m mod L for -(n-1) <= m_i <= n-1.  It is
zero at m = 0, which is the exclusion p != q of eq. 2.19.  It is also zero
at index n of any axis, which no pair of cells reaches (|j - m| <= n - 1).
The cyclic convolution of this table with the zero-padded field, cut back to
the first n entries per axis, is therefore the linear sum of eq. 3.3.7.
Every transform is a full 3-D FFT of L^3 points: no pruning of the zero
half, no octant of the spectrum.
"""

import math

import numpy as np
import scipy.fft

from . import ori_oracle
from .rows import default_workers


def green_spectrum(n, k, side=1.0, workers=None):
    """FFT of the (2n)^3 cyclic Green's table (eq. 3.3.8 applied to the
    table of eq. 3.3.7), complex128, shape (2n, 2n, 2n)."""
    L = 2 * n
    d = side / n
    i = np.arange(L)
    off = np.where(i < n, i, i - L).astype(np.float64)  # cyclic offset of index i
    sq = (d * off) ** 2
    g = np.empty((L, L, L), dtype=np.complex128)
    for a in range(L):
        r = np.sqrt(sq[a] + sq[:, None] + sq[None, :])
        if a == 0:
            r[0, 0] = 1.0  # overwritten with 0 below
        s = np.exp(1j * k * r) / (4.0 * math.pi * r)
        if a == 0:
            s[0, 0] = 0.0
        if a == n:
            s[:] = 0.0
        else:
            s[n, :] = 0.0
            s[:, n] = 0.0
        g[a] = s
    return scipy.fft.fftn(g, workers=workers or default_workers(), overwrite_x=True)


class GreenConvolution:
    """v -> G0 v on the n^3 cells (flat, p = (i1 n + i2) n + i3) through the
    (2n)^3 cyclic convolution; the spectrum is computed once."""

    def __init__(self, n, k, side=1.0, workers=None):
        self.n = n
        self.L = 2 * n
        self.workers = workers or default_workers()
        self.khat = green_spectrum(n, k, side, self.workers)
        self.buf = np.empty((self.L,) * 3, dtype=np.complex128)

    def __call__(self, v):
        n, L = self.n, self.L
        b = self.buf
        b.fill(0.0)
        b[:n, :n, :n] = np.asarray(v, dtype=np.complex128).reshape(n, n, n)
        f = scipy.fft.fftn(b, workers=self.workers, overwrite_x=True)
        f *= self.khat
        y = scipy.fft.ifftn(f, workers=self.workers, overwrite_x=True)
        return np.array(y[:n, :n, :n]).reshape(-1)


def scatter_fft(n, k, D, v, side=1.0, workers=None):
    """y = G0 (D v) through the cyclic convolution; flat in and out."""
    conv = GreenConvolution(n, k, side, workers)
    return conv(np.asarray(D, dtype=np.complex128) * np.asarray(v, dtype=np.complex128))


def solve_symmetrized_fft(n, k, D, u0, tol=1e-10, maxiter=1000, side=1.0, workers=None):
    """Solve (RED), eq. 2.19, by COCG on (I + S G0 S) w = S u0 with the
    convolution product, then u = u0 - G0 S w.  Returns (u, history)."""
    conv = GreenConvolution(n, k, side, workers)
    S = ori_oracle.symmetric_scale(D)
    w, hist = ori_oracle.cocg(lambda x: x + S * conv(S * x), S * u0, tol=tol, maxiter=maxiter)
    return u0 - conv(S * w), hist
