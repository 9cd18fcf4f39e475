"""The paper's own convolution route (Section 3), written out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

On the lattice x = d*(m1, m2, m3), m_i in [0, b) (eq. 3.3.5), the sum of
eq. 3.3.4 is the 3-D discrete convolution of eq. 3.3.7 with the table
g(m) = G(d*|m|), g(0) = 0 (the m != j exclusion).  Section 3 evaluates it
with the convolution theorem (eq. 3.3.8) after padding each axis in turn:
the Green's table is extended by mirroring (all entries except the first and
the last are appended in reverse order), the field is extended with zeros,
so both have 2b - 2 entries per axis; a cyclic convolution of the padded
arrays, cut back to the first b entries per axis, is the linear one.

This second route is pinned against the dense sum (``scatter_dense``) and
against the paper's 4x4 padding example.  ``numpy.fft`` is its only library
primitive.
"""

import math

import numpy as np


def mirror_pad_axis(g, axis):
    """Extend g along ``axis`` from b to 2b - 2 entries by mirroring.

    Entries 1 .. b-2 are appended in reverse order after the last one
    (Section 3, the 'For G' padding example).
    """
    g = np.asarray(g)
    b = g.shape[axis]
    if b <= 2:
        return g.copy()
    inner = np.take(g, np.arange(b - 2, 0, -1), axis=axis)
    return np.concatenate([g, inner], axis=axis)


def zero_pad_axis(u, axis, length):
    """Extend u along ``axis`` with zeros to ``length`` entries (the 'For u' example)."""
    u = np.asarray(u)
    pad = [(0, 0)] * u.ndim
    pad[axis] = (0, length - u.shape[axis])
    return np.pad(u, pad)


def green_table(b, d, k):
    """g[m1, m2, m3] = G(d*|m|) on [0, b)^3 with g[0, 0, 0] = 0 (eqs. 3.3.2, 3.3.7)."""
    m = np.indices((b, b, b)).astype(np.float64)
    r = d * np.sqrt(np.sum(m * m, axis=0))
    r[0, 0, 0] = 1.0
    g = np.exp(1j * k * r) / (4.0 * math.pi * r)
    g[0, 0, 0] = 0.0
    return g


def convolve_section3(g, u):
    """(G*u)(j) = sum_{m != j} g(j - m) u(m) on a b^3 cube, via eq. 3.3.8.

    Pads x, then y, then z (mirror for g, zeros for u), multiplies the FFTs,
    inverts and keeps the first b entries per axis.
    """
    u = np.asarray(u, dtype=np.complex128)
    b = u.shape[0]
    if b == 1:
        return np.zeros_like(u)
    gp = np.asarray(g, dtype=np.complex128)
    up = u
    for ax in range(3):
        gp = mirror_pad_axis(gp, ax)
        up = zero_pad_axis(up, ax, gp.shape[ax])
    y = np.fft.ifftn(np.fft.fftn(gp) * np.fft.fftn(up))
    return y[:b, :b, :b]


def scatter_section3(b, k, D, v, side=1.0):
    """y = G0 (D v) on the n = b lattice through the Section 3 route; flat in and out."""
    d = side / b
    Dv = (np.asarray(D, dtype=np.complex128) * np.asarray(v, dtype=np.complex128)).reshape(b, b, b)
    return convolve_section3(green_table(b, d, k), Dv).reshape(-1)
