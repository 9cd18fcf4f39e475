"""Seeded synthetic inputs for the solver and its oracle.

This module only draws inputs; it holds none of the solver's arithmetic.  It
is shared by the tests, the oracle-side checks and ``bench.py``.

Workload recipe (the paper's Section 4 experiment is a uniform particle
distribution in the unit cube, N = 1, spheres, a plane wave; the synthetic
cases keep that structure and add a +-10 % random boundary impedance):

* h_p = h0 * (1 + spread * xi_p), xi_p ~ U[-1, 1] drawn first, in p order,
  from ``numpy.random.default_rng(seed)``; default h0 = -1 + 0.5i.
* N_p = 1 (uniform distribution law, eq. 2.17 with N = 1).
* u0 = exp(i k alpha . x_p) at the cube centres (eq. 2.4), alpha a unit
  vector: given, or g / |g| with g = rng.standard_normal(3) drawn after xi.
* Fibonacci-sphere directions for multi-RHS cases:
  z_i = 1 - (2i + 1)/m, phi_i = i * pi * (3 - sqrt(5)).
"""

import math

import numpy as np


def random_direction(rng):
    g = rng.standard_normal(3)
    return g / np.linalg.norm(g)


def fibonacci_directions(m):
    i = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / m
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def centres(n, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5, dtype=np.float64):
    """Coordinates of the n^3 cube centres along each axis (i3 fastest)."""
    t = (np.arange(n, dtype=np.float64) + offset) * (side / n)
    return [origin[a] + t for a in range(3)]


def plane_wave(n, k, alpha, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5):
    """u0_p = exp(i k alpha . x_p), flat in p = (i1*n + i2)*n + i3."""
    x1, x2, x3 = centres(n, side, origin, offset)
    ph = (k * alpha[0] * x1)[:, None, None] + (k * alpha[1] * x2)[None, :, None] \
        + (k * alpha[2] * x3)[None, None, :]
    return np.exp(1j * ph).reshape(-1)


def make_case(n, k, seed, alpha=None, h0=-1.0 + 0.5j, spread=0.1, side=1.0,
              origin=(0.0, 0.0, 0.0), offset=0.5):
    """Return dict(h, N, u0, alpha, n, k, side, origin, offset) as NumPy arrays."""
    rng = np.random.default_rng(seed)
    P = n ** 3
    xi = rng.uniform(-1.0, 1.0, P)
    h = (h0 * (1.0 + spread * xi)).astype(np.complex128)
    if alpha is None:
        alpha = random_direction(rng)
    alpha = np.asarray(alpha, dtype=np.float64)
    N = np.ones(P, dtype=np.float64)
    u0 = plane_wave(n, k, alpha, side, origin, offset)
    return dict(h=h, N=N, u0=u0, alpha=alpha, n=n, k=k, side=side,
                origin=tuple(origin), offset=offset)


# Named workloads (n, k, seed, alpha): the unit cube, N = 1, h0 = -1 + 0.5i.
CASES = {
    # small parity case: dense LU finishes in seconds
    "n16_k1": dict(n=16, k=1.0, seed=0, alpha=(1.0, 0.0, 0.0)),
    # mixed-precision comparison
    "n128_k5": dict(n=128, k=5.0, seed=1, alpha=None),
    # headline measurement: 16.8 M unknowns, padded 512^3 FFT grid
    "n256_k5": dict(n=256, k=5.0, seed=5, alpha=None),
    # large single solve: padded 1024^3 grid
    "n512_k10": dict(n=512, k=10.0, seed=4, alpha=None),
}


def named_case(name):
    c = CASES[name]
    return make_case(c["n"], c["k"], c["seed"], alpha=c["alpha"])
