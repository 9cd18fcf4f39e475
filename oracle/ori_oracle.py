"""Dense CPU oracle for the reduced linear system (RED), eq. (2.19).

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU path never
imports this module.

What is computed (plain definitions, Section 2 of the paper):

* Cubes Delta_p of side ``side/n`` tile the cube [origin, origin + side]^3;
  the representative point x_p of Delta_p is ``origin + side*(i + offset)/n``
  with ``offset = 0.5`` (cube centres, the example choice next to eqs. 2.18
  and 2.19) or ``offset = 0`` (the lattice d*(m1, m2, m3) of eq. 3.3.5).
  The flat index is p = (i1*n + i2)*n + i3, i3 fastest.
* G(x, y) = exp(ik|x - y|) / (4 pi |x - y|)                     (eq. 2.6a)
* D_p = c_S h_p N_p |Delta_p|, with c_S = 4 pi for spheres (Section 2,
  after eq. 2.13; Section 4 uses spheres).
* (RED), eq. (2.19):  u_q + sum_{p != q} G(x_q, x_p) D_p u_p = u0_q,
  i.e. A u = u0 with A = I + G0 diag(D), where G0 is G with a zero diagonal
  (the sum excludes p = q).

Readings taken where the paper is silent:

* The self term p = q is excluded and nothing replaces it.
* The system is solved exactly as printed (minus sign in eq. 2.19).
* COCG itself is only cited by the paper; ``cocg`` below follows the
  published method of van der Vorst & Melissen (IEEE Trans. Magn. 26, 1990):
  CG with the unconjugated bilinear form x^T y for complex symmetric A.
* A = I + G0 D is complex symmetric only when D is constant; COCG is applied
  to the symmetrised system  (I + S G0 S) w = S u0,  S = sqrt(D) (any branch,
  S^2 = D), and u is recovered as  u = u0 - G0 S w.
"""

import math

import numpy as np

# c_S for spherical particles: |S_m| = c_S a^2 with c_S = 4 pi (Section 2, after eq. 2.13).
C_S = 4.0 * math.pi


# ---------------------------------------------------------------------------
# geometry and coefficients
# ---------------------------------------------------------------------------
def cell_points(n, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5):
    """Representative points x_p of the n^3 sub-cubes, shape (n^3, 3).

    Eqs. 2.18-2.19 (x_p a point of Delta_p, e.g. its centre) and eq. 3.3.5
    (lattice points d*m); p = (i1*n + i2)*n + i3.
    """
    i = np.indices((n, n, n)).reshape(3, -1).T.astype(np.float64)
    return np.asarray(origin, dtype=np.float64)[None, :] + side * (i + offset) / n


def cell_volume(n, side=1.0):
    """|Delta_p| = (side/n)^3 for the uniform partition (eq. 2.18)."""
    return (side / n) ** 3


def green(r, k):
    """Outgoing Helmholtz Green's function e^{ikr}/(4 pi r), eq. 2.6a / 3.3.2."""
    return np.exp(1j * k * r) / (4.0 * math.pi * r)


def coupling(h, N, n, side=1.0):
    """D_p = c_S h_p N_p |Delta_p|: the factor multiplying G_qp u_p in eq. 2.19."""
    h = np.asarray(h, dtype=np.complex128)
    N = np.ones(h.shape) if N is None else np.asarray(N, dtype=np.float64)
    return C_S * h * N * cell_volume(n, side)


def symmetric_scale(D):
    """S with S*S = D (principal complex square root).

    Any branch works: flipping the sign of S_p flips w_p = S_p u_p, and
    u = u0 - G0 S w is unchanged.
    """
    return np.sqrt(np.asarray(D, dtype=np.complex128))


# ---------------------------------------------------------------------------
# dense matrices (row blocks, NumPy)
# ---------------------------------------------------------------------------
def green_matrix(points, k, block=1024):
    """G0[q, p] = G(x_q, x_p) for p != q, 0 on the diagonal (eq. 2.19, p != q)."""
    P = points.shape[0]
    G0 = np.empty((P, P), dtype=np.complex128)
    for s in range(0, P, block):
        e = min(P, s + block)
        diff = points[s:e, None, :] - points[None, :, :]
        r = np.sqrt(np.sum(diff * diff, axis=2))
        rows = np.arange(s, e)
        r[rows - s, rows] = 1.0  # placeholder, overwritten below
        g = green(r, k)
        g[rows - s, rows] = 0.0
        G0[s:e] = g
    return G0


def system_matrix(points, k, D):
    """A = I + G0 diag(D): the matrix of (RED) written as A u = u0."""
    A = green_matrix(points, k) * np.asarray(D)[None, :]
    A[np.diag_indices_from(A)] += 1.0
    return A


def symmetric_system_matrix(points, k, S):
    """A_sym = I + S G0 S (complex symmetric), with S^2 = D."""
    S = np.asarray(S)
    A = S[:, None] * green_matrix(points, k) * S[None, :]
    A[np.diag_indices_from(A)] += 1.0
    return A


def solve_direct(A, rhs):
    """LU with partial pivoting (LAPACK zgesv via numpy.linalg.solve)."""
    return np.linalg.solve(A, rhs)


def scatter_dense(points, k, D, v, block=1024):
    """y = G0 (D v): the sum of eq. 2.19 for every q, by dense row blocks."""
    Dv = np.asarray(D) * np.asarray(v)
    P = points.shape[0]
    y = np.empty(P, dtype=np.complex128)
    for s in range(0, P, block):
        e = min(P, s + block)
        diff = points[s:e, None, :] - points[None, :, :]
        r = np.sqrt(np.sum(diff * diff, axis=2))
        rows = np.arange(s, e)
        r[rows - s, rows] = 1.0
        g = green(r, k)
        g[rows - s, rows] = 0.0
        y[s:e] = g @ Dv
    return y


def condition_number(A, method="svd"):
    """Condition number of the system matrix: the check that A is invertible.

    The paper's theory needs Im h <= 0, while its own experiment (Section 4)
    and the synthetic cases use Im h > 0, so invertibility is checked
    numerically rather than assumed.

    method="svd": the 2-norm condition number sigma_max / sigma_min from the
    singular values (LAPACK zgesdd via numpy.linalg.svd).
    method="gecon": LAPACK's estimate of the 1-norm condition number from an
    LU factorisation (zgetrf + zgecon), for sizes where an SVD is too slow.
    """
    A = np.asarray(A, dtype=np.complex128)
    if method == "svd":
        s = np.linalg.svd(A, compute_uv=False)
        return float(s[0] / s[-1])
    if method == "gecon":
        import scipy.linalg
        import scipy.linalg.lapack as lapack
        lu, _piv = scipy.linalg.lu_factor(A, check_finite=False)
        anorm = float(np.max(np.sum(np.abs(A), axis=0)))
        rcond, info = lapack.zgecon(lu, anorm, norm="1")
        if info != 0 or rcond <= 0.0:
            return math.inf
        return float(1.0 / rcond)
    raise ValueError(f"unknown method {method!r}")


def sample_scatter_rows(points, k, D, v, rows, chunk=1 << 20):
    """(G0 (D v))_q for the listed rows q, any size.

    Each row is a sum of P - 1 terms; terms are summed in chunks (NumPy's
    pairwise summation) and the chunk sums are added with math.fsum, so the
    result is accurate to a few ulps of the largest partial sum.
    """
    Dv = np.asarray(D, dtype=np.complex128) * np.asarray(v, dtype=np.complex128)
    P = points.shape[0]
    out = np.empty(len(rows), dtype=np.complex128)
    for t, q in enumerate(rows):
        q = int(q)
        re_parts, im_parts = [], []
        xq = points[q]
        for s in range(0, P, chunk):
            e = min(P, s + chunk)
            diff = points[s:e] - xq[None, :]
            r = np.sqrt(np.sum(diff * diff, axis=1))
            self_here = s <= q < e
            if self_here:
                r[q - s] = 1.0
            term = green(r, k) * Dv[s:e]
            if self_here:
                term[q - s] = 0.0
            re_parts.append(float(np.sum(term.real)))
            im_parts.append(float(np.sum(term.imag)))
        out[t] = complex(math.fsum(re_parts), math.fsum(im_parts))
    return out


def sample_residual_rows(points, k, D, u, u0, rows, chunk=1 << 20):
    """r_q = u0_q - u_q - (G0 D u)_q for the listed rows: the true residual of (RED)."""
    rows = np.asarray(rows, dtype=np.int64)
    s = sample_scatter_rows(points, k, D, u, rows, chunk=chunk)
    return np.asarray(u0)[rows] - np.asarray(u)[rows] - s


# ---------------------------------------------------------------------------
# brute force (pure Python, tiny n): pins the vectorised assembly and LAPACK
# ---------------------------------------------------------------------------
def brute_force_system(n, k, h, N, side=1.0, origin=(0.0, 0.0, 0.0), offset=0.5):
    """A as nested Python lists, term by term from eq. 2.19 (no NumPy)."""
    P = n * n * n
    pts = []
    for i1 in range(n):
        for i2 in range(n):
            for i3 in range(n):
                pts.append((origin[0] + side * (i1 + offset) / n,
                            origin[1] + side * (i2 + offset) / n,
                            origin[2] + side * (i3 + offset) / n))
    vol = (side / n) ** 3
    A = [[0j] * P for _ in range(P)]
    for q in range(P):
        for p in range(P):
            if p == q:
                A[q][p] = 1.0 + 0j
                continue
            dx = pts[q][0] - pts[p][0]
            dy = pts[q][1] - pts[p][1]
            dz = pts[q][2] - pts[p][2]
            r = math.sqrt(dx * dx + dy * dy + dz * dz)
            g = complex(math.cos(k * r), math.sin(k * r)) / (4.0 * math.pi * r)
            Np = 1.0 if N is None else float(N[p])
            A[q][p] = g * (4.0 * math.pi) * complex(h[p]) * Np * vol
    return A


def gauss_solve(A, b):
    """Gaussian elimination with partial pivoting on Python lists."""
    P = len(A)
    M = [list(row) + [complex(b[i])] for i, row in enumerate(A)]
    for c in range(P):
        piv = max(range(c, P), key=lambda i: abs(M[i][c]))
        M[c], M[piv] = M[piv], M[c]
        for i in range(c + 1, P):
            f = M[i][c] / M[c][c]
            if f != 0:
                for j in range(c, P + 1):
                    M[i][j] -= f * M[c][j]
    x = [0j] * P
    for i in range(P - 1, -1, -1):
        s = M[i][P]
        for j in range(i + 1, P):
            s -= M[i][j] * x[j]
        x[i] = s / M[i][i]
    return x


# ---------------------------------------------------------------------------
# COCG (van der Vorst & Melissen 1990; cited by the paper, Sections 1 and 3)
# ---------------------------------------------------------------------------
def cocg(apply_A, b, x0=None, tol=1e-10, maxiter=1000):
    """Conjugate Orthogonal Conjugate Gradient for complex symmetric A.

    CG with every inner product replaced by the unconjugated bilinear form
    x^T y.  Starts from x0 (default 0).  Stops when the recursively updated
    residual satisfies ||r||_2 / ||b||_2 < tol (the residual-based relative
    error of Section 4), or after ``maxiter`` iterations.

    Returns (x, history) with history[i] = ||r_i|| / ||b|| (history[0] is the
    initial residual).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    p = np.zeros_like(b)
    rho_old = None
    for it in range(maxiter):
        if hist[-1] < tol:
            break
        rho = np.sum(r * r)                 # r^T r, no conjugation
        beta = 0.0 if rho_old is None else rho / rho_old
        p = r + beta * p
        q = apply_A(p)
        mu = np.sum(p * q)                  # p^T A p, no conjugation
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        rho_old = rho
        hist.append(np.linalg.norm(r) / bnorm)
    return x, np.array(hist)


def solve_symmetrized_cocg(points, k, D, u0, tol=1e-10, maxiter=1000):
    """Solve (RED) by COCG on (I + S G0 S) w = S u0, then u = u0 - G0 S w.

    Dense operator; for small n only.  Returns (u, history).
    """
    S = symmetric_scale(D)
    G0 = green_matrix(points, k)

    def apply(w):
        return w + S * (G0 @ (S * w))

    w, hist = cocg(apply, S * u0, tol=tol, maxiter=maxiter)
    u = u0 - G0 @ (S * w)
    return u, hist


# ---------------------------------------------------------------------------
# adjoint gradient of J = sum |u - t|^2 with respect to h (material design)
# ---------------------------------------------------------------------------
def objective(u, t):
    """J = sum_j |u_j - t_j|^2."""
    e = np.asarray(u) - np.asarray(t)
    return float(np.sum(e.real ** 2 + e.imag ** 2))


def adjoint_gradient_dense(points, k, h, N, u0, t, n, side=1.0):
    """J and g with dJ = Re sum_p g_p dh_p, by the adjoint of eq. 2.19.

    A u = u0, A = I + G0 diag(c h), c_p = 4 pi N_p |Delta_p|.  Differentiating,
    A du = -G0 diag(c dh) u, so with A^T lam = conj(u - t) (A^T = I + D G0):
        dJ = 2 Re conj(u - t)^T du = Re sum_p g_p dh_p,
        g_p = -2 c_p u_p (G0 lam)_p.
    Hence dJ/dRe h_p = Re g_p and dJ/dIm h_p = -Im g_p.  Dense LU for both solves.
    """
    h = np.asarray(h, dtype=np.complex128)
    c = coupling(np.ones_like(h), N, n, side).real     # 4 pi N |Delta|
    D = c * h
    G0 = green_matrix(points, k)
    A = G0 * D[None, :]
    A[np.diag_indices_from(A)] += 1.0
    u = solve_direct(A, u0)
    e = u - np.asarray(t)
    lam = solve_direct(A.T, np.conj(e))
    g = -2.0 * c * u * (G0 @ lam)
    return objective(u, t), g, u
