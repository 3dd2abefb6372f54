"""Exact solutions of the bound-constrained QP, independent of GPCG.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The QP  min 1/2 x'Ax - b'x, l <= x <= u  with A SPD has a unique solution x*
(Section 2 of the paper), characterised by the Kuhn-Tucker conditions: with
g = A x - b, g_i = 0 where l_i < x_i < u_i, g_i >= 0 where x_i = l_i and
g_i <= 0 where x_i = u_i.  Any method that finds a point satisfying them has
found x*.  Two such methods live here; neither shares code with the GPCG
oracle:

* ``brute_force``: enumerate the 3^n faces (Section 5 counts them) for
  n <= 8 and keep the face whose equality-constrained minimiser satisfies the
  conditions above.
* ``pdas``: the primal-dual active-set iteration with sparse direct solves of
  the face systems A_FF x_F = b_F - A_FA x_A (SciPy SuperLU), the standard
  semismooth-Newton method for this problem class.  Used to polish an
  approximate solution into x* to rounding accuracy.
"""
from __future__ import annotations

import itertools
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def csr_matrix(csr, n=None):
    rowptr, colind, vals = csr
    n = n or len(rowptr) - 1
    return sp.csr_matrix((np.asarray(vals, np.float64), np.asarray(colind),
                          np.asarray(rowptr)), shape=(n, n))


def kkt_residual(A, b, l, u, x):
    """Largest violation of the Kuhn-Tucker conditions at x (0 at x*).

    Components: infeasibility max(l - x, x - u, 0), |g_i| on free variables,
    max(-g_i, 0) at lower bounds, max(g_i, 0) at upper bounds (fixed variables
    impose nothing on g).
    """
    g = A @ x - b
    infeas = np.maximum(np.maximum(l - x, x - u), 0.0)
    at_l = x == l
    at_u = x == u
    free = ~(at_l | at_u)
    r = np.zeros_like(x)
    r[free] = np.abs(g[free])
    only_l = at_l & ~at_u
    only_u = at_u & ~at_l
    r[only_l] = np.maximum(-g[only_l], 0.0)
    r[only_u] = np.maximum(g[only_u], 0.0)
    return float(max(infeas.max(initial=0.0), r.max(initial=0.0)))


def brute_force(Adense, b, l, u, tol=1e-12):
    """Solve a tiny QP (n <= 8) by enumerating every face.

    Each variable is at its lower bound, at its upper bound or free (infinite
    bounds are never active).  For each face the free part solves
    A_FF x_F = b_F - A_FA x_A; the face is kept if x is feasible and the
    multipliers have the signs the Kuhn-Tucker conditions demand.
    """
    A = np.asarray(Adense, np.float64)
    n = len(b)
    assert n <= 8
    best = None
    for choice in itertools.product((0, 1, 2), repeat=n):
        ch = np.array(choice)
        if np.any((ch == 1) & ~np.isfinite(l)) or np.any((ch == 2) & ~np.isfinite(u)):
            continue
        x = np.zeros(n)
        x[ch == 1] = l[ch == 1]
        x[ch == 2] = u[ch == 2]
        F = ch == 0
        if F.any():
            rhs = b[F] - A[np.ix_(F, ~F)] @ x[~F]
            x[F] = np.linalg.solve(A[np.ix_(F, F)], rhs)
        if np.any(x < l - tol) or np.any(x > u + tol):
            continue
        g = A @ x - b
        scale = 1.0 + np.abs(b).max()
        lo_ok = np.all(g[ch == 1] >= -tol * scale) if (ch == 1).any() else True
        up_ok = np.all(g[ch == 2] <= tol * scale) if (ch == 2).any() else True
        if lo_ok and up_ok:
            x = np.minimum(np.maximum(x, l), u)
            if best is None:
                best = x
            else:
                # x* is unique: every valid face must give the same point
                assert np.allclose(best, x, rtol=0, atol=1e-9), (best, x)
    return best


def pdas(A, b, l, u, x_init: Optional[np.ndarray] = None, max_iter: int = 500,
         c=None):
    """Primal-dual active-set method with sparse direct face solves.

    With lambda = A x - b, the sets predicted for the next iterate are
    L = {lambda + c (l - x) > 0} and U = {lambda + c (u - x) < 0}; fixed
    variables are always in L.  x is set to l on L and u on U and the free
    part solves A_II x_I = b_I - A_I,LU x_LU.  Stops when the sets repeat.
    c defaults to the diagonal of A, which makes the set prediction invariant
    to the scale of A.  Returns (x, iterations, converged).
    """
    A = sp.csr_matrix(A)
    if c is None:
        c = A.diagonal()
    n = len(b)
    x = np.zeros(n) if x_init is None else np.minimum(np.maximum(x_init, l), u)
    x = np.where(np.isfinite(x), x, 0.0)
    lam = A @ x - b
    fixed = l == u
    prevL = prevU = None
    for it in range(1, max_iter + 1):
        with np.errstate(invalid="ignore"):
            Lset = fixed | (np.isfinite(l) & (lam + c * (l - x) > 0))
            Uset = ~Lset & np.isfinite(u) & (lam + c * (u - x) < 0)
        if prevL is not None and np.array_equal(Lset, prevL) and np.array_equal(Uset, prevU):
            return x, it, True
        prevL, prevU = Lset, Uset
        x = np.zeros(n)
        x[Lset] = l[Lset]
        x[Uset] = u[Uset]
        I = ~(Lset | Uset)
        if I.any():
            Aii = A[I][:, I].tocsc()
            rhs = b[I] - A[I][:, ~I] @ x[~I]
            x[I] = spla.spsolve(Aii, rhs)
        lam = A @ x - b
        lam[I] = 0.0
    return x, max_iter, False


def polish(csr, b, l, u, x_approx: Optional[np.ndarray] = None):
    """x* to rounding accuracy, starting PDAS from an approximate solution."""
    A = csr_matrix(csr, len(b))
    x, it, ok = pdas(A, b, l, u, x_approx)
    if not ok:
        x, it, ok = pdas(A, b, l, u, None, max_iter=2000)
    return x, dict(iterations=it, converged=ok, kkt=kkt_residual(A, b, l, u, x))


def degenerate_set(x_star, g_star, l, u, rel: float = 1e-10):
    """Variables whose active/free status is ill-determined at x*.

    Free variables within rel * max(1, ||x*||_inf) of a bound, and active
    variables whose gradient is within rel * ||g*||_inf of zero.  Outside this
    set the active sets of two accurate solutions must agree exactly.
    """
    scale = max(1.0, float(np.abs(x_star).max(initial=0.0)))
    gap = np.minimum(x_star - l, u - x_star)
    act = (x_star == l) | (x_star == u)
    near = (~act) & (gap <= rel * scale)
    gmax = float(np.abs(g_star).max(initial=0.0))
    weak = act & (np.abs(g_star) <= rel * max(gmax, 1e-300))
    return near | weak


# ----------------------------------------------------------------------------
# Exact face solves for the constant five-point operator on a square grid.
#
# A = w (T (x) I + I (x) T), T = tridiag(-1, 2, -1) of order N (Dirichlet data
# outside the grid), is diagonalised by the orthonormal type-I discrete sine
# transform S along each axis: A = S Lam S with Lam_pq = w (4 - 2 cos(p pi h)
# - 2 cos(q pi h)), h = 1 / (N + 1), p, q = 1..N.  Given a face -- the active
# indices and the bound values there -- x* solves x_A = v, (A x - b)_F = 0.
# With mu = (A x - b)_A (the multipliers, zero on F), A x = b + E mu, so
# x = A^{-1} (b + E mu) and the conditions on A give the capacitance system
#     C mu = v - E' A^{-1} b,   C = E' A^{-1} E  (m x m, SPD).
# C_ab = sum_pq S_{i_a p} S_{j_a q} S_{i_b p} S_{j_b q} / Lam_pq.

def _dst_eigs(N: int, w: float):
    k = np.arange(1, N + 1)
    lam1 = 2.0 - 2.0 * np.cos(k * np.pi / (N + 1))
    return w * (lam1[:, None] + lam1[None, :])


def poisson_solve(N: int, w: float, rhs):
    """A^{-1} rhs for the constant five-point operator on an N x N grid (rows of
    N unknowns, index j N + i), by the orthonormal DST-I."""
    import scipy.fft
    R = np.asarray(rhs, np.float64).reshape(N, N)
    Y = scipy.fft.dstn(R, type=1, norm="ortho", workers=-1) / _dst_eigs(N, w)
    return scipy.fft.idstn(Y, type=1, norm="ortho", workers=-1).ravel()


def _green_block(N: int, w: float, idx):
    """C = E' A^{-1} E for the grid indices idx (m x m), from the closed-form
    eigenvectors S_{i p} = sqrt(2 h) sin(i' p pi h) (i' = i + 1)."""
    idx = np.asarray(idx, np.int64)
    m = len(idx)
    h = 1.0 / (N + 1)
    p = np.arange(1, N + 1)
    i, j = idx % N, idx // N
    si = np.sqrt(2 * h) * np.sin(np.outer(i + 1, p) * np.pi * h)  # m x N (column index)
    sj = np.sqrt(2 * h) * np.sin(np.outer(j + 1, p) * np.pi * h)  # m x N (row index)
    inv = 1.0 / _dst_eigs(N, w)                                   # [q (row), p (col)]
    C = np.empty((m, m))
    step = max(1, (1 << 27) // (N * N))  # rows of U per block: about 1 GB
    for a0 in range(0, m, step):
        a1 = min(m, a0 + step)
        U = (sj[a0:a1, :, None] * si[a0:a1, None, :]).reshape(a1 - a0, N * N)
        V = U * inv.ravel()[None, :]
        for b0 in range(0, m, step):
            b1 = min(m, b0 + step)
            W = (sj[b0:b1, :, None] * si[b0:b1, None, :]).reshape(b1 - b0, N * N)
            C[a0:a1, b0:b1] = V @ W.T
    return 0.5 * (C + C.T)


def face_solve_const(N: int, w: float, b, active_idx, active_val, refine: int = 2):
    """x with x_A = active_val and (A x - b)_F = 0 for the constant five-point
    operator (capacitance system above, then `refine` rounds of iterative
    refinement on the free residual).  Returns (x, mu)."""
    b = np.asarray(b, np.float64)
    idx = np.asarray(active_idx, np.int64)
    v = np.asarray(active_val, np.float64)
    if len(idx) == 0:
        return poisson_solve(N, w, b), np.zeros(0)
    C = _green_block(N, w, idx)
    Lc = np.linalg.cholesky(C)
    csolve = lambda r: np.linalg.solve(Lc.T, np.linalg.solve(Lc, r))

    def solve(rhs, vals):
        y = poisson_solve(N, w, rhs)
        mu = csolve(vals - y[idx])
        e = np.zeros_like(rhs)
        e[idx] = mu
        return poisson_solve(N, w, rhs + e), mu

    x, mu = solve(b, v)
    x[idx] = v
    A = stencil_const_csr(N, w)
    for _ in range(refine):
        r = b - A @ x
        r[idx] = 0.0
        dx, dmu = solve(r, np.zeros_like(v))
        dx[idx] = 0.0
        x += dx
        mu += dmu
    return x, mu


def stencil_const_csr(N: int, w: float):
    """The constant five-point operator as a SciPy CSR matrix."""
    T = sp.diags([-np.ones(N - 1), 2.0 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.identity(N)
    return (w * (sp.kron(I, T) + sp.kron(T, I))).tocsr()


def xstar_from_face(N: int, w: float, b, l, u, lower_idx, upper_idx):
    """x* of the QP with the constant five-point operator from a face
    certificate (lower- and upper-active indices), verified: the result is
    returned only if it satisfies the Kuhn-Tucker conditions -- then it is the
    unique solution whatever produced the certificate.  Returns (x, g, kkt)."""
    lower_idx = np.asarray(lower_idx, np.int64)
    upper_idx = np.asarray(upper_idx, np.int64)
    idx = np.concatenate([lower_idx, upper_idx])
    val = np.concatenate([np.asarray(l)[lower_idx], np.asarray(u)[upper_idx]])
    x, mu = face_solve_const(N, w, b, idx, val)
    x = np.minimum(np.maximum(x, l), u)
    A = stencil_const_csr(N, w)
    g = A @ x - b
    kkt = kkt_residual(A, b, l, u, x)
    # rounding level of a residual entry: |b| + 8 w |x|, times a few ulps
    scale = float(np.abs(b).max() + 8.0 * w * np.abs(x).max())
    if not kkt <= 64 * np.finfo(float).eps * scale:
        raise ValueError(f"face certificate does not give x*: KKT residual {kkt:.3e} "
                         f"(rounding level {np.finfo(float).eps * scale:.3e})")
    return x, g, kkt


def pdas_const(N: int, w: float, b, l, u, x_init, max_iter: int = 50):
    """The primal-dual active-set iteration of ``pdas`` with the face systems
    of the constant five-point operator solved by ``face_solve_const`` (for
    starts near x*, whose active sets are small).  Returns (x, iterations,
    converged)."""
    A = stencil_const_csr(N, w)
    c = A.diagonal()
    x = np.minimum(np.maximum(np.asarray(x_init, np.float64), l), u)
    lam = A @ x - b
    fixed = l == u
    prevL = prevU = None
    for it in range(1, max_iter + 1):
        with np.errstate(invalid="ignore"):
            Lset = fixed | (np.isfinite(l) & (lam + c * (l - x) > 0))
            Uset = ~Lset & np.isfinite(u) & (lam + c * (u - x) < 0)
        if prevL is not None and np.array_equal(Lset, prevL) and np.array_equal(Uset, prevU):
            return x, it, True
        prevL, prevU = Lset, Uset
        lo, up = np.flatnonzero(Lset), np.flatnonzero(Uset)
        x, _ = face_solve_const(N, w, b, np.concatenate([lo, up]),
                                np.concatenate([l[lo], u[up]]))
        lam = A @ x - b
        lam[~(Lset | Uset)] = 0.0
    return x, max_iter, False


def read_face(path):
    """(N, lower indices, upper indices) from a face certificate file: lines
    'N <int>', 'lower <count>' then the indices, 'upper <count>' then the
    indices; '#' starts a comment."""
    toks = []
    with open(path) as f:
        for line in f:
            toks += line.split("#", 1)[0].split()
    it = iter(toks)
    out = {}
    for key in it:
        cnt = int(next(it))
        out[key] = cnt if key == "N" else np.array([int(next(it)) for _ in range(cnt)], np.int64)
    return out["N"], out["lower"], out["upper"]
