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
