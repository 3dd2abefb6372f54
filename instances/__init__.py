"""Seeded synthetic GPCG problem instances.

This module only *generates inputs*: grids, operator coefficients, the
right-hand side b, the bounds l and u and the start x0.  It holds none of the
arithmetic of the method itself, and it is the one module that both the CPU
oracle (``oracle/``) and the HIP library (``paper_cs_0101018_amd``) are fed
from.

Problem form (the bound-constrained QP of Section 2 of the paper):

    minimise  q(x) = 1/2 x^T A x - b^T x     subject to  l <= x <= u

(the paper writes ``+ b^T x``; here the gradient is ``g = A x - b``).

Grid convention: an N x N interior grid with h = 1/(N+1), s_i = i h and
t_j = j h for i, j = 1..N, unknown index k = (j-1) N + (i-1) (s fastest),
homogeneous Dirichlet data outside the grid.

Operators are five-point stencils given by *edge weights*:

* ``wx`` has shape (N, N+1): ``wx[j, e]`` is the weight of the edge between
  grid columns e-1 and e of row j (0-based; columns -1 and N are the boundary).
* ``wy`` has shape (N+1, N): ``wy[e, i]`` is the weight of the edge between
  grid rows e-1 and e at column i.

      (A x)_k = sum over the 4 edges e of k of  w_e (x_k - x_nb(e)),
      x_nb = 0 outside the grid.

The constant-coefficient Laplacian is the special case w_e = 1/h^2, and the
variable-coefficient operator -div(c grad) puts c at edge midpoints, weight
c/h^2 (Section 5 of the paper describes the journal-bearing weight
(1 + eps cos xi_1)^3 that the variable-coefficient instances mimic).

Every random draw uses numpy's PCG64 ``default_rng``; the order of the draws
is part of each generator's definition.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

OP_CONST = "const"
OP_VAR = "var"


@dataclasses.dataclass
class Instance:
    """One bound-constrained QP on an N x N grid (or a small dense one)."""

    name: str
    N: int                       # grid side (0 for a dense/CSR-only instance)
    op: str                      # OP_CONST | OP_VAR | "csr"
    b: np.ndarray
    l: np.ndarray
    u: np.ndarray
    x0: np.ndarray
    w: float = 0.0               # OP_CONST: the single edge weight 1/h^2
    wx: Optional[np.ndarray] = None   # OP_VAR: (N, N+1)
    wy: Optional[np.ndarray] = None   # OP_VAR: (N+1, N)
    dense: Optional[np.ndarray] = None  # "csr" instances: the matrix itself
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.b.shape[0])

    # -- operator representations (input formats, not solver arithmetic) --
    def edge_weights(self):
        """(wx, wy) as full arrays, also for the constant operator."""
        if self.op == OP_CONST:
            N = self.N
            return (np.full((N, N + 1), self.w), np.full((N + 1, N), self.w))
        if self.op == OP_VAR:
            return self.wx, self.wy
        raise ValueError("instance has no stencil form")

    def csr(self):
        """The operator as CSR (rowptr int32, colind int32, vals float64).

        Columns are sorted ascending inside each row.
        """
        if self.dense is not None:
            return dense_to_csr(self.dense)
        wx, wy = self.edge_weights()
        return stencil_csr(self.N, wx, wy)


def dense_to_csr(D: np.ndarray):
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(D[i])[0]
        cols.append(nz.astype(np.int32))
        vals.append(D[i, nz])
        rowptr[i + 1] = rowptr[i] + len(nz)
    return rowptr, np.concatenate(cols), np.concatenate(vals)


def stencil_csr(N: int, wx: np.ndarray, wy: np.ndarray, rows=None):
    """Assemble the five-point edge-weight operator as CSR (sorted columns).

    Row k = j*N + i: diagonal wx[j,i] + wx[j,i+1] + wy[j,i] + wy[j+1,i];
    off-diagonals -wy[j,i] (row below), -wx[j,i] (left), -wx[j,i+1] (right),
    -wy[j+1,i] (row above), dropped where the neighbour is outside the grid.
    rows: None (every row) or sorted distinct row indices; the other rows of
    the n x n result are left empty (a sample of the operator's rows).
    """
    n = N * N
    k = np.arange(n, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    jj, ii = np.divmod(k, N)
    diag = wx[jj, ii] + wx[jj, ii + 1] + wy[jj, ii] + wy[jj + 1, ii]
    # candidate entries in sorted-column order: S, W, C, E, N
    cand_col = np.stack([
        (jj - 1) * N + ii, jj * N + ii - 1, jj * N + ii, jj * N + ii + 1,
        (jj + 1) * N + ii], axis=1)
    cand_val = np.stack([
        -wy[jj, ii], -wx[jj, ii], diag, -wx[jj, ii + 1], -wy[jj + 1, ii]], axis=1)
    valid = np.stack([jj > 0, ii > 0, np.ones(len(k), bool), ii < N - 1, jj < N - 1], axis=1)
    counts = np.zeros(n, dtype=np.int64)
    counts[k] = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cand_col[valid].astype(np.int32)
    vals = cand_val[valid].astype(np.float64)
    return rowptr.astype(np.int32), colind, vals


def grid_coords(N: int):
    """(s, t) of every unknown in index order k = (j-1) N + (i-1)."""
    h = 1.0 / (N + 1)
    idx = np.arange(1, N + 1, dtype=np.float64) * h
    t, s = np.meshgrid(idx, idx, indexing="ij")
    return s.ravel(), t.ravel(), h


def journal_weight(s, eps: float = 0.1):
    """c(s) = (1 + eps cos 2 pi s)^3, the journal-bearing-like coefficient."""
    return (1.0 + eps * np.cos(2.0 * np.pi * s)) ** 3


def varcoef_weights(N: int, eps: float = 0.1):
    """Edge weights of -div(c grad) with c(s) at edge midpoints, divided by h^2.

    x-edge e of any row sits at s = (e + 1/2) h (e = 0..N); a y-edge at column
    i sits at s = s_i, because c does not depend on t.
    """
    h = 1.0 / (N + 1)
    s_edge = (np.arange(N + 1, dtype=np.float64) + 0.5) * h
    s_col = np.arange(1, N + 1, dtype=np.float64) * h
    wx = np.broadcast_to(journal_weight(s_edge, eps) / h**2, (N, N + 1)).copy()
    wy = np.broadcast_to(journal_weight(s_col, eps) / h**2, (N + 1, N)).copy()
    return wx, wy


# ------------------------------------------------------- benchmark workloads

def _obstacle_lower(N, rng, amplitude=0.3):
    s, t, _ = grid_coords(N)
    z = rng.standard_normal(N * N)
    return amplitude * np.sin(np.pi * s) * np.sin(2.0 * np.pi * t) - 0.2 + 0.01 * z


def obstacle(N: int, seed: int = 0, *, amplitude: float = 0.3, u_random: bool = False,
             load: float = 1.0, name: Optional[str] = None) -> Instance:
    """Obstacle-type QP: constant 5-point Laplacian / h^2, b = load (1 by default).

    Draws, in order: z ~ N(0,1) for l (n values); then, if ``u_random``,
    w ~ U(0,1) for u = 0.25 + 0.05 w (n values).  Otherwise u = 0.25.
    Where the obstacle rises above u (large amplitudes) u is raised to l, which
    makes those variables fixed.  x0 = max(l, 0) clipped to u.
    """
    rng = np.random.default_rng(seed)
    n = N * N
    h = 1.0 / (N + 1)
    l = _obstacle_lower(N, rng, amplitude)
    if u_random:
        u = 0.25 + 0.05 * rng.uniform(0.0, 1.0, n)
    else:
        u = np.full(n, 0.25)
    u = np.maximum(u, l)
    x0 = np.minimum(np.maximum(l, 0.0), u)
    return Instance(name or f"obstacle{N}", N, OP_CONST, b=np.full(n, float(load)), l=l, u=u,
                    x0=x0, w=1.0 / h**2, meta=dict(seed=seed, amplitude=amplitude,
                                                   u_random=u_random, load=load))


def pressed(N: int, seed: int = 0, load: float = -10000.0) -> Instance:
    """An obstacle QP pressed onto its obstacle (b = load < 0, amplitude 0.3),
    the case of a small free set: at the solution 23 % of the unknowns are
    free for N = 512 and the default load, 25 % for N = 256 and load -2500."""
    return obstacle(N, seed, amplitude=0.3, load=load, name=f"pressed{N}")


def varcoef(N: int, seed: int = 0, *, eps: float = 0.1, name: Optional[str] = None) -> Instance:
    """Variable-coefficient QP: A = -div(c grad), c = (1 + eps cos 2 pi s)^3.

    b = 0.1 sin(2 pi s) + 0.01 v with v ~ U(-1,1) (n values, the only draw);
    l = 0, u = +inf, x0 = 0.
    """
    rng = np.random.default_rng(seed)
    n = N * N
    s, _, _ = grid_coords(N)
    b = 0.1 * np.sin(2.0 * np.pi * s) + 0.01 * rng.uniform(-1.0, 1.0, n)
    wx, wy = varcoef_weights(N, eps)
    return Instance(name or f"varcoef{N}", N, OP_VAR, b=b, l=np.zeros(n),
                    u=np.full(n, np.inf), x0=np.zeros(n), wx=wx, wy=wy,
                    meta=dict(seed=seed, eps=eps))


def obstacle50(seed: int = 0) -> Instance:
    """Plain FP64 obstacle QP on a 50 x 50 grid (n = 2,500)."""
    return obstacle(50, seed, name="obstacle50")


def varcoef256(seed: int = 0) -> Instance:
    """Plain FP64 variable-coefficient QP on a 256 x 256 grid (n = 65,536)."""
    return varcoef(256, seed, name="varcoef256")


def obstacle_ub(N: int = 1024, seed: int = 0) -> Instance:
    """Obstacle QP at scale (N = 1024 or 1600) with a random upper bound."""
    return obstacle(N, seed, u_random=True, name=f"obstacle{N}_ub")


def _mixed_member(ss: np.random.SeedSequence, nmin: int, nmax: int, idx: int) -> Instance:
    """One member of the mixed batches: N, operator, amplitude, then fields."""
    rng = np.random.default_rng(ss)
    N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    use_var = bool(rng.uniform() < 0.5)
    a = float(rng.uniform(0.1, 0.5))
    n = N * N
    h = 1.0 / (N + 1)
    if use_var:
        s, _, _ = grid_coords(N)
        b = 0.1 * np.sin(2.0 * np.pi * s) + 0.01 * rng.uniform(-1.0, 1.0, n)
        wx, wy = varcoef_weights(N)
        inst = Instance(f"m{idx}_varcoef{N}", N, OP_VAR, b=b, l=np.zeros(n),
                        u=np.full(n, np.inf), x0=np.zeros(n), wx=wx, wy=wy)
    else:
        l = _obstacle_lower(N, rng, a)
        u = np.maximum(np.full(n, 0.25), l)
        x0 = np.minimum(np.maximum(l, 0.0), u)
        inst = Instance(f"m{idx}_obstacle{N}", N, OP_CONST, b=np.ones(n), l=l, u=u,
                        x0=x0, w=1.0 / h**2)
    inst.meta = dict(index=idx, amplitude=a, varcoef=use_var)
    return inst


def batch512(seed: int = 0, count: int = 512, nmin: int = 32, nmax: int = 384):
    """512 independent QPs of uneven size (sides log-uniform in [32, 384])."""
    children = np.random.SeedSequence(seed).spawn(count)
    return [_mixed_member(c, nmin, nmax, i) for i, c in enumerate(children)]


def batch_member(seed: int, index: int, count: int = 512, nmin: int = 32,
                 nmax: int = 384) -> Instance:
    """Member ``index`` of ``batch512(seed, count, nmin, nmax)`` alone."""
    children = np.random.SeedSequence(seed).spawn(count)
    return _mixed_member(children[index], nmin, nmax, index)


def serve_trace(seed: int = 0, count: int = 4096, rate_hz: float = 200.0):
    """Poisson arrival times (seconds) for the serving workload."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    return np.cumsum(rng.exponential(1.0 / rate_hz, count))


def serve_request(seed: int, index: int, count: int = 4096,
                    nmin: int = 32, nmax: int = 512) -> Instance:
    """Request ``index`` of the serving workload (sides log-uniform in [32, 512])."""
    children = np.random.SeedSequence(seed).spawn(count)
    return _mixed_member(children[index], nmin, nmax, index)


# ------------------------------------------------------- small test instances

def tiny_dense(n: int, seed: int = 0, *, kinds=("box", "lower", "upper", "free", "fixed"),
               scale: float = 1.0) -> Instance:
    """A random dense SPD QP with n <= 8 and mixed bound types.

    Draws, in order: Q (n x n normal), b (n normal), the bound kind of each
    variable, two uniform values per variable for the bounds, x0 (n normal).
    """
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    A = Q.T @ Q + 0.5 * np.eye(n)
    b = scale * rng.standard_normal(n) * 2.0
    kind_idx = rng.integers(0, len(kinds), n)
    r = rng.uniform(-1.0, 1.0, (n, 2))
    l = np.full(n, -np.inf)
    u = np.full(n, np.inf)
    for i in range(n):
        k = kinds[kind_idx[i]]
        lo, hi = min(r[i]), max(r[i])
        if k == "box":
            l[i], u[i] = lo, hi
        elif k == "lower":
            l[i] = lo
        elif k == "upper":
            u[i] = hi
        elif k == "fixed":
            l[i] = u[i] = lo
    x0 = rng.standard_normal(n)
    return Instance(f"tiny{n}_{seed}", 0, "csr", b=b, l=l, u=u, x0=x0, dense=A,
                    meta=dict(seed=seed, kinds=[kinds[k] for k in kind_idx]))


def diagonal(n: int, seed: int = 0) -> Instance:
    """Diagonal SPD A with finite and infinite bounds (closed-form solution)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 4.0, n)
    b = rng.standard_normal(n)
    lo = rng.uniform(-0.6, 0.0, n)
    hi = rng.uniform(0.0, 0.6, n)
    which = rng.integers(0, 4, n)
    l = np.where((which == 0) | (which == 1), lo, -np.inf)
    u = np.where((which == 0) | (which == 2), hi, np.inf)
    x0 = np.zeros(n)
    return Instance(f"diag{n}_{seed}", 0, "csr", b=b, l=l, u=u, x0=x0, dense=np.diag(d),
                    meta=dict(seed=seed))


def unconstrained(N: int, op: str = OP_CONST, seed: int = 0) -> Instance:
    """l = -inf, u = +inf on a stencil operator (solution A^-1 b)."""
    rng = np.random.default_rng(seed)
    n = N * N
    s, t, h = grid_coords(N)
    b = np.sin(np.pi * s) * np.sin(np.pi * t) + 0.1 * rng.standard_normal(n)
    inst = Instance(f"free{N}_{op}", N, op, b=b, l=np.full(n, -np.inf),
                    u=np.full(n, np.inf), x0=np.zeros(n), w=1.0 / h**2)
    if op == OP_VAR:
        inst.wx, inst.wy = varcoef_weights(N)
    return inst


def manufactured(N: int, op: str = OP_CONST, seed: int = 0, *, frac_lower: float = 0.25,
                 frac_upper: float = 0.2) -> Instance:
    """A QP whose solution x* and active sets are known by construction.

    Draws, in order: the status of each variable (lower / upper / free), l, the
    gap u - l, the position of x* inside (l, u) for free variables, and the
    multiplier magnitudes.  x* sits on l (lower), on u (upper) or strictly
    inside; the gradient at x* is lambda with lambda > 0 on the lower set,
    lambda < 0 on the upper set and 0 on the free set, so b = A x* - lambda.
    The known answer is returned in ``meta`` (x_star, status).
    """
    rng = np.random.default_rng(seed)
    n = N * N
    h = 1.0 / (N + 1)
    r = rng.uniform(0.0, 1.0, n)
    status = np.where(r < frac_lower, 1, np.where(r < frac_lower + frac_upper, 2, 0))
    l = rng.uniform(-1.0, 0.0, n)
    gap = rng.uniform(0.2, 1.0, n)
    u = l + gap
    pos = rng.uniform(0.1, 0.9, n)
    lam_mag = rng.uniform(0.5, 2.0, n) * (1.0 / h**2) * 0.01
    x_star = np.where(status == 1, l, np.where(status == 2, u, l + pos * gap))
    lam = np.where(status == 1, lam_mag, np.where(status == 2, -lam_mag, 0.0))
    inst = Instance(f"manuf{N}_{op}", N, op, b=np.zeros(n), l=l, u=u, x0=l.copy(),
                    w=1.0 / h**2)
    if op == OP_VAR:
        inst.wx, inst.wy = varcoef_weights(N)
    import scipy.sparse as sp
    rowptr, colind, vals = inst.csr()
    A = sp.csr_matrix((vals, colind, rowptr), shape=(n, n))
    inst.b = A @ x_star - lam
    inst.meta = dict(seed=seed, x_star=x_star, status=status)
    return inst
