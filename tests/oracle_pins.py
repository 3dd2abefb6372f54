"""Pins of the GPCG oracle against facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with something that does not depend on the oracle:
closed forms, brute-force enumeration, an independent exact solver, textbook
CG written here from its definition, exact rational arithmetic, hand-derived
cases of the paper's definitions.  ``test_oracle_pins.py`` runs them against
the oracle; ``test_oracle_mutants.py`` runs them against builds of the oracle
with planted mistakes and requires every mistake to be caught.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import instances
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

TIGHT = dict(tol_rel=1e-13, max_outer=500)


def _load_cases():
    rows = []
    with open(os.path.join(GOLDEN, "proj_gradient_cases.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def _q(A, b, x):
    return 0.5 * x @ (A @ x) - b @ x


# ---------------------------------------------------------------- definitions

def pin_projection_is_median(o):
    """P[v] = mid(l, u, v), the componentwise median (Section 3)."""
    rng = np.random.default_rng(11)
    n = 4000
    a, c = rng.standard_normal(n), rng.standard_normal(n)
    l, u = np.minimum(a, c), np.maximum(a, c)
    l[:300] = -np.inf
    u[300:600] = np.inf
    u[600:700] = l[600:700]
    v = 2.0 * rng.standard_normal(n)
    v[700:800] = l[700:800]
    got = o.project(l, u, v)
    want = np.median(np.stack([l, u, v]), axis=0)
    assert np.array_equal(got, want)


def pin_projected_gradient_cases(o):
    """Hand cases of eq. (proj-gradient) and the binding set (Section 2)."""
    T = _load_cases()
    x, l, u, g, pg, act, bind = T.T
    got = o.proj_gradient(x, l, u, g)
    assert np.array_equal(got, pg), (got, pg)
    for k in range(len(x)):
        lo, up, nb = o.classify(x[k:k + 1], l[k:k + 1], u[k:k + 1], g[k:k + 1])
        assert lo + up == int(act[k]), k
        assert nb == int(act[k] and not bind[k]), k
    assert np.isclose(o.proj_gradient_norm(x, l, u, g), np.sqrt(np.sum(pg * pg)), rtol=1e-15)


def pin_gradient_matches_sparse_library(o):
    """g = A x - b against SciPy's CSR product."""
    inst = instances.varcoef256(seed=3)
    csr = inst.csr()
    A = exact.csr_matrix(csr)
    x = np.random.default_rng(2).standard_normal(inst.n)
    g = o.gradient(csr, x, inst.b)
    ref = A @ x - inst.b
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


# ------------------------------------------------------------- single steps

def pin_alpha0_minimises_along_projected_gradient(o):
    """alpha_0 of eq. (bqpls) is the minimiser of q(y - alpha P grad q(y))."""
    inst = instances.obstacle50(seed=5)
    csr = inst.csr()
    A = exact.csr_matrix(csr)
    y = inst.x0
    g = A @ y - inst.b
    dd, dAd = o.gp_alpha0(csr, y, inst.l, inst.u, g)
    a0 = dd / dAd
    d = o.proj_gradient(y, inst.l, inst.u, g)
    f = lambda a: _q(A, inst.b, y - a * d)
    assert a0 > 0
    for fac in (0.999, 1.001, 0.9, 1.1):
        assert f(a0) < f(fac * a0)


def pin_decrease_identity_exact(o):
    """q(y') - q(y) = g's + 1/2 s'As, checked in exact rational arithmetic."""
    inst = instances.tiny_dense(6, seed=21)
    A = inst.dense
    csr = inst.csr()
    y = np.clip(np.zeros(6), inst.l, inst.u)
    g = A @ y - inst.b
    ynew, gs, sAs, nchg = o.trial(csr, y, -g, 0.37, inst.l, inst.u, g)
    delta = o.decrease(gs, sAs)
    F = lambda v: [Fraction(float(t)) for t in v]
    Af = [[Fraction(float(t)) for t in row] for row in A]
    bf = F(inst.b)

    def qf(v):
        vf = F(v)
        Av = [sum(Af[i][j] * vf[j] for j in range(6)) for i in range(6)]
        return Fraction(1, 2) * sum(vf[i] * Av[i] for i in range(6)) - sum(bf[i] * vf[i] for i in range(6))

    exact_delta = float(qf(ynew) - qf(y))
    assert abs(delta - exact_delta) <= 1e-12 * (abs(exact_delta) + abs(gs))
    # the trial point is the projection of y - alpha g
    assert np.array_equal(ynew, np.median(np.stack([inst.l, inst.u, y - 0.37 * g]), axis=0))
    act_old = (y == inst.l) | (y == inst.u)
    act_new = (ynew == inst.l) | (ynew == inst.u)
    assert nchg == int(np.sum(act_old != act_new))


def _textbook_cg(A, rhs, iters):
    """Hestenes-Stiefel CG for A w = rhs from w = 0, written from the textbook."""
    w = np.zeros_like(rhs)
    r = rhs.copy()
    p = r.copy()
    out = []
    for _ in range(iters):
        Ap = A @ p
        a = (r @ r) / (p @ Ap)
        w = w + a * p
        r_new = r - a * Ap
        out.append(w.copy())
        if r_new @ r_new == 0:
            break
        p = r_new + (r_new @ r_new) / (r @ r) * p
        r = r_new
    return out


def pin_reduced_cg_is_textbook_cg(o):
    """Unconstrained face, eta -> 0: the iterates are textbook CG on A w = -g,
    the CG decreases equal q_k(w_{j-1}) - q_k(w_j), and m steps solve it."""
    inst = instances.tiny_dense(8, seed=4)
    A = inst.dense
    csr = inst.csr()
    g = np.random.default_rng(9).standard_normal(8)
    mask = np.ones(8, np.uint8)
    st, d, it, decs = o.reduced_cg(csr, mask, g, 1e-300)
    assert st == 0 and 1 <= it <= 8
    ref = _textbook_cg(A, -g, 8)
    assert np.allclose(d, ref[it - 1], rtol=1e-9, atol=1e-12)
    assert np.allclose(d, np.linalg.solve(A, -g), rtol=1e-8, atol=1e-10)
    qk = lambda w: 0.5 * w @ A @ w + g @ w
    prev = 0.0
    for j in range(it):
        cur = qk(ref[j])
        assert np.isclose(decs[j], prev - cur, rtol=1e-8), (j, decs[j], prev - cur)
        prev = cur
    # a few iterations with max_cg: again the textbook iterates
    st, d3, it3, _ = o.reduced_cg(csr, mask, g, 1e-300, max_cg=3)
    assert it3 == 3 and np.allclose(d3, ref[2], rtol=1e-10, atol=1e-13)


def pin_reduced_cg_stays_on_face(o):
    """With variables held fixed (mask 0) the direction is zero there and the
    free part solves A_FF d_F = -g_F (eq. (cg2))."""
    inst = instances.tiny_dense(8, seed=8)
    A = inst.dense
    g = np.random.default_rng(1).standard_normal(8)
    mask = np.array([1, 0, 1, 1, 0, 1, 0, 1], np.uint8)
    st, d, it, _ = o.reduced_cg(inst.csr(), mask, g, 1e-300)
    F = mask.astype(bool)
    assert st == 0 and np.all(d[~F] == 0.0) and it <= F.sum()
    assert np.allclose(d[F], np.linalg.solve(A[np.ix_(F, F)], -g[F]), rtol=1e-9, atol=1e-12)


def _textbook_pcg(A, rhs, dinv, iters):
    """Preconditioned CG for A w = rhs from w = 0 with M^{-1} = diag(dinv),
    written from the textbook; returns the iterates."""
    w = np.zeros_like(rhs)
    r = rhs.copy()
    z = dinv * r
    p = z.copy()
    out = []
    for _ in range(iters):
        Ap = A @ p
        a = (r @ z) / (p @ Ap)
        w = w + a * p
        r_new = r - a * Ap
        z_new = dinv * r_new
        out.append(w.copy())
        if r_new @ z_new == 0:
            break
        p = z_new + (r_new @ z_new) / (r @ z) * p
        r, z = r_new, z_new
    return out


def pin_reduced_pcg_is_textbook_pcg(o):
    """Diagonal preconditioner on a badly scaled SPD matrix: the iterates are
    textbook preconditioned CG with M = diag(A_k), the decreases equal
    q_k(w_{j-1}) - q_k(w_j), and on a free subset the preconditioner is the
    diagonal of the reduced matrix (eq. (cg2))."""
    rng = np.random.default_rng(21)
    Q = rng.standard_normal((8, 8))
    S = np.diag(10.0 ** rng.uniform(-2, 2, 8))
    A = S @ (Q.T @ Q + 0.5 * np.eye(8)) @ S  # SPD, diagonal spread over 1e8
    csr = instances.dense_to_csr(A)
    g = rng.standard_normal(8)
    mask = np.ones(8, np.uint8)
    ref = _textbook_pcg(A, -g, 1.0 / np.diag(A), 8)
    for k in (1, 2, 3):
        st, d, it, _ = o.reduced_cg(csr, mask, g, 1e-300, max_cg=k, precond=1)
        assert st == 0 and it == k
        assert np.allclose(d, ref[k - 1], rtol=1e-9, atol=1e-12 * np.abs(ref[k - 1]).max())
    st, d, it, decs = o.reduced_cg(csr, mask, g, 1e-300, precond=1)
    assert st == 0 and 1 <= it <= 8
    assert np.allclose(d, np.linalg.solve(A, -g), rtol=1e-7)
    qk = lambda w: 0.5 * w @ A @ w + g @ w
    prev = 0.0
    for j in range(min(it, 3)):
        cur = qk(ref[j])
        assert np.isclose(decs[j], prev - cur, rtol=1e-7), (j, decs[j], prev - cur)
        prev = cur
    # the unpreconditioned iterates differ on this matrix: the option is live
    st0, d0, _, _ = o.reduced_cg(csr, mask, g, 1e-300, max_cg=2)
    assert not np.allclose(d0, ref[1], rtol=1e-6)
    # a free subset: the preconditioner is the diagonal of A_FF
    F = np.array([1, 1, 0, 1, 0, 1, 1, 0], bool)
    refF = _textbook_pcg(A[np.ix_(F, F)], -g[F], 1.0 / np.diag(A)[F], 5)
    st, d, it, _ = o.reduced_cg(csr, F.astype(np.uint8), g, 1e-300, max_cg=2, precond=1)
    assert st == 0 and np.all(d[~F] == 0.0)
    assert np.allclose(d[F], refF[1], rtol=1e-9, atol=1e-12 * np.abs(refF[1]).max())


def pin_pcg_decrease_identity_exact(o):
    """For preconditioned CG, 1/2 alpha_j rho_j'z_j = q_k(w_{j-1}) - q_k(w_j)
    holds exactly: the recurrence run in rational arithmetic on a small SPD
    system, and the oracle's floating-point decreases agree with it."""
    from fractions import Fraction as Fr
    rng = np.random.default_rng(5)
    n = 5
    Q = rng.integers(-3, 4, (n, n))
    Ai = Q.T @ Q + np.diag(rng.integers(1, 9, n))
    gi = rng.integers(-5, 6, n)
    A = [[Fr(int(v)) for v in row] for row in Ai]
    g = [Fr(int(v)) for v in gi]
    dinv = [1 / A[i][i] for i in range(n)]
    mv = lambda v: [sum(A[i][k] * v[k] for k in range(n)) for i in range(n)]
    dot = lambda a, b: sum(x * y for x, y in zip(a, b))
    qk = lambda w: Fr(1, 2) * dot(w, mv(w)) + dot(g, w)
    w = [Fr(0)] * n
    r = [-v for v in g]
    z = [di * ri for di, ri in zip(dinv, r)]
    p = list(z)
    exact_decs = []
    for _ in range(n):
        Ap = mv(p)
        rz = dot(r, z)
        a = rz / dot(p, Ap)
        w_new = [wi + a * pi for wi, pi in zip(w, p)]
        dec = Fr(1, 2) * a * rz
        assert dec == qk(w) - qk(w_new)
        exact_decs.append(dec)
        r = [ri - a * api for ri, api in zip(r, Ap)]
        z = [di * ri for di, ri in zip(dinv, r)]
        w = w_new
        if dot(r, z) == 0:
            break
        p = [zi + dot(r, z) / rz * pi for zi, pi in zip(z, p)]
    csr = instances.dense_to_csr(Ai.astype(float))
    st, d, it, decs = o.reduced_cg(csr, np.ones(n, np.uint8), gi.astype(float), 1e-300,
                                   max_cg=len(exact_decs), precond=1)
    assert st == 0
    for j in range(it):
        assert abs(decs[j] - float(exact_decs[j])) <= 1e-11 * abs(float(exact_decs[j])), j


def pin_jacobi_gpcg_same_solution(o):
    """GPCG with the diagonal preconditioner reaches the same x* as without it
    (x* does not depend on the preconditioner), on the obstacle problem and on
    a strongly varying coefficient, where it needs far fewer CG iterations."""
    inst = instances.obstacle50(0)
    xs, info = exact.polish(inst.csr(), inst.b, inst.l, inst.u, None)
    assert info["converged"]
    x1, _, st1 = o.solve_instance(inst, precond=1, **TIGHT)
    assert st1["status"] == 0
    assert np.abs(x1 - xs).max() <= 1e-9 * max(1.0, np.abs(xs).max())
    vc = instances.varcoef(40, 2, eps=0.9)
    vc.l = np.full(vc.n, -np.inf)  # unconstrained: x* = A^{-1} b
    vc.u = np.full(vc.n, np.inf)
    want = np.linalg.solve(exact.csr_matrix(vc.csr()).toarray(), vc.b)
    x0, _, s0 = o.solve_instance(vc, **TIGHT)
    xj, _, sj = o.solve_instance(vc, precond=1, **TIGHT)
    for x in (x0, xj):
        assert np.abs(x - want).max() <= 1e-9 * np.abs(want).max()
    assert sj["cg_iters"] < 0.5 * s0["cg_iters"], (sj["cg_iters"], s0["cg_iters"])


def pin_residual_cg_stop(o):
    """The residual test (cg_stop = 1): CG stops at the first iterate whose
    residual ||r_k + A_k w_j|| is at most eta ||r_k||, found here by running
    textbook CG; with the Jacobi preconditioner the norm is the M^{-1} norm."""
    inst = instances.tiny_dense(8, seed=12, scale=3.0)
    A = inst.dense
    csr = inst.csr()
    g = np.random.default_rng(3).standard_normal(8)
    mask = np.ones(8, np.uint8)
    for eta in (0.5, 0.1, 1e-3):
        ref = _textbook_cg(A, -g, 8)
        r0 = np.linalg.norm(g)
        want = next(j for j, w in enumerate(ref) if np.linalg.norm(g + A @ w) <= eta * r0) + 1
        st, d, it, _ = o.reduced_cg(csr, mask, g, eta, cg_stop=1)
        assert st == 0 and it == want, (eta, it, want)
        assert np.allclose(d, ref[it - 1], rtol=1e-9, atol=1e-12)
    dinv = 1.0 / np.diag(A)
    refp = _textbook_pcg(A, -g, dinv, 8)
    mnorm = lambda r: np.sqrt(r @ (dinv * r))
    want = next(j for j, w in enumerate(refp) if mnorm(-g - A @ w) <= 0.1 * mnorm(-g)) + 1
    st, d, it, _ = o.reduced_cg(csr, mask, g, 0.1, cg_stop=1, precond=1)
    assert st == 0 and it == want
    # the whole method reaches the same x* with either test
    inst = instances.obstacle50(2)
    xs, info = exact.polish(inst.csr(), inst.b, inst.l, inst.u, None)
    x, _, st = o.solve_instance(inst, cg_stop=1, **TIGHT)
    assert info["converged"] and st["status"] == 0
    assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()



# ------------------------------------------------------------ stopping rules

def _spd(seed, n=10, decades=4.0):
    """An SPD matrix with eigenvalues spread over `decades` decades (random
    orthogonal basis) and a vector g, both from the seed."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(10.0 ** rng.uniform(0.0, decades, n)) @ Q.T
    return 0.5 * (A + A.T), rng.standard_normal(n)


def _direct_decreases(A, g, iterates):
    """q_k(w_{j-1}) - q_k(w_j) along the iterates, from w_0 = 0, with
    q_k(w) = 1/2 w'Aw + g'w evaluated directly (not by the CG identity)."""
    qk = lambda w: 0.5 * w @ (A @ w) + g @ w
    vals = [0.0] + [qk(w) for w in iterates]
    return np.array([vals[j] - vals[j + 1] for j in range(len(iterates))])


def _ratio_stop(decs, eta, frozen=False):
    """1-based index of the first j >= 2 with dec_j <= eta * max_{l<j} dec_l,
    the relative-decrease test of eqs. (pgstop2) and (cgstop1); None when no
    iterate passes it.  frozen: the misreading that compares with the first
    decrease instead of the largest earlier one."""
    for j in range(1, len(decs)):
        ref = decs[0] if frozen else np.max(decs[:j])
        if decs[j] <= eta * ref:
            return j + 1
    return None


# (seed of _spd, eta): cases where the running max and the first decrease give
# different stopping iterations
CG_RATIO_CASES = [(0, 0.05), (1, 0.5), (3, 0.5), (4, 0.5), (5, 0.2)]


def pin_cg_ratio_stop(o):
    """Eq. (cgstop1): the reduced CG stops at the first iterate j >= 2 whose
    decrease q_k(w_{j-1}) - q_k(w_j) is at most eta_2 times the largest
    earlier decrease.  The decreases come from textbook CG iterates and a
    direct evaluation of q_k; every case is one where the decreases are not
    monotone, so comparing with the first decrease would stop elsewhere."""
    for seed, eta in CG_RATIO_CASES:
        A, g = _spd(seed)
        n = len(g)
        ref = _textbook_cg(A, -g, n)
        decs = _direct_decreases(A, g, ref)
        want = _ratio_stop(decs, eta)
        assert want is not None and want < len(ref), (seed, eta)
        assert want != _ratio_stop(decs, eta, frozen=True), (seed, eta)
        for j in range(1, want):  # no decision within rounding of the threshold
            r = decs[j] / np.max(decs[:j])
            assert abs(r - eta) > 1e-6 * eta, (seed, eta, j, r)
        st, d, it, odecs = o.reduced_cg(instances.dense_to_csr(A), np.ones(n, np.uint8), g, eta)
        assert st == 0 and it == want, (seed, eta, it, want)
        assert np.allclose(d, ref[it - 1], rtol=1e-8, atol=1e-10 * np.abs(ref[it - 1]).max())
        assert np.allclose(odecs, decs[:it], rtol=1e-7), (seed, eta)


def _proj_grad_def(x, l, u, g):
    """Eq. (proj-gradient) written out: g_i on free variables, min(g_i, 0) at
    a lower bound, max(g_i, 0) at an upper bound, 0 when l_i = u_i."""
    p = g.copy()
    at_l, at_u = x == l, x == u
    p[at_l & at_u] = 0.0
    only_l, only_u = at_l & ~at_u, at_u & ~at_l
    p[only_l] = np.minimum(g[only_l], 0.0)
    p[only_u] = np.maximum(g[only_u], 0.0)
    return p


def _gp_phase(A, b, l, u, x, eta1, mu=0.01, max_gp=50, max_backtrack=60):
    """One gradient-projection phase of Algorithm GPCG, written here from
    Section 3: y_{j+1} = P[y_j - alpha_j grad q(y_j)] with alpha_j the first
    of alpha_0, alpha_0/2, ... giving sufficient decrease (eq. (gplsstop),
    q evaluated directly), alpha_0 the minimiser of q along -P grad q(y_j);
    stop when the active set repeats (pgstop1), on the relative-decrease test
    with eta1 (pgstop2), or after max_gp iterates.  Returns (iterates, the
    decreases, reason, smallest relative margin of a backtracking decision)."""
    q = lambda v: 0.5 * v @ (A @ v) - b @ v
    y = np.minimum(np.maximum(x, l), u)
    decs, margin = [], np.inf
    while True:
        g = A @ y - b
        d = _proj_grad_def(y, l, u, g)
        if not d.any():
            return len(decs), decs, "optimal", margin
        a = (d @ d) / (d @ (A @ d))
        for _ in range(max_backtrack + 1):
            yn = np.minimum(np.maximum(y - a * g, l), u)
            gs = g @ (yn - y)
            slack = q(yn) - q(y) - mu * gs
            margin = min(margin, abs(slack) / max(abs(gs), 1e-300))
            if slack <= 0.0:
                break
            a *= 0.5
        else:
            return len(decs), decs, "backtrack", margin
        dec = q(y) - q(yn)
        same_face = np.array_equal((y == l) | (y == u), (yn == l) | (yn == u))
        j = len(decs) + 1
        ratio = dec <= eta1 * max(decs) if decs else False
        decs.append(dec)
        y = yn
        if same_face:
            return j, decs, "pgstop1", margin
        if ratio:
            return j, decs, "pgstop2", margin
        if j >= max_gp:
            return j, decs, "cap", margin


def _gp_case(seed, n=40):
    """A dense box-constrained QP started at its upper bounds, where the first
    gradient-projection phase runs several iterates."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(10.0 ** rng.uniform(0.0, 2.5, n)) @ Q.T
    A = 0.5 * (A + A.T)
    b = 20.0 * rng.standard_normal(n)
    l = rng.uniform(-1.0, 0.0, n)
    u = l + rng.uniform(0.2, 1.5, n)
    return A, b, l, u, u.copy()


def pin_gp_ratio_stop(o):
    """Eq. (pgstop2): the gradient-projection phase stops at the first iterate
    j >= 2 whose decrease is at most eta_1 times the largest earlier one.  The
    phase is run independently here; the oracle's first phase (max_outer = 1)
    must take as many iterates, with the paper's eta_1 = 0.1, eta_2 = 0.05 and
    with eta_1 = 0.3, eta_2 = 0.01.  Every case stops by pgstop2, and with
    eta_2 in place of eta_1 it would stop at another iterate."""
    for seed in (0, 1, 4, 7, 8, 14):
        A, b, l, u, x0 = _gp_case(seed)
        csr = instances.dense_to_csr(A)
        for eta1, eta2 in ((0.1, 0.05), (0.3, 0.01)):
            want, decs, why, margin = _gp_phase(A, b, l, u, x0, eta1)
            other = _gp_phase(A, b, l, u, x0, eta2)[0]
            assert why == "pgstop2" and other != want, (seed, eta1, why, other)
            assert margin > 1e-9, (seed, margin)
            for j in range(1, want):
                r = decs[j] / max(decs[:j])
                assert abs(r - eta1) > 1e-6 * eta1, (seed, j, r)
            st = o.gpcg(csr, b, l, u, x0, max_outer=1, eta1=eta1, eta2=eta2)[2]
            assert st["gp_iters"] == want, (seed, eta1, st["gp_iters"], want)


def pin_eta2_schedule(o):
    """Eq. (cgstop3) and the reading of it: when the binding set equals the
    active set after a projected search, CG runs again on that face with eta_2
    multiplied by eta2_reduce; whenever a gradient-projection phase has run,
    the next CG phase uses the initial eta_2 again.  Checked on the trace of
    every CG phase (the eta its stopping test used, and its decreases, which
    must meet eq. (cgstop1) with that eta) of solves with chains of face
    repeats and with a gradient-projection phase after a repeat."""
    cases = [(instances.obstacle(12, 0, amplitude=0.5, u_random=True), {}),
             (instances.obstacle(16, 5, amplitude=0.5, u_random=True), dict(eta2=0.3)),
             (instances.obstacle50(0), dict(eta2_reduce=0.5)),
             (instances.obstacle50(0), {})]
    after_repeat = 0
    for inst, kw in cases:
        opts = dict(TIGHT, **kw)
        eta2 = kw.get("eta2", 0.05)
        red = kw.get("eta2_reduce", 0.1)
        _, _, st = o.solve_instance(inst, cg_trace_cap=400, dec_per=256, **opts)
        tr = st["cg_phases_trace"]
        assert st["status"] == 0 and len(tr) == st["cg_phases"]
        assert tr[0]["repeat"] == 0
        assert sum(t["repeat"] for t in tr) == st["face_repeats"] >= 2
        for i, t in enumerate(tr):
            if t["repeat"]:
                assert t["eta"] == tr[i - 1]["eta"] * red, (inst.name, i, t["eta"])
            else:
                assert t["eta"] == eta2, (inst.name, i, t["eta"])
                after_repeat += int(i > 0 and tr[i - 1]["repeat"] == 1)
            if t["iters"] <= len(t["decs"]):
                stop = _ratio_stop(t["decs"], t["eta"])
                # the test fired at the last iteration, or never (rho = 0 / cap)
                assert stop in (t["iters"], None), (inst.name, i, stop, t["iters"])
    assert after_repeat >= 2


def pin_objective(o):
    """q(x) = 1/2 x'Ax - b'x (Section 2, sign of b as in g = Ax - b): the
    oracle's objective against exact rational arithmetic on a tiny QP, and the
    q its solves report against a sparse-library evaluation at the answer."""
    inst = instances.tiny_dense(7, seed=31)
    x = np.random.default_rng(8).standard_normal(7)
    Af = [[Fraction(float(v)) for v in row] for row in inst.dense]
    xf = [Fraction(float(v)) for v in x]
    bf = [Fraction(float(v)) for v in inst.b]
    qx = Fraction(1, 2) * sum(xf[i] * sum(Af[i][j] * xf[j] for j in range(7)) for i in range(7)) \
        - sum(bf[i] * xf[i] for i in range(7))
    got = o.objective(inst.csr(), inst.b, x)
    assert abs(got - float(qx)) <= 1e-13 * (1.0 + abs(float(qx)))
    for inst in (instances.obstacle50(3), instances.varcoef(48, 2)):
        A = exact.csr_matrix(inst.csr())
        x, _, st = o.solve_instance(inst)
        want = 0.5 * x @ (A @ x) - inst.b @ x
        assert abs(st["q"] - want) <= 1e-12 * (abs(want) + abs(inst.b @ x)), (inst.name, st["q"], want)


# ---------------------------------------------------------------- whole method

def pin_brute_force_tiny(o, count=40):
    """Tiny QPs (n <= 8, mixed bound kinds incl. +-inf and l = u): GPCG's x
    equals the solution found by enumerating all 3^n faces."""
    for seed in range(count):
        n = 1 + seed % 8
        inst = instances.tiny_dense(n, seed=100 + seed)
        ref = exact.brute_force(inst.dense, inst.b, inst.l, inst.u)
        assert ref is not None
        x, _, st = o.solve_instance(inst, **TIGHT)
        assert st["status"] == 0, (seed, st)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(x - ref).max() <= 1e-9 * scale, (seed, x, ref)
        assert np.all(x >= inst.l) and np.all(x <= inst.u)


def pin_diagonal_closed_form(o):
    """Diagonal A: x*_i = mid(l_i, u_i, b_i / a_ii)."""
    inst = instances.diagonal(200, seed=3)
    x, _, st = o.solve_instance(inst, **TIGHT)
    d = np.diag(inst.dense)
    want = np.minimum(np.maximum(inst.b / d, inst.l), inst.u)
    assert st["status"] == 0
    assert np.allclose(x, want, rtol=1e-12, atol=1e-13)


def pin_unconstrained_laplacian_dst(o):
    """l = -inf, u = +inf on the 5-point Laplacian: x* = A^{-1} b, computed by
    the discrete sine transform that diagonalises A (closed-form eigenvalues
    4/h^2 (sin^2(p pi h/2) + sin^2(q pi h/2)))."""
    N = 31
    inst = instances.unconstrained(N, instances.OP_CONST, seed=2)
    h = 1.0 / (N + 1)
    k = np.arange(1, N + 1)
    lam1 = np.sin(k * np.pi * h / 2) ** 2
    Lam = 4.0 / h**2 * (lam1[:, None] + lam1[None, :])
    B = inst.b.reshape(N, N)
    X = scipy.fft.idstn(scipy.fft.dstn(B, type=1) / Lam, type=1)
    x, _, st = o.solve_instance(inst, **TIGHT)
    assert st["status"] == 0
    assert st["gp_iters"] == 1  # A(x) stays empty: pgstop1 ends GP at j = 1
    # with no active bound the exact 1-D minimiser (GP) and the unit CG step
    # (projected search) both satisfy sufficient decrease: no backtracking
    assert st["backtracks"] == 0
    assert np.abs(x - X.ravel()).max() <= 1e-9 * np.abs(X).max()


def pin_unconstrained_varcoef_direct(o):
    """Unconstrained variable-coefficient operator against a sparse direct solve."""
    inst = instances.unconstrained(40, instances.OP_VAR, seed=6)
    A = exact.csr_matrix(inst.csr())
    want = spla.spsolve(A.tocsc(), inst.b)
    x, _, st = o.solve_instance(inst, **TIGHT)
    assert st["status"] == 0
    assert np.abs(x - want).max() <= 1e-9 * np.abs(want).max()


def pin_manufactured(o):
    """Problems built around a known x* and known lower/upper/free sets."""
    for op in (instances.OP_CONST, instances.OP_VAR):
        inst = instances.manufactured(24, op, seed=7)
        xs, status = inst.meta["x_star"], inst.meta["status"]
        x, g, st = o.solve_instance(inst, **TIGHT)
        assert st["status"] == 0, st
        assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max(), op
        assert np.array_equal(x == inst.l, status == 1), op
        assert np.array_equal(x == inst.u, status == 2), op
        assert st["n_upper"] == int(np.sum(status == 2))


def pin_matches_independent_exact_solver(o):
    """The obstacle problem (n = 2500) against primal-dual active set + sparse
    direct solves, a method sharing nothing with GPCG."""
    inst = instances.obstacle50(seed=1)
    csr = inst.csr()
    x, g, st = o.solve_instance(inst, **TIGHT)
    xs, info = exact.polish(csr, inst.b, inst.l, inst.u, None)
    assert info["converged"] and st["status"] == 0
    assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()
    assert np.array_equal(x == inst.l, xs == inst.l)


def pin_invariants(o):
    """q decreases at every projected search (sufficient decrease), the active
    set does not shrink across a CG step + projected search (the CG direction
    is zero on A(x_k)), and the answer is feasible."""
    inst = instances.obstacle50(seed=2)
    x, g, st = o.solve_instance(inst, trace_cap=1000)
    tq = st["trace_q"]
    assert len(tq) == st["outer_iters"] >= 2
    assert np.all(np.diff(tq) < 0)
    act = st["trace_act"]
    assert np.all(act[:, 1] >= act[:, 0])
    assert np.all(x >= inst.l) and np.all(x <= inst.u)


ALL_PINS = [
    pin_projection_is_median,
    pin_projected_gradient_cases,
    pin_gradient_matches_sparse_library,
    pin_alpha0_minimises_along_projected_gradient,
    pin_decrease_identity_exact,
    pin_reduced_cg_is_textbook_cg,
    pin_reduced_cg_stays_on_face,
    pin_reduced_pcg_is_textbook_pcg,
    pin_pcg_decrease_identity_exact,
    pin_residual_cg_stop,
    pin_brute_force_tiny,
    pin_diagonal_closed_form,
    pin_unconstrained_laplacian_dst,
    pin_unconstrained_varcoef_direct,
    pin_manufactured,
    pin_matches_independent_exact_solver,
    pin_invariants,
    pin_jacobi_gpcg_same_solution,
    pin_cg_ratio_stop,
    pin_gp_ratio_stop,
    pin_eta2_schedule,
    pin_objective,
]
