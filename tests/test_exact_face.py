"""The exact face solver of the constant five-point operator (capacitance
system over the DST-diagonalised Laplacian) that rebuilds x* of the large
obstacle problems from a face certificate, pinned against SciPy's sparse
direct solver and the primal-dual active-set method; a wrong certificate is
refused by the Kuhn-Tucker check."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import instances
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_poisson_solve_matches_sparse_direct():
    N, w = 37, 38.0 ** 2
    rhs = np.random.default_rng(0).standard_normal(N * N)
    A = exact.stencil_const_csr(N, w)
    want = spla.spsolve(A.tocsc(), rhs)
    got = exact.poisson_solve(N, w, rhs)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the assembled operator is the instances' five-point operator
    inst = instances.obstacle(N, 0)
    assert abs(exact.stencil_const_csr(N, inst.w) - exact.csr_matrix(inst.csr())).max() == 0.0


def test_face_solve_matches_sparse_direct_on_a_random_face():
    N, w = 48, 49.0 ** 2
    rng = np.random.default_rng(1)
    n = N * N
    b = rng.standard_normal(n)
    act = np.sort(rng.choice(n, 60, replace=False))
    val = rng.uniform(-0.1, 0.1, act.size)
    x, mu = exact.face_solve_const(N, w, b, act, val)
    A = exact.stencil_const_csr(N, w)
    F = np.ones(n, bool)
    F[act] = False
    want = np.zeros(n)
    want[act] = val
    want[F] = spla.spsolve(A[F][:, F].tocsc(), b[F] - A[F][:, ~F] @ val)
    assert np.array_equal(x[act], val)
    assert np.abs(x - want).max() <= 1e-12 * np.abs(want).max()
    # mu are the multipliers: (A x - b) on the face
    assert np.allclose(mu, (A @ x - b)[act], rtol=1e-9, atol=1e-9 * np.abs(b).max())


@pytest.mark.parametrize("N", [64, 96])
def test_pdas_with_face_solves_equals_pdas_with_superlu(N):
    inst = instances.obstacle_ub(N, 0)
    A = exact.csr_matrix(inst.csr())
    x1, _, ok1 = exact.pdas(A, inst.b, inst.l, inst.u, inst.x0)
    x2, _, ok2 = exact.pdas_const(N, inst.w, inst.b, inst.l, inst.u, inst.x0)
    assert ok1 and ok2
    assert np.array_equal(x1 == inst.l, x2 == inst.l)
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()


def test_wrong_certificate_is_refused():
    N = 64
    inst = instances.obstacle_ub(N, 0)
    A = exact.csr_matrix(inst.csr())
    xs, _, _ = exact.pdas(A, inst.b, inst.l, inst.u, inst.x0)
    lo = np.flatnonzero(xs == inst.l)
    assert lo.size >= 2
    x, g, kkt = exact.xstar_from_face(N, inst.w, inst.b, inst.l, inst.u, lo, [])
    assert np.abs(x - xs).max() <= 1e-12 * np.abs(xs).max()
    with pytest.raises(ValueError):  # one active variable missing: infeasible
        exact.xstar_from_face(N, inst.w, inst.b, inst.l, inst.u, lo[1:], [])
    free = np.flatnonzero((xs > inst.l) & (xs < inst.u))
    far = free[np.argmax(xs[free] - inst.l[free])]
    with pytest.raises(ValueError):  # a free variable pinned: wrong multiplier sign
        exact.xstar_from_face(N, inst.w, inst.b, inst.l, inst.u, np.append(lo, far), [])


def test_committed_face_of_1024_gives_x_star():
    inst = instances.obstacle_ub(1024, 0)
    N, lo, up = exact.read_face(os.path.join(GOLDEN, "face_obstacle_ub_1024_seed0.txt"))
    assert N == 1024 and lo.size > 0
    x, g, kkt = exact.xstar_from_face(N, inst.w, inst.b, inst.l, inst.u, lo, up)
    assert np.all(x >= inst.l) and np.all(x <= inst.u)
    assert kkt <= 1e-8
