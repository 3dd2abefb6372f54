"""The single-reduction CG recurrence for p'Ap in FP32 (CPU only).

The GPU's reduced CG gets p_{j+1}'A p_{j+1} from the recurrence
delta_{j+1} - beta_{j+1} gamma_{j+1} / alpha_j (Chronopoulos and Gear) with
the sums gamma = rho'rho and delta = rho'A rho accumulated in FP32 in the mixed
form.  Once rho has nearly vanished the recurrence can turn non-positive by
rounding although A is positive definite; the device then ends the CG phase
with the current iterate instead of declaring the operator indefinite.  This
test reproduces the situation in NumPy FP32 on the face of a 2-D Laplacian and
checks that the iterate at that point is a descent direction of the reduced
quadratic q_k(w) = 1/2 w'A w + g'w (the projected search along it is sound).
"""
import numpy as np
import scipy.sparse as sp


def _laplacian(N):
    T = sp.diags([-np.ones(N - 1), 2.0 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.eye(N)
    return (sp.kron(I, T) + sp.kron(T, I)).tocsr()


def _single_reduction_cg_f32(A, g, iters):
    """CG from w = 0 on A w = -g in the single-reduction form, FP32 vectors
    and sums; returns (iteration at which the recurrence for p'Ap first fails
    to be positive or None, w, that value)."""
    f = np.float32
    A = A.astype(f)
    rho = (-g).astype(f)
    w = np.zeros_like(rho)
    p = np.zeros_like(rho)
    s = np.zeros_like(rho)
    u = A @ rho
    gam, dl = f(rho @ rho), f(rho @ u)
    al, be = gam / dl, f(0)
    for j in range(iters):
        s = u if j == 0 else u + be * s
        p = rho if j == 0 else rho + be * p
        w = w + al * p
        rho = rho - al * s
        u = A @ rho
        gn, dn = f(rho @ rho), f(rho @ u)
        be = gn / gam
        pAp = dn - be * gn / al
        if not pAp > 0:
            return j + 1, w, float(pAp)
        al, gam = gn / pAp, gn
    return None, w, None


def test_fp32_recurrence_loses_positivity_with_a_descent_iterate():
    N = 64
    A = _laplacian(N)
    g = np.random.default_rng(0).standard_normal(N * N)
    j, w, pAp = _single_reduction_cg_f32(A, g, 5000)
    assert j is not None and pAp <= 0.0  # the situation the device guards against
    w64 = w.astype(np.float64)
    qk = 0.5 * w64 @ (A @ w64) + g @ w64
    # the exact minimiser of q_k reaches -1/2 g'A^-1 g; the iterate is a descent
    # direction that has gone most of the way
    import scipy.sparse.linalg as spla
    qmin = -0.5 * g @ spla.spsolve(A.tocsc(), g)
    assert qk < 0.0 and qk <= 0.99 * qmin
