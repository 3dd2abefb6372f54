"""Full-size obstacle problems (1024^2 and 1600^2 unknowns) on the GPU, through
the same solver path the benchmark times.

1024^2: the reference x* is the CPU oracle's answer polished by the exact
solver (primal-dual active set with sparse direct face solves) -- no GPU output
is used -- and the FP64 / mixed answers at tight tolerances must match it to
1e-8 / 1e-6 with identical faces off the degenerate set.
1600^2: properties that hold at any size -- feasibility, the termination test
re-evaluated on the CPU with the oracle's FP64 gradient, and agreement of the
FP64 and mixed answers.
"""
import numpy as np
import pytest

import instances
import oracle
from oracle import exact
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

_XSTAR = {}


def xstar(N):
    if N not in _XSTAR:
        inst = instances.obstacle_ub(N, 0)
        xo, _, _ = oracle.default().solve_instance(inst, tol_rel=1e-10)
        xs, info = exact.polish(inst.csr(), inst.b, inst.l, inst.u, xo)
        assert info["converged"]
        A = exact.csr_matrix(inst.csr())
        _XSTAR[N] = (inst, xs, A @ xs - inst.b)
    return _XSTAR[N]


def cpu_pg(inst, x):
    ora = oracle.default()
    g = ora.gradient(inst.csr(), x, inst.b)
    return ora.proj_gradient_norm(x, inst.l, inst.u, g)


@pytest.mark.timeout(900)
def test_obstacle1024_matches_exact_solution():
    import paper_cs_0101018_amd as gpcg
    inst, xs, gs = xstar(1024)
    print(f"1024^2: x* ready, |x*|_inf={np.abs(xs).max():.4f}", flush=True)
    deg = exact.degenerate_set(xs, gs, inst.l, inst.u)
    for prec, tol, bar in ((gpcg.GPCG_PREC_FP64, 1e-12, 1e-8),
                           (gpcg.GPCG_PREC_MIXED, 1e-10, 1e-6)):
        x, g, st = G.solve(inst, precision=prec, tol_rel=tol)
        err = G.rel_inf(x, xs)
        print(f"  prec={prec} status={st['status']} outer={st['outer_iters']} "
              f"cg={st['cg_iters']} pg={st['pg']:.3e} err={err:.3e}", flush=True)
        assert st["status"] in (gpcg.GPCG_OK, gpcg.GPCG_STAGNATED), st
        assert np.all(x >= inst.l) and np.all(x <= inst.u)
        assert err <= bar
        act = (x == inst.l) | (x == inst.u)
        act_s = (xs == inst.l) | (xs == inst.u)
        assert not ((act != act_s) & ~deg).any()


@pytest.mark.timeout(600)
def test_obstacle1600_properties():
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle_ub(1600, 0)
    res = {}
    for prec in (gpcg.GPCG_PREC_FP64, gpcg.GPCG_PREC_MIXED):
        x, g, st = G.solve(inst, precision=prec)
        pg = cpu_pg(inst, x)
        print(f"  1600^2 prec={prec} status={st['status']} outer={st['outer_iters']} "
              f"cg={st['cg_iters']} pg_gpu={st['pg']:.3e} pg_cpu={pg:.3e} tau={st['tau']:.3e}",
              flush=True)
        assert st["status"] == gpcg.GPCG_OK, st
        assert np.all(x >= inst.l) and np.all(x <= inst.u)
        assert pg <= st["tau"] * 1.001
        res[prec] = x
    # both answers satisfy the same termination test; on this instance that
    # bounds their distance well below the mixed-form bar
    assert G.rel_inf(res[1], res[0]) <= 1e-4
