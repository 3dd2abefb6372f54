"""The oracle against its pins (CPU only)."""
import numpy as np
import pytest

import instances
import oracle
from oracle import exact
from tests import oracle_pins


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(ora, pin):
    pin(ora)


def test_paper_constants(ora):
    """eta_1 = 0.1 and eta_2 = 0.05 are the values used in Section 5."""
    o = ora.options()
    assert o.eta1 == 0.1 and o.eta2 == 0.05
    assert 0.0 < o.mu < 0.5  # eq. (gplsstop) asks for mu in (0, 1/2)


def test_start_outside_box_is_projected(ora):
    inst = instances.obstacle50(seed=4)
    x_ref, _, st_ref = ora.solve_instance(inst)
    x0 = inst.x0.copy()
    x0[::7] = 5.0  # above u = 0.25
    x, _, st = ora.gpcg(inst.csr(), inst.b, inst.l, inst.u, x0)
    assert st["x0_projected"] == 1 and st_ref["x0_projected"] == 0
    assert st["status"] == 0
    xs, _ = exact.polish(inst.csr(), inst.b, inst.l, inst.u, x_ref)
    assert np.abs(x - xs).max() <= 1e-5 * np.abs(xs).max()


def test_errors(ora):
    inst = instances.tiny_dense(5, seed=3)
    csr = inst.csr()
    l, u = inst.l.copy(), inst.u.copy()
    l[2], u[2] = 1.0, 0.0
    assert ora.gpcg(csr, inst.b, l, u, inst.x0)[2]["status"] == oracle.ERR_BOUNDS
    b = inst.b.copy()
    b[1] = np.nan
    assert ora.gpcg(csr, b, inst.l, inst.u, inst.x0)[2]["status"] == oracle.ERR_NAN
    # an indefinite matrix is caught by the curvature guards
    D = -np.eye(5)
    bad = instances.dense_to_csr(D)
    st = ora.gpcg(bad, np.ones(5), np.full(5, -np.inf), np.full(5, np.inf), np.zeros(5))[2]
    assert st["status"] == oracle.ERR_NOT_SPD


def test_iteration_caps(ora):
    inst = instances.obstacle50(seed=0)
    st = ora.solve_instance(inst, max_outer=1)[2]
    assert st["status"] == oracle.MAXIT and st["outer_iters"] == 1
    st = ora.solve_instance(inst, max_cg=1)[2]
    assert st["status"] in (oracle.OK, oracle.MAXIT)


def test_free_fraction_matches_stated_sanity(ora):
    """Sanity only (parity unpinned): the variable-coefficient instance ends
    with about two thirds of its variables free, the same regime as the
    paper's eps = 0.1 journal bearing (about 68% free, Section 5)."""
    inst = instances.varcoef256()
    x, g, st = ora.solve_instance(inst)
    frac = st["n_free"] / inst.n
    assert 0.55 < frac < 0.75
