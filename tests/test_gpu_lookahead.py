"""Trial passes that look ahead (the fused form evaluates eq. (bqpls) at the
trial point inside the trial pass): the iterates are bitwise those of the
plain pass sequence, every count but the passes is unchanged, and each
look-ahead saves exactly one pass."""
import numpy as np
import pytest

import instances
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

COUNTS = ("outer_iters", "gp_iters", "cg_iters", "backtracks", "face_repeats", "cg_phases",
          "n_lower", "n_upper")


def _pair(inst, kind=None, **opts):
    import paper_cs_0101018_amd as gpcg
    on = G.solve(inst, kind, form=gpcg.GPCG_FORM_FUSED, lookahead=gpcg.GPCG_LOOKAHEAD_ON, **opts)
    off = G.solve(inst, kind, form=gpcg.GPCG_FORM_FUSED, lookahead=gpcg.GPCG_LOOKAHEAD_OFF,
                  **opts)
    return on, off


def _same(on, off):
    (x1, g1, s1), (x0, g0, s0) = on, off
    assert s1["status"] == s0["status"] == 0, (s1["status"], s0["status"])
    assert np.array_equal(x1, x0) and np.array_equal(g1, g0)
    for k in COUNTS:
        assert s1[k] == s0[k], k
    assert s0["lookaheads"] == 0
    assert s1["passes"] + s1["lookaheads"] == s0["passes"]
    return s1


@pytest.mark.parametrize("N", [1, 2, 3, 5, 16, 37, 77, 256, 300])
@pytest.mark.parametrize("op", [instances.OP_CONST, instances.OP_VAR])
def test_lookahead_bitwise(N, op):
    """Grids narrower than a tile (a tile spans several rows), one tile per
    row, rows wider than a tile, ragged last tiles."""
    inst = (instances.obstacle(N, 3, amplitude=0.4) if op == instances.OP_CONST
            else instances.varcoef(N, 2))
    print(f"lookahead N={N} op={op}", flush=True)
    s1 = _same(*_pair(inst))
    # every accepted iterate that continues its phase saves its step-length pass
    assert s1["lookaheads"] <= s1["gp_iters"]
    if N >= 16:
        assert s1["lookaheads"] > 0


@pytest.mark.parametrize("prec", [0, 1])
def test_lookahead_mixed_and_preconditioned(prec):
    import paper_cs_0101018_amd as gpcg
    inst = instances.varcoef(96, 5, eps=0.5)
    _same(*_pair(inst, precision=prec, precond=gpcg.GPCG_PRECOND_JACOBI))
    _same(*_pair(inst, precision=prec, cg_stop=gpcg.GPCG_CGSTOP_RESIDUAL))


@pytest.mark.parametrize("nx,ny", [(257, 3), (3, 200), (600, 40), (1, 700), (700, 1)])
def test_lookahead_rectangular(nx, ny):
    """Rectangular grids, including single rows and columns: a stencil
    neighbour two rows away is outside the grid or far from the tile."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    rng = np.random.default_rng(nx * 1000 + ny)
    n = nx * ny
    b = rng.standard_normal(n)
    l = np.where(rng.uniform(size=n) < 0.5, -0.05 * rng.uniform(size=n), -np.inf)
    u = np.where(rng.uniform(size=n) < 0.3, 0.05 * rng.uniform(size=n), np.inf)
    wx = 0.5 + rng.uniform(size=(ny, nx + 1))
    wy = 0.5 + rng.uniform(size=(ny + 1, nx))
    out = []
    for la in (gpcg.GPCG_LOOKAHEAD_ON, gpcg.GPCG_LOOKAHEAD_OFF):
        for var in (False, True):
            op = (gpcg.Operator.stencil_var(nx, ny, G.to_dev(wx.ravel()), G.to_dev(wy.ravel()))
                  if var else gpcg.Operator.stencil_const(nx, ny, 1.0))
            s = gpcg.Solver(op, device=dev, form=gpcg.GPCG_FORM_FUSED, lookahead=la)
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            g = torch.empty_like(x)
            st = s.solve(G.to_dev(b), G.to_dev(l), G.to_dev(u), x, g)
            torch.cuda.synchronize()
            out.append((x.cpu().numpy(), g.cpu().numpy(), st))
            s.close()
    _same(out[0], out[2])
    _same(out[1], out[3])


def test_lookahead_fused_equals_split():
    """The split form does not look ahead: the same iterates, and its extra
    passes are exactly the fused form's look-aheads."""
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(140, 7, amplitude=0.45, u_random=True)
    xf, gf, sf = G.solve(inst, form=gpcg.GPCG_FORM_FUSED)
    xs, gs, ss = G.solve(inst, form=gpcg.GPCG_FORM_SPLIT)
    assert np.array_equal(xf, xs) and np.array_equal(gf, gs)
    assert sf["lookaheads"] > 0 and ss["lookaheads"] == 0
    assert sf["passes"] + sf["lookaheads"] == ss["passes"]
    for k in COUNTS:
        assert sf[k] == ss[k], k


def test_lookahead_off_for_csr_and_wide_tiles():
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(60, 1)
    for kind, opts in (("csr", {}), (None, {"tile": 512})):
        x, g, st = G.solve(inst, kind, form=gpcg.GPCG_FORM_FUSED,
                           lookahead=gpcg.GPCG_LOOKAHEAD_ON, **opts)
        assert st["status"] == 0 and st["lookaheads"] == 0
