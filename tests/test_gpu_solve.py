"""Whole GPCG solves on the GPU against the FP64 oracle (through the C ABI).

Parity bar: ||x - x*||_inf / ||x*||_inf <= 1e-8 (FP64 form) and <= 1e-6 (mixed
form) against the polished oracle solution x*, with identical active sets
outside the degenerate set (free variables within 1e-10 of a bound, active
variables with |g| within 1e-10 of zero).  The claim is made at a projected-
gradient tolerance tight enough for it to follow: on the face of x*,
||x - x*||_2 <= ||P grad q(x)||_2 / lambda_min(A) with lambda_min ~ 2 pi^2 for
both grid operators, so tol_rel = 1e-12 suffices for every instance here.
"""
import numpy as np
import pytest

import instances
import oracle
from oracle import exact
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

TIGHT = 1e-12
_REF = {}


def reference(name, inst):
    """Polished x* (oracle GPCG at a tight tolerance, then exact face solve)."""
    if name not in _REF:
        xo, go, st = oracle.default().solve_instance(inst, tol_rel=1e-12)
        xs, info = exact.polish(inst.csr(), inst.b, inst.l, inst.u, xo)
        assert info["converged"] and info["kkt"] < 1e-8 * max(1.0, np.abs(inst.b).max())
        A = exact.csr_matrix(inst.csr())
        _REF[name] = (xs, A @ xs - inst.b, st)
    return _REF[name]


def check_faces(x, xs, gs, inst):
    deg = exact.degenerate_set(xs, gs, inst.l, inst.u)
    act_gpu = (x == inst.l) | (x == inst.u)
    act_ref = (xs == inst.l) | (xs == inst.u)
    bad = (act_gpu != act_ref) & ~deg
    assert not bad.any(), f"{bad.sum()} active-set mismatches off the degenerate set"


def cpu_projected_gradient_norm(inst, x):
    ora = oracle.default()
    g = ora.gradient(inst.csr(), x, inst.b)
    return ora.proj_gradient_norm(x, inst.l, inst.u, g)


CASES = [
    ("c0", lambda: instances.obstacle50(0), None),
    ("c0_csr", lambda: instances.obstacle50(0), "csr"),
    ("c1", lambda: instances.varcoef256(0), None),
    ("c1_csr", lambda: instances.varcoef256(0), "csr"),
    ("obst_ragged", lambda: instances.obstacle(77, 3, amplitude=0.45, u_random=True), None),
]


@pytest.mark.parametrize("name,make,kind", CASES, ids=[c[0] for c in CASES])
def test_fp64_matches_oracle(name, make, kind):
    inst = make()
    print(f"solve fp64 {name} n={inst.n}", flush=True)
    xs, gs, st_ref = reference(name.split("_csr")[0], inst)
    x, g, st = G.solve(inst, kind, tol_rel=TIGHT)
    assert st["status"] == 0, st
    assert np.all(x >= inst.l) and np.all(x <= inst.u)
    err = G.rel_inf(x, xs)
    print(f"  outer={st['outer_iters']} gp={st['gp_iters']} cg={st['cg_iters']} err={err:.2e} "
          f"(oracle outer={st_ref['outer_iters']} cg={st_ref['cg_iters']})", flush=True)
    assert err <= 1e-8
    check_faces(x, xs, gs, inst)
    # the returned gradient is g = Ax - b at the answer
    A = exact.csr_matrix(inst.csr())
    assert np.allclose(g, A @ x - inst.b, rtol=0, atol=1e-9 * np.abs(inst.b).max() + 1e-12)


@pytest.mark.parametrize("name,make", [("c0", lambda: instances.obstacle50(0)),
                                       ("c1", lambda: instances.varcoef256(0))])
def test_metric_tolerance_holds_on_cpu(name, make):
    """At the metric tolerance (1e-8 relative) the answer satisfies the
    termination test when its projected gradient is recomputed on the CPU."""
    inst = make()
    x, g, st = G.solve(inst)
    assert st["status"] == 0
    pg = cpu_projected_gradient_norm(inst, x)
    assert pg <= st["tau"] * 1.001 + 1e-14, (pg, st["tau"])
    xs, gs, _ = reference(name, inst)
    print(f"  metric tol: err vs x* = {G.rel_inf(x, xs):.2e}", flush=True)


def test_mixed_precision_matches_oracle():
    import paper_cs_0101018_amd as gpcg
    inst = instances.varcoef256(0)
    xs, gs, _ = reference("c1", inst)
    x, g, st = G.solve(inst, precision=gpcg.GPCG_PREC_MIXED, tol_rel=1e-10)
    err = G.rel_inf(x, xs)
    print(f"  mixed: status={st['status']} outer={st['outer_iters']} cg={st['cg_iters']} "
          f"err={err:.2e}", flush=True)
    assert st["status"] == 0
    assert err <= 1e-6
    check_faces(x, xs, gs, inst)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_brute_force(seed):
    n = 1 + seed % 8
    inst = instances.tiny_dense(n, seed=500 + seed)
    ref = exact.brute_force(inst.dense, inst.b, inst.l, inst.u)
    x, g, st = G.solve(inst, "csr", tol_rel=1e-13)
    assert st["status"] == 0, st
    assert np.abs(x - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("op", [instances.OP_CONST, instances.OP_VAR])
@pytest.mark.parametrize("N", [24, 100])
def test_manufactured(op, N):
    """Known x* with lower- and upper-active variables."""
    inst = instances.manufactured(N, op, seed=N)
    xs, status = inst.meta["x_star"], inst.meta["status"]
    x, g, st = G.solve(inst, tol_rel=1e-13)
    assert st["status"] == 0, st
    assert G.rel_inf(x, xs) <= 1e-9
    assert np.array_equal(x == inst.l, status == 1)
    assert np.array_equal(x == inst.u, status == 2)
    assert st["n_upper"] == int(np.sum(status == 2))


def test_unconstrained_matches_direct_solve():
    import scipy.sparse.linalg as spla
    inst = instances.unconstrained(45, instances.OP_VAR, seed=1)
    want = spla.spsolve(exact.csr_matrix(inst.csr()).tocsc(), inst.b)
    x, g, st = G.solve(inst, tol_rel=1e-13)
    assert st["status"] == 0 and st["gp_iters"] == 1
    assert G.rel_inf(x, want) <= 1e-9


def test_deterministic_and_graph_invariant():
    inst = instances.obstacle50(2)
    x1, g1, s1 = G.solve(inst)
    x2, g2, s2 = G.solve(inst)
    x3, g3, s3 = G.solve(inst, use_graph=0, chunk=6)
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)
    for k in ("outer_iters", "gp_iters", "cg_iters", "backtracks", "passes"):
        assert s1[k] == s2[k] == s3[k], k


@pytest.mark.parametrize("case", ["c0", "c0_csr", "c1s", "ragged_mixed", "ragged_csr_mixed",
                                  "many_tiles", "many_tiles_mixed", "wide_auto_tiles",
                                  "wide_auto_tiles_mixed"])
def test_fused_and_split_forms_agree_bitwise(case):
    """The two launch forms use the same tiles and summation orders."""
    import paper_cs_0101018_amd as gpcg
    inst, kind, prec = {
        "c0": (instances.obstacle50(0), None, gpcg.GPCG_PREC_FP64),
        "c0_csr": (instances.obstacle50(0), "csr", gpcg.GPCG_PREC_FP64),
        "c1s": (instances.varcoef(96, 3), None, gpcg.GPCG_PREC_FP64),
        "ragged_mixed": (instances.obstacle(77, 5), None, gpcg.GPCG_PREC_MIXED),
        "ragged_csr_mixed": (instances.obstacle(77, 5), "csr", gpcg.GPCG_PREC_MIXED),
        # more tiles than threads per workgroup: every slot sum has a tail
        "many_tiles": (instances.obstacle(601, 1), None, gpcg.GPCG_PREC_FP64),
        "many_tiles_mixed": (instances.varcoef(333, 2), None, gpcg.GPCG_PREC_MIXED),
        # beyond 1024 x 256 unknowns the library's tiles hold several chunks
        # of 256 (512 unknowns per tile)
        "wide_auto_tiles": (instances.obstacle(1100, 2), None, gpcg.GPCG_PREC_FP64),
        "wide_auto_tiles_mixed": (instances.varcoef(530, 4), None, gpcg.GPCG_PREC_MIXED),
    }[case]
    res = [G.solve(inst, kind, precision=prec, form=f)
           for f in (gpcg.GPCG_FORM_FUSED, gpcg.GPCG_FORM_SPLIT)]
    res.append(G.solve(inst, kind, precision=prec, form=gpcg.GPCG_FORM_SPLIT,
                       use_graph=0, chunk=10))
    res.append(G.solve(inst, kind, precision=prec, form=gpcg.GPCG_FORM_SPLIT, tiles_per_wg=3))
    # the CG iterations in a data kernel of their own
    res.append(G.solve(inst, kind, precision=prec, form=gpcg.GPCG_FORM_SPLIT,
                       cg_kernel=gpcg.GPCG_CGK_ON))
    res.append(G.solve(inst, kind, precision=prec, form=gpcg.GPCG_FORM_SPLIT, tiles_per_wg=2,
                       cg_kernel=gpcg.GPCG_CGK_ON, prefetch=gpcg.GPCG_PREFETCH_OFF))
    (x1, g1, s1) = res[0]
    assert s1["status"] == gpcg.GPCG_OK
    for x, g, st in res[1:]:
        assert np.array_equal(x, x1) and np.array_equal(g, g1)
        for k in ("outer_iters", "gp_iters", "cg_iters", "backtracks"):
            assert st[k] == s1[k], k
        # the fused form's trial passes look ahead; the split form's do not
        assert st["passes"] + st["lookaheads"] == s1["passes"] + s1["lookaheads"]


@pytest.mark.parametrize("tile,mixed", [(512, False), (1024, False), (2048, False),
                                        (1024, True), (2048, True)],
                         ids=["512", "1024", "2048", "1024_mixed", "2048_mixed"])
def test_wider_tiles(tile, mixed):
    """Tiles of several 256-unknown chunks (no early loads; 512: two chunks
    loaded together, 1024 and 2048: the library's tiles on the largest grids,
    the mixed form's from 1024^2 on, chunks one after the other) on a ragged
    grid whose last tile is partly empty: the parity bar of the precision
    (FP64 1e-8, mixed 1e-6 against x*), and the launch forms agree bitwise."""
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(77, 3, amplitude=0.45, u_random=True)
    xs, gs, _ = reference("obst_ragged", inst)
    prec = gpcg.GPCG_PREC_MIXED if mixed else gpcg.GPCG_PREC_FP64
    x, g, st = G.solve(inst, tol_rel=1e-10 if mixed else TIGHT, tile=tile, precision=prec)
    assert st["status"] == gpcg.GPCG_OK, st
    assert G.rel_inf(x, xs) <= (1e-6 if mixed else 1e-8)
    check_faces(x, xs, gs, inst)
    xf, _, _ = G.solve(inst, tile=tile, precision=prec, form=gpcg.GPCG_FORM_FUSED)
    xp, _, _ = G.solve(inst, tile=tile, precision=prec, form=gpcg.GPCG_FORM_SPLIT)
    xq, _, _ = G.solve(inst, tile=tile, precision=prec, form=gpcg.GPCG_FORM_SPLIT,
                       tiles_per_wg=2)
    assert np.array_equal(xf, xp) and np.array_equal(xf, xq)


def test_start_outside_box_is_projected():
    inst = instances.obstacle50(4)
    inst.x0 = inst.x0.copy()
    inst.x0[::5] = 3.0
    x, g, st = G.solve(inst, tol_rel=TIGHT)
    assert st["x0_projected"] == 1 and st["status"] == 0
    xs, gs, _ = reference("c0s4", instances.obstacle50(4))
    assert G.rel_inf(x, xs) <= 1e-8


def test_errors():
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(20, 1)
    bad = instances.obstacle(20, 1)
    bad.l = bad.l.copy()
    bad.l[17] = 1.0  # above u = 0.25
    with pytest.raises(gpcg.GpcgError) as e:
        G.solve(bad)
    assert e.value.status == gpcg.GPCG_ERR_BOUNDS
    nan = instances.obstacle(20, 1)
    nan.b = nan.b.copy()
    nan.b[3] = np.nan
    with pytest.raises(gpcg.GpcgError) as e:
        G.solve(nan)
    assert e.value.status == gpcg.GPCG_ERR_NAN
    neg = instances.tiny_dense(5, 3)
    neg.dense = -np.eye(5)
    neg.l, neg.u = np.full(5, -np.inf), np.full(5, np.inf)
    with pytest.raises(gpcg.GpcgError) as e:
        G.solve(neg, "csr")
    assert e.value.status == gpcg.GPCG_ERR_NOT_SPD
    x, g, st = G.solve(inst, max_outer=1)
    assert st["status"] == gpcg.GPCG_MAXIT and st["outer_iters"] == 1


@pytest.mark.parametrize("form", [1, 2], ids=["fused", "split"])
def test_repeated_solves_on_one_handle(form):
    """Several solves on one handle and workspace (the state of the last one
    still in the caches) give the same answer every time.  A 1024^2 grid in
    the fused form has 2048 tiles, so every workgroup also sums the slots of
    tiles beyond the first 256."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    inst = instances.obstacle_ub(1024, 0)
    b, l, u, x0 = (G.to_dev(a) for a in (inst.b, inst.l, inst.u, inst.x0))
    s = gpcg.Solver(gpcg.Operator.stencil_const(1024, 1024, inst.w), device=dev, form=form)
    first = None
    for rep in range(6):
        print(f"repeated solve form={form} rep={rep}", flush=True)
        x = x0.clone()
        st = s.solve(b, l, u, x)
        torch.cuda.synchronize()
        assert st["status"] == 0, st
        xh = x.cpu().numpy()
        if first is None:
            first = (xh, st["passes"])
        else:
            assert np.array_equal(xh, first[0]) and st["passes"] == first[1]
    s.close()
