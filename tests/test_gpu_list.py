"""The compacted free-list form of the reduced CG (free_set = LIST) against the
polished oracle x*, to the same bar as the mask form; both launch forms of
the list form agree bitwise.

In the list form a set-up pass compacts the free mask of the face into an
ascending index list (prefix sums of the per-tile free counts, then ballots
inside each tile), and every CG iteration sweeps only the list.  The sums
run over list tiles instead of grid tiles, so the iterates agree with the
mask form only to rounding; the answers meet the same parity bar.
"""
import numpy as np
import pytest

import instances
from tests import gpu_util as G
from tests.test_gpu_solve import TIGHT, check_faces, reference

pytestmark = pytest.mark.gpu

CASES = [
    ("c0", lambda: instances.obstacle50(0), None, 0),
    ("c1", lambda: instances.varcoef256(0), None, 0),
    ("c1_csr", lambda: instances.varcoef256(0), "csr", 0),
    ("obst_ragged", lambda: instances.obstacle(77, 3, amplitude=0.45, u_random=True), None, 0),
    ("c1_mixed", lambda: instances.varcoef256(0), None, 1),
    ("obst_ragged_csr_mixed",
     lambda: instances.obstacle(77, 3, amplitude=0.45, u_random=True), "csr", 1),
]


@pytest.mark.parametrize("name,make,kind,prec", CASES, ids=[c[0] for c in CASES])
def test_list_form_matches_oracle(name, make, kind, prec):
    import paper_cs_0101018_amd as gpcg
    inst = make()
    base = name.split("_csr")[0].split("_mixed")[0]
    xs, gs, _ = reference(base, inst)
    tol, bar = (TIGHT, 1e-8) if prec == 0 else (1e-10, 1e-6)
    print(f"list form {name} n={inst.n}", flush=True)
    x, g, st = G.solve(inst, kind, precision=prec, tol_rel=tol,
                       free_set=gpcg.GPCG_FREESET_LIST)
    err = G.rel_inf(x, xs)
    print(f"  status={st['status']} outer={st['outer_iters']} cg={st['cg_iters']} "
          f"err={err:.2e}", flush=True)
    assert st["status"] == gpcg.GPCG_OK, st
    assert np.all(x >= inst.l) and np.all(x <= inst.u)
    assert err <= bar
    check_faces(x, xs, gs, inst)


@pytest.mark.parametrize("prec", [0, 1])
def test_list_form_fused_split_bitwise(prec):
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(77, 5, amplitude=0.45)
    res = [G.solve(inst, precision=prec, free_set=gpcg.GPCG_FREESET_LIST, form=f)
           for f in (gpcg.GPCG_FORM_FUSED, gpcg.GPCG_FORM_SPLIT)]
    assert res[0][2]["status"] == gpcg.GPCG_OK
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][2]["cg_iters"] == res[1][2]["cg_iters"]


def test_list_form_fixed_and_free_extremes():
    """Every variable fixed (l = u: nothing is ever free), a third of them
    fixed in runs of seven (the list skips those runs), and every variable
    free (unconstrained)."""
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(40, 2)
    inst.u = inst.l.copy()
    inst.x0 = inst.l.copy()
    x, g, st = G.solve(inst, free_set=gpcg.GPCG_FREESET_LIST)
    assert st["status"] == gpcg.GPCG_OK and np.array_equal(x, inst.l)

    half = instances.obstacle(61, 4, amplitude=0.4)
    half.u = half.u.copy()
    fixed = (np.arange(half.n) // 7) % 3 == 0
    half.u[fixed] = half.l[fixed]
    half.x0 = np.minimum(np.maximum(half.x0, half.l), half.u)
    xs, gs, _ = reference("obst61_runs_fixed", half)
    x, g, st = G.solve(half, tol_rel=TIGHT, free_set=gpcg.GPCG_FREESET_LIST)
    assert st["status"] == gpcg.GPCG_OK, st
    assert G.rel_inf(x, xs) <= 1e-8
    check_faces(x, xs, gs, half)

    free = instances.unconstrained(45, instances.OP_VAR, seed=1)
    xm, _, _ = G.solve(free, tol_rel=1e-13)
    xl, _, sl = G.solve(free, tol_rel=1e-13, free_set=gpcg.GPCG_FREESET_LIST)
    assert sl["status"] == gpcg.GPCG_OK
    assert G.rel_inf(xl, xm) <= 1e-10


def test_list_form_in_a_batch_matches_alone():
    import paper_cs_0101018_amd as gpcg
    insts = [instances.obstacle(N, 7 + N, amplitude=0.4) for N in (33, 64, 90)]
    alone = [G.solve(i, free_set=gpcg.GPCG_FREESET_LIST)[0] for i in insts]
    torch, dev = G.torch_dev()
    ops = [G.operator_for(i) for i in insts]
    solvers = [gpcg.Solver(op, device=dev, free_set=gpcg.GPCG_FREESET_LIST) for op in ops]
    xs = [G.to_dev(i.x0) for i in insts]
    probs = [(G.to_dev(i.b), G.to_dev(i.l), G.to_dev(i.u), x) for i, x in zip(insts, xs)]
    b = gpcg.Batch(solvers, device=dev)
    stats = b.solve(probs, mode=gpcg.GPCG_BATCH_STEPPED)
    torch.cuda.synchronize()
    for x, a, st in zip(xs, alone, stats):
        assert st["status"] == gpcg.GPCG_OK
        assert np.array_equal(x.cpu().numpy(), a)
    b.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_list_form_large_grid(prec):
    """Beyond 262,144 unknowns the mask form uses 512-unknown tiles; the list
    form keeps 256 (its compaction works one unknown per thread).  Its answer
    meets the parity bar against the mask form's, and both launch forms agree
    bitwise."""
    import paper_cs_0101018_amd as gpcg
    inst = instances.obstacle(530, 6, amplitude=0.4)
    tol, bar = (TIGHT, 1e-8) if prec == 0 else (1e-10, 1e-6)
    xm, gm, sm = G.solve(inst, precision=0, tol_rel=TIGHT)
    outs = [G.solve(inst, precision=prec, tol_rel=tol, free_set=gpcg.GPCG_FREESET_LIST, form=f)
            for f in (gpcg.GPCG_FORM_FUSED, gpcg.GPCG_FORM_SPLIT)]
    for x, g, st in outs:
        assert st["status"] == gpcg.GPCG_OK, st
        assert G.rel_inf(x, xm) <= bar
    assert np.array_equal(outs[0][0], outs[1][0])
