"""Jacobi-preconditioned reduced CG (options.precond = GPCG_PRECOND_JACOBI, the
diagonal of A on the free set; the paper's point Jacobi preconditioner).

x* does not depend on the preconditioner: the answers meet the same parity bar
against the polished oracle solution as the plain form.  Every launch form,
the batch and the tuner candidates stay bitwise equal to the solo answer."""
import numpy as np
import pytest

import instances
import oracle
from tests import gpu_util as G
from tests.test_gpu_solve import TIGHT, check_faces, reference

pytestmark = pytest.mark.gpu

CASES = [
    ("c0", lambda: instances.obstacle50(0), None, 0),
    ("c1", lambda: instances.varcoef256(0), None, 0),
    ("c1_csr", lambda: instances.varcoef256(0), "csr", 0),
    ("obst_ragged", lambda: instances.obstacle(77, 3, amplitude=0.45, u_random=True), None, 0),
    ("bearing_e09", lambda: instances.varcoef(90, 1, eps=0.9), None, 0),
    ("c1_mixed", lambda: instances.varcoef256(0), None, 1),
    ("bearing_e09_mixed", lambda: instances.varcoef(90, 1, eps=0.9), None, 1),
]


@pytest.mark.parametrize("name,make,kind,prec", CASES, ids=[c[0] for c in CASES])
def test_jacobi_matches_oracle(name, make, kind, prec):
    import paper_cs_0101018_amd as gpcg
    inst = make()
    base = name.split("_csr")[0].split("_mixed")[0]
    xs, gs, _ = reference(base, inst)
    tol, bar = (TIGHT, 1e-8) if prec == 0 else (1e-10, 1e-6)
    x, g, st = G.solve(inst, kind, precision=prec, tol_rel=tol,
                       precond=gpcg.GPCG_PRECOND_JACOBI)
    err = G.rel_inf(x, xs)
    print(f"jacobi {name}: status={st['status']} cg={st['cg_iters']} err={err:.2e}", flush=True)
    assert st["status"] == gpcg.GPCG_OK, st
    assert np.all(x >= inst.l) and np.all(x <= inst.u)
    assert err <= bar
    check_faces(x, xs, gs, inst)


def test_jacobi_cuts_cg_iterations_like_the_oracle():
    """On a strongly varying coefficient the preconditioner cuts the CG
    iterations, on the GPU as in the oracle (counts within 20 %)."""
    import paper_cs_0101018_amd as gpcg
    inst = instances.varcoef(90, 1, eps=0.9)
    _, _, s0 = G.solve(inst)
    _, _, s1 = G.solve(inst, precond=gpcg.GPCG_PRECOND_JACOBI)
    _, _, o1 = oracle.default().solve_instance(inst, precond=1)
    print(f"cg iterations: plain {s0['cg_iters']}, jacobi {s1['cg_iters']}, "
          f"oracle jacobi {o1['cg_iters']}", flush=True)
    assert s1["cg_iters"] < 0.5 * s0["cg_iters"]
    assert abs(s1["cg_iters"] - o1["cg_iters"]) <= 0.2 * o1["cg_iters"] + 5


@pytest.mark.parametrize("prec", [0, 1])
def test_jacobi_forms_bitwise(prec):
    import paper_cs_0101018_amd as gpcg
    inst = instances.varcoef(77, 4, eps=0.5)
    J = gpcg.GPCG_PRECOND_JACOBI
    res = [G.solve(inst, precision=prec, precond=J, form=gpcg.GPCG_FORM_FUSED),
           G.solve(inst, precision=prec, precond=J, form=gpcg.GPCG_FORM_SPLIT),
           G.solve(inst, precision=prec, precond=J, form=gpcg.GPCG_FORM_SPLIT, tiles_per_wg=3),
           G.solve(inst, precision=prec, precond=J, prefetch=gpcg.GPCG_PREFETCH_OFF),
           G.solve(inst, "csr", precision=prec, precond=J)]
    x0 = res[0][0]
    assert res[0][2]["status"] == gpcg.GPCG_OK
    for x, _, st in res[1:4]:
        assert np.array_equal(x, x0)
        assert st["cg_iters"] == res[0][2]["cg_iters"]
    # the CSR operator assembles the same matrix; its sums run in another order
    assert G.rel_inf(res[4][0], x0) <= 1e-6


@pytest.mark.parametrize("mode", [0, 1], ids=["stepped", "persistent"])
def test_jacobi_batch_equals_alone(mode):
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    J = gpcg.GPCG_PRECOND_JACOBI
    insts = [instances.varcoef(40, 2, eps=0.9), instances.obstacle(55, 3),
             instances.varcoef(63, 5)]
    precs = [J, 0, J]  # a batch may mix preconditioned and plain QPs
    alone = [G.solve(i, precond=p)[0] for i, p in zip(insts, precs)]
    solvers = [gpcg.Solver(G.operator_for(i), device=dev, precond=p) for i, p in zip(insts, precs)]
    xs = [G.to_dev(i.x0) for i in insts]
    probs = [(G.to_dev(i.b), G.to_dev(i.l), G.to_dev(i.u), x) for i, x in zip(insts, xs)]
    bt = gpcg.Batch(solvers, device=dev)
    stats = bt.solve(probs, mode=mode)
    torch.cuda.synchronize()
    for x, a, st in zip(xs, alone, stats):
        assert st["status"] == gpcg.GPCG_OK
        assert np.array_equal(x.cpu().numpy(), a)
    bt.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("name,make,prec,pc", [
    ("c0", lambda: instances.obstacle50(0), 0, 0),
    ("c1", lambda: instances.varcoef256(0), 0, 0),
    ("c1_jacobi", lambda: instances.varcoef256(0), 0, 1),
    ("c1_mixed", lambda: instances.varcoef256(0), 1, 0),
])
def test_residual_cg_stop_matches_oracle(name, make, prec, pc):
    """The residual CG test (cg_stop = GPCG_CGSTOP_RESIDUAL) against the
    polished x*; its CG counts track the oracle's with the same test."""
    import paper_cs_0101018_amd as gpcg
    inst = make()
    xs, gs, _ = reference(name.split("_")[0], inst)
    tol, bar = (TIGHT, 1e-8) if prec == 0 else (1e-10, 1e-6)
    x, g, st = G.solve(inst, precision=prec, tol_rel=tol, precond=pc,
                       cg_stop=gpcg.GPCG_CGSTOP_RESIDUAL)
    err = G.rel_inf(x, xs)
    print(f"residual stop {name}: status={st['status']} cg={st['cg_iters']} err={err:.2e}",
          flush=True)
    assert st["status"] == gpcg.GPCG_OK, st
    assert err <= bar
    check_faces(x, xs, gs, inst)
    if prec == 0:
        _, _, so = oracle.default().solve_instance(inst, precond=pc, cg_stop=1)
        _, _, sg = G.solve(inst, precond=pc, cg_stop=gpcg.GPCG_CGSTOP_RESIDUAL)
        assert abs(sg["cg_iters"] - so["cg_iters"]) <= 0.2 * so["cg_iters"] + 5, (sg, so)
    # the launch forms agree bitwise under this test as well
    xa, _, _ = G.solve(inst, precision=prec, precond=pc, cg_stop=1, form=gpcg.GPCG_FORM_FUSED)
    xb, _, _ = G.solve(inst, precision=prec, precond=pc, cg_stop=1, form=gpcg.GPCG_FORM_SPLIT)
    assert np.array_equal(xa, xb)
