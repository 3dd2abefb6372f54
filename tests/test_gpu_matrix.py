"""The matrix free set (free_set = MATRIX, CSR operators): once per CG phase
the reduced matrix A_F of the paper's technique 1 is written out as CSR over
the free list (a count pass and a fill pass after the list pass), and every CG
iteration reads only its nonzeros.  Against the polished oracle x* to the
parity bar, and bitwise against the list form: the products skip only terms
whose vector entry is an exact zero, in the same order."""
import numpy as np
import pytest

import instances
from tests import gpu_util as G
from tests.test_gpu_solve import TIGHT, check_faces, reference

pytestmark = pytest.mark.gpu

CASES = [
    ("c0", lambda: instances.obstacle50(0), 0),
    ("c1", lambda: instances.varcoef256(0), 0),
    ("obst_ragged", lambda: instances.obstacle(77, 3, amplitude=0.45, u_random=True), 0),
    ("pressed", lambda: instances.pressed(256, 0, load=-2500.0), 0),
    ("c1_mixed", lambda: instances.varcoef256(0), 1),
    ("pressed_mixed", lambda: instances.pressed(256, 0, load=-2500.0), 1),
]


@pytest.mark.parametrize("name,make,prec", CASES, ids=[c[0] for c in CASES])
def test_matrix_form_matches_oracle_and_list(name, make, prec):
    import paper_cs_0101018_amd as gpcg
    inst = make()
    base = name.split("_mixed")[0]
    xs, gs, _ = reference(base, inst)
    tol, bar = (TIGHT, 1e-8) if prec == 0 else (1e-10, 1e-6)
    print(f"matrix form {name} n={inst.n}", flush=True)
    x, g, st = G.solve(inst, "csr", precision=prec, tol_rel=tol,
                       free_set=gpcg.GPCG_FREESET_MATRIX)
    err = G.rel_inf(x, xs)
    print(f"  status={st['status']} cg={st['cg_iters']} err={err:.2e}", flush=True)
    assert st["status"] == gpcg.GPCG_OK, st
    assert np.all(x >= inst.l) and np.all(x <= inst.u)
    assert err <= bar
    check_faces(x, xs, gs, inst)
    xl, gl, sl = G.solve(inst, "csr", precision=prec, tol_rel=tol,
                         free_set=gpcg.GPCG_FREESET_LIST)
    assert np.array_equal(x, xl) and np.array_equal(g, gl)
    for k in ("outer_iters", "gp_iters", "cg_iters", "cg_phases"):
        assert st[k] == sl[k], k
    # two more passes (count, fill) per CG phase than the list form
    assert st["passes"] + st["lookaheads"] == sl["passes"] + sl["lookaheads"] + 2 * st["cg_phases"]


@pytest.mark.parametrize("prec", [0, 1])
def test_matrix_form_launch_forms_agree(prec):
    import paper_cs_0101018_amd as gpcg
    inst = instances.pressed(300, 2, load=-3000.0)
    res = [G.solve(inst, "csr", precision=prec, free_set=gpcg.GPCG_FREESET_MATRIX, form=f, **o)
           for f, o in ((gpcg.GPCG_FORM_FUSED, {}), (gpcg.GPCG_FORM_SPLIT, {}),
                        (gpcg.GPCG_FORM_SPLIT, {"tiles_per_wg": 3}),
                        (gpcg.GPCG_FORM_SPLIT, {"cg_kernel": gpcg.GPCG_CGK_ON}))]
    x0, g0, s0 = res[0]
    assert s0["status"] == gpcg.GPCG_OK
    for x, g, st in res[1:]:
        assert np.array_equal(x, x0) and np.array_equal(g, g0)
        assert st["cg_iters"] == s0["cg_iters"]


@pytest.mark.parametrize("mode", [0, 1], ids=["stepped", "persistent"])
def test_matrix_form_in_a_batch(mode):
    """A batch mixing matrix-form CSR members with mask-form stencil members:
    each answer bitwise equal to the same QP solved alone."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    insts = [instances.pressed(120, 1, load=-800.0), instances.obstacle(60, 2),
             instances.varcoef(90, 3), instances.pressed(200, 4, load=-2000.0)]
    kinds = ["csr", None, None, "csr"]
    sets = [gpcg.GPCG_FREESET_MATRIX, gpcg.GPCG_FREESET_MASK, gpcg.GPCG_FREESET_MASK,
            gpcg.GPCG_FREESET_MATRIX]
    solvers = [gpcg.Solver(G.operator_for(i, k), device=dev, free_set=f)
               for i, k, f in zip(insts, kinds, sets)]
    batch = gpcg.Batch(solvers, device=dev)
    data = [(G.to_dev(i.b), G.to_dev(i.l), G.to_dev(i.u), G.to_dev(i.x0)) for i in insts]
    stats = batch.solve(data, mode=mode)
    torch.cuda.synchronize()
    for inst, kind, fs, d, st in zip(insts, kinds, sets, data, stats):
        xa, ga, sa = G.solve(inst, kind, free_set=fs)
        assert st["status"] == sa["status"] == 0
        assert np.array_equal(d[3].cpu().numpy(), xa), inst.name
        assert st["cg_iters"] == sa["cg_iters"], inst.name
    batch.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_matrix_form_with_jacobi_and_residual_stop(prec):
    """The preconditioned CG and the residual stopping test on A_F: bitwise
    the list form's answer."""
    import paper_cs_0101018_amd as gpcg
    inst = instances.varcoef(120, 4, eps=0.5)
    for opts in ({"precond": gpcg.GPCG_PRECOND_JACOBI},
                 {"cg_stop": gpcg.GPCG_CGSTOP_RESIDUAL},
                 {"precond": gpcg.GPCG_PRECOND_JACOBI, "cg_stop": gpcg.GPCG_CGSTOP_RESIDUAL}):
        xm, gm, sm = G.solve(inst, "csr", precision=prec, free_set=gpcg.GPCG_FREESET_MATRIX,
                             **opts)
        xl, gl, sl = G.solve(inst, "csr", precision=prec, free_set=gpcg.GPCG_FREESET_LIST, **opts)
        assert sm["status"] == sl["status"] == gpcg.GPCG_OK, (sm["status"], sl["status"])
        assert np.array_equal(xm, xl) and np.array_equal(gm, gl)
        assert sm["cg_iters"] == sl["cg_iters"]
