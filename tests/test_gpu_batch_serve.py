"""Batched and served solves equal the same QP solved alone (bitwise: each QP
keeps its own tile size, so its reductions run in the same order), and match
the oracle."""
import numpy as np
import pytest

import instances
import oracle
from oracle import exact
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def mix(count, seed=7, nmin=20, nmax=90):
    children = np.random.SeedSequence(seed).spawn(count)
    return [instances._mixed_member(c, nmin, nmax, i) for i, c in enumerate(children)]


def solo(inst, **opts):
    return G.solve(inst, **opts)


def _batch(insts, mode, **opts):
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    solvers = [gpcg.Solver(G.operator_for(i), device=dev, **opts) for i in insts]
    batch = gpcg.Batch(solvers, device=dev)
    data = [(G.to_dev(i.b), G.to_dev(i.l), G.to_dev(i.u), G.to_dev(i.x0)) for i in insts]
    stats = batch.solve(data, mode=mode)
    torch.cuda.synchronize()
    xs = [d[3].cpu().numpy() for d in data]
    batch.close()
    for s in solvers:
        s.close()
    return xs, stats


@pytest.mark.parametrize("mixed", [0, 1])
@pytest.mark.parametrize("mode,form", [(0, 1), (0, 2), (1, 0)],
                         ids=["stepped_fused", "stepped_split", "persistent"])
def test_batch_equals_alone(mode, form, mixed):
    """Stepped batches in the fused form (one launch per pass, every
    workgroup folds its own QP's slots) and in the split form, and the
    persistent form."""
    insts = mix(9, seed=11 + mixed)
    print(f"batch mode={mode} form={form} mixed={mixed} sizes={[i.N for i in insts]}", flush=True)
    xs, stats = _batch(insts, mode, precision=mixed, form=form)
    for inst, x, st in zip(insts, xs, stats):
        xa, ga, sa = solo(inst, precision=mixed)
        assert st["status"] == sa["status"] == 0, (st, sa)
        assert np.array_equal(x, xa), inst.name
        for k in ("outer_iters", "gp_iters", "cg_iters"):
            assert st[k] == sa[k], (inst.name, k)
        # batches never look ahead; a QP alone (fused form) may
        assert st["passes"] == sa["passes"] + sa["lookaheads"], inst.name


@pytest.mark.parametrize("cgk", [0, 1], ids=["one_data_kernel", "cg_kernel"])
@pytest.mark.parametrize("mixed", [0, 1])
def test_batch_equals_alone_many_tiles(mixed, cgk):
    """Members with more tiles than threads per workgroup (their slot sums
    have tails): the batch (split form) equals each one alone (fused form),
    with the CG iterations in the data kernel of every pass or in one of
    their own."""
    import paper_cs_0101018_amd as gpcg
    insts = [instances.obstacle(300, 4, amplitude=0.4), instances.varcoef(270, 1),
             instances.obstacle(45, 2), instances.obstacle(560, 3)]  # 560^2: 512-unknown tiles
    ck = gpcg.GPCG_CGK_ON if cgk else gpcg.GPCG_CGK_OFF
    xs, stats = _batch(insts, 0, precision=mixed, cg_kernel=ck, form=gpcg.GPCG_FORM_SPLIT)
    for inst, x, st in zip(insts, xs, stats):
        xa, ga, sa = solo(inst, precision=mixed)
        assert st["status"] == sa["status"] == 0, (st, sa)
        assert np.array_equal(x, xa), inst.name
        assert st["cg_iters"] == sa["cg_iters"], inst.name


@pytest.mark.parametrize("mixed", [0, 1])
def test_batch_fused_many_tiles(mixed):
    """The fused form of a stepped batch with members whose slot sums have
    tails (more tiles than threads per workgroup, 512-unknown tiles): each
    workgroup folds its own QP's slots; bitwise each QP alone."""
    import paper_cs_0101018_amd as gpcg
    insts = [instances.obstacle(300, 4, amplitude=0.4), instances.obstacle(45, 2),
             instances.obstacle(560, 3), instances.varcoef(130, 5)]
    xs, stats = _batch(insts, 0, precision=mixed, form=gpcg.GPCG_FORM_FUSED)
    for inst, x, st in zip(insts, xs, stats):
        xa, ga, sa = solo(inst, precision=mixed)
        assert st["status"] == sa["status"] == 0, (st, sa)
        assert np.array_equal(x, xa), inst.name
        assert st["cg_iters"] == sa["cg_iters"], inst.name


def test_batch_matches_oracle():
    insts = mix(5, seed=3)
    xs, stats = _batch(insts, 1, tol_rel=1e-12)
    ora = oracle.default()
    for inst, x in zip(insts, xs):
        xo, _, _ = ora.solve_instance(inst, tol_rel=1e-12)
        xstar, info = exact.polish(inst.csr(), inst.b, inst.l, inst.u, xo)
        assert G.rel_inf(x, xstar) <= 1e-8, inst.name


def test_server_mix_equals_alone():
    """Requests admitted while others run (4 slots, more requests than fit),
    each answer bitwise equal to the same request solved alone."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    insts = mix(14, seed=5, nmin=16, nmax=64)
    ops = [G.operator_for(i) for i in insts]
    foot = [gpcg.Server.footprint(o, gpcg.GPCG_PREC_MIXED) for o in ops]
    arena = 3 * max(foot) + 65536
    srv = gpcg.Server(arena, max_slots=4, precision=gpcg.GPCG_PREC_MIXED, tol_rel=1e-8,
                      quantum=16, device=dev)
    outs = {}
    for k, (inst, op) in enumerate(zip(insts, ops)):
        x_out = torch.zeros(inst.n, dtype=torch.float64, device=dev)
        outs[k] = x_out
        rc = srv.submit(k, op, G.to_dev(inst.b), G.to_dev(inst.l), G.to_dev(inst.u),
                        G.to_dev(inst.x0), x_out)
        assert rc == 0
    done = []
    max_resident = 0
    for _ in range(100000):
        active = srv.step()
        done += srv.poll()
        if active == 0:
            break
    assert len(done) == len(insts)
    admits = sorted(c["t_admit"] for c in done)
    finishes = sorted(c["t_done"] for c in done)
    # continuous batching: some request was admitted after another finished
    assert admits[-1] >= finishes[0]
    for c in done:
        inst = insts[c["tag"]]
        assert c["status"] == 0
        xa, ga, sa = solo(inst, precision=gpcg.GPCG_PREC_MIXED, tol_rel=1e-8,
                          tile=gpcg.GPCG_SERVER_TILE)
        assert np.array_equal(outs[c["tag"]].cpu().numpy(), xa), inst.name
        assert c["stats"]["cg_iters"] == sa["cg_iters"]
    # a request that can never fit is refused
    big = instances.obstacle(400, 0)
    op = gpcg.Operator.stencil_const(400, 400, big.w)
    z = torch.zeros(big.n, dtype=torch.float64, device=dev)
    assert srv.submit(999, op, z, z, z, z, z) == gpcg.GPCG_ERR_NOSPACE
    srv.close()
