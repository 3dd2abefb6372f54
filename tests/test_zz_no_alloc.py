"""The allocation-free projected-gradient entry point against the one with a
handle and workspace, through the C ABI: two calls in a row on one GPU (the
second smaller, so that it finds the first call's partial sums in the shared
scratch array), each bitwise equal to gpcg_projected_gradient and to the
oracle's elementwise definitions."""
import numpy as np
import pytest

import oracle
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _case(n, seed):
    rng = np.random.default_rng(seed)
    a, c = rng.standard_normal(n), rng.standard_normal(n)
    l, u = np.minimum(a, c), np.maximum(a, c)
    l[rng.uniform(size=n) < 0.1] = -np.inf
    u[rng.uniform(size=n) < 0.1] = np.inf
    fx = rng.uniform(size=n) < 0.05
    u[fx] = l[fx]
    x = np.clip(rng.standard_normal(n), l, u)
    pick = rng.uniform(size=n)
    x = np.where(pick < 0.3, np.where(np.isfinite(l), l, x), x)
    x = np.where(pick > 0.8, np.where(np.isfinite(u), u, x), x)
    g = rng.standard_normal(n)
    g[rng.uniform(size=n) < 0.05] = 0.0
    return x, l, u, g


def _with_handle(gpcg, torch, dev, x, l, u, g):
    n = len(x)
    s = gpcg.Solver(gpcg.Operator.csr(G.to_dev(np.arange(n + 1, dtype=np.int32)),
                                      G.to_dev(np.arange(n, dtype=np.int32)),
                                      G.to_dev(np.ones(n))), device=dev)
    pg = torch.empty(n, dtype=torch.float64, device=dev)
    out = s.projected_gradient(G.to_dev(x), G.to_dev(l), G.to_dev(u), G.to_dev(g), pg)
    torch.cuda.synchronize()
    s.close()
    return out, pg.cpu().numpy()


def test_noalloc_matches_workspace_entry_point():
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    ora = oracle.default()
    # 3,000,001 unknowns fill all 2048 workgroups of partial sums; the second
    # call's 70,001 use 69 of them and must not pick up the first call's rest
    for n, seed in ((3_000_001, 11), (70_001, 12)):
        print(f"noalloc projected gradient n={n} seed={seed}", flush=True)
        x, l, u, g = _case(n, seed)
        ref, pg_ref = _with_handle(gpcg, torch, dev, x, l, u, g)
        pg = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
        got = gpcg.projected_gradient_noalloc(G.to_dev(x), G.to_dev(l), G.to_dev(u),
                                              G.to_dev(g), pg)
        torch.cuda.synchronize()
        assert got == ref, (got, ref)  # the same kernels and grid: bitwise the same sums
        pg_got = pg.cpu().numpy()
        assert np.array_equal(pg_got, pg_ref)
        want = ora.proj_gradient(x, l, u, g)
        assert np.array_equal(pg_got, want)
        assert got[1:] == ora.classify(x, l, u, g)
        assert np.isclose(got[0], np.sum(want * want), rtol=1e-13)
    # without the pg output and on a stream of its own
    x, l, u, g = _case(1000, 13)
    ref, _ = _with_handle(gpcg, torch, dev, x, l, u, g)
    st = torch.cuda.Stream(device=dev)
    xd, ld, ud, gd = (G.to_dev(a) for a in (x, l, u, g))
    torch.cuda.synchronize()
    got = gpcg.projected_gradient_noalloc(xd, ld, ud, gd, None, stream=st)
    assert got == ref
