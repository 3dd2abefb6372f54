"""Building blocks of the HIP path against the oracle (through the C ABI)."""
import numpy as np
import pytest

import instances
import oracle
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 4, 37, 50, 64, 129]


def _inst(N, op, seed=0):
    if op == instances.OP_VAR:
        return instances.varcoef(N, seed)
    return instances.obstacle(N, seed)


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("kind", ["const", "var", "csr"])
def test_spmv_fp64(N, kind):
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    base = instances.OP_VAR if kind == "var" else instances.OP_CONST
    inst = _inst(N, base)
    print(f"spmv fp64 N={N} kind={kind}", flush=True)
    s = gpcg.Solver(G.operator_for(inst, kind), device=dev)
    rng = np.random.default_rng(N)
    v = rng.standard_normal(inst.n)
    ref = oracle.default().matvec(inst.csr(), v)
    vd = G.to_dev(v)
    y = torch.empty_like(vd)
    s.spmv(vd, y)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    scale = np.abs(inst.csr()[2]).max() * np.abs(v).max()
    assert np.abs(got - ref).max() <= 1e-14 * scale * 8
    mask = (rng.uniform(size=inst.n) < 0.6).astype(np.uint8)
    s.spmv(vd, y, G.to_dev(mask))
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    assert np.all(got[mask == 0] == 0.0)
    assert np.abs(got - ref * mask).max() <= 1e-14 * scale * 8
    s.close()


@pytest.mark.parametrize("N", [61, 64])
@pytest.mark.parametrize("kind", ["const", "var", "csr"])
def test_spmv_fp32(N, kind):
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    base = instances.OP_VAR if kind == "var" else instances.OP_CONST
    inst = _inst(N, base)
    s = gpcg.Solver(G.operator_for(inst, kind), device=dev, precision=gpcg.GPCG_PREC_MIXED)
    v = np.random.default_rng(1).standard_normal(inst.n).astype(np.float32)
    ref = oracle.default().matvec(inst.csr(), v.astype(np.float64))
    vd = G.to_dev(v)
    y = torch.empty_like(vd)
    s.spmv(vd, y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    scale = np.abs(inst.csr()[2]).max() * np.abs(v).max()
    assert np.abs(got - ref).max() <= 1e-5 * scale
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["const", "var"])
@pytest.mark.parametrize("N", [2, 4, 8, 100])
def test_spmv_vector_kernel_bitwise(N, kind, prec):
    """The vector-load stencil kernel (grid width a multiple of the vector
    width, aligned arrays) and the scalar kernel (the same arrays at an odd
    element offset) give bitwise equal products, masked and unmasked."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    base = instances.OP_VAR if kind == "var" else instances.OP_CONST
    inst = _inst(N, base, seed=3)
    s = gpcg.Solver(G.operator_for(inst, kind), device=dev, precision=prec)
    dt = torch.float32 if prec else torch.float64
    rng = np.random.default_rng(N)
    n = inst.n
    v = torch.from_numpy(rng.standard_normal(n)).to(dt).to(dev)
    m = torch.from_numpy((rng.uniform(size=n) < 0.6).astype(np.uint8)).to(dev)
    vb = torch.zeros(n + 1, dtype=dt, device=dev)
    mb = torch.zeros(n + 1, dtype=torch.uint8, device=dev)
    vb[1:] = v
    mb[1:] = m
    for mask, mask_odd in ((None, None), (m, mb[1:])):
        y_vec = torch.empty(n, dtype=dt, device=dev)
        y_odd = torch.zeros(n + 1, dtype=dt, device=dev)
        s.spmv(v, y_vec, mask)
        s.spmv(vb[1:], y_odd[1:], mask_odd)
        torch.cuda.synchronize()
        assert torch.equal(y_vec, y_odd[1:])
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["const", "var"])
def test_spmv_row_marching_large_grid(kind, prec):
    """Grids whose v, y and mask exceed the 256 MB last-level cache take the
    row-marching kernel (rows of v kept in registers, neighbours from adjacent
    lanes).  Its product equals the one-row scalar kernel's bitwise (the same
    arrays at an odd element offset), masked, and the oracle's product on
    sampled rows: the grid border, the ragged last segment and row block, and
    rows inside."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    # FP64: 17 B per unknown, 4098^2 = 16.8 M unknowns (285 MB), 4098 = 8 * 512 + 2
    # FP32: 9 B per unknown, 5464^2 = 29.9 M unknowns (269 MB), 5464 = 5 * 1024 + 344
    N = 5464 if prec else 4098
    n = N * N
    print(f"spmv row marching N={N} kind={kind} prec={prec}", flush=True)
    if kind == "var":
        wx, wy = instances.varcoef_weights(N)
        rng_w = np.random.default_rng(5)
        wx = wx * rng_w.uniform(0.5, 1.5, size=wx.shape)
        wy = wy * rng_w.uniform(0.5, 1.5, size=wy.shape)
        op = gpcg.Operator.stencil_var(N, N, G.to_dev(wx.ravel()), G.to_dev(wy.ravel()))
    else:
        w = float((N + 1) ** 2)
        wx, wy = np.full((N, N + 1), w), np.full((N + 1, N), w)
        op = gpcg.Operator.stencil_const(N, N, w)
    s = gpcg.Solver(op, device=dev, precision=prec)
    dt = torch.float32 if prec else torch.float64
    rng = np.random.default_rng(N + prec)
    v_np = rng.standard_normal(n).astype(np.float32 if prec else np.float64)
    m_np = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    v = torch.from_numpy(v_np).to(dev)
    m = torch.from_numpy(m_np).to(dev)
    vb = torch.zeros(n + 1, dtype=dt, device=dev)
    mb = torch.zeros(n + 1, dtype=torch.uint8, device=dev)
    vb[1:] = v
    mb[1:] = m
    jrows = sorted({0, 1, 2, 3, 4, 5, N // 2 - 1, N // 2, N // 2 + 1, N - 3, N - 2, N - 1})
    rows = (np.asarray(jrows, dtype=np.int64)[:, None] * N + np.arange(N)[None, :]).ravel()
    ref = oracle.default().matvec(instances.stencil_csr(N, wx, wy, rows),
                                  v_np.astype(np.float64))[rows]
    scale = 4.0 * max(wx.max(), wy.max()) * np.abs(v_np).max()
    tol = 1e-5 * scale if prec else 8e-14 * scale
    for mask, mask_odd in ((None, None), (m, mb[1:])):
        y_vec = torch.empty(n, dtype=dt, device=dev)
        y_odd = torch.zeros(n + 1, dtype=dt, device=dev)
        s.spmv(v, y_vec, mask)
        s.spmv(vb[1:], y_odd[1:], mask_odd)
        torch.cuda.synchronize()
        assert torch.equal(y_vec, y_odd[1:])
        got = y_vec.cpu().numpy().astype(np.float64)[rows]
        want = ref if mask is None else ref * m_np[rows]
        if mask is not None:
            assert np.all(got[m_np[rows] == 0] == 0.0)
        assert np.abs(got - want).max() <= tol
        del y_vec, y_odd
    s.close()


def test_spmv_bench_size_8192():
    """The SpMV bandwidth figure's largest grid (8192^2, constant stencil, FP64,
    mask of ones as timed): the row-marching product equals the one-row
    kernel's bitwise and the oracle's product on sampled rows."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    N = 8192
    n = N * N
    print(f"spmv bench size N={N}", flush=True)
    w = float((N + 1) ** 2)
    s = gpcg.Solver(gpcg.Operator.stencil_const(N, N, w), device=dev)
    v = torch.randn(n, dtype=torch.float64, device=dev)
    m = torch.ones(n, dtype=torch.uint8, device=dev)
    y = torch.empty_like(v)
    s.spmv(v, y, m)
    vb = torch.zeros(n + 1, dtype=torch.float64, device=dev)
    mb = torch.zeros(n + 1, dtype=torch.uint8, device=dev)
    vb[1:] = v
    mb[1:] = m
    y_odd = torch.zeros(n + 1, dtype=torch.float64, device=dev)
    s.spmv(vb[1:], y_odd[1:], mb[1:])
    torch.cuda.synchronize()
    assert torch.equal(y, y_odd[1:])
    del vb, mb, y_odd
    jrows = [0, 1, 3, 4, 5, N // 2, N - 5, N - 4, N - 1]
    rows = (np.asarray(jrows, dtype=np.int64)[:, None] * N + np.arange(N)[None, :]).ravel()
    wx, wy = np.full((N, N + 1), w), np.full((N + 1, N), w)
    v_np = v.cpu().numpy()
    ref = oracle.default().matvec(instances.stencil_csr(N, wx, wy, rows), v_np)[rows]
    got = y.cpu().numpy()[rows]
    assert np.abs(got - ref).max() <= 8e-14 * 4.0 * w * np.abs(v_np).max()
    s.close()


@pytest.mark.parametrize("offset", [0, 1], ids=["aligned16", "aligned8"])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 5000, 70001, 5_000_001])
def test_projected_gradient_exact(n, offset):
    """Projected gradient and face counts are compare/select work: bit-exact.
    offset 1 passes arrays one element into their buffers (8-byte aligned
    only): the kernel's 8-byte-load path instead of its unknown-pair path."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = G.torch_dev()
    rng = np.random.default_rng(n)
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
    ora = oracle.default()
    inst = instances.obstacle(1, 0)
    s = gpcg.Solver(gpcg.Operator.csr(G.to_dev(np.arange(n + 1, dtype=np.int32)),
                                      G.to_dev(np.arange(n, dtype=np.int32)),
                                      G.to_dev(np.ones(n))), device=dev)
    def dev_vec(a):
        t = torch.zeros(n + offset, dtype=torch.float64, device=dev)
        t[offset:] = G.to_dev(a)
        return t[offset:]
    pg = dev_vec(np.zeros(n))
    n2, lo, up, nb = s.projected_gradient(dev_vec(x), dev_vec(l), dev_vec(u), dev_vec(g), pg)
    want = ora.proj_gradient(x, l, u, g)
    assert np.array_equal(pg.cpu().numpy(), want)
    assert (lo, up, nb) == ora.classify(x, l, u, g)
    assert np.isclose(n2, np.sum(want * want), rtol=1e-13)
    s.close()
