"""Helpers for the GPU tests: instances to device tensors and solvers."""
from __future__ import annotations

import numpy as np

import instances


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def to_dev(a, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def operator_for(inst, kind=None):
    """The instance's operator as a device Operator: 'const', 'var' or 'csr'."""
    import paper_cs_0101018_amd as gpcg
    kind = kind or inst.op
    if kind == "csr" or inst.op == "csr":
        rowptr, colind, vals = inst.csr()
        return gpcg.Operator.csr(to_dev(rowptr), to_dev(colind), to_dev(vals))
    if kind == instances.OP_CONST:
        return gpcg.Operator.stencil_const(inst.N, inst.N, inst.w)
    wx, wy = inst.edge_weights()
    return gpcg.Operator.stencil_var(inst.N, inst.N, to_dev(wx.ravel()), to_dev(wy.ravel()))


def solve(inst, kind=None, **opts):
    """Solve on the GPU; returns (x numpy, g numpy, stats)."""
    import paper_cs_0101018_amd as gpcg
    torch, dev = torch_dev()
    op = operator_for(inst, kind)
    s = gpcg.Solver(op, device=dev, **opts)
    x = to_dev(inst.x0)
    g = torch.empty_like(x)
    st = s.solve(to_dev(inst.b), to_dev(inst.l), to_dev(inst.u), x, g)
    torch.cuda.synchronize()
    out = x.cpu().numpy(), g.cpu().numpy(), st
    s.close()
    return out


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
