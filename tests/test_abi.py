"""The C ABI library loads and exports every function include/gpcg.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpcg.h")
LIB = os.path.join(ROOT, "paper_cs_0101018_amd", "libgpcg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpcg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gpcg_create", "gpcg_solve", "gpcg_destroy", "gpcg_workspace_bytes",
                 "gpcg_batch_solve", "gpcg_server_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libgpcg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_cs_0101018_amd as gpcg
    assert sorted(gpcg.EXPORTED) == declared_functions()


def test_host_side_validation_without_gpu():
    """Descriptor and option checks run on the host before any device call."""
    import paper_cs_0101018_amd as gpcg
    op = gpcg.gpcg_operator(kind=gpcg.GPCG_OP_STENCIL5_CONST, nx=10, ny=10, w=-1.0)
    nbytes = ctypes.c_size_t()
    rc = gpcg.gpcg_workspace_bytes(ctypes.byref(op), None, ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_ERR_ARG
    op.w = 121.0
    rc = gpcg.gpcg_workspace_bytes(ctypes.byref(op), None, ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_OK and nbytes.value > 100 * 8 * 6
    opt = gpcg.default_options(mu=0.7)
    rc = gpcg.gpcg_workspace_bytes(ctypes.byref(op), ctypes.byref(opt), ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_ERR_ARG
    opt = gpcg.default_options(tile=300)
    rc = gpcg.gpcg_workspace_bytes(ctypes.byref(op), ctypes.byref(opt), ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_ERR_ARG
    # a workspace that is too small is refused before any device work
    h = ctypes.c_void_p()
    rc = gpcg.gpcg_create(ctypes.byref(op), None, ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert rc == gpcg.GPCG_ERR_WORKSPACE
    # the server refuses CSR operators and over-sized requests up front
    csr = gpcg.gpcg_operator(kind=gpcg.GPCG_OP_CSR, n=4, nnz=4, rowptr=8, colind=8, vals=8)
    rc = gpcg.gpcg_server_footprint(ctypes.byref(csr), 0, ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_ERR_ARG
    assert gpcg.status_string(gpcg.GPCG_ERR_NOT_SPD).startswith("operator")


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_default_tile_rule(mixed):
    """The library's tile is a function of n and the precision alone: 256
    unknowns up to 1024 tiles of 256, then 512, then 1024 once the grid holds
    8192 tiles of 1024 (mixed: 1024 of them), and 2048 once it holds 8192
    tiles of 2048.  The workspace holds one slot block per tile, so the
    default layout matches the explicit tile the rule names and no other."""
    import paper_cs_0101018_amd as gpcg
    nbytes = ctypes.c_size_t()
    prec = gpcg.GPCG_PREC_MIXED if mixed else gpcg.GPCG_PREC_FP64

    def ws(nx, ny, tile):
        op = gpcg.gpcg_operator(kind=gpcg.GPCG_OP_STENCIL5_CONST, nx=nx, ny=ny, w=121.0)
        opt = gpcg.default_options(tile=tile, precision=prec)
        assert gpcg.gpcg_workspace_bytes(ctypes.byref(op), ctypes.byref(opt),
                                         ctypes.byref(nbytes)) == gpcg.GPCG_OK
        return nbytes.value

    cases = [((512, 512), 256), ((512, 513), 512), ((1024, 1023), 512),
             ((1024, 1024), 1024 if mixed else 512), ((1600, 1600), 1024 if mixed else 512),
             ((2048, 4095), 1024 if mixed else 512), ((2048, 4096), 1024),
             ((4096, 4095), 1024), ((4096, 4096), 2048), ((8192, 8192), 2048)]
    for (nx, ny), tile in cases:
        auto = ws(nx, ny, 0)
        assert auto == ws(nx, ny, tile), (nx, ny, tile)
        for other in {256, 512, 1024, 2048} - {tile}:
            assert auto != ws(nx, ny, other), (nx, ny, other)


def test_free_set_forms_host_checks():
    """The matrix free set needs a CSR operator and 256-unknown tiles; its
    workspace holds A_F (row offsets, column indices, values) on top of the
    list form's."""
    import paper_cs_0101018_amd as gpcg
    nbytes = ctypes.c_size_t()
    stencil = gpcg.gpcg_operator(kind=gpcg.GPCG_OP_STENCIL5_CONST, nx=10, ny=10, w=121.0)
    opt = gpcg.default_options(free_set=gpcg.GPCG_FREESET_MATRIX)
    rc = gpcg.gpcg_workspace_bytes(ctypes.byref(stencil), ctypes.byref(opt), ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_ERR_ARG
    n, nnz = 1000, 4960
    csr = gpcg.gpcg_operator(kind=gpcg.GPCG_OP_CSR, n=n, nnz=nnz, rowptr=8, colind=8, vals=8)
    sizes = {}
    for fs in (gpcg.GPCG_FREESET_MASK, gpcg.GPCG_FREESET_LIST, gpcg.GPCG_FREESET_MATRIX):
        opt = gpcg.default_options(free_set=fs)
        rc = gpcg.gpcg_workspace_bytes(ctypes.byref(csr), ctypes.byref(opt), ctypes.byref(nbytes))
        assert rc == gpcg.GPCG_OK
        sizes[fs] = nbytes.value
    assert sizes[gpcg.GPCG_FREESET_LIST] >= sizes[gpcg.GPCG_FREESET_MASK] + 4 * n
    assert sizes[gpcg.GPCG_FREESET_MATRIX] >= sizes[gpcg.GPCG_FREESET_LIST] + 4 * (n + 1) + 12 * nnz
    opt = gpcg.default_options(free_set=gpcg.GPCG_FREESET_MATRIX, tile=512)
    rc = gpcg.gpcg_workspace_bytes(ctypes.byref(csr), ctypes.byref(opt), ctypes.byref(nbytes))
    assert rc == gpcg.GPCG_ERR_ARG


def test_binding_rejects_bad_tensors_before_the_library():
    """The binding checks device, dtype, contiguity and length of every array
    before a pointer reaches the C ABI (a wrong one would make the kernels read
    or write out of bounds)."""
    import torch
    import paper_cs_0101018_amd as gpcg
    f64 = (torch.float64,)
    with pytest.raises(ValueError, match="GPU"):
        gpcg._check_vec(torch.zeros(10, dtype=torch.float64), 10, f64, "b")
    with pytest.raises(ValueError, match="required"):
        gpcg._check_vec(None, 10, f64, "x")
    gpcg._check_vec(None, 10, f64, "g_out", optional=True)
    with pytest.raises(ValueError, match="torch tensor"):
        gpcg._check_vec([0.0] * 10, 10, f64, "l")


class _FakeCudaTensor:
    """Enough of a torch.Tensor's interface for the checks, on a 'cuda' device."""

    def __init__(self, t, device="cuda"):
        self._t = t
        self.device = torch_device(device)
        self.dtype = t.dtype

    def is_contiguous(self):
        return self._t.is_contiguous()

    def numel(self):
        return self._t.numel()


def torch_device(s):
    import torch
    return torch.device(s)


def test_binding_checks_dtype_contiguity_and_length(monkeypatch):
    import torch
    import paper_cs_0101018_amd as gpcg
    monkeypatch.setattr(torch, "Tensor", _FakeCudaTensor)
    f64 = (torch.float64,)
    ok = _FakeCudaTensor(torch.zeros(12, dtype=torch.float64))
    gpcg._check_vec(ok, 12, f64, "x")
    with pytest.raises(ValueError, match="12 elements"):
        gpcg._check_vec(_FakeCudaTensor(torch.zeros(11, dtype=torch.float64)), 12, f64, "x")
    with pytest.raises(ValueError, match="dtype"):
        gpcg._check_vec(_FakeCudaTensor(torch.zeros(12, dtype=torch.float32)), 12, f64, "x")
    with pytest.raises(ValueError, match="contiguous"):
        gpcg._check_vec(_FakeCudaTensor(torch.zeros(24, dtype=torch.float64)[::2]), 12, f64, "x")


def test_noalloc_size_limit_checked_on_host():
    """The allocation-free entry point refuses sizes outside [1, GPCG_NOALLOC_MAX_N]
    before any device work (the pointers below are never dereferenced)."""
    import paper_cs_0101018_amd as gpcg
    fake = ctypes.c_void_p(4096)
    n2 = ctypes.c_double()
    for n in (0, -5, gpcg.GPCG_NOALLOC_MAX_N + 1):
        rc = gpcg.gpcg_projected_gradient_noalloc(n, fake, fake, fake, fake, None,
                                                  ctypes.byref(n2), None, None, None, None)
        assert rc == gpcg.GPCG_ERR_ARG
        assert "n must be in" in gpcg.gpcg_last_error().decode()
