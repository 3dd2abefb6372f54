"""MI355X-native GPCG: Python binding of the C ABI in ``include/gpcg.h``.

This module only marshals arguments: every step of the solve runs in the
HIP kernels of ``libgpcg.so`` (built in-tree by ``paper_cs_0101018_amd/build.py``).
PyTorch supplies device memory and streams.  If the library is missing the
import fails; there is no CPU fallback.

Low-level names mirror the C ABI (``gpcg_create``, ``gpcg_solve``, ...).  The
``Solver``, ``Batch`` and ``Server`` classes wrap them for torch tensors.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpcg.so")

# torch is imported first so that the HIP runtime it ships is the one
# libgpcg.so binds to (same SONAME): one process, one HIP runtime.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libgpcg.so not found at {LIB_PATH}; build it with "
        "`python paper_cs_0101018_amd/build.py` (hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
GPCG_OK, GPCG_MAXIT, GPCG_STAGNATED = 0, 1, 2
GPCG_ERR_ARG, GPCG_ERR_BOUNDS, GPCG_ERR_NAN, GPCG_ERR_NOT_SPD = -1, -2, -3, -4
GPCG_ERR_WORKSPACE, GPCG_ERR_HIP, GPCG_ERR_NOSPACE, GPCG_ERR_HANG = -5, -6, -7, -8
GPCG_OP_STENCIL5_CONST, GPCG_OP_STENCIL5_VAR, GPCG_OP_CSR = 1, 2, 3
GPCG_PREC_FP64, GPCG_PREC_MIXED = 0, 1
GPCG_FREESET_MASK, GPCG_FREESET_LIST, GPCG_FREESET_MATRIX = 0, 1, 2
GPCG_BATCH_STEPPED, GPCG_BATCH_PERSISTENT = 0, 1
GPCG_FORM_AUTO, GPCG_FORM_FUSED, GPCG_FORM_SPLIT = 0, 1, 2
GPCG_PREFETCH_AUTO, GPCG_PREFETCH_ON, GPCG_PREFETCH_OFF = 0, 1, 2
GPCG_PRECOND_NONE, GPCG_PRECOND_JACOBI = 0, 1
GPCG_CGSTOP_DECREASE, GPCG_CGSTOP_RESIDUAL = 0, 1
GPCG_LOOKAHEAD_AUTO, GPCG_LOOKAHEAD_ON, GPCG_LOOKAHEAD_OFF = 0, 1, 2
GPCG_CGK_AUTO, GPCG_CGK_ON, GPCG_CGK_OFF = 0, 1, 2
GPCG_SERVER_TILE = 512  # tile of every served request


class gpcg_operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("w", C.c_double),
                ("wx", C.c_void_p), ("wy", C.c_void_p), ("n", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("vals", C.c_void_p)]


class gpcg_options(C.Structure):
    _fields_ = [("tol_rel", C.c_double), ("tol_abs", C.c_double), ("eta1", C.c_double),
                ("eta2", C.c_double), ("eta2_reduce", C.c_double), ("mu", C.c_double),
                ("max_outer", C.c_int32), ("max_gp", C.c_int32), ("max_backtrack", C.c_int32),
                ("max_cg", C.c_int32), ("precision", C.c_int32), ("free_set", C.c_int32),
                ("tile", C.c_int32), ("chunk", C.c_int32), ("use_graph", C.c_int32),
                ("max_stall", C.c_int32), ("form", C.c_int32),
                ("tiles_per_wg", C.c_int32), ("prefetch", C.c_int32),
                ("precond", C.c_int32), ("cg_stop", C.c_int32), ("cg_kernel", C.c_int32),
                ("lookahead", C.c_int32)]


class gpcg_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("gp_iters", C.c_int32),
                ("cg_iters", C.c_int32), ("backtracks", C.c_int32), ("face_repeats", C.c_int32),
                ("cg_phases", C.c_int32), ("x0_projected", C.c_int32), ("pg0", C.c_double),
                ("pg", C.c_double), ("tau", C.c_double), ("q", C.c_double),
                ("n_free", C.c_int64), ("n_lower", C.c_int64), ("n_upper", C.c_int64),
                ("passes", C.c_int64), ("lookaheads", C.c_int64), ("launches", C.c_int64),
                ("host_checks", C.c_int64),
                ("bytes", C.c_double), ("ms_total", C.c_double), ("ms_cg", C.c_double),
                ("ms_gp", C.c_double), ("ms_search", C.c_double), ("ms_other", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gpcg_problem(C.Structure):
    _fields_ = [("b", C.c_void_p), ("l", C.c_void_p), ("u", C.c_void_p), ("x", C.c_void_p),
                ("g_out", C.c_void_p)]


class gpcg_server_options(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("precision", C.c_int32), ("tol_rel", C.c_double), ("quantum", C.c_int32)]


class gpcg_request(C.Structure):
    _fields_ = [("op", gpcg_operator), ("b", C.c_void_p), ("l", C.c_void_p),
                ("u", C.c_void_p), ("x0", C.c_void_p), ("x_out", C.c_void_p),
                ("tag", C.c_uint64)]


class gpcg_completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("stats", gpcg_stats),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


GPCG_TUNE_MAX = 32


class gpcg_tune_entry(C.Structure):
    _fields_ = [("form", C.c_int32), ("tiles_per_wg", C.c_int32), ("prefetch", C.c_int32),
                ("chunk", C.c_int32), ("shrink", C.c_int32), ("cg_kernel", C.c_int32),
                ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gpcg_tune_report(C.Structure):
    _fields_ = [("count", C.c_int32), ("mismatches", C.c_int32), ("chosen", gpcg_tune_entry),
                ("cand", gpcg_tune_entry * GPCG_TUNE_MAX)]

    def as_dict(self):
        return {"count": self.count, "mismatches": self.mismatches,
                "chosen": self.chosen.as_dict(),
                "candidates": [self.cand[i].as_dict() for i in range(self.count)]}


_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_P = C.POINTER
_SIGS = {
    "gpcg_options_default": (None, [_P(gpcg_options)]),
    "gpcg_workspace_bytes": (C.c_int, [_P(gpcg_operator), _P(gpcg_options), _P(_sz)]),
    "gpcg_create": (C.c_int, [_P(gpcg_operator), _P(gpcg_options), _vp, _sz, _vp, _P(_vp)]),
    "gpcg_solve": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _P(gpcg_stats)]),
    "gpcg_destroy": (C.c_int, [_vp]),
    "gpcg_spmv": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gpcg_spmv_f32": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gpcg_projected_gradient": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _P(C.c_double),
                                          _P(_i64), _P(_i64), _P(_i64)]),
    "gpcg_projected_gradient_noalloc": (C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp,
                                                  _P(C.c_double), _P(_i64), _P(_i64),
                                                  _P(_i64), _vp]),
    "gpcg_batch_workspace_bytes": (C.c_int, [C.c_int, C.c_void_p, _P(_sz)]),
    "gpcg_batch_create": (C.c_int, [C.c_int, _P(_vp), _vp, _sz, _vp, _P(_vp)]),
    "gpcg_batch_solve": (C.c_int, [_vp, _P(gpcg_problem), C.c_int, _P(gpcg_stats)]),
    "gpcg_batch_destroy": (C.c_int, [_vp]),
    "gpcg_autotune": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _P(gpcg_tune_report)]),
    "gpcg_batch_autotune": (C.c_int, [_vp, _P(gpcg_problem), _P(_vp), _P(gpcg_tune_report)]),
    "gpcg_server_footprint": (C.c_int, [_P(gpcg_operator), C.c_int, _P(_sz)]),
    "gpcg_server_create": (C.c_int, [_P(gpcg_server_options), _vp, _P(_vp)]),
    "gpcg_server_submit": (C.c_int, [_vp, _P(gpcg_request)]),
    "gpcg_server_step": (C.c_int, [_vp, _P(C.c_int)]),
    "gpcg_server_poll": (C.c_int, [_vp, _P(gpcg_completion), C.c_int, _P(C.c_int)]),
    "gpcg_server_destroy": (C.c_int, [_vp]),
    "gpcg_status_string": (C.c_char_p, [C.c_int]),
    "gpcg_last_error": (C.c_char_p, []),
    "gpcg_build_info": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_SIGS)


class GpcgError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.gpcg_last_error().decode() or _lib.gpcg_status_string(status).decode()
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise GpcgError(status, where)
    return status


# ------------------------------------------------------------ torch helpers

def _torch():
    import torch
    return torch


def _dptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _check_vec(t, n: int, dtypes, name: str, optional: bool = False):
    """Raises ValueError unless t is a contiguous CUDA tensor of one of
    `dtypes` with exactly n elements: the kernels index every array up to n
    and would read or write out of bounds otherwise."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device, got {t.device}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(map(str, dtypes))}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")


def _f64():
    return (_torch().float64,)


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _workspace(nbytes: int, device):
    """A 256-byte aligned device buffer (torch uint8) and its aligned address."""
    torch = _torch()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    return buf, (base + 255) // 256 * 256


def default_options(**kw) -> gpcg_options:
    o = gpcg_options()
    _lib.gpcg_options_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Operator:
    """A device-resident operator description (keeps its tensors alive)."""

    def __init__(self, desc: gpcg_operator, keep: Sequence):
        self.desc = desc
        self.keep = list(keep)

    @property
    def n(self) -> int:
        d = self.desc
        return d.n if d.kind == GPCG_OP_CSR else d.nx * d.ny

    @staticmethod
    def stencil_const(nx: int, ny: int, w: float) -> "Operator":
        return Operator(gpcg_operator(kind=GPCG_OP_STENCIL5_CONST, nx=nx, ny=ny, w=w), [])

    @staticmethod
    def stencil_var(nx: int, ny: int, wx, wy) -> "Operator":
        """wx: ny*(nx+1) FP64 device tensor; wy: (ny+1)*nx FP64 device tensor."""
        wx, wy = wx.contiguous(), wy.contiguous()
        _check_vec(wx, ny * (nx + 1), _f64(), "wx")
        _check_vec(wy, (ny + 1) * nx, _f64(), "wy")
        return Operator(gpcg_operator(kind=GPCG_OP_STENCIL5_VAR, nx=nx, ny=ny,
                                      wx=_dptr(wx), wy=_dptr(wy)), [wx, wy])

    @staticmethod
    def csr(rowptr, colind, vals) -> "Operator":
        """int32 rowptr (n+1), int32 colind (nnz), FP64 vals (nnz) on the device."""
        rowptr, colind, vals = rowptr.contiguous(), colind.contiguous(), vals.contiguous()
        torch = _torch()
        n = rowptr.numel() - 1
        _check_vec(rowptr, n + 1, (torch.int32,), "rowptr")
        _check_vec(colind, colind.numel(), (torch.int32,), "colind")
        _check_vec(vals, colind.numel(), _f64(), "vals")
        return Operator(gpcg_operator(kind=GPCG_OP_CSR, n=n, nnz=colind.numel(),
                                      rowptr=_dptr(rowptr), colind=_dptr(colind),
                                      vals=_dptr(vals)), [rowptr, colind, vals])


class Solver:
    """One GPCG context (gpcg_create / gpcg_solve / gpcg_destroy)."""

    def __init__(self, op: Operator, device="cuda", stream=None, **options):
        self.op = op
        self.opt = default_options(**options)
        self.stream = stream
        nbytes = C.c_size_t()
        check(_lib.gpcg_workspace_bytes(C.byref(op.desc), C.byref(self.opt), C.byref(nbytes)),
              "gpcg_workspace_bytes")
        self.ws_bytes = nbytes.value
        self._ws, self._ws_ptr = _workspace(self.ws_bytes, device)
        h = C.c_void_p()
        check(_lib.gpcg_create(C.byref(op.desc), C.byref(self.opt), self._ws_ptr,
                               self.ws_bytes, _stream_ptr(stream), C.byref(h)), "gpcg_create")
        self.handle = h

    def solve(self, b, l, u, x, g_out=None) -> dict:
        """x holds x0 on entry and the answer on return (FP64 device tensors)."""
        n = self.op.n
        for t, name in ((b, "b"), (l, "l"), (u, "u"), (x, "x")):
            _check_vec(t, n, _f64(), name)
        _check_vec(g_out, n, _f64(), "g_out", optional=True)
        st = gpcg_stats()
        rc = _lib.gpcg_solve(self.handle, _dptr(b), _dptr(l), _dptr(u), _dptr(x),
                             _dptr(g_out), C.byref(st))
        check(rc, "gpcg_solve")
        return st.as_dict()

    def autotune(self, b, l, u, x0, x_work=None) -> dict:
        """Times the launch configurations on this problem and keeps the
        fastest (gpcg_autotune); returns the report.  x0 is not modified."""
        n = self.op.n
        for t, name in ((b, "b"), (l, "l"), (u, "u"), (x0, "x0")):
            _check_vec(t, n, _f64(), name)
        x = x_work if x_work is not None else _torch().empty_like(x0)
        _check_vec(x, n, _f64(), "x_work")
        rep = gpcg_tune_report()
        check(_lib.gpcg_autotune(self.handle, _dptr(b), _dptr(l), _dptr(u), _dptr(x0),
                                 _dptr(x), C.byref(rep)), "gpcg_autotune")
        return rep.as_dict()

    def spmv(self, v, y, mask=None):
        torch, n = _torch(), self.op.n
        _check_vec(v, n, (torch.float64, torch.float32), "v")
        _check_vec(y, n, (v.dtype,), "y")
        _check_vec(mask, n, (torch.uint8,), "mask", optional=True)
        fn = _lib.gpcg_spmv_f32 if v.dtype.itemsize == 4 else _lib.gpcg_spmv
        check(fn(self.handle, _dptr(v), _dptr(y), _dptr(mask)), "gpcg_spmv")

    def projected_gradient(self, x, l, u, g, pg=None):
        n = self.op.n
        for t, name in ((x, "x"), (l, "l"), (u, "u"), (g, "g")):
            _check_vec(t, n, _f64(), name)
        _check_vec(pg, n, _f64(), "pg", optional=True)
        n2 = C.c_double()
        lo, up, nb = C.c_int64(), C.c_int64(), C.c_int64()
        check(_lib.gpcg_projected_gradient(self.handle, _dptr(x), _dptr(l), _dptr(u), _dptr(g),
                                           _dptr(pg), C.byref(n2), C.byref(lo), C.byref(up),
                                           C.byref(nb)), "gpcg_projected_gradient")
        return n2.value, lo.value, up.value, nb.value

    def close(self):
        if self.handle:
            _lib.gpcg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many handles advanced together (gpcg_batch_*)."""

    def __init__(self, solvers: Sequence[Solver], device="cuda", stream=None):
        self.solvers = list(solvers)
        cnt = len(self.solvers)
        nbytes = C.c_size_t()
        arr = (C.c_void_p * cnt)(*[s.handle.value for s in self.solvers])
        check(_lib.gpcg_batch_workspace_bytes(cnt, arr, C.byref(nbytes)),
              "gpcg_batch_workspace_bytes")
        self._ws, ptr = _workspace(nbytes.value, device)
        h = C.c_void_p()
        check(_lib.gpcg_batch_create(cnt, arr, ptr, nbytes.value, _stream_ptr(stream),
                                     C.byref(h)), "gpcg_batch_create")
        self.handle = h

    def solve(self, problems, mode=GPCG_BATCH_STEPPED):
        """problems: list of (b, l, u, x) device tensors; returns per-QP stats."""
        cnt = len(self.solvers)
        if len(problems) != cnt:
            raise ValueError(f"{cnt} problems expected, got {len(problems)}")
        probs = (gpcg_problem * cnt)()
        for i, p in enumerate(problems):
            b, l, u, x = p[:4]
            g = p[4] if len(p) > 4 else None
            n = self.solvers[i].op.n
            for t, name in ((b, "b"), (l, "l"), (u, "u"), (x, "x")):
                _check_vec(t, n, _f64(), f"problems[{i}].{name}")
            _check_vec(g, n, _f64(), f"problems[{i}].g_out", optional=True)
            probs[i] = gpcg_problem(_dptr(b), _dptr(l), _dptr(u), _dptr(x), _dptr(g))
        stats = (gpcg_stats * cnt)()
        check(_lib.gpcg_batch_solve(self.handle, probs, mode, stats), "gpcg_batch_solve")
        return [s.as_dict() for s in stats]

    def autotune(self, problems, x0s) -> dict:
        """Times the stepped-form launch configurations (gpcg_batch_autotune)
        and keeps the fastest; x0s are copied into the problems' x first."""
        cnt = len(self.solvers)
        if len(problems) != cnt or len(x0s) != cnt:
            raise ValueError(f"{cnt} problems and starts expected")
        probs = (gpcg_problem * cnt)()
        for i, p in enumerate(problems):
            b, l, u, x = p[:4]
            n = self.solvers[i].op.n
            for t, name in ((b, "b"), (l, "l"), (u, "u"), (x, "x"), (x0s[i], "x0")):
                _check_vec(t, n, _f64(), f"problems[{i}].{name}")
            probs[i] = gpcg_problem(_dptr(b), _dptr(l), _dptr(u), _dptr(x), None)
        arr = (C.c_void_p * cnt)(*[_dptr(x) for x in x0s])
        rep = gpcg_tune_report()
        check(_lib.gpcg_batch_autotune(self.handle, probs, arr, C.byref(rep)),
              "gpcg_batch_autotune")
        return rep.as_dict()

    def close(self):
        if self.handle:
            _lib.gpcg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GPCG_NOALLOC_MAX_N = 1 << 34


def projected_gradient_noalloc(x, l, u, g, pg=None, stream=None):
    """gpcg_projected_gradient_noalloc: ||P grad q(x)||^2 and the face counts
    of x without a handle or workspace (the library's fixed per-GPU scratch;
    nothing is allocated).  Returns (norm2, n_lower, n_upper, n_nonbinding)."""
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        raise ValueError("x must be a torch tensor")
    n = x.numel()
    for t, name in ((x, "x"), (l, "l"), (u, "u"), (g, "g")):
        _check_vec(t, n, _f64(), name)
    _check_vec(pg, n, _f64(), "pg", optional=True)
    n2 = C.c_double()
    lo, up, nb = C.c_int64(), C.c_int64(), C.c_int64()
    check(_lib.gpcg_projected_gradient_noalloc(n, _dptr(x), _dptr(l), _dptr(u), _dptr(g),
                                               _dptr(pg), C.byref(n2), C.byref(lo),
                                               C.byref(up), C.byref(nb), _stream_ptr(stream)),
          "gpcg_projected_gradient_noalloc")
    return n2.value, lo.value, up.value, nb.value


def status_string(code: int) -> str:
    return _lib.gpcg_status_string(code).decode()


def build_info() -> str:
    return _lib.gpcg_build_info().decode()


class Server:
    """Continuous-batching solve service (gpcg_server_*).

    Requests are admitted by arena footprint and free slots while others are
    running; each request's state stays resident in the arena until done.
    """

    def __init__(self, arena_bytes: int, max_slots: int, precision=GPCG_PREC_MIXED,
                 tol_rel=1e-8, quantum=0, device="cuda", stream=None):
        self._arena, ptr = _workspace(arena_bytes, device)
        self.opt = gpcg_server_options(arena=ptr, arena_bytes=arena_bytes, max_slots=max_slots,
                                       precision=precision, tol_rel=tol_rel, quantum=quantum)
        h = C.c_void_p()
        check(_lib.gpcg_server_create(C.byref(self.opt), _stream_ptr(stream), C.byref(h)),
              "gpcg_server_create")
        self.handle = h
        self._pending = {}

    @staticmethod
    def footprint(op: Operator, precision=GPCG_PREC_MIXED) -> int:
        nbytes = C.c_size_t()
        check(_lib.gpcg_server_footprint(C.byref(op.desc), precision, C.byref(nbytes)),
              "gpcg_server_footprint")
        return nbytes.value

    def submit(self, tag: int, op: Operator, b, l, u, x0, x_out) -> int:
        """Queues a request; returns the C status (GPCG_ERR_NOSPACE if it can
        never fit).  The tensors are kept alive until completion."""
        n = op.n
        for t, name in ((b, "b"), (l, "l"), (u, "u"), (x0, "x0")):
            _check_vec(t, n, _f64(), name)
        _check_vec(x_out, n, _f64(), "x_out", optional=True)
        req = gpcg_request(op=op.desc, b=_dptr(b), l=_dptr(l), u=_dptr(u), x0=_dptr(x0),
                           x_out=_dptr(x_out), tag=tag)
        rc = _lib.gpcg_server_submit(self.handle, C.byref(req))
        if rc == GPCG_OK:
            self._pending[tag] = (op, b, l, u, x0, x_out)
        return rc

    def step(self) -> int:
        active = C.c_int()
        check(_lib.gpcg_server_step(self.handle, C.byref(active)), "gpcg_server_step")
        return active.value

    def poll(self, max_items: int = 256):
        buf = (gpcg_completion * max_items)()
        got = C.c_int()
        check(_lib.gpcg_server_poll(self.handle, buf, max_items, C.byref(got)), "gpcg_server_poll")
        out = []
        for i in range(got.value):
            c = buf[i]
            out.append(dict(tag=c.tag, status=c.status, stats=c.stats.as_dict(),
                            t_submit=c.t_submit, t_admit=c.t_admit, t_done=c.t_done))
            self._pending.pop(c.tag, None)
        return out

    def close(self):
        if self.handle:
            _lib.gpcg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
