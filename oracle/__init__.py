"""Plain FP64 CPU oracle for GPCG -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_cs_0101018_amd``) never imports, links or runs it, and it shares no
code with that library: the only common module is ``instances`` (seeded input
generators).

Contents
--------
* ``gpcg_ref.c``: Algorithm GPCG (Section 3 of the paper) in plain C on CSR,
  sequential sums, no FMA contraction, plus its building blocks (projection,
  projected gradient, active / binding classification, the exact 1-D step,
  projected-search trial points, reduced-matrix CG).  Loaded through ctypes.
* ``exact.py``: an *independent* exact solver (primal-dual active set +
  sparse direct solves) used to deliver the polished solution x* that the
  GPU results are compared with, and brute-force face enumeration for n <= 8.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import tempfile
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpcg_ref.c")
_BUILD = os.path.join(_HERE, "_build")
LIB_PATH = os.path.join(_BUILD, "libgpcg_ref.so")

OK, MAXIT, STAGNATED = 0, 1, 2
ERR_ARG, ERR_BOUNDS, ERR_NAN, ERR_NOT_SPD = -1, -2, -3, -4


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("vals", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("tol_rel", C.c_double), ("tol_abs", C.c_double), ("eta1", C.c_double),
                ("eta2", C.c_double), ("eta2_reduce", C.c_double), ("mu", C.c_double),
                ("max_outer", C.c_int32), ("max_gp", C.c_int32),
                ("max_backtrack", C.c_int32), ("max_cg", C.c_int32), ("max_stall", C.c_int32),
                ("precond", C.c_int32), ("cg_stop", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("gp_iters", C.c_int32),
                ("cg_iters", C.c_int32), ("backtracks", C.c_int32),
                ("face_repeats", C.c_int32), ("cg_phases", C.c_int32),
                ("x0_projected", C.c_int32), ("pg0", C.c_double), ("pg", C.c_double),
                ("tau", C.c_double), ("q", C.c_double), ("n_free", C.c_int64),
                ("n_lower", C.c_int64), ("n_upper", C.c_int64),
                ("trace_q", C.c_void_p), ("trace_act", C.c_void_p),
                ("trace_cap", C.c_int32), ("trace_len", C.c_int32),
                ("trace_cg_eta", C.c_void_p), ("trace_cg_iters", C.c_void_p),
                ("trace_cg_repeat", C.c_void_p), ("trace_cg_dec", C.c_void_p),
                ("trace_cg_cap", C.c_int32), ("trace_cg_len", C.c_int32),
                ("trace_dec_per", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("trace_")}


def build(out: Optional[str] = None, mutant: int = 0) -> str:
    """Compile the oracle with gcc; returns the shared-library path."""
    out = out or LIB_PATH
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", out + ".tmp", _SRC, "-lm"]
    if mutant:
        cmd.insert(1, f"-DORA_MUTANT={int(mutant)}")
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """ctypes front end to one build of ``gpcg_ref.c``."""

    def __init__(self, lib_path: Optional[str] = None):
        path = lib_path or LIB_PATH
        if lib_path is None and (not os.path.exists(path) or
                                 os.path.getmtime(path) < os.path.getmtime(_SRC)):
            build(path)
        self.lib = C.CDLL(path)
        L = self.lib
        vp, i64, d = C.c_void_p, C.c_int64, C.c_double
        L.ora_default_options.argtypes = [vp]
        L.ora_matvec.argtypes = [vp, vp, vp]
        L.ora_dot.argtypes = [i64, vp, vp]
        L.ora_dot.restype = d
        L.ora_gradient.argtypes = [vp, vp, vp, vp]
        L.ora_objective.argtypes = [vp, vp, vp]
        L.ora_objective.restype = d
        L.ora_project.argtypes = [i64, vp, vp, vp, vp]
        L.ora_proj_gradient.argtypes = [i64, vp, vp, vp, vp, vp]
        L.ora_proj_gradient_norm.argtypes = [i64, vp, vp, vp, vp]
        L.ora_proj_gradient_norm.restype = d
        L.ora_classify.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        L.ora_gp_alpha0.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.ora_trial.argtypes = [vp, vp, vp, d, vp, vp, vp, vp, vp, vp, vp]
        L.ora_reduced_cg.argtypes = [vp, vp, vp, d, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp,
                                     C.c_int32]
        L.ora_reduced_cg.restype = C.c_int
        L.ora_decrease.argtypes = [d, d]
        L.ora_decrease.restype = d
        L.ora_gpcg.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ora_gpcg.restype = C.c_int

    # -- operator handling
    def _csr(self, csr):
        rowptr, colind, vals = csr
        keep = (np.ascontiguousarray(rowptr, dtype=np.int32),
                np.ascontiguousarray(colind, dtype=np.int32), _f64(vals))
        s = _Csr(len(keep[0]) - 1, keep[0].ctypes.data, keep[1].ctypes.data,
                 keep[2].ctypes.data)
        return s, keep

    def options(self, **kw) -> Options:
        o = Options()
        self.lib.ora_default_options(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    # -- building blocks
    def matvec(self, csr, x):
        A, keep = self._csr(csr)
        x = _f64(x)
        y = np.empty_like(x)
        self.lib.ora_matvec(C.byref(A), _ptr(x), _ptr(y))
        return y

    def gradient(self, csr, x, b):
        A, keep = self._csr(csr)
        x, b = _f64(x), _f64(b)
        g = np.empty_like(x)
        self.lib.ora_gradient(C.byref(A), _ptr(x), _ptr(b), _ptr(g))
        return g

    def objective(self, csr, b, x):
        A, keep = self._csr(csr)
        b, x = _f64(b), _f64(x)
        return self.lib.ora_objective(C.byref(A), _ptr(b), _ptr(x))

    def project(self, l, u, v):
        l, u, v = _f64(l), _f64(u), _f64(v)
        out = np.empty_like(v)
        self.lib.ora_project(len(v), _ptr(l), _ptr(u), _ptr(v), _ptr(out))
        return out

    def proj_gradient(self, x, l, u, g):
        x, l, u, g = _f64(x), _f64(l), _f64(u), _f64(g)
        out = np.empty_like(x)
        self.lib.ora_proj_gradient(len(x), _ptr(x), _ptr(l), _ptr(u), _ptr(g), _ptr(out))
        return out

    def proj_gradient_norm(self, x, l, u, g):
        x, l, u, g = _f64(x), _f64(l), _f64(u), _f64(g)
        return self.lib.ora_proj_gradient_norm(len(x), _ptr(x), _ptr(l), _ptr(u), _ptr(g))

    def classify(self, x, l, u, g):
        x, l, u, g = _f64(x), _f64(l), _f64(u), _f64(g)
        lo, up, nb = C.c_int64(), C.c_int64(), C.c_int64()
        self.lib.ora_classify(len(x), _ptr(x), _ptr(l), _ptr(u), _ptr(g), C.byref(lo),
                              C.byref(up), C.byref(nb))
        return lo.value, up.value, nb.value

    def gp_alpha0(self, csr, y, l, u, g):
        A, keep = self._csr(csr)
        y, l, u, g = _f64(y), _f64(l), _f64(u), _f64(g)
        dd, dAd = C.c_double(), C.c_double()
        self.lib.ora_gp_alpha0(C.byref(A), _ptr(y), _ptr(l), _ptr(u), _ptr(g), C.byref(dd),
                               C.byref(dAd))
        return dd.value, dAd.value

    def trial(self, csr, y, direction, alpha, l, u, g):
        A, keep = self._csr(csr)
        y, dr, l, u, g = _f64(y), _f64(direction), _f64(l), _f64(u), _f64(g)
        ynew = np.empty_like(y)
        gs, sAs, nchg = C.c_double(), C.c_double(), C.c_int64()
        self.lib.ora_trial(C.byref(A), _ptr(y), _ptr(dr), float(alpha), _ptr(l), _ptr(u),
                           _ptr(g), _ptr(ynew), C.byref(gs), C.byref(sAs), C.byref(nchg))
        return ynew, gs.value, sAs.value, nchg.value

    def decrease(self, gs, sAs):
        return self.lib.ora_decrease(float(gs), float(sAs))

    def reduced_cg(self, csr, free_mask, g, eta, max_cg=0, dec_cap=4096, precond=0, cg_stop=0):
        A, keep = self._csr(csr)
        fm = np.ascontiguousarray(free_mask, dtype=np.uint8)
        g = _f64(g)
        d = np.empty_like(g)
        it = C.c_int32()
        decs = np.zeros(dec_cap)
        st = self.lib.ora_reduced_cg(C.byref(A), _ptr(fm), _ptr(g), float(eta), int(max_cg),
                                     int(precond), int(cg_stop), _ptr(d), C.byref(it),
                                     _ptr(decs), dec_cap)
        return st, d, it.value, decs[:min(it.value, dec_cap)]

    # -- the whole method
    def gpcg(self, csr, b, l, u, x0, trace_cap: int = 0, cg_trace_cap: int = 0,
             dec_per: int = 64, **opts):
        """Run Algorithm GPCG; returns (x, g, stats-dict).

        trace_cap > 0 adds ``trace_q`` and ``trace_act`` (one entry per
        projected search); cg_trace_cap > 0 adds ``cg_phases_trace``: per CG
        phase the eta of its stopping test, its iterations, whether it repeats
        CG on the previous face (eq. (cgstop3)), and its first dec_per CG
        decreases."""
        A, keep = self._csr(csr)
        b, l, u, x0 = _f64(b), _f64(l), _f64(u), _f64(x0)
        x = np.empty_like(x0)
        g = np.empty_like(x0)
        o = self.options(**opts)
        st = Stats()
        trace = np.zeros(max(trace_cap, 1))
        trace_act = np.zeros(2 * max(trace_cap, 1), dtype=np.int64)
        if trace_cap:
            st.trace_q = trace.ctypes.data
            st.trace_act = trace_act.ctypes.data
            st.trace_cap = trace_cap
        ccap = max(cg_trace_cap, 1)
        cg_eta = np.zeros(ccap)
        cg_it = np.zeros(ccap, dtype=np.int32)
        cg_rep = np.zeros(ccap, dtype=np.int32)
        cg_dec = np.full(ccap * dec_per, np.nan)
        if cg_trace_cap:
            st.trace_cg_eta = cg_eta.ctypes.data
            st.trace_cg_iters = cg_it.ctypes.data
            st.trace_cg_repeat = cg_rep.ctypes.data
            st.trace_cg_dec = cg_dec.ctypes.data
            st.trace_cg_cap = cg_trace_cap
            st.trace_dec_per = dec_per
        self.lib.ora_gpcg(C.byref(A), _ptr(b), _ptr(l), _ptr(u), _ptr(x0), C.byref(o),
                          _ptr(x), _ptr(g), C.byref(st))
        out = st.as_dict()
        if trace_cap:
            out["trace_q"] = trace[:st.trace_len].copy()
            out["trace_act"] = trace_act[:2 * st.trace_len].reshape(-1, 2).copy()
        if cg_trace_cap:
            k = st.trace_cg_len
            decs = cg_dec.reshape(ccap, dec_per)
            out["cg_phases_trace"] = [
                dict(eta=float(cg_eta[i]), iters=int(cg_it[i]), repeat=int(cg_rep[i]),
                     decs=decs[i, :min(int(cg_it[i]), dec_per)].copy())
                for i in range(k)]
        return x, g, out

    def solve_instance(self, inst, **opts):
        return self.gpcg(inst.csr(), inst.b, inst.l, inst.u, inst.x0, **opts)


_default: Optional[Oracle] = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def build_mutant(k: int, directory: Optional[str] = None) -> str:
    """Build the oracle with planted mistake number k (tests of the pins)."""
    directory = directory or tempfile.mkdtemp(prefix="gpcg_mutant_")
    return build(os.path.join(directory, f"libgpcg_ref_m{k}.so"), mutant=k)
