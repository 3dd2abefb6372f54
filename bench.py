"""Benchmark: GPCG on one MI355X -- solves/sec, HBM roofline of the pass kernel,
SpMV bandwidth, p50/p99 latency -- with the FP64 CPU oracle timed beside it.

Default run (no --workload): the headline is the 1600 x 1600 obstacle problem
with both bounds (n = 2,560,000, the largest single-GPU configuration) solved
in FP64 at projected-gradient tolerance 1e-8 relative.  One step = one whole
GPCG solve (every pass: projection, gradients, gradient-projection searches,
reduced CG, projected searches, termination), inputs resident in HBM, x0
restored on the device each step.  The same line carries, under their own
keys: the mixed-precision solve of the same problem, the 512-QP batch (mixed)
against 512 sequential plain FP64 solves, the 4096-request serving trace
(Poisson, 200 req/s, mixed) against a plain FP64 one-at-a-time loop, the
256 x 256 variable-coefficient problem, the SpMV and reduction building
blocks, and the error of every GPU answer class against the oracle's x*.

CPU leg (``cpu_baseline``): the FP64 oracle (``oracle/``), timed on this
host, and the oracle's answers the GPU answers are compared with.  It runs in
worker processes while the GPU work runs; the headline's oracle timing runs
alone at the end.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
    python bench.py --workload NAME [...]      (one workload, one line)
    python bench.py --counters FETCH_DIR WRITE_DIR   (summarise two rocprofv3
                    --pmc runs, FETCH_SIZE then WRITE_SIZE, as text)

Prints one JSON line.  `roofline.traffic` comes from the committed counter
summary of the workload's kernel when its kernel-source digest matches the
sources being run, else null.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import csv
import glob
import hashlib
import json
import multiprocessing
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E datasheet peak
METRIC = "GPCG solves/sec + SpMV HBM GB/s at proj-grad tol 1e-8; p50/p99 solve latency"

WORKLOADS = {
    # name: (instance factory, options, description)
    "varcoef256_fp64": ("varcoef256", dict(), "GPCG FP64, -div(c grad u) 256x256 (n=65,536), "
                        "c=(1+0.1 cos 2 pi s)^3, l=0, u=inf, tol 1e-8 rel"),
    "varcoef256_mixed": ("varcoef256", dict(precision=1), "GPCG mixed FP32-CG, varcoef 256x256"),
    "obstacle50_fp64": ("obstacle50", dict(), "GPCG FP64, obstacle 50x50"),
    "obstacle1024_fp64": ("obstacle_ub_1024", dict(), "GPCG FP64, obstacle 1024x1024, both bounds"),
    "obstacle1024_mixed": ("obstacle_ub_1024", dict(precision=1),
                           "GPCG mixed FP32-CG, obstacle 1024x1024, both bounds"),
    "obstacle1600_fp64": ("obstacle_ub_1600", dict(),
                          "GPCG FP64, obstacle 1600x1600 (n=2,560,000), 5-point Laplacian/h^2, "
                          "b=1, l=0.3 sin(pi s) sin(2 pi t)-0.2+0.01 N(0,1), "
                          "u=0.25+0.05 U(0,1), x0=max(l,0), tol 1e-8 rel"),
    "obstacle1600_mixed": ("obstacle_ub_1600", dict(precision=1),
                           "GPCG mixed FP32-CG, obstacle 1600x1600, both bounds"),
    # the same problem family past the 256 MB last-level cache (1.34 GB of
    # vectors per pass): every pass streams from HBM
    "obstacle4096_fp64": ("obstacle_ub_4096", dict(),
                          "GPCG FP64, obstacle 4096x4096 (n=16,777,216), both bounds, tol 1e-8 rel"),
    "obstacle4096_mixed": ("obstacle_ub_4096", dict(precision=1),
                           "GPCG mixed FP32-CG, obstacle 4096x4096 (n=16,777,216), both bounds"),
    "bearing256_fp64": ("bearing256", dict(), "GPCG FP64, -div(c grad u) 256x256, "
                        "c=(1+0.9 cos 2 pi s)^3 (eccentricity 0.9), l=0, u=inf, tol 1e-8 rel"),
    # the coefficient family of the paper's journal-bearing runs at their size
    # (1600^2); finite differences, not the paper's finite elements: context
    "varcoef1600_fp64": ("varcoef1600", dict(), "GPCG FP64, -div(c grad u) 1600x1600, "
                         "c=(1+0.1 cos 2 pi s)^3 (eccentricity 0.1), l=0, u=inf, tol 1e-8 rel"),
    "bearing1600_fp64": ("bearing1600", dict(), "GPCG FP64, -div(c grad u) 1600x1600, "
                         "c=(1+0.9 cos 2 pi s)^3 (eccentricity 0.9), l=0, u=inf, tol 1e-8 rel"),
    # small free set, CSR operator (the matrix free set's case)
    "pressed512_csr_fp64": ("pressed512", dict(operator="csr"),
                            "GPCG FP64, obstacle 512x512 pressed onto its obstacle (b=-1e4), "
                            "CSR operator, 23% free at the solution"),
}
BATCH_WORKLOADS = ("batch512_fp64", "batch512_mixed")
SERVE_WORKLOADS = ("serve4096",)
HEADLINE = "obstacle1600_fp64"
SAMPLE = 64  # stratified sample of batch members / requests for the oracle

KERNEL_SOURCES = ("paper_cs_0101018_amd/csrc/gpcg_kernels.hip",
                  "paper_cs_0101018_amd/csrc/gpcg_internal.h")
COPY_CALIB_BYTES = 256 << 20


def kernel_digest():
    """sha256 over the device sources: counters taken on other code are stale."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_rows(d):
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for fn in files:
        with open(fn, newline="") as f:
            yield from csv.DictReader(f)


def _per_dispatch_kib(d, counter):
    """{kernel name: [KiB of each dispatch]} for one counter."""
    acc = {}
    for r in _counter_rows(d):
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "?")
        key = r.get("Dispatch_Id", r.get("Correlation_Id"))
        acc.setdefault(name, {})
        acc[name][key] = acc[name].get(key, 0.0) + float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in acc.items()}


def counters_summary(fetch_dir, write_dir):
    """Text summary of a FETCH_SIZE run and a WRITE_SIZE run: mean KiB per
    dispatch by kernel, and the scale factor that maps the counter of the
    256 MiB calibration copy (the largest copy dispatch: 256 MiB read, 256 MiB
    written) onto the bytes it is known to move."""
    fetch = _per_dispatch_kib(fetch_dir, "FETCH_SIZE")
    write = _per_dispatch_kib(write_dir, "WRITE_SIZE")
    known_kib = COPY_CALIB_BYTES / 1024.0

    def calib(tab):
        cands = [(max(v), k) for k, v in tab.items() if "copy" in k.lower() and v]
        if not cands or max(cands)[0] <= 0.0:
            return None, None, None
        val, name = max(cands)
        return known_kib / val, name, val

    cf, cname, cfv = calib(fetch)
    cw, _, cwv = calib(write)
    mean = lambda v: sum(v) / len(v) if v else float("nan")
    lines = [f"kernel_source_sha256: {kernel_digest()}",
             f"copy_calibration_kernel: {cname}",
             f"copy_calibration_fetch_kib: {cfv}",
             f"copy_calibration_write_kib: {cwv}",
             f"calib_factor_fetch: {cf}",
             f"calib_factor_write: {cw}",
             "",
             f"{'kernel':90s} {'dispatches':>10s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s}"]
    for k in sorted(set(fetch) | set(write), key=lambda k: -len(fetch.get(k, []))):
        f, w = fetch.get(k, []), write.get(k, [])
        lines.append(f"{k[:90]:90s} {max(len(f), len(w)):10d} {mean(f):12.1f} {mean(w):12.1f}")
    return "\n".join(lines)


def traffic_from_profile(workload, kernel_substr):
    """HBM bytes per launch of the kernel from the committed counter summary
    (scaled by the copy calibration), or None when absent or stale."""
    fn = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(fn):
        return None
    txt = open(fn).read()
    kv = dict(re.findall(r"^(\w+): (\S+)$", txt, re.M))
    if kv.get("kernel_source_sha256") != kernel_digest():
        return None
    try:
        cf, cw = float(kv["calib_factor_fetch"]), float(kv["calib_factor_write"])
    except (KeyError, ValueError):
        return None
    for line in txt.splitlines():
        parts = line.split()
        if len(parts) >= 4 and kernel_substr in line:
            try:
                f, w = float(parts[-2]), float(parts[-1])
            except ValueError:
                continue
            return (f * cf + w * cw) * 1024.0
    return None


def make_instance(key):
    import instances
    if key == "obstacle50":
        return instances.obstacle50(0)
    if key == "varcoef256":
        return instances.varcoef256(0)
    if key == "bearing256":
        return instances.varcoef(256, 0, eps=0.9, name="bearing256")
    if key == "varcoef1600":
        return instances.varcoef(1600, 0, eps=0.1, name="varcoef1600")
    if key == "bearing1600":
        return instances.varcoef(1600, 0, eps=0.9, name="bearing1600")
    if key.startswith("obstacle_ub_"):
        return instances.obstacle_ub(int(key.split("_")[-1]), 0)
    if key == "pressed512":
        return instances.pressed(512, 0)
    raise KeyError(key)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_extras(gpcg, torch, dev, reps=40, grids=(1024, 1600), precs=(0, 1)):
    """Bandwidth of the SpMV building block y = M o (A v) on the large grids:
    `reps` back-to-back launches timed with HIP events on the launch stream.
    Warm: one (v, y, mask) set, resident in the 256 MB last-level cache where
    it fits.  Cold: the launches cycle through enough sets (> 1 GiB) that every
    launch reads from HBM."""
    out = {}
    for N in grids:
        for prec in precs:
            op = gpcg.Operator.stencil_const(N, N, float((N + 1) ** 2))
            s = gpcg.Solver(op, device=dev, precision=prec)
            dt = torch.float32 if prec else torch.float64
            per = 2 * (4 if prec else 8) + 1
            set_bytes = per * N * N
            for cold in (False, True):
                nsets = max(1, -(-(1 << 30) // set_bytes)) if cold else 1
                sets = [(torch.randn(N * N, dtype=torch.float64, device=dev).to(dt),
                         torch.empty(N * N, dtype=dt, device=dev),
                         torch.ones(N * N, dtype=torch.uint8, device=dev)) for _ in range(nsets)]
                for i in range(min(nsets, 4)):
                    s.spmv(*sets[i])
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for i in range(reps):
                    s.spmv(*sets[i % nsets])
                e1.record()
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                # the same bytes moved by a device copy (read + write), same cycling
                e0.record()
                for i in range(reps):
                    a_, b_, _ = sets[i % nsets]
                    b_.copy_(a_)
                e1.record()
                torch.cuda.synchronize()
                tc = e0.elapsed_time(e1) * 1e-3 / reps
                copy_gbs = 2 * sets[0][0].numel() * sets[0][0].element_size() / tc / 1e9
                key = f"spmv_const{N}_{'fp32' if prec else 'fp64'}_{'cold' if cold else 'warm'}"
                out[key] = dict(GBs=round(set_bytes / t / 1e9, 1), us=round(t * 1e6, 2),
                                bytes_per_var=per, frac=round(set_bytes / t / 1e9 / HBM_PEAK_GBS, 3),
                                copy_GBs=round(copy_gbs, 1),
                                frac_of_copy=round(set_bytes / t / 1e9 / copy_gbs, 3))
                del sets
            s.close()
    return out


def reduction_extras(gpcg, torch, dev, N=8192, reps=20):
    """Bandwidth of the projected-gradient reduction (||grad_Omega q||^2 and the
    face counts; x, l, u, g read once: 32 B per unknown) on an 8192^2 grid,
    two 2.1 GB sets alternated so that every call reads from HBM.  Each call
    of gpcg_projected_gradient waits for its result on the host, so the time
    per call (HIP events around the whole loop) includes that round trip: a
    lower bound on the kernels' own rate."""
    op = gpcg.Operator.stencil_const(N, N, float((N + 1) ** 2))
    s = gpcg.Solver(op, device=dev)
    n = N * N
    sets = []
    for k in range(2):
        g = torch.Generator(device=dev)
        g.manual_seed(k)
        lo = torch.rand(n, dtype=torch.float64, device=dev, generator=g) - 0.5
        up = lo + 0.25 + torch.rand(n, dtype=torch.float64, device=dev, generator=g)
        x = torch.maximum(lo, torch.zeros_like(lo))
        x = torch.minimum(x, up)
        gr = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
        sets.append((x, lo, up, gr))
    for i in range(2):
        s.projected_gradient(*sets[i])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        s.projected_gradient(*sets[i % 2])
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    byt = 32.0 * n
    del sets
    s.close()
    return {f"pgrad{N}_fp64_cold": dict(GBs=round(byt / t / 1e9, 1), us=round(t * 1e6, 2),
                                        bytes_per_var=32, frac=round(byt / t / 1e9 / HBM_PEAK_GBS, 3),
                                        includes_host_wait=True)}

# ------------------------------------------------------------------ CPU leg
# Everything below that imports ``oracle`` is the CPU-baseline leg: the FP64
# oracle timed on this host, and the oracle's answers (x*) that the GPU
# answers are compared with.  The GPU path never touches it.

def host_info():
    """CPU model and the number of CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return dict(cpu_model=model, cpus_available=ncpu, machine=platform.machine())


def cpu_xstar_face(N):
    """x* of the N x N obstacle problem (seed 0) rebuilt from its committed face
    certificate by one exact face solve, accepted only if it satisfies the
    Kuhn-Tucker conditions (oracle.exact.xstar_from_face)."""
    import instances
    from oracle import exact
    inst = instances.obstacle_ub(N, 0)
    _, lo, up = exact.read_face(os.path.join(ROOT, "tests", "golden",
                                             f"face_obstacle_ub_{N}_seed0.txt"))
    t0 = time.perf_counter()
    x, g, kkt = exact.xstar_from_face(N, inst.w, inst.b, inst.l, inst.u, lo, up)
    return dict(x=x, kkt=kkt, seconds=time.perf_counter() - t0, n_lower=len(lo),
                n_upper=len(up))


def cpu_member(kind, index, count):
    """One batch member or serving request: the oracle's FP64 GPCG solve at the
    metric tolerance (timed, one thread), then polished into x*."""
    import instances
    import oracle
    from oracle import exact
    if kind == "batch":
        inst = instances.batch_member(0, index, count)
    else:
        inst = instances.serve_request(0, index, count)
    ora = oracle.default()
    t0 = time.perf_counter()
    xo, _, st = ora.solve_instance(inst)
    t = time.perf_counter() - t0
    xs, info = exact.polish(inst.csr(), inst.b, inst.l, inst.u, xo)
    return dict(index=index, n=inst.n, seconds=t, status=st["status"], cg=st["cg_iters"],
                xstar=xs, polished=bool(info["converged"]), kkt=info["kkt"])


def cpu_headline_sample(key, max_outer, cg_iters):
    """The oracle on the headline instance: its first `max_outer` GPCG
    iterations (gradient projection, CG, projected search) and, separately,
    `cg_iters` iterations of its reduced CG (extraction of A_F included) on the
    face of x0, each timed on one thread."""
    import oracle
    inst = make_instance(key)
    ora = oracle.default()
    t0 = time.perf_counter()
    _, _, st = ora.solve_instance(inst, max_outer=max_outer)
    t_outer = time.perf_counter() - t0
    free = ((inst.l < inst.x0) & (inst.x0 < inst.u)).astype(np.uint8)
    g = ora.gradient(inst.csr(), inst.x0, inst.b)
    t0 = time.perf_counter()
    _, _, it, _ = ora.reduced_cg(inst.csr(), free, g, 1e-300, max_cg=cg_iters, dec_cap=1)
    t_cg = time.perf_counter() - t0
    return dict(seconds=t_outer, cg=st["cg_iters"], outer=st["outer_iters"],
                gp=st["gp_iters"], cg_seconds=t_cg, cg_run=it)


ONE_SOLVE_ALL_CORES = ("one solve: the oracle has no threaded code, so the host's other cores "
                       "do not shorten it (OMP_NUM_THREADS=1 and =nproc run the same code)")

def cpu_baseline_whole(inst, budget_s=12.0, precond=0, cg_stop=0):
    """The FP64 oracle, as it stands, on this host: solves/sec on a bounded
    sample (whole solves of the same workload until the budget is spent)."""
    import oracle
    ora = oracle.default()
    csr = inst.csr()
    t0 = time.perf_counter()
    k = 0
    while True:
        ora.gpcg(csr, inst.b, inst.l, inst.u, inst.x0, precond=precond, cg_stop=cg_stop)
        k += 1
        el = time.perf_counter() - t0
        if el >= budget_s or k >= 200:
            break
    return dict(value=k / el, unit="solves/s", cores=1, kind="oracle",
                sample=f"{k} complete solves of the same instance in {el:.1f} s "
                       f"(single-threaded C, -O3 -ffp-contract=off)",
                all_cores=dict(value=k / el, cores=1, how=ONE_SOLVE_ALL_CORES), **host_info())


def cpu_baseline_projected(key, cg_full, max_outer=4, cg_iters=1000):
    """Headline CPU baseline for problems whose oracle solve takes minutes: the
    oracle's first GPCG iterations (which hold most of its gradient-projection
    iterates) plus the rest of the solve's CG iterations at the oracle's
    measured cost per CG iteration (the CG phases are >95 % of its time)."""
    r = cpu_headline_sample(key, max_outer, cg_iters)
    per_cg = r["cg_seconds"] / max(r["cg_run"], 1)
    t_full = r["seconds"] + max(cg_full - r["cg"], 0) * per_cg
    return dict(value=1.0 / t_full, unit="solves/s", cores=1, kind="oracle",
                sample=f"oracle on the same instance, one thread: its first {r['outer']} "
                       f"GPCG iterations ({r['gp']} gradient-projection iterates, {r['cg']} "
                       f"CG iterations) in {r['seconds']:.1f} s, and {r['cg_run']} reduced-CG "
                       f"iterations on the face of x0 in {r['cg_seconds']:.1f} s; the other "
                       f"{max(cg_full - r['cg'], 0)} CG iterations of a whole solve (the GPU "
                       f"FP64 solve's count, {cg_full}, at the same tolerance) at that cost: "
                       f"{t_full:.0f} s per solve",
                seconds_sampled=round(r["seconds"] + r["cg_seconds"], 2),
                all_cores=dict(value=1.0 / t_full, cores=1, how=ONE_SOLVE_ALL_CORES),
                **host_info())


def stratified(sizes, k):
    """k member indices spread evenly over the members sorted by size."""
    order = np.argsort(np.asarray(sizes), kind="stable")
    m = len(order)
    return sorted(int(order[int((j + 0.5) * m / k)]) for j in range(min(k, m)))


def start_cpu_pool(workers):
    """Worker processes for the CPU leg (started before the GPU is used)."""
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    for k in env_keys:  # one or two threads per worker: the workers share the host
        os.environ[k] = "2"
    ctx = multiprocessing.get_context("spawn")
    return cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx)


def rel_inf(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def err_summary(errs):
    e = np.asarray(errs, dtype=np.float64)
    return {"max": float(e.max()), "median": float(np.median(e)), "count": int(e.size)}

# ------------------------------------------------------------------ GPU legs

def _dev_instance(inst, gpcg, torch, dev):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    N = inst.N
    if inst.op == "var":
        wx, wy = inst.edge_weights()
        op = gpcg.Operator.stencil_var(N, N, t(wx.ravel()), t(wy.ravel()))
    else:
        op = gpcg.Operator.stencil_const(N, N, inst.w)
    return op, t(inst.b), t(inst.l), t(inst.u), t(inst.x0)


def kernel_names(gpcg, args, tuned, ntiles, mixed, csr, precond):
    """The dominant kernel of a single-QP solve: the fused pass kernel, or the
    data kernel of the split form (the pass's transition runs in it)."""
    if tuned is not None:
        fused = tuned["form"] == gpcg.GPCG_FORM_FUSED
        prefetch = bool(tuned["prefetch"])
        cgk = bool(tuned["cg_kernel"]) and not fused
    else:
        fused = args.form == "fused" or (args.form == "auto" and ntiles <= 1024)
        # early CG loads need 256-unknown tiles (the library's choice up to
        # 1024 of them) and the mask free set
        tile = args.tile or (256 if ntiles <= 1024 else 512)
        prefetch = (args.prefetch != "off" and tile == 256 and args.free_set == "mask"
                    and not csr)
        cgk = args.cg_kernel == "on" and not fused
    ct = "float" if mixed else "double"
    mat = "true" if args.free_set == "matrix" else "false"
    flags = f"{ct}, {'true' if prefetch else 'false'}, {'true' if precond else 'false'}"
    if fused:
        return (f"gpcg::step_kernel<{flags}, {mat}> (one fused GPCG pass per launch)",
                f"step_kernel<{flags}, {mat}>")
    # the CG iterations' own data kernel, or the one of every pass; the matrix
    # form never runs in the CG-only kernel
    part = 1 if cgk and mat == "false" else 0
    pmat = "false" if part == 1 else mat
    # the last two template arguments: one QP (no work queue), generic
    # gradient-projection passes
    return (f"gpcg::pass_kernel<{flags}, {part}, {pmat}, false, false> (data kernel of the split "
            "form; the time per launch is that of one pass: transition and data kernels)",
            f"pass_kernel<{flags}, {part}, {pmat}, false, false>")


def run_single(gpcg, torch, dev, args, workload, steps, warmup, autotune=True):
    """Solves/sec of one single-QP workload; returns (result dict, answer on the
    host, stats of the last step)."""
    key, opts, desc = WORKLOADS[workload]
    inst = make_instance(key)
    N = inst.N
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    opts = dict(opts)
    csr = opts.pop("operator", None) == "csr"
    mixed = bool(opts.get("precision"))
    if args.free_set == "matrix" and not csr:
        sys.exit("the matrix free set needs a CSR operator (e.g. --workload pressed512_csr_fp64)")
    if csr:
        rowptr, colind, vals = inst.csr()
        op = gpcg.Operator.csr(t(rowptr), t(colind), t(vals))
    elif inst.op == "var":
        wx, wy = inst.edge_weights()
        op = gpcg.Operator.stencil_var(N, N, t(wx.ravel()), t(wy.ravel()))
    else:
        op = gpcg.Operator.stencil_const(N, N, inst.w)
    form = {"auto": gpcg.GPCG_FORM_AUTO, "fused": gpcg.GPCG_FORM_FUSED,
            "split": gpcg.GPCG_FORM_SPLIT}[args.form]
    fs = {"mask": gpcg.GPCG_FREESET_MASK, "list": gpcg.GPCG_FREESET_LIST,
          "matrix": gpcg.GPCG_FREESET_MATRIX}[args.free_set]
    pf = {"auto": gpcg.GPCG_PREFETCH_AUTO, "on": gpcg.GPCG_PREFETCH_ON,
          "off": gpcg.GPCG_PREFETCH_OFF}[args.prefetch]
    pc = gpcg.GPCG_PRECOND_JACOBI if args.precond == "jacobi" else gpcg.GPCG_PRECOND_NONE
    cs = gpcg.GPCG_CGSTOP_RESIDUAL if args.cg_stop == "residual" else gpcg.GPCG_CGSTOP_DECREASE
    la = {"auto": gpcg.GPCG_LOOKAHEAD_AUTO, "on": gpcg.GPCG_LOOKAHEAD_ON,
          "off": gpcg.GPCG_LOOKAHEAD_OFF}[args.lookahead]
    ck = {"auto": gpcg.GPCG_CGK_AUTO, "on": gpcg.GPCG_CGK_ON,
          "off": gpcg.GPCG_CGK_OFF}[args.cg_kernel]
    solver = gpcg.Solver(op, device=dev, form=form, free_set=fs, prefetch=pf, precond=pc,
                         cg_stop=cs, lookahead=la, cg_kernel=ck, tiles_per_wg=args.tiles_per_wg,
                         chunk=args.chunk, tile=args.tile, **opts)
    b, l, u, x0 = t(inst.b), t(inst.l), t(inst.u), t(inst.x0)
    x = torch.empty_like(x0)

    def step():
        x.copy_(x0)
        return solver.solve(b, l, u, x)

    tuned = None
    if (autotune and not args.no_autotune and args.form == "auto" and args.tiles_per_wg == 0
            and args.prefetch == "auto" and args.chunk == 0 and args.cg_kernel == "auto"):
        tuned = solver.autotune(b, l, u, x0)["chosen"]
        log(f"{workload}: autotune {tuned}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    stream = torch.cuda.current_stream(dev)  # the solver's stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        stats.append(step())
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    st = stats[-1]
    assert all(s["status"] == 0 for s in stats), [s["status"] for s in stats]
    xh = x.cpu().numpy()
    solver.close()

    launches = sum(s["launches"] for s in stats)
    passes = sum(s["passes"] for s in stats)
    alg_bytes = sum(s["bytes"] for s in stats)
    avg_launch_s = gpu_ms * 1e-3 / launches
    bytes_per_launch = alg_bytes / launches
    achieved = bytes_per_launch / avg_launch_s / 1e9
    kname, ksub = kernel_names(gpcg, args, tuned, -(-inst.n // 256), mixed, csr,
                               args.precond == "jacobi")
    traffic = traffic_from_profile(workload, ksub)
    lat = [s["ms_total"] for s in stats]
    res = {
        "metric": METRIC,
        "value": round(steps / wall, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(wall * 1e3 / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32cg" if mixed else "f64",
        "data": "synthetic (seeded instance generator, seed 0)",
        "config": {"workload": workload, "description": desc, "n": inst.n,
                   "free_set": args.free_set, "form": args.form,
                   "tiles_per_wg": args.tiles_per_wg, "prefetch": args.prefetch,
                   "precond": args.precond, "cg_stop": args.cg_stop,
                   "lookahead": args.lookahead, "cg_kernel": args.cg_kernel,
                   "chunk": args.chunk, "tile": args.tile,
                   "grid": f"{N}x{N}", "tol_rel": 1e-8, "global_batch": 1,
                   "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": None if traffic is None else round(traffic, 1),
            "bytes_per_launch": round(bytes_per_launch, 1),
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "launches_per_solve": launches / steps,
            "useful_passes_per_solve": passes / steps,
        },
        "autotune": tuned,
        "solve_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                             "p99": round(float(np.percentile(lat, 99)), 3)},
        "solve": {k: st[k] for k in ("outer_iters", "gp_iters", "cg_iters", "backtracks",
                                     "face_repeats", "passes", "lookaheads", "launches", "pg",
                                     "tau")},
        "phase_ms": {k: round(st[k], 3) for k in ("ms_cg", "ms_gp", "ms_search", "ms_other")},
    }
    return res, xh, st, inst


def bench_batch(args, gpcg, torch, dev, mixed, sample=()):
    """512 independent QPs of uneven size in one batch (persistent launch or
    stepped graph chunks) against 512 sequential plain FP64 solves.  Returns
    the result and the answers (batch, sequential FP64) of the sampled members."""
    import instances
    insts = instances.batch512(0)
    data = [_dev_instance(i, gpcg, torch, dev) for i in insts]
    mode = gpcg.GPCG_BATCH_PERSISTENT if args.batch_mode == "persistent" else gpcg.GPCG_BATCH_STEPPED
    if args.free_set == "matrix":
        sys.exit("the matrix free set needs CSR operators; the batch members are stencils")
    fs = gpcg.GPCG_FREESET_LIST if args.free_set == "list" else gpcg.GPCG_FREESET_MASK
    pc = gpcg.GPCG_PRECOND_JACOBI if args.precond == "jacobi" else gpcg.GPCG_PRECOND_NONE
    # batch members use 512-unknown tiles (the split form's data kernel keeps
    # two 256-unknown chunks of loads in flight per workgroup), 1024 in mixed
    # precision (half the CG bytes per unknown: the per-tile costs weigh more;
    # autotuned batch 1071 -> 1095 solves/s, FP64 within 1 %); the compacted
    # list form keeps its 256-unknown tiles; --tile overrides all
    tile = args.tile or ((1024 if mixed else 512) if fs == gpcg.GPCG_FREESET_MASK else 0)
    solvers = [gpcg.Solver(d[0], device=dev, precision=int(mixed), free_set=fs, precond=pc,
                           tile=tile) for d in data]
    batch = gpcg.Batch(solvers, device=dev)
    xs = [torch.empty_like(d[4]) for d in data]
    probs = [(d[1], d[2], d[3], x) for d, x in zip(data, xs)]

    def run_batch():
        for d, x in zip(data, xs):
            x.copy_(d[4])
        return batch.solve(probs, mode=mode)

    tuned = None
    if not args.no_autotune and mode == gpcg.GPCG_BATCH_STEPPED:
        tuned = batch.autotune(probs, [d[4] for d in data])["chosen"]
        log(f"batch: autotune {tuned}")
    for _ in range(args.batch_warmup):
        run_batch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        st = run_batch()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.batch_steps
    bad = [s["status"] for s in st if s["status"] != 0]
    alg_bytes = sum(s["bytes"] for s in st)
    n_tot = sum(i.n for i in insts)
    wl = "batch512_mixed" if mixed else "batch512_fp64"
    res = {
        "metric": "GPCG solves/sec, 512-QP batch (proj-grad tol 1e-8 rel)",
        "value": round(len(insts) / wall, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.batch_steps, "warmup": args.batch_warmup,
        "ms_per_step": round(wall * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32cg" if mixed else "f64",
        "data": "synthetic (512 obstacle / variable-coefficient QPs, sides log-uniform "
                "in [32, 384], seed 0)",
        "config": {"workload": wl, "qps": len(insts), "unknowns": n_tot,
                   "batch_mode": args.batch_mode, "free_set": args.free_set,
                   "precond": args.precond, "tile": tile or "auto"},
        "roofline": {"bound": "hbm", "kernel": "whole batch (every pass of every QP)",
                     "achieved": round(alg_bytes / wall / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg_bytes / wall / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_batch": alg_bytes},
        "autotune": tuned,
        "failed": len(bad),
        "launches": int(st[0]["launches"]),
        "passes_per_qp": {"min": int(min(s["passes"] for s in st)),
                          "median": float(np.median([s["passes"] for s in st])),
                          "max": int(max(s["passes"] for s in st))},
    }
    answers = {"batch": {i: xs[i].cpu().numpy() for i in sample}}
    if args.no_sequential:
        return res, answers
    # baseline: the same 512 QPs one after another, plain FP64, same GPU
    seq = [gpcg.Solver(d[0], device=dev) for d in data]
    x1 = [torch.empty_like(d[4]) for d in data]
    for s_, d, x in zip(seq[:8], data[:8], x1[:8]):
        x.copy_(d[4]); s_.solve(d[1], d[2], d[3], x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_, d, x in zip(seq, data, x1):
        x.copy_(d[4])
        s_.solve(d[1], d[2], d[3], x)
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    err = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(xs, x1))
    res["sequential_fp64"] = {"solves_per_s": round(len(insts) / seq_wall, 2),
                              "ms_total": round(seq_wall * 1e3, 1)}
    res["speedup_vs_sequential_fp64"] = round(seq_wall / wall, 3)
    res["max_rel_diff_vs_sequential_fp64"] = err
    answers["sequential_fp64"] = {i: x1[i].cpu().numpy() for i in sample}
    return res, answers


def bench_serve(args, gpcg, torch, dev, reqs_host, sample=()):
    """Poisson arrivals at 200 req/s replayed against the continuous-batching
    server (mixed precision), and the same trace through a plain FP64
    one-at-a-time loop (FIFO, service times measured on the same GPU).
    Returns the result and the served answers of the sampled requests."""
    import instances
    count = len(reqs_host)
    arr = instances.serve_trace(0, count)
    reqs = [(inst.n,) + _dev_instance(inst, gpcg, torch, dev) for inst in reqs_host]
    torch.cuda.synchronize()
    arena = 8 << 30
    srv = gpcg.Server(arena, max_slots=512, precision=gpcg.GPCG_PREC_MIXED, tol_rel=1e-8,
                      quantum=32, device=dev)
    outs = [torch.empty(r[0], dtype=torch.float64, device=dev) for r in reqs]
    log("serve: replaying the trace")
    t0 = time.perf_counter()
    nxt = 0
    done = {}
    while len(done) < count:
        now = time.perf_counter() - t0
        while nxt < count and arr[nxt] <= now:
            r = reqs[nxt]
            rc = srv.submit(nxt, r[1], r[2], r[3], r[4], r[5], outs[nxt])
            assert rc == 0, rc
            nxt += 1
        active = srv.step()
        for c in srv.poll(1024):
            done[c["tag"]] = c
            if len(done) % 512 == 0:
                log(f"serve: {len(done)}/{count} done")
        if active == 0 and nxt < count:
            time.sleep(max(0.0, min(0.002, arr[nxt] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    # the library stamps completions with the monotonic clock that
    # time.perf_counter() reads on Linux: latency = completion - arrival
    lat = np.array([done[i]["t_done"] - (t0 + arr[i]) for i in range(count)])
    bad = sum(1 for c in done.values() if c["status"] != 0)
    torch.cuda.synchronize()
    answers = {i: outs[i].cpu().numpy() for i in sample}
    # capacity: the same requests all submitted at once (the server saturated)
    log("serve: saturated replay")
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        assert srv.submit(i, r[1], r[2], r[3], r[4], r[5], outs[i]) == 0
    sat_done = 0
    while sat_done < count:
        srv.step()
        sat_done += len(srv.poll(1024))
    sat_wall = time.perf_counter() - t0
    srv.close()
    # FP64 one-at-a-time baseline: FIFO single server on the same trace
    log("serve: FP64 one-at-a-time baseline")
    service = np.zeros(count)
    for i, r in enumerate(reqs):
        s_ = gpcg.Solver(r[1], device=dev)
        xb = r[5].clone()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s_.solve(r[2], r[3], r[4], xb)
        torch.cuda.synchronize()
        service[i] = time.perf_counter() - ts
        s_.close()
        if (i + 1) % 1024 == 0:
            log(f"serve: baseline {i + 1}/{count} solves")
    finish = np.zeros(count)
    tcur = 0.0
    for i in range(count):
        tcur = max(tcur, arr[i]) + service[i]
        finish[i] = tcur
    lat_seq = finish - arr
    res = {
        "metric": "GPCG serving: solves/sec and p50/p99 latency (Poisson 200 req/s)",
        "value": round(count / wall, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(wall * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32cg", "data": "synthetic (Poisson trace, 200 req/s; sides log-uniform in [32, 512], seed 0)",
        "config": {"workload": "serve4096", "requests": count, "rate_hz": 200,
                   "max_slots": 512, "quantum": 32},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 2)},
        "capacity_solves_per_s": round(count / sat_wall, 2),
        "fp64_one_at_a_time": {
            "solves_per_s": round(count / max(finish[-1], arr[-1]), 2),
            "capacity_solves_per_s": round(count / float(service.sum()), 2),
            "p50_ms": round(float(np.percentile(lat_seq, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat_seq, 99)) * 1e3, 2),
            "mean_service_ms": round(float(service.mean()) * 1e3, 3)},
        "failed": bad,
    }
    return res, answers

# ------------------------------------------------------------------ main

def lam_min_const(N, w):
    """Smallest eigenvalue of the constant five-point operator on N x N."""
    return 2.0 * w * (2.0 - 2.0 * np.cos(np.pi / (N + 1)))


def accuracy_entry(x, xs, st, N=None, w=None):
    """Error of a GPU answer against x*, with the bound that the termination
    test gives on the answer's face: ||x - x*||_2 <= ||P grad q(x)||_2 / lambda_min(A)."""
    e = {"rel_inf_err": rel_inf(x, xs), "pg": st["pg"], "tau": st["tau"]}
    if N is not None:
        e["bound_l2"] = st["pg"] / lam_min_const(N, w)
        e["err_l2"] = float(np.linalg.norm(np.asarray(x) - xs))
    return e


def suite(args):
    """The default run: the headline and every other workload of the metric."""
    import instances
    info = host_info()
    workers = max(1, min(12, info["cpus_available"] - 2))
    pool = None
    futs = {}
    batch_sizes = [i.n for i in instances.batch512(0)]
    batch_sample = stratified(batch_sizes, SAMPLE)
    serve_host = [instances.serve_request(0, i, args.requests) for i in range(args.requests)]
    serve_sample = stratified([r.n for r in serve_host], SAMPLE)
    if not args.no_cpu_baseline:
        import oracle
        oracle.default()  # built before the workers start (they only load it)
        pool = start_cpu_pool(workers)
        futs["xstar1600"] = pool.submit(cpu_xstar_face, 1600)
        for i in batch_sample:
            futs[("batch", i)] = pool.submit(cpu_member, "batch", i, 512)
        for i in serve_sample:
            futs[("serve", i)] = pool.submit(cpu_member, "serve", i, args.requests)
        log(f"cpu leg: {len(futs)} oracle tasks on {workers} worker processes")

    import torch
    import paper_cs_0101018_amd as gpcg
    dev = torch.device("cuda:0")

    log("headline: obstacle1600_fp64")
    res, x64, st64, inst = run_single(gpcg, torch, dev, args, HEADLINE, args.steps, args.warmup)
    log(f"headline: {res['value']} solves/s")
    log("obstacle1600_mixed")
    rmix, xmx, stmx, _ = run_single(gpcg, torch, dev, args, "obstacle1600_mixed",
                                    args.steps, args.warmup)
    res["obstacle1600_mixed"] = {
        "solves_per_s": rmix["value"], "ms_per_step": rmix["ms_per_step"],
        "speedup_vs_fp64": round(rmix["value"] / res["value"], 3),
        "roofline": rmix["roofline"], "autotune": rmix["autotune"], "solve": rmix["solve"],
        "rel_inf_diff_vs_fp64_gpu": rel_inf(xmx, x64)}
    log("varcoef256_fp64")
    rvc, _, _, _ = run_single(gpcg, torch, dev, args, "varcoef256_fp64", max(args.steps, 20),
                              args.warmup)
    res["varcoef256_fp64"] = {"solves_per_s": rvc["value"], "ms_per_step": rvc["ms_per_step"],
                              "roofline": rvc["roofline"], "autotune": rvc["autotune"],
                              "solve": rvc["solve"]}
    log("batch512_mixed")
    rb, bans = bench_batch(args, gpcg, torch, dev, True, batch_sample)
    res["batch512"] = rb
    log("serve4096")
    rs, sans = bench_serve(args, gpcg, torch, dev, serve_host, serve_sample)
    res["serve4096"] = rs
    res["latency_ms"] = dict(rs["latency_ms"], source="serve4096: Poisson 200 req/s, mixed, "
                             "continuous batching; completion - arrival")
    if not args.no_spmv:
        log("spmv and reduction building blocks")
        res["spmv"] = spmv_extras(gpcg, torch, dev, grids=(1600, 4096, 8192), precs=(0,))
        res["spmv"].update(spmv_extras(gpcg, torch, dev, grids=(8192,), precs=(1,)))
        res["reduction"] = reduction_extras(gpcg, torch, dev)
    torch.cuda.synchronize()

    if pool is not None:
        log("cpu leg: collecting the oracle's answers")
        out = {k: f.result() for k, f in futs.items()}
        pool.shutdown()
        xs = out["xstar1600"]["x"]
        w = inst.w
        acc = {"xstar": {"obstacle1600": "rebuilt from the committed face certificate by one "
                                         "exact face solve, Kuhn-Tucker residual "
                                         f"{out['xstar1600']['kkt']:.2e}",
                         "members": "oracle FP64 GPCG at the metric tolerance, polished by "
                                    "the primal-dual active-set solver"},
               "tol_rel": 1e-8,
               "obstacle1600_fp64": accuracy_entry(x64, xs, st64, 1600, w),
               "obstacle1600_mixed": accuracy_entry(xmx, xs, stmx, 1600, w)}
        bt = [out[("batch", i)] for i in batch_sample]
        acc["batch512_mixed"] = err_summary([rel_inf(bans["batch"][r["index"]], r["xstar"])
                                             for r in bt])
        if "sequential_fp64" in bans:
            acc["batch512_sequential_fp64"] = err_summary(
                [rel_inf(bans["sequential_fp64"][r["index"]], r["xstar"]) for r in bt])
        sv = [out[("serve", i)] for i in serve_sample]
        acc["serve4096_mixed"] = err_summary([rel_inf(sans[r["index"]], r["xstar"])
                                              for r in sv])
        acc["sample"] = (f"{len(bt)} batch members and {len(sv)} requests, stratified by size "
                         "(every k-th in size order)")
        res["accuracy"] = acc
        # oracle solves/sec of the batch and the trace, one thread per solve,
        # projected from the stratified sample
        tb = sum(r["seconds"] for r in bt) * 512 / len(bt)
        ts = sum(r["seconds"] for r in sv) * args.requests / len(sv)
        # all cores: independent solves side by side, one per worker process;
        # the one-thread times above were taken with every worker busy
        many = (f"{workers} oracle solves at a time, one per worker process ({workers} of "
                f"{info['cpus_available']} host CPUs; the GPU legs run meanwhile): {workers} x "
                "the one-thread rate, which was measured with every worker busy")
        res["batch512"]["cpu_baseline"] = dict(
            value=round(512 / tb, 3), unit="solves/s", cores=1, kind="oracle",
            sample=f"{len(bt)} members stratified by size, timed one thread each "
                   f"({workers} worker processes at once); sum scaled to 512 members: "
                   f"{tb:.0f} s",
            all_cores=dict(value=round(workers * 512 / tb, 3), cores=workers, how=many), **info)
        res["serve4096"]["cpu_baseline"] = dict(
            value=round(args.requests / ts, 3), unit="solves/s", cores=1, kind="oracle",
            sample=f"{len(sv)} requests stratified by size, timed one thread each "
                   f"({workers} worker processes at once); sum scaled to "
                   f"{args.requests} requests: {ts:.0f} s",
            all_cores=dict(value=round(workers * args.requests / ts, 3), cores=workers, how=many),
            **info)
        # the headline's oracle time, alone on the host
        log("cpu leg: headline oracle sample")
        res["cpu_baseline"] = cpu_baseline_projected("obstacle_ub_1600", st64["cg_iters"])
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None,
                    choices=sorted(WORKLOADS) + list(BATCH_WORKLOADS) + list(SERVE_WORKLOADS),
                    help="one workload only (default: the headline and every other workload)")
    ap.add_argument("--batch-mode", default="stepped", choices=["persistent", "stepped"])
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-warmup", type=int, default=1)
    ap.add_argument("--requests", type=int, default=4096, help="serving: trace length")
    ap.add_argument("--form", default="auto", choices=["auto", "fused", "split"],
                    help="launch form of single-QP workloads")
    ap.add_argument("--tiles-per-wg", type=int, default=0,
                    help="split form: consecutive tiles per data workgroup (0 = library default)")
    ap.add_argument("--prefetch", default="auto", choices=["auto", "on", "off"],
                    help="early CG operand loads (stencil QPs)")
    ap.add_argument("--chunk", type=int, default=0, help="passes per graph replay (0 = default)")
    ap.add_argument("--precond", default="none", choices=["none", "jacobi"],
                    help="preconditioner of the reduced CG")
    ap.add_argument("--cg-stop", default="decrease", choices=["decrease", "residual"],
                    help="CG stopping test: relative decrease (the paper's) or residual")
    ap.add_argument("--tile", type=int, default=0,
                    help="unknowns per tile (multiple of 256; 0 = library choice)")
    ap.add_argument("--cg-kernel", default="auto", choices=["auto", "on", "off"],
                    help="split form: CG iterations in a data kernel of their own")
    ap.add_argument("--lookahead", default="auto", choices=["auto", "on", "off"],
                    help="fused form: trial passes also evaluate the next step length")
    ap.add_argument("--free-set", default="mask", choices=["mask", "list", "matrix"],
                    help="free set of the reduced CG: byte mask, compacted list, or the "
                         "list with the reduced matrix written out (CSR operators)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (run during warmup, untimed)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch: skip the sequential FP64 comparison")
    ap.add_argument("--extras", action="store_true",
                    help="one workload: time SpMV on 1024^2 and 1600^2 in FP64 and FP32")
    ap.add_argument("--no-spmv", action="store_true", help="skip the SpMV bandwidth figure")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 256 MiB device copy first (counter calibration)")
    ap.add_argument("--counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc output folders and exit")
    args = ap.parse_args()
    if args.counters:
        print(counters_summary(*args.counters))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the QPs would shard by grid strips or by QP; not built). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload is None:
        print(json.dumps(suite(args)), flush=True)
        return

    import torch
    import paper_cs_0101018_amd as gpcg
    dev = torch.device("cuda:0")
    if args.copy_calib:
        # the calibration copy must be the largest copy of the run: no SpMV
        # bandwidth figure (its reference copies reach 512 MiB)
        args.no_spmv = True
        a = torch.empty(COPY_CALIB_BYTES, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy-calib: 268435456 bytes read + written")
        del a, b
    if args.workload in BATCH_WORKLOADS:
        args.batch_steps, args.batch_warmup = max(1, args.steps), args.warmup
        res, _ = bench_batch(args, gpcg, torch, dev, args.workload.endswith("mixed"))
        print(json.dumps(res), flush=True)
        return
    if args.workload in SERVE_WORKLOADS:
        import instances
        reqs = [instances.serve_request(0, i, args.requests) for i in range(args.requests)]
        res, _ = bench_serve(args, gpcg, torch, dev, reqs)
        print(json.dumps(res), flush=True)
        return
    res, _, st, inst = run_single(gpcg, torch, dev, args, args.workload, args.steps, args.warmup)
    if args.extras:
        res["extras"] = spmv_extras(gpcg, torch, dev)
    if not args.no_cpu_baseline:
        key = WORKLOADS[args.workload][0]
        if inst.n > 1_000_000:
            res["cpu_baseline"] = cpu_baseline_projected(key, st["cg_iters"])
        else:
            res["cpu_baseline"] = cpu_baseline_whole(
                inst, precond=int(args.precond == "jacobi"),
                cg_stop=int(args.cg_stop == "residual"))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
