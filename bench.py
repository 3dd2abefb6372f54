"""Benchmark: GPCG solves/sec on one MI355X, with the roofline of the pass
kernel and the FP64 CPU oracle timed beside it.

One step = one complete GPCG solve (every pass of Algorithm GPCG: projection,
gradients, gradient-projection searches, reduced CG, projected searches,
termination) of the 256 x 256 variable-coefficient problem at projected-
gradient tolerance 1e-8 relative, FP64, from x0 = 0.  Inputs are resident in
HBM before the timed region; each step restores x0 on the device.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--extras] [--copy-calib]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E datasheet peak

WORKLOADS = {
    # name: (instance factory, options, description)
    "varcoef256_fp64": ("config1", dict(), "GPCG FP64, -div(c grad u) 256x256 (n=65,536), "
                        "c=(1+0.1 cos 2 pi s)^3, l=0, u=inf, tol 1e-8 rel"),
    "varcoef256_mixed": ("config1", dict(precision=1), "GPCG mixed FP32-CG, varcoef 256x256"),
    "obstacle50_fp64": ("config0", dict(), "GPCG FP64, obstacle 50x50"),
    "obstacle1024_fp64": ("config2_1024", dict(), "GPCG FP64, obstacle 1024x1024"),
    "obstacle1024_mixed": ("config2_1024", dict(precision=1), "GPCG mixed, obstacle 1024x1024"),
    "obstacle1600_fp64": ("config2_1600", dict(), "GPCG FP64, obstacle 1600x1600"),
    "obstacle1600_mixed": ("config2_1600", dict(precision=1), "GPCG mixed, obstacle 1600x1600"),
}


def make_instance(key):
    import instances
    if key == "config0":
        return instances.config0(0)
    if key == "config1":
        return instances.config1(0)
    if key.startswith("config2_"):
        return instances.config2(int(key.split("_")[1]), 0)
    raise KeyError(key)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(inst, budget_s=12.0):
    """The FP64 oracle, as it stands, on this host: solves/sec on a bounded
    sample (whole solves of the same workload until the budget is spent)."""
    import oracle
    ora = oracle.default()
    csr = inst.csr()
    t0 = time.perf_counter()
    k = 0
    while True:
        ora.gpcg(csr, inst.b, inst.l, inst.u, inst.x0)
        k += 1
        el = time.perf_counter() - t0
        if el >= budget_s or k >= 200:
            break
    return dict(value=k / el, unit="solves/s", cores=1, kind="oracle",
                sample=f"{k} complete solves of the same instance in {el:.1f} s "
                       f"(single-threaded C, -O2 -ffp-contract=off)")


def spmv_extras(gpcg, torch, dev):
    """SpMV bandwidth of the building-block kernel on the large grids, warm and
    with the 256 MB last-level cache flushed before each launch."""
    out = {}
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    for N in (1024, 1600):
        for prec in (0, 1):
            op = gpcg.Operator.stencil_const(N, N, float((N + 1) ** 2))
            s = gpcg.Solver(op, device=dev, precision=prec)
            dt = torch.float32 if prec else torch.float64
            v = torch.randn(N * N, dtype=torch.float64, device=dev).to(dt)
            y = torch.empty_like(v)
            mask = torch.ones(N * N, dtype=torch.uint8, device=dev)
            per = 2 * v.element_size() + 1
            for cold in (False, True):
                times = []
                for it in range(12):
                    if cold:
                        flush.fill_(it & 0xFF)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    s.spmv(v, y, mask)
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                t = float(np.median(times[2:])) * 1e-3
                key = f"spmv_const{N}_{'fp32' if prec else 'fp64'}_{'cold' if cold else 'warm'}"
                out[key] = dict(GBs=round(per * N * N / t / 1e9, 1), us=round(t * 1e6, 2),
                                bytes_per_var=per)
            s.close()
    del flush
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="varcoef256_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time SpMV on 1024^2/1600^2")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 256 MiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_cs_0101018_amd as gpcg

    dev = torch.device("cuda:0")
    key, opts, desc = WORKLOADS[args.workload]
    inst = make_instance(key)
    N = inst.N
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    if args.copy_calib:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy-calib: 268435456 bytes read + written")
        del a, b

    if inst.op == "var":
        wx, wy = inst.edge_weights()
        op = gpcg.Operator.stencil_var(N, N, t(wx.ravel()), t(wy.ravel()))
    else:
        op = gpcg.Operator.stencil_const(N, N, inst.w)
    solver = gpcg.Solver(op, device=dev, **opts)
    b, l, u, x0 = t(inst.b), t(inst.l), t(inst.u), t(inst.x0)
    x = torch.empty_like(x0)

    def step():
        x.copy_(x0)
        return solver.solve(b, l, u, x)

    for _ in range(args.warmup):
        st = step()
    torch.cuda.synchronize()
    stats = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        stats.append(step())
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    st = stats[-1]
    assert all(s["status"] == 0 for s in stats), [s["status"] for s in stats]

    launches = sum(s["launches"] for s in stats)
    passes = sum(s["passes"] for s in stats)
    alg_bytes = sum(s["bytes"] for s in stats)
    avg_launch_s = gpu_ms * 1e-3 / launches
    bytes_per_launch = alg_bytes / launches
    achieved = bytes_per_launch / avg_launch_s / 1e9
    solves_per_s = args.steps / wall

    res = {
        "metric": "GPCG solves/sec (proj-grad tol 1e-8 rel)",
        "value": round(solves_per_s, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not opts.get("precision") else "f64+f32cg",
        "data": "synthetic (seeded instance generator, seed 0)",
        "config": {"workload": args.workload, "description": desc, "n": inst.n,
                   "grid": f"{N}x{N}", "tol_rel": 1e-8, "global_batch": 1,
                   "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm",
            "kernel": "gpcg::step_kernel (one fused GPCG pass per launch)",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": None,
            "bytes_per_launch": round(bytes_per_launch, 1),
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "launches_per_solve": launches / args.steps,
            "useful_passes_per_solve": passes / args.steps,
        },
        "solve": {k: st[k] for k in ("outer_iters", "gp_iters", "cg_iters", "backtracks",
                                     "face_repeats", "passes", "launches", "pg", "tau")},
        "phase_ms": {k: round(st[k], 3) for k in ("ms_cg", "ms_gp", "ms_search", "ms_other")},
    }
    if args.extras:
        res["extras"] = spmv_extras(gpcg, torch, dev)
    solver.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
