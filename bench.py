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
BATCH_WORKLOADS = ("batch512_fp64", "batch512_mixed")
SERVE_WORKLOADS = ("serve4096",)


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


def _dev_instance(inst, gpcg, torch, dev):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    N = inst.N
    if inst.op == "var":
        wx, wy = inst.edge_weights()
        op = gpcg.Operator.stencil_var(N, N, t(wx.ravel()), t(wy.ravel()))
    else:
        op = gpcg.Operator.stencil_const(N, N, inst.w)
    return op, t(inst.b), t(inst.l), t(inst.u), t(inst.x0)


def bench_batch(args, gpcg, torch, dev):
    """512 independent QPs of uneven size in one batch (persistent launch or
    stepped graph chunks) against 512 sequential plain FP64 solves."""
    import instances
    mixed = args.workload.endswith("mixed")
    insts = instances.config3(0)
    data = [_dev_instance(i, gpcg, torch, dev) for i in insts]
    mode = gpcg.GPCG_BATCH_PERSISTENT if args.batch_mode == "persistent" else gpcg.GPCG_BATCH_STEPPED
    solvers = [gpcg.Solver(d[0], device=dev, precision=int(mixed)) for d in data]
    batch = gpcg.Batch(solvers, device=dev)
    xs = [torch.empty_like(d[4]) for d in data]
    probs = [(d[1], d[2], d[3], x) for d, x in zip(data, xs)]

    def run_batch():
        for d, x in zip(data, xs):
            x.copy_(d[4])
        return batch.solve(probs, mode=mode)

    for _ in range(args.warmup):
        run_batch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = run_batch()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    bad = [s["status"] for s in st if s["status"] != 0]
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
    n_tot = sum(i.n for i in insts)
    err = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(xs, x1))
    return {
        "metric": "GPCG solves/sec, 512-QP batch (proj-grad tol 1e-8 rel)",
        "value": round(len(insts) / wall, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32cg" if mixed else "f64", "data": "synthetic (config-3 generator, seed 0)",
        "config": {"workload": args.workload, "qps": len(insts), "unknowns": n_tot,
                   "batch_mode": args.batch_mode},
        "sequential_fp64": {"solves_per_s": round(len(insts) / seq_wall, 2),
                            "ms_total": round(seq_wall * 1e3, 1)},
        "speedup_vs_sequential_fp64": round(seq_wall / wall, 3),
        "max_rel_diff_vs_sequential_fp64": err,
        "failed": len(bad),
    }


def bench_serve(args, gpcg, torch, dev):
    """Poisson arrivals at 200 req/s replayed against the continuous-batching
    server (mixed precision), and the same trace through a plain FP64
    one-at-a-time loop (FIFO, service times measured on the same GPU)."""
    import instances
    count = args.requests
    arr = instances.config4_trace(0, count)
    log(f"serve: generating {count} requests")
    reqs = []
    for i in range(count):
        inst = instances.config4_request(0, i, count)
        reqs.append((inst.n,) + _dev_instance(inst, gpcg, torch, dev))
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
        if active == 0 and nxt < count:
            time.sleep(max(0.0, min(0.002, arr[nxt] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    # the library stamps completions with the monotonic clock that
    # time.perf_counter() reads on Linux: latency = completion - arrival
    lat = np.array([done[i]["t_done"] - (t0 + arr[i]) for i in range(count)])
    bad = sum(1 for c in done.values() if c["status"] != 0)
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
    finish = np.zeros(count)
    tcur = 0.0
    for i in range(count):
        tcur = max(tcur, arr[i]) + service[i]
        finish[i] = tcur
    lat_seq = finish - arr
    return {
        "metric": "GPCG serving: solves/sec and p50/p99 latency (Poisson 200 req/s)",
        "value": round(count / wall, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(wall * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32cg", "data": "synthetic (config-4 generator and trace, seed 0)",
        "config": {"workload": "serve4096", "requests": count, "rate_hz": 200,
                   "max_slots": 512, "quantum": 32},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 2)},
        "fp64_one_at_a_time": {
            "solves_per_s": round(count / max(finish[-1], arr[-1]), 2),
            "p50_ms": round(float(np.percentile(lat_seq, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat_seq, 99)) * 1e3, 2),
            "mean_service_ms": round(float(service.mean()) * 1e3, 3)},
        "failed": bad,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="varcoef256_fp64",
                    choices=sorted(WORKLOADS) + list(BATCH_WORKLOADS) + list(SERVE_WORKLOADS))
    ap.add_argument("--batch-mode", default="persistent", choices=["persistent", "stepped"])
    ap.add_argument("--requests", type=int, default=4096, help="serving: trace length")
    ap.add_argument("--form", default="auto", choices=["auto", "fused", "split"],
                    help="launch form of single-QP workloads")
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
    if args.workload in BATCH_WORKLOADS:
        print(json.dumps(bench_batch(args, gpcg, torch, dev)), flush=True)
        return
    if args.workload in SERVE_WORKLOADS:
        print(json.dumps(bench_serve(args, gpcg, torch, dev)), flush=True)
        return
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
    form = {"auto": gpcg.GPCG_FORM_AUTO, "fused": gpcg.GPCG_FORM_FUSED,
            "split": gpcg.GPCG_FORM_SPLIT}[args.form]
    solver = gpcg.Solver(op, device=dev, form=form, **opts)
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
