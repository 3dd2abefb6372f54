"""Writes the face certificates of the large obstacle problems (the active set
of x*), which tests rebuild x* from by one exact face solve and verify with
the Kuhn-Tucker conditions (``oracle.exact.xstar_from_face``).

Calls only the seeded input generator and ``oracle/``: the FP64 GPCG oracle at
a tight tolerance, then the primal-dual active-set iteration with exact face
solves from its answer until the active set repeats.

    python tests/golden/make_faces.py 1024 1600
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import instances  # noqa: E402
import oracle  # noqa: E402
from oracle import exact  # noqa: E402


def face_file(N, seed=0):
    return os.path.join(HERE, f"face_obstacle_ub_{N}_seed{seed}.txt")


def main(sizes):
    for N in sizes:
        inst = instances.obstacle_ub(N, 0)
        t0 = time.time()
        xo, _, st = oracle.default().solve_instance(inst, tol_rel=1e-10)
        print(f"{N}: oracle {time.time() - t0:.1f} s, status {st['status']}, "
              f"pg {st['pg']:.3e}", flush=True)
        x, it, ok = exact.pdas_const(N, inst.w, inst.b, inst.l, inst.u, xo)
        assert ok
        lo = np.flatnonzero(x == inst.l)
        up = np.flatnonzero((x == inst.u) & (x != inst.l))
        xs, g, kkt = exact.xstar_from_face(N, inst.w, inst.b, inst.l, inst.u, lo, up)
        print(f"{N}: PDAS {it} iterations, {len(lo)} lower / {len(up)} upper active, "
              f"KKT residual {kkt:.3e}, |x*|_inf {np.abs(xs).max():.6f}", flush=True)
        with open(face_file(N), "w") as f:
            f.write(f"# Face of x* for the obstacle problem with both bounds, {N}x{N}, seed 0\n"
                    f"# (5-point Laplacian / h^2, b = 1; l and u from the seeded generator).\n"
                    f"# Written by tests/golden/make_faces.py from the FP64 GPCG oracle at\n"
                    f"# tol_rel 1e-10 and a primal-dual active-set polish; x* is rebuilt from\n"
                    f"# it by one exact face solve and accepted only if it satisfies the\n"
                    f"# Kuhn-Tucker conditions.  Indices k = j N + i.\n")
            f.write(f"N {N}\n")
            for name, arr in (("lower", lo), ("upper", up)):
                f.write(f"{name} {len(arr)}\n")
                for k0 in range(0, len(arr), 10):
                    f.write(" ".join(str(int(v)) for v in arr[k0:k0 + 10]) + "\n")


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1024, 1600])
