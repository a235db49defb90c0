"""Writes cfg3_oracle_energy.json: the FP64 oracle's Davidson ground-state
energy of the D = 4096 synthetic workload (L = 54, N = 54, 2Sz = 0, mean
sector 64, max 512, 3000 random terms in adjoint pairs plus the gapped
diagonal terms, seed 3), started from the same vector as the device runs.

Calls only the oracle (sigma by the definition of Eq. (2), Davidson's
iteration) on inputs from the seeded generator; nothing here touches the
GPU library.  Takes about an hour on eight cores and ~50 GB of memory.

    python tests/golden/make_cfg3_energy.py [--threads N]
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from synth import synthetic_problem, gapped_guess  # noqa: E402
from oracle import heff  # noqa: E402
from oracle.davidson import davidson  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg3_oracle_energy.json")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--tol-res", type=float, default=1e-7)
    args = ap.parse_args()
    t0 = time.time()
    P = synthetic_problem(54, 54, 0, 4096, 64, 512, 3000, seed=3, gapped=True, threads=args.threads)
    print("generated %d terms, %d blocks (%.0f s)" % (P.nTerms, P.nBlk, time.time() - t0), flush=True)
    t0 = time.time()
    tasks = heff.enumerate_tasks(P)
    tasks.sort(key=lambda t: t[0])  # canonical table order (stable by output sector)
    flops = heff.total_flops(tasks)
    d = heff.diagonal(P, tasks)
    print("tasks %d, %.3f TFLOP per product (%.0f s)" % (len(tasks), flops / 1e12, time.time() - t0), flush=True)
    times = []

    def mv(x):
        t = time.time()
        y, _ = heff.sigma_threaded(P, x, tasks, threads=args.threads)
        times.append(time.time() - t)
        print("  product %d: %.1f s" % (len(times), times[-1]), flush=True)
        return y

    x0 = gapped_guess(P, 2)
    t0 = time.time()
    e, x, info = davidson(mv, d, x0, tol_res=args.tol_res, tol_e=1e-12, max_sub=32, keep=8, max_iter=200)
    wall = time.time() - t0
    rec = {
        "workload": "L=54 N=54 2Sz=0 D=4096 per block (mean sector 64, max 512), 3000 terms + gapped diagonal, "
                    "seed 3; start vector gapped_guess(seed 2)",
        "energy": float(e), "iters": int(info["iters"]), "matvecs": int(info["matvecs"]),
        "res_norm": float(info["res"]), "tol_res": args.tol_res, "tol_e": 1e-12, "max_sub": 32, "keep": 8,
        "davidson_seconds": round(wall, 1), "seconds_per_product": round(float(np.median(times)), 2),
        "flops_per_product": flops, "oracle_tflops": round(flops / float(np.median(times)) / 1e12, 4),
        "threads": args.threads, "cpu_model": cpu_model(),
        "written_by": "tests/golden/make_cfg3_energy.py (oracle only)",
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
