#!/usr/bin/env python3
"""Write the oracle's field on a 5 x 5 subset of the 900 x 900 target mesh of the
random space-filling example as the paper runs it (10^6 random sources, targets on
the separate mesh, T = 8): tests/golden/cfg7_oracle_samples.txt.

The values are the plain definition of the field (Sec. 1, eqs. solnRep, Green;
Sec. 7, eq. exactSol) evaluated by the CPU oracle with the analytic signatures of
eq. exampleDensities.  No target coincides with a source.  Nothing here runs or
reads the GPU library.

Sample: the mesh points (ix, iy) with ix, iy in {90, 270, 450, 630, 810} (a regular
5 x 5 subset of the mesh, the size of the paper's error check at T = 8), at the
final step 7150 (T = 8) and at step 3575 (t = 4).

Run time: about 40 minutes on 8 cores.  Progress is appended to a partial file
after each step, so an interrupted run resumes where it stopped.

    python tests/golden/make_cfg7_golden.py [--threads N]
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from wfp_workloads import config  # noqa: E402

OUT = os.path.join(HERE, "cfg7_oracle_samples.txt")
PARTIAL = OUT + ".partial"
SUB = [90, 270, 450, 630, 810]
STEPS = [3575, 7150]


def sample_targets() -> np.ndarray:
    return np.array(sorted(iy * 900 + ix for iy in SUB for ix in SUB))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    w = config(7)
    delta = w.W * w.dt                 # eq. W
    b = math.log(1.0 / w.tol)          # Sec. 2.1
    ti = sample_targets()
    done = {}
    if os.path.exists(PARTIAL):
        for line in open(PARTIAL):
            i, n, v = line.split()
            done[(int(i), int(n))] = v
    for n in sorted(STEPS, reverse=True):
        if all((int(i), n) in done for i in ti):
            continue
        t0 = time.time()
        u = oracle.u_workload(w, ti, [n * w.dt], self_mode=0, delta=delta, b=b, nthreads=args.threads)[:, 0]
        with open(PARTIAL, "a") as f:
            for i, v in zip(ti, u):
                f.write(f"{int(i)} {n} {float(v)!r}\n")
                done[(int(i), n)] = repr(float(v))
        print(f"step {n}: {time.time() - t0:.0f} s, |u| max {np.abs(u).max():.3e}", flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle field u(x_i, t_n) of the seeded random space-filling example as the paper runs it\n")
        f.write("# (10^6 sources, eq. exampleDensities signatures, dt = 8/7150, T = 8, targets on the 900 x 900\n")
        f.write("# mesh).  Plain definition of Sec. 1 eqs. solnRep, Green and Sec. 7 eq. exactSol by the CPU\n")
        f.write("# oracle.  Written by make_cfg7_golden.py.\n")
        f.write("# targets: mesh points iy * 900 + ix with ix, iy in {90, 270, 450, 630, 810}\n")
        f.write("# columns: target_index step u\n")
        for n in STEPS:
            for i in ti:
                f.write(f"{int(i)} {n} {done[(int(i), n)]}\n")
    os.remove(PARTIAL)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
