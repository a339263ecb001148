#!/usr/bin/env python3
"""Write the oracle's field at a seeded sample of (target, step) pairs of the
10^6-source, 300 x 300-wavelength workload: tests/golden/cfg4_oracle_samples.txt.

The values are the plain definition of the field (Sec. 1, eqs. solnRep, Green;
Sec. 7, eq. exactSol) evaluated by the CPU oracle with the analytic signatures
of eq. exampleDensities.  Sources = targets, so each target coincides with one
source: that pair contributes its windowed history (the oracle's self_mode = 1,
with delta = W dt of eq. W and b = ln(1/eps) of Sec. 2.1).  Nothing here runs
or reads the GPU library.

Sample: 32 targets drawn by numpy default_rng(4040) without replacement, at the
steps listed in STEPS: two before the far history starts (step LA = 4300 at this
workload), three between its onset and the benchmark window, three inside the
window 5801..6000 (step 6000, the window's last, included).

Run time: about 2.5 hours on 8 cores (the cost of one sample grows with t; one
sample at step 6000 is ~450 core-seconds).  Progress is appended to a partial
file after each step, so an interrupted run resumes where it stopped.

    python tests/golden/make_cfg4_golden.py [--threads N]
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

OUT = os.path.join(HERE, "cfg4_oracle_samples.txt")
PARTIAL = OUT + ".partial"
N_TARGETS = 32
TARGET_SEED = 4040
STEPS = [1200, 3000, 4400, 5000, 5600, 5850, 5950, 6000]


def sample_targets(M: int) -> np.ndarray:
    return np.sort(np.random.default_rng(TARGET_SEED).choice(M, size=N_TARGETS, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    w = config(4)
    delta = w.W * w.dt                 # eq. W
    b = math.log(1.0 / w.tol)          # Sec. 2.1
    ti = sample_targets(w.M)
    done = {}
    if os.path.exists(PARTIAL):
        for line in open(PARTIAL):
            i, n, v = line.split()
            done[(int(i), int(n))] = v
    for n in sorted(STEPS, reverse=True):        # the benchmark window first
        if all((int(i), n) in done for i in ti):
            continue
        t0 = time.time()
        u = oracle.u_workload(w, ti, [n * w.dt], self_mode=1, delta=delta, b=b, nthreads=args.threads)[:, 0]
        with open(PARTIAL, "a") as f:
            for i, v in zip(ti, u):
                f.write(f"{int(i)} {n} {float(v)!r}\n")
                done[(int(i), n)] = repr(float(v))
        print(f"step {n}: {time.time() - t0:.0f} s, |u| max {np.abs(u).max():.3e}", flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle field u(x_i, t_n) of the seeded 10^6-source workload (300 x 300 wavelengths,\n")
        f.write("# eq. exampleDensities signatures, dt = 8/7150, W = 16, eps = 1e-7; sources = targets,\n")
        f.write("# coincident pair as its windowed history).  Plain definition of Sec. 1 eqs. solnRep,\n")
        f.write("# Green and Sec. 7 eq. exactSol by the CPU oracle.  Written by make_cfg4_golden.py.\n")
        f.write(f"# targets: default_rng({TARGET_SEED}).choice(M, {N_TARGETS}, replace=False), sorted\n")
        f.write("# columns: target_index step u\n")
        for n in STEPS:
            for i in ti:
                f.write(f"{int(i)} {n} {done[(int(i), n)]}\n")
    os.remove(PARTIAL)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
