"""Parity at the benchmark's full size (GPU): 10^6 random sources = targets, 300 x 300
wavelengths, dt = 8/7150, W = 16, p = 20, eps = 1e-7, run through all 6000 steps in the
launch configuration the benchmark times.

The reference values are the oracle's field at 32 seeded targets and 8 steps
(tests/golden/cfg4_oracle_samples.txt, written by make_cfg4_golden.py beside it from the
plain definition of Sec. 1 eqs. solnRep, Green with the signatures of Sec. 7 eq.
exampleDensities): two steps before the far history starts (its onset is step 4300 here),
three between its onset and the benchmark's timed window, three inside the window.

Bar: relative L2 error over the 32 samples of each step at most 1e-6 (the accuracy the
throughput figure is quoted at) for the mixed form; the FP64 form, whose error is the
method's own (about 10 eps, Sec. 7.1), at most 1e-7.

Without look-ahead the local part interpolates sigma from past levels only, as eq.
sigInterp is written (levels t_{n - nm + l}, l = 1..nm): at delays below p/2 steps the
p-point stencil is one-sided, whose interpolation error is several orders larger than
the centred stencil's (the Lagrange basis grows towards the stencil's end).  Measured on
MI355X at this workload: 3.4e-5 at step 1200, 7e-6 .. 1.2e-5 from step 3000 on (the
look-ahead form: 1.6e-7 .. 2.6e-7).  Its bar is 1e-4, and the look-ahead form must be
at least 10 times more accurate.
"""
import gc
import os

import numpy as np
import pytest

from gpu_helpers import rel_l2, run_plan

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg4_oracle_samples.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        i, n, v = line.split()
        vals.setdefault(int(n), {})[int(i)] = float(v)
    return vals


def _check(precision, bar, **kw):
    import torch
    from wfp_workloads import config
    g = _golden()
    steps = sorted(g)
    assert len(steps) == 8 and all(len(g[n]) == 32 for n in steps)
    w = config(4)
    plan, out = run_plan(w, precision=precision, nsteps=max(steps), record=set(steps), **kw)
    info = plan.info()
    del plan
    gc.collect()
    torch.cuda.empty_cache()
    errs = {}
    for n in steps:
        ti = np.array(sorted(g[n]))
        ref = np.array([g[n][i] for i in ti])
        errs[n] = rel_l2(out[n][ti], ref)
    print(f"{precision} lookahead {info['lookahead']}: rel L2 per step",
          {n: f"{e:.2e}" for n, e in errs.items()})
    assert max(errs.values()) <= bar, errs
    _ERRS[(precision, info["lookahead"])] = max(errs.values())
    return info


_ERRS = {}


def test_cfg4_mixed_matches_oracle():
    info = _check("mixed", 1e-6)
    assert info["lookahead"] == 9 and info["local_path"] == 2


def test_cfg4_fp64_matches_oracle():
    info = _check("fp64", 1e-7)
    assert info["local_path"] == 2


def test_cfg4_mixed_without_lookahead_matches_oracle():
    info = _check("mixed", 1e-4, lookahead=0)
    assert info["lookahead"] == 0
    if ("mixed", 9) in _ERRS:
        assert _ERRS[("mixed", 9)] * 10 <= _ERRS[("mixed", 0)], _ERRS
