"""Convergence in dt (Sec. 7.1), FP64 form (GPU).

M = 100 random sources, signatures of eq. exampleDensities with t0 in [1.5, 7] and
omega uniform in [0, 10 pi], eps = 1e-8, W = 24; the error at T = 8 on a regular
10 x 10 target mesh against the oracle, for interpolation orders p = 2, 4, ..., 10.
The paper reports rates matching the design order p down to a plateau about one
digit above eps; the local part's time interpolation (eq. sigInterp) is what sets
the order.  eq. dt bounds the step here by (pi - 2b/W)/K0 = 0.0216, so the sweep
runs from dt = 0.02 down.
"""
import math

import numpy as np
import pytest

from gpu_helpers import oracle_field, rel_l2

pytestmark = pytest.mark.gpu

T_FINAL = 8.0
EPS = 1e-8
DTS = [0.02, 0.01, 0.005]


def _workload(dt):
    from wfp_workloads import family_e_workload, grid_targets
    rng = np.random.default_rng(51)
    src = rng.uniform(-1.0, 1.0, size=(100, 2))
    nt = int(round(T_FINAL / dt))
    w = family_e_workload("conv_M100", rng, src, L=10.0, nt=nt, dt=dt, W=24, tol=EPS, T_ref=8.0,
                          tgt=grid_targets(10))
    w.omega = 10.0 * math.pi * np.random.default_rng(52).uniform(0.0, 1.0, size=100)
    return w


def _error(p, dt):
    import torch
    import paper_2604_07170_amd as pa
    w = _workload(dt)
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision="fp64", interp_order=p)
    info = plan.info()
    L = info["lookahead"]
    dev = torch.device("cuda", 0)
    params = w.torch_params(dev)
    u = torch.empty(w.Nx, dtype=torch.float64, device=dev)
    for n in range(1, w.nt + L + 1):
        plan.step(w.sigma_torch(n * w.dt, dev, params))
    plan.evaluate(u)
    torch.cuda.synchronize()
    assert plan.info()["step_reported"] == w.nt
    got = u.cpu().numpy()
    ref = oracle_field(w, info, np.arange(w.Nx), [w.nt], self_mode=0)[:, 0]
    return rel_l2(got, ref)


# time steps per order: down to where the error meets the plateau
DTS_P = {2: [0.02, 0.01, 0.005], 4: [0.02, 0.01, 0.005], 6: [0.02, 0.01, 0.005],
         8: [0.02, 0.016, 0.0125, 0.01, 0.008], 10: [0.02, 0.016, 0.0125, 0.01]}


@pytest.mark.parametrize("p", [2, 4, 6, 8, 10])
def test_convergence_order_in_dt(p):
    dts = DTS_P[p]
    errs = [_error(p, dt) for dt in dts]
    rates = [math.log(errs[i] / errs[i + 1]) / math.log(dts[i] / dts[i + 1]) for i in range(len(errs) - 1)]
    print(f"p = {p}: errors {['%.2e' % e for e in errs]}, observed orders {['%.2f' % r for r in rates]}")
    # measured (MI355X, FP64) at dt = 0.02, 0.016, 0.0125, 0.01, 0.008, 0.005:
    #   p = 2:  1.75e-3 1.10e-3 5.86e-4 3.32e-4 1.76e-4 3.75e-5
    #   p = 4:  9.28e-5 3.72e-5 1.19e-5 4.48e-6 1.49e-6 1.13e-7
    #   p = 6:  6.34e-6 1.64e-6 3.21e-7 7.80e-8 1.63e-8 4.87e-10
    #   p = 8:  4.72e-7 7.87e-8 9.45e-9 1.48e-9 1.94e-10 9.80e-12
    #   p = 10: 3.67e-8 3.95e-9 2.94e-10 3.39e-11 1.26e-11 9.59e-12
    # (orders over the first interval 2.08, 4.10, 6.06, 8.03, 9.99)
    for r in rates:
        assert p - 0.5 <= r <= p + 2.5, rates
    if p >= 6:
        assert _error(p, 0.005) <= 10 * EPS       # at or below the plateau the paper reports (about 10 eps)


def test_error_plateau_at_small_dt():
    """The highest order reaches the method's error floor: halving dt from 0.01 no longer
    gives order 10, and the floor lies below the paper's ~10 eps."""
    e = [_error(10, dt) for dt in (0.01, 0.008, 0.005)]
    print("p = 10 errors at dt = 0.01, 0.008, 0.005:", ["%.2e" % x for x in e])
    assert e[2] > 0.5 * e[1]                      # flat: order 10 would give (0.625)^10 = 0.009
    assert max(e[1:]) <= 10 * EPS
