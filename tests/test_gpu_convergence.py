"""Convergence in dt (Sec. 5.1), FP64 form (GPU).

M = 100 random sources, signatures of eq. exampleDensities with t0 in [1.5, 7] and
omega uniform in [0, 10 pi], eps = 1e-8, W = 24; the error at T = 8 on a regular
10 x 10 target mesh against the oracle, for interpolation orders p.  The paper
reports rates matching the design order p down to a plateau about one digit above
eps; the local part's time interpolation (eq. sigInterp) is what sets the order.
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


@pytest.mark.parametrize("p", [2, 4, 6])
def test_convergence_order_in_dt(p):
    errs = [_error(p, dt) for dt in DTS]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"p = {p}: errors {['%.2e' % e for e in errs]}, observed orders {['%.2f' % r for r in rates]}")
    # measured (MI355X, FP64): p = 2: 1.75e-3, 3.3e-4, 3.8e-5 (orders 2.4, 3.1); p = 4: 9.3e-5,
    # 4.5e-6, 1.1e-7 (4.4, 5.3); p = 6: 6.3e-6, 7.8e-8, 4.9e-10 (6.3, 7.3)
    for r in rates:
        assert p - 0.5 <= r <= p + 2.5, rates
    if p == 6:
        assert errs[-1] <= 10 * EPS          # at or below the plateau the paper reports (about 10 eps)
