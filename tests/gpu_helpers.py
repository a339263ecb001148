"""Shared helpers of the GPU tests: run a workload through the HIP path, sample the oracle."""
import numpy as np


def run_plan(w, precision="mixed", nsteps=None, record=None, **kw):
    """Step a workload through the library; returns (plan, {m: u(t_m) as numpy}).

    record: set of m (reported steps) to keep; default all.  The plan reports
    u(t_{n - lookahead}) after the n-th step, so it is stepped nsteps + lookahead times.
    """
    import torch
    import paper_2604_07170_amd as pa
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p, **kw)
    info = plan.info()
    L = info["lookahead"]
    nt = w.nt if nsteps is None else nsteps
    dev = torch.device("cuda", 0)
    params = w.torch_params(dev)
    out = {}
    u = torch.empty(w.Nx, dtype=torch.float64, device=dev)
    for n in range(1, nt + L + 1):
        plan.step(w.sigma_torch(n * w.dt, dev, params))
        m = n - L
        if m >= 1 and (record is None or m in record):
            plan.evaluate(u)
            out[m] = u.cpu().numpy().copy()
    torch.cuda.synchronize()
    return plan, out


def oracle_field(w, plan_info, target_idx, steps, self_mode=1, **kw):
    import oracle
    return oracle.u_workload(w, target_idx, np.asarray(steps) * w.dt, self_mode=self_mode,
                             delta=plan_info["delta"], b=plan_info["b"], **kw)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
