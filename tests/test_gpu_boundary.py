"""Boundary options of the C ABI on the GPU: non-finite samples (check_finite) and
host-pointer sample/field buffers (host_pointers), against the plain device-pointer plan."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(w, nsteps, bad_step=None, bad_index=0, bad_value=np.nan, **kw):
    """u(t_m) after every step of a plan (device pointers); the sample of `bad_index` at
    `bad_step` replaced by `bad_value`.  Returns ([fields], [statuses of evaluate])."""
    import torch
    import paper_2604_07170_amd as pa
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision="fp64", interp_order=w.p, **kw)
    dev = torch.device("cuda", 0)
    params = w.torch_params(dev)
    out, errs = [], []
    for n in range(1, nsteps + 1):
        s = w.sigma_torch(n * w.dt, dev, params)
        if n == bad_step:
            s[bad_index] = bad_value
        plan.step(s)
        u = torch.empty(w.Nx, dtype=torch.float64, device=dev)
        try:
            plan.evaluate(u)
            errs.append(0)
        except pa.Wfp2dError as e:
            errs.append(e.code)
        out.append(u.cpu().numpy())
    return plan, out, errs


def test_nonfinite_sample_is_reported_once_and_taken_as_zero():
    import paper_2604_07170_amd as pa
    from wfp_workloads import config
    w = config(0)
    n_bad, j_bad = 30, 5
    plan, got, errs = _run(w, 50, bad_step=n_bad, bad_index=j_bad, bad_value=np.nan, check_finite=True)
    # the count is copied back after each evaluation: reported at the step's evaluation or a later one
    reported = [n + 1 for n, e in enumerate(errs) if e == pa.ERR_NONFINITE]
    assert len(reported) <= 1 and (not reported or n_bad <= reported[0] <= n_bad + 2)
    if not reported:
        with pytest.raises(pa.Wfp2dError) as ei:
            plan.info()                                 # synchronises, then reports
        assert ei.value.code == pa.ERR_NONFINITE
    plan.info()                                         # reported once: no error any more
    plan.close()
    ref_plan, ref, ref_errs = _run(w, 50, bad_step=n_bad, bad_index=j_bad, bad_value=0.0)
    ref_plan.close()
    assert all(e == 0 for e in ref_errs)
    # same arithmetic; the local part's atomic sums may add in another order
    for a, b in zip(got, ref):
        assert np.all(np.isfinite(a))
        assert np.linalg.norm(a - b) <= 1e-12 * max(np.linalg.norm(b), 1e-300)


def test_infinite_sample_with_check_off_is_not_reported():
    import paper_2604_07170_amd as pa
    from wfp_workloads import config
    w = config(0)
    plan, got, errs = _run(w, 12, bad_step=3, bad_index=0, bad_value=np.inf)
    assert all(e == 0 for e in errs)
    plan.info()
    plan.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_host_pointer_plan_matches_device_pointer_plan(precision):
    import torch
    import paper_2604_07170_amd as pa
    from wfp_workloads import tiny
    w = tiny(seed=3, M=20, L=2.0)
    dev = torch.device("cuda", 0)
    params = w.torch_params(dev)
    pd = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p)
    ph = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p, host_pointers=True)
    try:
        for n in range(1, 41):
            s = w.sigma_torch(n * w.dt, dev, params)
            pd.step(s)
            sh = s.cpu().numpy()
            ph.step(sh)
            sh[:] = np.nan                       # the library copied the samples before returning
            ud = pd.evaluate().cpu().numpy()
            uh = ph.evaluate()                   # numpy, written on return
            assert isinstance(uh, np.ndarray)
            assert np.linalg.norm(ud - uh) <= 1e-12 * max(np.linalg.norm(ud), 1e-300), n
        assert np.linalg.norm(ud) > 0
        with pytest.raises(pa.Wfp2dError) as ei:
            ph.graph_capture(torch.zeros(w.M, dtype=torch.float64, device=dev),
                             torch.zeros(w.Nx, dtype=torch.float64, device=dev))
        assert ei.value.code == -6
    finally:
        pd.close()
        ph.close()
