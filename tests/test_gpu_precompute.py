"""Set-up computed on the device (GPU): the Hankel coefficients of eq. H (the contraction of
J0(kappa r) with the r-quadrature on the device) against the host's evaluation of the same
definition (wfp2d_host_eval 3, pinned to Table 1 on the CPU), and the set-up phases the plan
reports.  The NUFFT kernel weights, also made on the device, are covered by every end-to-end
parity test and by the type-1 stage test against the direct Fourier sum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [0, 4])
def test_hankel_table_on_device_matches_host(cfg):
    import paper_2604_07170_amd as pa
    from wfp_workloads import config
    w = config(cfg)
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision="mixed", interp_order=w.p)
    info = plan.info()
    rows = plan.debug(pa.STAGE.HANKEL)
    plan.close()
    assert rows.shape == (info["n_far_classes"], 641)
    pick = np.sort(np.random.default_rng(3).choice(len(rows), size=min(64, len(rows)), replace=False))
    kap = rows[pick, 0]
    host = pa.host_eval(3, [info["A"], 1.0, 30.0] + list(kap), len(kap) * 640).reshape(len(kap), 640)
    err = np.abs(rows[pick, 1:] - host).max() / np.abs(host).max()
    print(f"config {cfg}: {len(rows)} classes, device vs host Hankel table {err:.2e} (of the largest |H|)")
    assert err <= 1e-12
    ms = info["init_ms"]
    print("set-up phases (ms):", [round(x, 1) for x in ms])
    assert ms[6] > 0 and all(x >= 0 for x in ms) and sum(ms[:6]) <= ms[6] * 1.001
