"""The local part from stored pair lists (the default) against the per-step pair
search, and against the oracle (GPU).

Both paths evaluate the same pairs with the same panel and coordinate (Sec. 6,
eq. local2).  With the same number of Chebyshev terms only the order of the
per-target additions differs, so the fields agree to rounding; a mixed-precision
plan may drop trailing terms whose sum is at most 1e-3 tol of the largest
coefficient, and the fields must then still agree to 0.05 tol.  A workload with targets placed
within dt/2 of sources covers the dyadic sub-panels, which have lists of
their own.
"""
import numpy as np
import pytest

from gpu_helpers import oracle_field, rel_l2

pytestmark = pytest.mark.gpu


def _lockstep(w, precision, steps, **kw):
    """Step a pair-list plan and a pair-search plan on the same samples; fields at `steps`."""
    import torch
    import paper_2604_07170_amd as pa
    a = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p, **kw)
    b = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p, local_pairs=False, **kw)
    ia, ib = a.info(), b.info()
    L = ia["lookahead"]
    dev = torch.device("cuda", 0)
    params = w.torch_params(dev)
    ua = torch.empty(w.Nx, dtype=torch.float64, device=dev)
    ub = torch.empty_like(ua)
    out_a, out_b = {}, {}
    for n in range(1, max(steps) + L + 1):
        s = w.sigma_torch(n * w.dt, dev, params)
        a.step(s)
        b.step(s)
        if n - L in steps:
            a.evaluate(ua)
            b.evaluate(ub)
            out_a[n - L], out_b[n - L] = ua.cpu().numpy(), ub.cpu().numpy()
    torch.cuda.synchronize()
    return ia, ib, out_a, out_b


def _agreement(ia, ib, w):
    """Bound on the relative difference of the two paths' fields."""
    return 1e-12 if ia["cheb_degree"] == ib["cheb_degree"] else 0.05 * w.tol


def _near_coincident(n_src=256, seed=31):
    """Uniform sources, 4 wavelengths (dt = 0.05); each target sits at a distance in
    [0.01, 0.9] dt from its source, so that both dyadic (r < dt/2) and regular pairs occur."""
    from wfp_workloads import family_g_workload
    rng = np.random.default_rng(seed)
    L = 4.0
    dt = 2.0 / L / 10.0
    src = rng.uniform(-0.9, 0.9, size=(n_src, 2))
    rad = dt * rng.uniform(0.01, 0.9, size=n_src)
    ang = rng.uniform(0.0, 2 * np.pi, size=n_src)
    tgt = src + np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
    w = family_g_workload("near_coincident", rng, src, L=L, nt=60, tgt=tgt)
    assert abs(w.dt - dt) < 1e-15
    return w


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_lists_match_pair_search_config0(precision):
    from wfp_workloads import config
    w = config(0)
    steps = {40, 120, 200}
    ia, ib, ua, ub = _lockstep(w, precision, steps)
    assert ia["local_path"] == 2 and ia["local_pair_bytes"] > 0
    assert ib["local_path"] == 1 and ib["local_pair_bytes"] == 0
    assert ib["cheb_degree"] == 20 and (ia["cheb_degree"] == 20 if precision == "fp64" else ia["cheb_degree"] <= 20)
    assert abs(ia["n_local_pairs"] - ib["n_local_pairs"]) <= max(2, 1e-6 * ib["n_local_pairs"])
    print(f"config0 {precision}: Chebyshev terms {ia['cheb_degree']} (pair lists) vs {ib['cheb_degree']} (search)")
    for m in sorted(steps):
        d = rel_l2(ua[m], ub[m])
        print(f"config0 {precision} step {m}: pair lists vs search rel diff {d:.2e}")
        assert d <= _agreement(ia, ib, w)


def test_pair_lists_match_pair_search_config2():
    """65536 uniform sources: many cells and chunks, some cells with two chunks."""
    from wfp_workloads import config
    w = config(2)
    steps = {780, 820}                  # the signatures start at t >= 2.25 (step 750)
    ia, ib, ua, ub = _lockstep(w, "mixed", steps)
    assert ia["local_path"] == 2
    for m in sorted(steps):
        assert np.isfinite(ua[m]).all() and np.linalg.norm(ub[m]) > 0
        d = rel_l2(ua[m], ub[m])
        print(f"config2 mixed step {m}: pair lists vs search rel diff {d:.2e}")
        assert d <= _agreement(ia, ib, w)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_lists_dyadic_pairs_against_oracle(precision):
    w = _near_coincident()
    steps = {15, 45}
    ia, ib, ua, ub = _lockstep(w, precision, steps)
    assert ia["local_path"] == 2
    idx = np.arange(w.Nx)
    for m in sorted(steps):
        assert np.isfinite(ua[m]).all() and np.linalg.norm(ub[m]) > 0
        d = rel_l2(ua[m], ub[m])
        assert d <= _agreement(ia, ib, w), d
    U = np.array([ua[m] for m in sorted(steps)]).T
    Uo = oracle_field(w, ia, idx, sorted(steps), self_mode=0)
    err = rel_l2(U, Uo)
    print(f"near-coincident {precision}: rel L2 vs oracle {err:.3e}")
    assert err <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_lists_several_target_batches(precision):
    """4096 sources = targets clustered in a 0.2 x 0.2 square: one cell's 5 x 5 block holds
    all 4096 targets, more than one batch of 1024, so each chunk's pairs come in four
    segments flushed one after the other.  Against the per-step search (which batches
    512 targets at a time) and the oracle."""
    from wfp_workloads import family_g_workload
    rng = np.random.default_rng(41)
    src = np.array([0.3, -0.2]) + rng.uniform(-0.1, 0.1, size=(4096, 2))
    w = family_g_workload("cluster4096", rng, src, L=4.0, nt=40)
    steps = {20, 40}
    ia, ib, ua, ub = _lockstep(w, precision, steps)
    assert ia["local_path"] == 2
    for m in sorted(steps):
        assert np.isfinite(ua[m]).all() and np.linalg.norm(ub[m]) > 0
        d = rel_l2(ua[m], ub[m])
        print(f"cluster {precision} step {m}: pair lists vs search rel diff {d:.2e}")
        assert d <= _agreement(ia, ib, w)
    tg = np.sort(rng.choice(w.Nx, size=24, replace=False))
    U = np.array([ua[m][tg] for m in sorted(steps)]).T
    Uo = oracle_field(w, ia, tg, sorted(steps))
    err = rel_l2(U, Uo)
    print(f"cluster {precision}: rel L2 vs oracle {err:.3e}")
    assert err <= 1e-6
