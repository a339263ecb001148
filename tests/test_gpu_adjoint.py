"""The adjoint: transposition, gradients with respect to source strengths,
checkpoints (GPU).

* dot-product test: <g, K sigma> = <K^T g, sigma> for random sigma and g,
  with K the plan's discrete operator and K^T the transposed plan run on
  time-reversed input;
* central finite differences of a quadratic loss on 32 strengths (exact to
  rounding for a quadratic: the loss is a quadratic form in A);
* the oracle's transpose: for a linear loss sum g u, dL/dA_j equals
  sum_{i,m} g_i(t_m) u_ij(t_m), with u_ij the oracle's field of source j alone;
* the checkpointed loss (forward state saved every few steps, u recomputed
  segment by segment in the backward) gives the stored-field gradient;
* saving and loading the plan state reproduces the continuation.
"""
import dataclasses

import numpy as np
import pytest

from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


def _unit_signatures(w, n_max, dev):
    """s_j(t_l), l = 1..n_max, as a table on the device (unit strengths)."""
    import torch
    wu = dataclasses.replace(w, amp=np.ones(w.M))
    params = wu.torch_params(dev)
    S = torch.stack([wu.sigma_torch(l * w.dt, dev, params) for l in range(1, n_max + 1)])
    return lambda l: S[l - 1]


def _plan(w, precision, **kw):
    import paper_2604_07170_amd as pa
    return pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p, **kw)


def _dot_product(w, precision, nt, seed):
    import torch
    dev = torch.device("cuda", 0)
    plan = _plan(w, precision)
    adj = plan.adjoint()
    la = plan.info()["lookahead"]
    assert adj.info()["lookahead"] == la and adj.M == w.Nx and adj.Nx == w.M
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn((nt + la, w.M), generator=g, dtype=torch.float64).to(dev)   # sigma(t_l)
    G = torch.randn((nt, w.Nx), generator=g, dtype=torch.float64).to(dev)       # g(t_m)
    U = torch.empty((nt, w.Nx), dtype=torch.float64, device=dev)
    for n in range(1, nt + la + 1):
        plan.step(X[n - 1])
        if n > la:
            plan.evaluate(U[n - la - 1])
    SB = torch.empty((nt + la, w.M), dtype=torch.float64, device=dev)
    zero = torch.zeros(w.Nx, dtype=torch.float64, device=dev)
    for n in range(1, nt + 2 * la + 1):
        m = nt + la + 1 - n
        adj.step(G[m - 1] if 1 <= m <= nt else zero)
        if n > la:
            adj.evaluate(SB[nt + 2 * la - n])          # sigma-bar(t_l), l = nt + 2 la + 1 - n
    lhs = float((G * U).sum())
    rhs = float((SB * X).sum())
    scale = float(G.norm() * U.norm())
    plan.close()
    adj.close()
    return lhs, rhs, scale


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_dot_product_config0(precision, tol):
    from wfp_workloads import config
    w = config(0, displaced_targets=True)
    lhs, rhs, scale = _dot_product(w, precision, nt=150, seed=3)
    print(f"config0 {precision}: <g,K s> = {lhs:.12e}, <K^T g, s> = {rhs:.12e}, rel {abs(lhs - rhs) / scale:.1e}")
    assert abs(lhs - rhs) <= tol * scale


def test_dot_product_config2_mixed():
    from wfp_workloads import config
    w = config(2)
    lhs, rhs, scale = _dot_product(w, "mixed", nt=40, seed=4)
    print(f"config2 mixed: rel {abs(lhs - rhs) / scale:.1e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def _fd_check(w, precision, nt, m0, h, tol, n_check=32):
    import torch
    from paper_2604_07170_amd.adjoint import StrengthRun, strength_field
    dev = torch.device("cuda", 0)
    plan = _plan(w, precision)
    la = plan.info()["lookahead"]
    run = StrengthRun(plan, _unit_signatures(w, nt + la, dev), nt=nt, m0=m0)
    A0 = torch.as_tensor(w.amp, dtype=torch.float64, device=dev)
    A = A0.clone().requires_grad_(True)
    u = strength_field(A, run)
    L = 0.5 * (u * u).sum()
    L.backward()
    grad = A.grad.detach().cpu().numpy()
    idx = np.sort(np.random.default_rng(32).choice(w.M, size=n_check, replace=False))
    fd = np.zeros(n_check)
    for k, j in enumerate(idx):
        e = torch.zeros_like(A0)
        e[j] = h
        up = run.forward_field(A0 + e)
        um = run.forward_field(A0 - e)
        fd[k] = float(0.5 * ((up * up).sum() - (um * um).sum())) / (2 * h)
    assert np.linalg.norm(fd) > 0
    err = rel_l2(grad[idx], fd)
    print(f"{w.name} {precision}: FD on {n_check} strengths, rel L2 {err:.2e} (|grad| {np.linalg.norm(fd):.3e})")
    run.close()
    plan.close()
    assert err <= tol


def test_fd_32_strengths_config0_fp64():
    """Window t_101..t_150 lies past the far-history onset (L_A + W < 101)."""
    from wfp_workloads import config
    w = config(0, displaced_targets=True)
    _fd_check(w, "fp64", nt=150, m0=101, h=0.5, tol=1e-9)


def test_fd_32_strengths_config2_fp64():
    """Config 2's geometry and signatures with onsets moved into the first steps
    (its own onsets come after t = 2.25, beyond this short window)."""
    from wfp_workloads import config
    w = config(2)
    w = dataclasses.replace(w, t0=np.random.default_rng(21).uniform(0.0, 0.05, size=w.M))
    _fd_check(w, "fp64", nt=50, m0=31, h=1.0, tol=1e-8)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gradient_against_oracle_transpose(precision):
    """dL/dA_j for L = sum_{i,m} g_i(t_m) u_i(t_m): the oracle's field of source j alone,
    contracted with g, is the j-th row of the transposed operator applied to g."""
    import torch
    import oracle
    from paper_2604_07170_amd.adjoint import StrengthRun, strength_field
    from wfp_workloads import config
    w = config(0, displaced_targets=True)
    dev = torch.device("cuda", 0)
    nt = 120
    plan = _plan(w, precision)
    info = plan.info()
    run = StrengthRun(plan, _unit_signatures(w, nt + info["lookahead"], dev), nt=nt, m0=1)
    G = np.random.default_rng(9).standard_normal((nt, w.Nx))
    A = torch.as_tensor(w.amp, dtype=torch.float64, device=dev).requires_grad_(True)
    u = strength_field(A, run)
    (torch.as_tensor(G, device=dev) * u).sum().backward()
    grad = A.grad.cpu().numpy()
    idx = np.sort(np.random.default_rng(10).choice(w.M, size=32, replace=False))
    times = np.arange(1, nt + 1) * w.dt
    xs = np.repeat(w.tgt, nt, axis=0)
    ts = np.tile(times, w.Nx)
    ref = np.zeros(len(idx))
    for k, j in enumerate(idx):
        uj = oracle.u_direct(w.src[j:j + 1], w.family[j:j + 1], np.ones(1), w.t0[j:j + 1], w.omega[j:j + 1],
                             w.s[j:j + 1], xs, ts, self_mode=1, delta=info["delta"], b=info["b"])
        ref[k] = float((G.T.reshape(-1) * uj).sum())      # uj is ordered (target, time)
    err = rel_l2(grad[idx], ref)
    print(f"oracle transpose {precision}: rel L2 {err:.2e} over 32 strengths")
    run.close()
    plan.close()
    assert err <= 1e-6


@pytest.mark.parametrize("spectral", [False, True])
def test_checkpointed_loss_matches_stored_field(spectral):
    import torch
    from paper_2604_07170_amd.adjoint import StrengthRun, strength_field, strength_loss_checkpointed
    from wfp_workloads import config
    w = config(0, displaced_targets=True)
    dev = torch.device("cuda", 0)
    nt, m0 = 140, 61
    plan = _plan(w, "mixed")
    la = plan.info()["lookahead"]
    run = StrengthRun(plan, _unit_signatures(w, nt + la, dev), nt=nt, m0=m0)
    Y = torch.as_tensor(np.random.default_rng(5).standard_normal((nt - m0 + 1, w.Nx)) * 1e-2, device=dev)
    wts = torch.linspace(0.5, 1.5, nt - m0 + 1, dtype=torch.float64, device=dev)

    def loss_fn(m, um):
        k = m - m0
        return 0.5 * wts[k] * ((um - Y[k]) ** 2).sum()

    A1 = torch.as_tensor(w.amp, dtype=torch.float64, device=dev).requires_grad_(True)
    u = strength_field(A1, run)
    L1 = (0.5 * wts[:, None] * (u - Y) ** 2).sum()
    L1.backward()
    A2 = torch.as_tensor(w.amp, dtype=torch.float64, device=dev).requires_grad_(True)
    L2 = strength_loss_checkpointed(A2, run, loss_fn, every=17, spectral=spectral)
    L2.backward()
    dl = abs(float(L1) - float(L2)) / abs(float(L1))
    dg = rel_l2(A2.grad.cpu().numpy(), A1.grad.cpu().numpy())
    print(f"checkpointed (spectral {spectral}, sigma ring of {plan.info()['sigma_depth']} steps) vs stored: "
          f"loss rel {dl:.1e}, grad rel {dg:.1e}")
    run.close()
    plan.close()
    assert dl <= 1e-12 and dg <= 1e-12


def test_fd_32_strengths_config4_spectral_checkpoints():
    """The 10^6-source, 300-wavelength geometry (sources = targets, dt = 8/7150), FP64, with
    the signature onsets moved into the first steps so that a short window carries signal:
    the gradient of loss = 1/2 sum_m |u(t_m)|^2 over m = 21..40 through spectral checkpoints
    every 8 steps (the Fourier history without the sigma ring, refilled from the signatures
    on restore) against central differences on 32 seeded strengths (exact for this
    quadratic loss up to rounding)."""
    import dataclasses
    import torch
    import paper_2604_07170_amd as pa
    from paper_2604_07170_amd.adjoint import StrengthRun, strength_field, strength_loss_checkpointed
    from wfp_workloads import config
    dev = torch.device("cuda", 0)
    w = config(4)
    w = dataclasses.replace(w, t0=np.random.default_rng(21).uniform(0.0, 0.02, size=w.M))
    nt, m0 = 40, 21
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision="fp64", interp_order=w.p)
    la = plan.info()["lookahead"]
    full, spec = plan.state_bytes(), plan.spectral_state_bytes()
    print(f"state blob {full / 2**30:.1f} GiB, spectral {spec / 2**30:.1f} GiB")
    assert spec < 0.25 * full
    wu = dataclasses.replace(w, amp=np.ones(w.M))
    params = wu.torch_params(dev)
    S = torch.stack([wu.sigma_torch(l * w.dt, dev, params) for l in range(1, nt + la + 1)])
    run = StrengthRun(plan, lambda l: S[l - 1], nt=nt, m0=m0)

    def loss_fn(m, um):
        return 0.5 * (um * um).sum()

    A0 = torch.as_tensor(w.amp, dtype=torch.float64, device=dev)
    A = A0.clone().requires_grad_(True)
    L = strength_loss_checkpointed(A, run, loss_fn, every=8)
    L.backward()
    grad = A.grad.detach().cpu().numpy()
    idx = np.sort(np.random.default_rng(32).choice(w.M, size=32, replace=False))
    h = 1.0
    fd = np.zeros(len(idx))
    for k, j in enumerate(idx):
        e = torch.zeros_like(A0)
        e[j] = h
        up = strength_field(A0 + e, run)
        um = strength_field(A0 - e, run)
        fd[k] = float(0.5 * ((up * up).sum() - (um * um).sum())) / (2 * h)
    err = rel_l2(grad[idx], fd)
    print(f"config 4 geometry, FP64, spectral checkpoints: adjoint vs central differences {err:.2e} "
          f"over 32 strengths (|fd| {np.linalg.norm(fd):.3e})")
    run.close()
    plan.close()
    assert np.linalg.norm(fd) > 0 and err <= 1e-8


def test_spectral_checkpoint_kind_and_sigma_reach():
    """A spectral blob loads only as spectral (and a full one only as full); put_sigma takes
    only steps the ring holds."""
    import torch
    import paper_2604_07170_amd as pa
    from wfp_workloads import config
    w = config(0)
    dev = torch.device("cuda", 0)
    plan = _plan(w, "fp64")
    s = torch.ones(w.M, dtype=torch.float64, device=dev)
    for _ in range(5):
        plan.step(s)
    spec, full = plan.save_spectral_state(), plan.save_state()
    with pytest.raises(pa.Wfp2dError):
        plan.load_state(spec)
    with pytest.raises(pa.Wfp2dError):
        plan.load_spectral_state(full)
    plan.load_spectral_state(spec)
    assert plan.info()["steps_ingested"] == 5
    for bad in (0, 6):
        with pytest.raises(pa.Wfp2dError):
            plan.put_sigma(bad, s)
    for l in range(1, 6):
        plan.put_sigma(l, s)
    plan.close()


def test_state_save_load_and_reset():
    import torch
    import paper_2604_07170_amd as pa
    from wfp_workloads import config
    w = config(0, displaced_targets=True)
    dev = torch.device("cuda", 0)
    params = w.torch_params(dev)
    plan = _plan(w, "fp64")
    twin = _plan(w, "fp64")
    for n in range(1, 91):
        plan.step(w.sigma_torch(n * w.dt, dev, params))
    blob = plan.save_state()
    assert blob.numel() == plan.state_bytes()

    def cont(p, n0, k=30):
        out = []
        for n in range(n0, n0 + k):
            p.step(w.sigma_torch(n * w.dt, dev, params))
            out.append(p.evaluate().cpu().numpy())
        return np.array(out)

    a = cont(plan, 91)
    plan.load_state(blob)
    assert plan.info()["steps_ingested"] == 90
    b = cont(plan, 91)
    twin.load_state(blob)                       # another plan of the same geometry
    c = cont(twin, 91)
    assert rel_l2(b, a) <= 1e-14 and rel_l2(c, a) <= 1e-14
    other = pa.Wfp2d(w.src[:32], w.tgt[:32], w.dt, w.W, w.tol, precision="fp64")
    with pytest.raises(pa.Wfp2dError):
        other.load_state(blob)                  # foreign geometry
    plan.reset()
    assert plan.info()["steps_ingested"] == 0
    fresh = _plan(w, "fp64")
    d = cont(plan, 1, 40)
    e = cont(fresh, 1, 40)
    assert rel_l2(d[-10:], e[-10:]) <= 1e-14
    for p in (plan, twin, other, fresh):
        p.close()


def test_reset_clears_a_history_ring_beyond_2_32_elements():
    """At 10^6 sources the sigma ring holds 4.3e9 doubles, more than one dispatch
    of one work-item per element can cover: after a reset, a rerun must match the
    run of the freshly allocated plan (whose memory the allocator zeroed)."""
    import torch
    from wfp_workloads import config
    w = config(4)
    dev = torch.device("cuda", 0)
    plan = _plan(w, "mixed")
    info = plan.info()
    assert info["sigma_depth"] * w.M > 2**32
    j = int(np.random.default_rng(4).integers(w.M))
    x = torch.as_tensor(np.random.default_rng(3).standard_normal(40), device=dev)

    def run():
        plan.reset()
        e = torch.zeros(w.M, dtype=torch.float64, device=dev)
        for n in range(1, 25):
            e.zero_()
            e[j] = x[n - 1]
            plan.step(e)
        return plan.evaluate().cpu().numpy(), plan.debug(2)      # u and the lag transform S_lag

    u0, lag0 = run()
    u1, lag1 = run()
    assert np.abs(lag1).max() <= 1e-6 * max(np.abs(lag0).max(), 1.0)   # sigma(t <= 0) = 0 behind the lag
    assert rel_l2(u1, u0) <= 1e-13
    plan.close()
