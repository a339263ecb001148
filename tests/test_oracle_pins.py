"""Pins of the reference evaluator against facts fixed by the paper and by mathematics.

Each test targets a plausible mistake in the oracle: a wrong singular
substitution (closed forms at small r), a dropped 1/2pi or sign (closed forms),
a causality leak, a window that does not partition unity, a mis-sized panel for
oscillatory signatures (independent QUADPACK integration), the blending
function (its closed-form Fourier transform from Sec. 2.1), and the Green's
function as a whole (the spatial Fourier transform of a one-source field
against sin(|k| t)/|k|).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from wfp_workloads import FAMILY_E, FAMILY_G, FAMILY_RAMP, FAMILY_STEP, config


def one(fam, A=1.0, t0=0.0, w=0.0, s=0.0):
    return dict(family=[fam], amp=[A], t0=[t0], omega=[w], s=[s])


def u1(src, tgt, t, sig, **kw):
    return oracle.u_direct(np.array([src]), sig["family"], sig["amp"], sig["t0"], sig["omega"], sig["s"],
                           np.array([tgt]), [t], **kw)[0]


@pytest.mark.parametrize("r,t", [(0.3, 1.0), (1e-6, 0.5), (1e-9, 3.0), (1.2, 5.0), (2.5, 2.6), (0.5, 0.7)])
def test_step_signature_closed_form(r, t):
    # sigma = H(t): u = (1/2pi) acosh(t/r) for t > r  (from eqs. solnRep and Green)
    src = (0.125, -0.25)
    tgt = (src[0] + r, src[1])
    rr = math.hypot(tgt[0] - src[0], tgt[1] - src[1])
    u = u1(src, tgt, t, one(FAMILY_STEP))
    assert u == pytest.approx(math.acosh(t / rr) / (2 * math.pi), rel=1e-13)


def _ramp_closed(r, t):
    # (1/2pi)[t acosh(t/r) - sqrt(t^2-r^2)] = (r/2pi)(V cosh V - sinh V), t = r cosh V
    V = math.acosh(t / r)
    if V < 1e-2:
        g = sum(V ** (2 * k + 1) * (1.0 / math.factorial(2 * k) - 1.0 / math.factorial(2 * k + 1))
                for k in range(1, 8))
    else:
        g = V * math.cosh(V) - math.sinh(V)
    return r * g / (2 * math.pi)


@pytest.mark.parametrize("r,t", [(0.3, 1.0), (1e-5, 0.5), (0.5, 0.50001), (1.0, 4.0)])
def test_ramp_signature_closed_form(r, t):
    src = (-0.5, 0.25)
    tgt = (src[0], src[1] + r)
    rr = abs(tgt[1] - src[1])
    u = u1(src, tgt, t, one(FAMILY_RAMP))
    assert u == pytest.approx(_ramp_closed(rr, t), rel=1e-12)


def test_causality_and_onset():
    # G = 0 outside the light cone (eq. Green); sigma = 0 before its onset
    sig = one(FAMILY_G, A=1.3, t0=0.4, w=4 * math.pi, s=0.25)
    r = 0.7
    for t in [0.05, 0.5, 1.0, 1.0999]:       # t - r < t0
        assert u1((0, 0), (r, 0), t, sig) == 0.0
    assert abs(u1((0, 0), (r, 0), 1.6, sig)) > 0.0


def test_linearity_and_radial_symmetry():
    rng = np.random.default_rng(3)
    src = np.array([[0.1, 0.2], [0.1, 0.2]])
    fam = [FAMILY_E, FAMILY_E]
    th = rng.uniform(0, 2 * np.pi, 6)
    tg = np.stack([0.1 + 0.37 * np.cos(th), 0.2 + 0.37 * np.sin(th)], 1)
    ua = oracle.u_direct(src, fam, [0.7, -1.9], [0.3, 0.3], [20.0, 20.0], [0, 0], tg, 2.0)
    ub = oracle.u_direct(src[:1], fam[:1], [0.7 - 1.9], [0.3], [20.0], [0], tg, 2.0)
    np.testing.assert_allclose(ua, ub, rtol=1e-13)
    np.testing.assert_allclose(ub, ub[0], rtol=1e-13)   # radial symmetry of G


@pytest.mark.parametrize("fam,w,s,t0,r,t", [
    (FAMILY_E, 31.4, 0.0, 0.6, 0.21, 2.3),
    (FAMILY_E, 94.2, 0.0, 0.2, 0.05, 1.7),
    (FAMILY_G, 4 * math.pi, 0.25, 0.3, 0.4, 3.1),
    (FAMILY_G, 20 * math.pi, 0.05, 0.1, 0.013, 0.9),
])
def test_against_quadpack(fam, w, s, t0, r, t):
    # independent integration: QUADPACK's algebraic-weight rule handles (tau - r)^(-1/2)
    sig = one(fam, A=1.0, t0=t0, w=w, s=s)
    from wfp_workloads import sigma_np
    f = lambda tau: sigma_np(np.array([fam]), np.array([1.0]), np.array([t0]), np.array([w]),
                             np.array([s]), t - tau)[0] / math.sqrt(tau + r)
    val, err = integrate.quad(f, r, t, weight="alg", wvar=(-0.5, 0.0), limit=5000, epsabs=1e-15,
                              epsrel=1e-13)
    u = u1((0.0, 0.0), (r, 0.0), t, sig)
    assert u == pytest.approx(val / (2 * math.pi), rel=2e-11, abs=1e-15)


def test_refinement_invariance_config0():
    w = config(0)
    ti = np.arange(0, 64, 9)
    ts = w.dt * np.array([37, 80, 150, 200])
    a = oracle.u_workload(w, ti, ts)
    b = oracle.u_workload(w, ti, ts, npp=24, hscale=0.5)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def _kb_ft_closed(om, delta, b):
    # Sec. 2.1: FT of phi' = b/sinh(b) sinc(sqrt((delta om/2)^2 - b^2)) times a phase.  The
    # paper prints e^{-i delta om/2}; with its stated kernel e^{+i om t} (same section) and
    # phi' supported on [0, delta] and symmetric about delta/2 the phase is e^{+i delta om/2},
    # which is the reading pinned here.
    z2 = (delta * om / 2) ** 2 - b * b
    if z2 >= 0:
        z = math.sqrt(z2)
        sinc = math.sin(z) / z if z > 0 else 1.0
    else:
        z = math.sqrt(-z2)
        sinc = math.sinh(z) / z
    return b * np.exp(+1j * delta * om / 2) / math.sinh(b) * sinc


@pytest.mark.parametrize("delta,b", [(1.2, math.log(1e7)), (0.0179, math.log(1e7)), (1.0, 30.0)])
def test_blending_function_fourier_closed_form(delta, b):
    x, wq = np.polynomial.legendre.leggauss(200)
    t = 0.5 * delta * (x + 1)
    _, dphi = oracle.phi(t, delta, b)
    for om in [0.0, 3.0 / delta, 20.0 / delta, 2 * b / delta, 60.0 / delta]:
        ft = 0.5 * delta * np.sum(wq * dphi * np.exp(1j * om * t))
        ref = _kb_ft_closed(om, delta, b)
        assert abs(ft - ref) <= 1e-12 * max(1.0, abs(ref))
    p, _ = oracle.phi(np.array([0.0, 0.5 * delta, delta, 2 * delta]), delta, b)
    np.testing.assert_allclose(p, [0.0, 0.5, 1.0, 1.0], atol=1e-14)   # symmetry of the bump


def test_windows_partition_unity():
    # eq. split: u_l + u_nh + u_fh = u for targets in B (r > 0), for any blending parameters
    w = config(0)
    delta, b, Ap = 1.2, math.log(1e7), 6.0
    ti = np.array([0, 5, 33])
    ts = np.array([2.0, 6.2, 9.7])
    kw = dict(delta=delta, b=b, Aplus=Ap)
    full = oracle.u_workload(w, ti, ts, **kw)
    parts = sum(oracle.u_workload(w, ti, ts, window=k, **kw) for k in (1, 2, 3))
    np.testing.assert_allclose(parts, full, rtol=1e-12, atol=1e-14 * np.abs(full).max())
    hist = oracle.u_workload(w, ti, ts, window=oracle.WIN_HISTORY, **kw)
    loc = oracle.u_workload(w, ti, ts, window=oracle.WIN_LOCAL, **kw)
    np.testing.assert_allclose(hist + loc, full, rtol=1e-12, atol=1e-14 * np.abs(full).max())


def test_coincident_self_term_is_the_r_to_zero_limit_of_the_history():
    # the windowed self history at r = 0 is the r -> 0 limit of the history component
    sig = one(FAMILY_E, A=1.0, t0=0.5, w=25.0)
    delta, b = 0.3, math.log(1e7)
    t = 2.2
    at0 = u1((0.2, 0.2), (0.2, 0.2), t, sig, self_mode=1, delta=delta, b=b)
    near0 = u1((0.2, 0.2), (0.2 + 1e-9, 0.2), t, sig, window=oracle.WIN_HISTORY, delta=delta, b=b)
    assert at0 == pytest.approx(near0, rel=1e-8)
    # and it is excluded when self_mode = 0 (eq. exactSol omits r_j = 0)
    assert u1((0.2, 0.2), (0.2, 0.2), t, sig) == 0.0


def test_thread_count_does_not_change_the_sum():
    w = config(0)
    a = oracle.u_workload(w, [3, 7], [4.0, 8.0], nthreads=1)
    b = oracle.u_workload(w, [3, 7], [4.0, 8.0], nthreads=4)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("k", [0.5, 3.0, 7.5, 15.0, 24.0])
def test_spatial_fourier_transform_closed_form(k):
    """The spatial Fourier transform of the 2D Green's function (eq. Green) is
    sin(|k| t)/|k| for t > 0, so the field of one source with signature sigma has
    transform int_0^t sigma(t - tau) sin(|k| tau)/|k| dtau.  The oracle's field is
    radial about the source, so its transform is 2 pi int_0^R u(r, t) J0(|k| r) r dr,
    R = t - t0 (causality); that integral is taken here by Gauss-Legendre in
    r = R v^2, which absorbs the logarithmic behaviour of u at r -> 0."""
    from scipy import special
    t, t0, s, w = 0.9, 0.05, 0.05, 20.0
    sig = one(FAMILY_G, A=1.0, t0=t0, w=w, s=s)
    R = t - t0
    v, gw = np.polynomial.legendre.leggauss(400)
    v = 0.5 * (v + 1.0)
    gw = 0.5 * gw
    r = R * v * v
    xs = np.stack([r, np.zeros_like(r)], 1)
    u = oracle.u_direct(np.zeros((1, 2)), sig["family"], sig["amp"], sig["t0"], sig["omega"], sig["s"],
                        xs, np.full(r.size, t))
    uhat = 2 * math.pi * np.sum(gw * u * special.j0(k * r) * r * 2 * R * v)

    c = t0 + 8.5 * s
    sigma = lambda tt: math.exp(-(tt - c) ** 2 / (2 * s * s)) * math.sin(w * (tt - c)) if tt > t0 else 0.0
    closed, _ = integrate.quad(lambda tau: sigma(t - tau) * math.sin(k * tau) / k, 0.0, R,
                               limit=400, epsabs=1e-15, epsrel=1e-13)
    print(f"k = {k}: transform of the oracle field {uhat:.12e}, closed form {closed:.12e}, "
          f"rel diff {abs(uhat - closed) / abs(closed):.1e}")
    assert abs(closed) > 1e-4 and abs(uhat - closed) <= 1e-11 * abs(closed)   # measured 2e-14


# ---------------------------------------------------------------------------
# The signature-support cut-offs.  The oracle takes family E as exactly zero for
# t <= t0 - 2 (when t0 > 2) and family G as exactly zero for t >= t0 + 22.5 s.
# These tests place the cut inside the integration range, so a cut moved inward
# (dropping a non-negligible part of sigma) changes u beyond the QUADPACK bound.
# ---------------------------------------------------------------------------

def _erfc_half(x):
    return 0.5 * math.erfc(x)


@pytest.mark.parametrize("t0", [3.0, 5.0, 2.0001])
def test_family_e_support_start_is_below_1e40(t0):
    # eq. exampleDensities: sigma = A (1 + erf(5 (t - t0)))/2 sin(...), so below the cut
    # |sigma| <= |A| erfc(5 (t0 - t))/2 <= erfc(10)/2 ~ 1e-45
    start, end = oracle.sig_support(FAMILY_E, 1.0, t0, 50.0)
    assert start == pytest.approx(t0 - 2.0, abs=1e-15) and math.isinf(end)
    assert _erfc_half(5.0 * (t0 - start)) < 1e-40
    # the cut is as far in as a 1e-40 bound allows, up to a margin: not at t0 - 1.5 or closer
    assert start <= t0 - 1.9


def test_family_e_support_start_is_zero_for_early_onsets():
    start, _ = oracle.sig_support(FAMILY_E, 1.0, 1.3, 50.0)
    assert start == 0.0            # sigma(t <= 0) = 0 (eq. wave2d: zero initial data)


@pytest.mark.parametrize("s", [0.25, 0.05])
def test_family_g_support_end_is_below_1e40(s):
    t0 = 0.4
    start, end = oracle.sig_support(FAMILY_G, 1.0, t0, 4 * math.pi, s)
    assert start == t0
    assert end == pytest.approx(t0 + 22.5 * s, rel=1e-15)
    c = t0 + 8.5 * s
    assert math.exp(-((end - c) ** 2) / (2 * s * s)) < 1e-40
    assert end >= t0 + 22.0 * s


@pytest.mark.parametrize("t0,w,r,t", [
    (3.0, 31.4, 0.21, 4.6),       # the cut at t0 - 2 = 1 lies inside [r, t]: tau up to 3.6
    (5.0, 47.1, 0.05, 6.3),       # tau up to 3.3 reaches below the cut at 3
    (2.6, 94.2, 0.4, 3.9),
])
def test_family_e_late_onset_against_quadpack(t0, w, r, t):
    """Independent integration of the untruncated eq. exampleDensities signature.
    With t0 > 2 the oracle starts each integral at t - tau = t0 - 2; QUADPACK sees the
    whole of [r, t].  A cut moved inward by 0.5 or more leaves out erfc(7.5)/2-sized or
    larger pieces of the erf ramp; one at t0 - 1 already shifts u by ~1e-12 relative,
    and anything above the 2e-11 tolerance fails here."""
    from wfp_workloads import sigma_np
    sig = one(FAMILY_E, A=1.0, t0=t0, w=w)
    f = lambda tau: sigma_np(np.array([FAMILY_E]), np.array([1.0]), np.array([t0]), np.array([w]),
                             np.array([0.0]), t - tau)[0] / math.sqrt(tau + r)
    # split at the erf ramp so that QUADPACK resolves it
    pts = sorted({r, max(r, t - t0 - 0.6), max(r, t - t0 + 0.6), t})
    val = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        if b > a:
            v, _ = integrate.quad(lambda x: f(x) * (1.0 / math.sqrt(x - r) if a > r else 1.0), a, b,
                                  **({} if a > r else dict(weight="alg", wvar=(-0.5, 0.0))),
                                  limit=5000, epsabs=1e-15, epsrel=1e-13)
            val += v
    u = u1((0.0, 0.0), (r, 0.0), t, sig)
    assert abs(val) > 1e-3
    assert u == pytest.approx(val / (2 * math.pi), rel=2e-11, abs=1e-15)
    # and the ramp below the cut is what a wrongly placed cut would drop: its size
    lost = abs(integrate.quad(lambda x: f(x) / math.sqrt(x - r), t - t0 + 0.2, t - t0 + 2.0,
                              limit=2000)[0])
    assert lost > 1e-6 * abs(val)


@pytest.mark.parametrize("s,w,t0,r,extra", [(0.25, 4 * math.pi, 0.3, 0.4, 1.0),
                                             (0.05, 20 * math.pi, 0.1, 0.013, 0.37)])
def test_family_g_after_envelope_against_mpmath(s, w, t0, r, extra):
    """t - r beyond t0 + 22.5 s: the whole envelope lies inside [r, t], and the oracle starts
    each integral at t - tau = t0 + 22.5 s.  The reference is 30-digit tanh-sinh quadrature
    (mpmath) of the signature over its whole envelope, in the variable x = t - tau where the
    kernel 1/sqrt(tau^2 - r^2) is smooth; QUADPACK in double precision loses ~1e-12 of this
    cancelling integral to roundoff.  A support end moved inward to t0 + 14 s would drop a
    tail of relative size 1e-9 or more (checked below), far above the 1e-12 tolerance."""
    import mpmath as mp
    sig = one(FAMILY_G, A=1.0, t0=t0, w=w, s=s)
    t = r + t0 + 22.5 * s + extra
    c = t0 + 8.5 * s
    with mp.workdps(30):
        f = lambda x: mp.exp(-(x - c) ** 2 / (2 * s * s)) * mp.sin(w * (x - c)) / mp.sqrt((t - x) ** 2 - r * r)
        pts = [t0] + [c + k * s / 4 for k in range(-33, 57)] + [t0 + 22.5 * s, t0 + 24 * s]
        val = float(mp.quad(f, pts))
        tail = float(mp.quad(f, [t0 + 14 * s + k * s / 4 for k in range(0, 35)]))
    u = u1((0.0, 0.0), (r, 0.0), t, sig)
    assert abs(val) > 1e-6
    assert u == pytest.approx(val / (2 * math.pi), rel=1e-12, abs=1e-18)
    assert abs(tail) > 1e-9 * abs(val)
