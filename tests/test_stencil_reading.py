"""Why the local part delays its output by ceil(p/2) - 1 steps (the look-ahead reading of
Sec. 6, eq. sigInterp): interpolating a signature of the benchmark's top frequency from the
p = 20 grid samples nearest the node (centred) against from the 20 newest past samples only
(one-sided), at delays below one step.  Plain Lagrange interpolation, no library code."""
import math

import numpy as np


def _lagrange_error(nodes, omega_dt, s):
    """|interpolant - sin| at s of sin(omega_dt x) through the integer nodes."""
    L = np.ones(len(nodes))
    for i, xi in enumerate(nodes):
        for j, xj in enumerate(nodes):
            if i != j:
                L[i] *= (s - xj) / (xi - xj)
    return abs(float(np.dot(L, np.sin(omega_dt * nodes))) - math.sin(omega_dt * s))


def test_one_sided_stencil_is_orders_less_accurate():
    # 300 wavelengths across [-1, 1]^2: omega up to 300 pi, plus the erf's 10 sqrt(ln 1/eps)
    # (Sec. 7, the eps-bandwidth K0), at dt = 8/7150 and eps = 1e-7
    dt = 8.0 / 7150.0
    omega_dt = (300.0 * math.pi + 10.0 * math.sqrt(math.log(1e7))) * dt
    delays = np.linspace(0.0, 1.0, 21)                   # in steps; the node sits at time -delay
    past = -np.arange(20, dtype=float)                   # times t_n, t_{n-1}, ..., t_{n-19}
    centred = np.arange(-10, 10, dtype=float)            # times t_{n-10} .. t_{n+9} (9 steps ahead)
    e_one = max(_lagrange_error(past, omega_dt, -d) for d in delays)
    e_cen = max(_lagrange_error(centred, omega_dt, -d) for d in delays)
    assert e_one > 1e-3          # measured 6.3e-3
    assert e_cen < 1e-6          # measured 2.5e-7
    assert e_one > 1e3 * e_cen
