"""The seeded synthetic inputs (CPU): sizes, domain, time steps and signature
parameters of each workload as the design notes state them, and determinism."""
import math

import numpy as np
import pytest

from wfp_workloads import FAMILY_E, FAMILY_G, batch_instances, config


def _in_b(x):
    return bool(np.all(np.abs(x) <= 1.0))


@pytest.mark.parametrize("idx,M,Nx,dt,W,nt,fam", [
    (0, 64, 64, 0.05, 24, 200, FAMILY_G),
    (1, 4096, 4096, 0.01, 24, 2000, FAMILY_G),
    (2, 65536, 65536, 0.003, 16, 4000, FAMILY_E),
    (4, 1_000_000, 1_000_000, 8 / 7150, 16, 6000, FAMILY_E),
    (5, 100_000, 810_000, 8 / 7150, 16, 7150, FAMILY_E),
    (6, 1_000_000, 810_000, 8 / 7150, 16, 7150, FAMILY_E),
    (7, 1_000_000, 810_000, 8 / 7150, 16, 7150, FAMILY_E),
])
def test_configuration_recipe(idx, M, Nx, dt, W, nt, fam):
    w = config(idx)
    assert (w.M, w.Nx, w.W, w.nt, w.p, w.tol) == (M, Nx, W, nt, 20, 1e-7)
    assert w.dt == pytest.approx(dt, rel=1e-12)
    assert _in_b(w.src) and _in_b(w.tgt)
    assert np.all(w.family == fam)
    if idx in (0, 1, 2, 4):
        assert np.array_equal(w.src, w.tgt)                 # sources = targets
    if fam == FAMILY_E:
        L = w.meta["L"]
        assert np.all((w.omega >= 0) & (w.omega <= math.pi * L))
    if idx in (2, 4, 7):
        T = w.dt * w.nt
        assert np.all((w.t0 >= 1.5 * T / 8) & (w.t0 <= 7.0 * T / 8))
    if idx == 7:
        # Sec. 7.2 as run in the paper: T = 8, t0 in [1.5, 7], omega = 300 pi z^(1/3)
        assert w.dt * w.nt == pytest.approx(8.0)
        assert np.median(w.omega) == pytest.approx(300 * math.pi * 0.5 ** (1 / 3), rel=0.01)
    if idx in (5, 6):
        frac = np.arange(M) / M
        assert np.allclose(w.t0, 1.5 + 5.5 * frac)
    if idx in (5, 6, 7):
        # the 900 x 900 mesh: cell centres of a 900 x 900 partition of B
        xs = np.unique(w.tgt[:, 0])
        assert xs.size == 900 and np.allclose(np.diff(xs), 2 / 900)
    if idx == 5:
        # the circle of radius 0.8 about (0.2, 0.2), touching the edge of B
        assert np.allclose(np.hypot(w.src[:, 0] - 0.2, w.src[:, 1] - 0.2), 0.8)
        assert np.allclose(w.omega, 300 * math.pi * np.arange(M) / M)


@pytest.mark.parametrize("idx", [0, 2])
def test_configurations_are_seeded(idx):
    a, b = config(idx), config(idx)
    for f in ("src", "tgt", "amp", "t0", "omega", "s"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


def test_displaced_targets_leave_the_sources():
    w = config(0, displaced_targets=True)
    d = np.hypot(*(w.tgt - w.src).T)
    assert _in_b(w.tgt) and np.all(d > 0)


def test_batched_instances():
    ws = batch_instances(64)
    Ms = np.array([w.M for w in ws])
    Ls = np.array([w.meta["L"] for w in ws])
    assert len(ws) == 64 and Ms.min() >= 500 and Ms.max() < 20000
    assert Ls.min() >= 10 and Ls.max() <= 50
    assert len(set(w.dt for w in ws)) == 64                 # each instance has its own time step
    assert all(w.nt == 1000 and w.W == 16 and _in_b(w.src) for w in ws)
    assert [w.M for w in batch_instances(64)] == Ms.tolist()
