"""Seeded synthetic workloads for the 2D wave-potential evaluation problem.

This module only *describes inputs*: source/target positions, the closed-form
parameters of each source's time signature, and the time grid.  It holds none
of the fast method's arithmetic and none of the reference evaluator's, so both
the GPU path and the CPU oracle may draw their inputs from it.

Signature families (Sec. 7, eq. exampleDensities, and the Gaussian-modulated
carrier used by the small configurations):

* family 0 ("G"): sigma(t) = A exp(-(t-c)^2 / (2 s^2)) sin(w (t-c)) for t > t0,
  exactly 0 for t <= t0, with c = t0 + 8.5 s (so the jump at t0 is below 2e-16 |A|).
* family 1 ("E"): sigma(t) = A * 0.5 (erf(5 (t - t0)) + 1) sin(w (t - t0)) for
  t > 0, exactly 0 for t <= 0 (eq. exampleDensities).
* family 2 (step):  sigma(t) = A for t > t0, else 0   (closed-form tests only).
* family 3 (ramp):  sigma(t) = A (t - t0) for t > t0   (closed-form tests only).

The problem is posed in the paper's units: sources and targets in B = [-1, 1]^2,
wave speed 1 (Sec. 1, eq. wave2d).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FAMILY_G, FAMILY_E, FAMILY_STEP, FAMILY_RAMP = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    src: np.ndarray            # (M, 2) float64 source positions in [-1, 1]^2
    tgt: np.ndarray            # (Nx, 2) float64 target positions in [-1, 1]^2
    family: np.ndarray         # (M,) int32
    amp: np.ndarray            # (M,) float64
    t0: np.ndarray             # (M,) float64
    omega: np.ndarray          # (M,) float64
    s: np.ndarray              # (M,) float64 (Gaussian envelope width; unused for E)
    dt: float
    nt: int
    W: int
    tol: float = 1e-7
    p: int = 20
    K0: float = 0.0            # eps-bandwidth of the signatures
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.src.shape[0])

    @property
    def Nx(self) -> int:
        return int(self.tgt.shape[0])

    def sigma(self, t: float) -> np.ndarray:
        """All M signature values at time t (float64)."""
        return sigma_np(self.family, self.amp, self.t0, self.omega, self.s, float(t))

    def sigma_torch(self, t: float, device, params=None):
        """Same closed form evaluated with torch (float64) on ``device``."""
        import torch
        if params is None:
            params = self.torch_params(device)
        fam, amp, t0, om, s = params
        present = self._families_present()
        t = torch.as_tensor(float(t), dtype=torch.float64, device=device)
        out = torch.zeros_like(amp)
        g = fam == FAMILY_G
        if present[FAMILY_G]:
            c = t0 + 8.5 * s
            v = amp * torch.exp(-((t - c) ** 2) / (2 * s * s)) * torch.sin(om * (t - c))
            out = torch.where(g & (t > t0), v, out)
        e = fam == FAMILY_E
        if present[FAMILY_E]:
            v = amp * 0.5 * (torch.erf(5.0 * (t - t0)) + 1.0) * torch.sin(om * (t - t0))
            out = torch.where(e & (t > 0), v, out)
        st = fam == FAMILY_STEP
        if present[FAMILY_STEP]:
            out = torch.where(st & (t > t0), amp, out)
        rp = fam == FAMILY_RAMP
        if present[FAMILY_RAMP]:
            out = torch.where(rp & (t > t0), amp * (t - t0), out)
        return out

    def _families_present(self):
        """Which signature families occur (host-side, so evaluating on a device never waits)."""
        key = (id(self.family), self.family.shape)
        cached = self.__dict__.get("_present")
        if cached is None or cached[0] != key:
            cached = (key, [bool(np.any(self.family == f)) for f in range(4)])
            self.__dict__["_present"] = cached
        return cached[1]

    def torch_params(self, device):
        import torch
        return (torch.as_tensor(self.family, device=device),
                torch.as_tensor(self.amp, dtype=torch.float64, device=device),
                torch.as_tensor(self.t0, dtype=torch.float64, device=device),
                torch.as_tensor(self.omega, dtype=torch.float64, device=device),
                torch.as_tensor(self.s, dtype=torch.float64, device=device))


def _erf(x):
    from scipy.special import erf
    return erf(x)


def sigma_np(family, amp, t0, omega, s, t: float) -> np.ndarray:
    out = np.zeros(amp.shape, dtype=np.float64)
    g = family == FAMILY_G
    if g.any():
        c = t0[g] + 8.5 * s[g]
        v = amp[g] * np.exp(-((t - c) ** 2) / (2 * s[g] ** 2)) * np.sin(omega[g] * (t - c))
        out[g] = np.where(t > t0[g], v, 0.0)
    e = family == FAMILY_E
    if e.any() and t > 0:
        out[e] = amp[e] * 0.5 * (_erf(5.0 * (t - t0[e])) + 1.0) * np.sin(omega[e] * (t - t0[e]))
    st = family == FAMILY_STEP
    if st.any():
        out[st] = np.where(t > t0[st], amp[st], 0.0)
    rp = family == FAMILY_RAMP
    if rp.any():
        out[rp] = np.where(t > t0[rp], amp[rp] * (t - t0[rp]), 0.0)
    return out


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def uniform_square(rng, M: int) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(M, 2))


def star_curve(M: int, r0: float = 1.0, amp: float = 0.3, lobes: int = 5,
               scale: float | None = None) -> np.ndarray:
    """M points equispaced in angle on r(th) = r0 + amp cos(lobes th), scaled into B."""
    th = 2.0 * math.pi * np.arange(M) / M
    r = r0 + amp * np.cos(lobes * th)
    if scale is None:
        scale = 1.0 / (r0 + amp)
    # keep strictly inside the closed box
    scale = min(scale, (1.0 - 1e-12) / (r0 + amp))
    return np.stack([scale * r * np.cos(th), scale * r * np.sin(th)], axis=1)


def grid_targets(n: int = 900) -> np.ndarray:
    """A regular n x n mesh of targets over B (cell centres, row-major in y then x)."""
    c = -1.0 + (2.0 * np.arange(n) + 1.0) / n
    X, Y = np.meshgrid(c, c)
    return np.stack([X.ravel(), Y.ravel()], 1)


def circle_sources(M: int) -> np.ndarray:
    """M points equispaced in s on [0.8 cos s + 0.2, 0.8 sin s + 0.2] (touches the edge of B)."""
    s = 2.0 * np.pi * np.arange(M) / M
    return np.clip(np.stack([0.8 * np.cos(s) + 0.2, 0.8 * np.sin(s) + 0.2], 1), -1.0, 1.0)


def wiggly_sources(M: int) -> np.ndarray:
    """M points equispaced in s on r(s) = 0.61 + 0.2 cos 60s - 0.1 sin 20s + 0.05 cos 30s - 0.1 cos 40s.

    The curve reaches |x| = 1.0029 near s = 0 and s = pi; those points are clipped onto the
    edge of B (the library takes points in [-1, 1]^2)."""
    s = 2.0 * np.pi * np.arange(M) / M
    r = 0.61 + 0.2 * np.cos(60 * s) - 0.1 * np.sin(20 * s) + 0.05 * np.cos(30 * s) - 0.1 * np.cos(40 * s)
    return np.clip(np.stack([r * np.cos(s), r * np.sin(s)], 1), -1.0, 1.0)


def displaced(rng, pts: np.ndarray, frac: float = 0.3) -> np.ndarray:
    """Targets = points moved by a seeded offset of about frac x mean spacing."""
    M = pts.shape[0]
    h = 2.0 / math.sqrt(max(M, 1))
    off = rng.uniform(-frac * h, frac * h, size=pts.shape)
    return np.clip(pts + off, -1.0, 1.0)


# --------------------------------------------------------------------------
# parameter rules for the signature families
# --------------------------------------------------------------------------

def k0_family_g(omega_c: float, s: float, tol: float) -> float:
    """eps-bandwidth of a Gaussian-modulated carrier: |sigma^(w)| ~ exp(-(w-wc)^2 s^2/2)."""
    return omega_c + math.sqrt(2.0 * math.log(1.0 / tol)) / s


def k0_family_e(omega_max: float, tol: float) -> float:
    """eps-bandwidth of eq. exampleDensities: max|w| + 10 sqrt(log(1/eps)) (Sec. 7)."""
    return omega_max + 10.0 * math.sqrt(math.log(1.0 / tol))


def window_for(K0: float, dt: float, tol: float) -> int:
    """Smallest W with dt <= (pi - 2b/W)/K0 (eq. dt), b = ln(1/eps)."""
    b = math.log(1.0 / tol)
    gap = math.pi - K0 * dt
    if gap <= 0:
        raise ValueError("time step above the signature Nyquist limit")
    return int(math.ceil(2.0 * b / gap))


def dt_for(K0: float, W: int, tol: float, margin: float = 0.9757) -> float:
    """Time step from eq. dt with the margin used in Sec. 7.2 (8/7150 vs the bound)."""
    b = math.log(1.0 / tol)
    return margin * (math.pi - 2.0 * b / W) / K0


# --------------------------------------------------------------------------
# the configurations
# --------------------------------------------------------------------------

def family_g_workload(name, rng, src, L: float, nt: int, tol=1e-7, p=20, t0_range=(0.0, 1.0),
                      tgt=None) -> Workload:
    M = src.shape[0]
    omega_c = math.pi * L                    # L wavelengths across the side 2 of B
    period = 2.0 / L
    s = 0.5 * period                         # envelope width: half a period (std dev)
    dt = period / 10.0                       # 10 steps per period
    t0 = rng.uniform(*t0_range, size=M)
    amp = rng.standard_normal(M)
    K0 = k0_family_g(omega_c, s, tol)
    W = window_for(K0, dt, tol)
    return Workload(name=name, src=src, tgt=src.copy() if tgt is None else tgt,
                    family=np.full(M, FAMILY_G, np.int32), amp=amp, t0=t0,
                    omega=np.full(M, omega_c), s=np.full(M, s), dt=dt, nt=nt, W=W,
                    tol=tol, p=p, K0=K0, meta=dict(L=L, family="G"))


def family_e_workload(name, rng, src, L: float, nt: int, dt: float | None = None, W: int = 16,
                      tol=1e-7, p=20, T_ref: float | None = None, tgt=None) -> Workload:
    M = src.shape[0]
    omega_max = math.pi * L
    K0 = k0_family_e(omega_max, tol)
    if dt is None:
        dt = dt_for(K0, W, tol)
    T = dt * nt if T_ref is None else T_ref
    t0 = rng.uniform(1.5, 7.0, size=M) * (T / 8.0)     # Sec. 7.2 offsets, scaled to T
    z = rng.uniform(0.0, 1.0, size=M)
    omega = omega_max * np.cbrt(z)                        # Sec. 7.2: 300 pi z^(1/3)
    return Workload(name=name, src=src, tgt=src.copy() if tgt is None else tgt,
                    family=np.full(M, FAMILY_E, np.int32), amp=np.ones(M), t0=t0,
                    omega=omega, s=np.zeros(M), dt=dt, nt=nt, W=W, tol=tol, p=p, K0=K0,
                    meta=dict(L=L, family="E"))


def config(idx: int, displaced_targets: bool = False) -> Workload:
    """The seeded workloads (numbering follows the benchmark's configuration list)."""
    rng = np.random.default_rng(1000 + idx)
    if idx == 0:
        src = uniform_square(rng, 64)
        w = family_g_workload("cfg0_M64_4wl_G", rng, src, L=4.0, nt=200)
    elif idx == 1:
        src = star_curve(4096)
        w = family_g_workload("cfg1_M4096_star_20wl_G", rng, src, L=20.0, nt=2000)
    elif idx == 2:
        src = uniform_square(rng, 65536)
        w = family_e_workload("cfg2_M65536_100wl_E", rng, src, L=100.0, nt=4000, dt=0.003)
    elif idx == 4:
        src = uniform_square(rng, 1_000_000)
        w = family_e_workload("cfg4_M1e6_300wl_E", rng, src, L=300.0, nt=6000, dt=8.0 / 7150.0,
                              T_ref=8.0 / 7150.0 * 6000)
    elif idx == 7:
        # the random space-filling example of Sec. 7.2 as the paper runs it: the 10^6 random
        # sources of the 300-wavelength workload's recipe with T = 8 (t0 in [1.5, 7]), targets
        # on the separate 900 x 900 mesh (no target on a source)
        src = uniform_square(rng, 1_000_000)
        w = family_e_workload("cfg7_random_M1e6_grid900", rng, src, L=300.0, nt=7150, dt=8.0 / 7150.0, T_ref=8.0,
                              tgt=grid_targets(900))
    elif idx in (5, 6):
        # the curve examples of Sec. 7: the Sec. 7.2 step, window and final time T = 8, a
        # 900 x 900 target mesh (no target on a source), t0 rising from 1.5 to 7 along the
        # curve; on the circle omega rises linearly to 300 pi along it, on the wiggly curve
        # omega = 300 pi z^(1/3) with z uniform
        M = 100_000 if idx == 5 else 1_000_000
        src = circle_sources(M) if idx == 5 else wiggly_sources(M)
        name = "cfg5_circle_M1e5_grid900" if idx == 5 else "cfg6_wiggly_M1e6_grid900"
        w = family_e_workload(name, rng, src, L=300.0, nt=7150, dt=8.0 / 7150.0, T_ref=8.0, tgt=grid_targets(900))
        frac = np.arange(M) / M
        w.t0 = 1.5 + 5.5 * frac
        if idx == 5:
            w.omega = 300.0 * np.pi * frac
    else:
        raise ValueError(f"no such configuration {idx}")
    if displaced_targets:
        w.tgt = displaced(np.random.default_rng(2000 + idx), w.src)
        w.name += "_disp"
    return w


def batch_instances(n: int = 64, nt: int = 1000, W: int = 16, tol: float = 1e-7,
                    m_range=(500, 20000), l_range=(10.0, 50.0)) -> list:
    """Independent scatterers of uneven size: star curves with M_i log-uniform in m_range
    and L_i ~ U(l_range) wavelengths across B, family E signatures, the time step of
    eq. dt with the Sec. 7.2 margin for each instance's bandwidth."""
    rng = np.random.default_rng(1003)
    L = rng.uniform(*l_range, size=n)
    M = np.floor(np.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1]), size=n))).astype(np.int64)
    out = []
    for i in range(n):
        r = np.random.default_rng(1003000 + i)
        src = star_curve(int(M[i]))
        out.append(family_e_workload(f"cfg3_inst{i}_M{int(M[i])}_{L[i]:.1f}wl_E", r, src, L=float(L[i]), nt=nt,
                                     W=W, tol=tol))
    return out


def tiny(seed: int = 7, M: int = 16, L: float = 2.0, nt: int = 60, family: str = "G",
         displaced_targets: bool = True) -> Workload:
    """A few-source case small enough for exhaustive oracle checks."""
    rng = np.random.default_rng(seed)
    src = uniform_square(rng, M)
    if family == "G":
        w = family_g_workload(f"tiny_G_{seed}", rng, src, L=L, nt=nt)
    else:
        w = family_e_workload(f"tiny_E_{seed}", rng, src, L=L, nt=nt, W=20)
    if displaced_targets:
        w.tgt = displaced(np.random.default_rng(seed + 1), src)
    return w
