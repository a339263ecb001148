"""Reference (oracle) evaluators for the 2D wave potential — TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never does, and this
package imports nothing from it: the two share no code.

Contents
--------
* :func:`u_direct` — the plain definition of the field (Sec. 1, eqs. solnRep,
  Green; Sec. 7, eq. exactSol) by composite Gauss-Legendre quadrature with the
  analytic signatures, FP64, OpenMP over (sample, source block), fixed-order
  compensated summation.  Optional windows give the local / near / far /
  history components of eq. split.
* :func:`phi` — the blending function of eq. KBblending.

The stage check of the type-1 transform compares with the direct Fourier sum
of eq. sighat, written out in that test (a matrix-vector product in numpy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

WIN_FULL, WIN_LOCAL, WIN_NEAR, WIN_FAR, WIN_HISTORY = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain C, no fast-math)."""
    src = os.path.join(_HERE, "direct.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_u.argtypes = [ctypes.c_int64, d, i32, d, d, d, d, ctypes.c_int64, d, d,
                                 ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, d]
        lib.oracle_u.restype = ctypes.c_int
        lib.oracle_phi.argtypes = [ctypes.c_int64, d, ctypes.c_double, ctypes.c_double, d, d]
        lib.oracle_phi.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_sig_support.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, d, d]
        lib.oracle_sig_support.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads() -> int:
    return int(_load().oracle_threads())


def u_direct(src, family, amp, t0, omega, s, xs, ts, window=WIN_FULL, delta=0.0, b=0.0,
             Aplus=0.0, self_mode=0, npp=16, hscale=1.0, nthreads=0):
    """u at sample points xs (n,2) and times ts (n,). All arrays float64.

    ``self_mode=1`` adds, for a target that coincides with a source, that
    source's windowed history (1/2pi) int sigma(t-tau) phi(tau)/tau dtau (the
    part of a coincident pair that the fast method's Fourier history keeps);
    ``self_mode=0`` omits coincident pairs as eq. exactSol does.
    """
    lib = _load()
    src = np.ascontiguousarray(src, np.float64).reshape(-1, 2)
    M = src.shape[0]
    fam = np.ascontiguousarray(family, np.int32).reshape(M)
    amp = np.ascontiguousarray(amp, np.float64).reshape(M)
    t0 = np.ascontiguousarray(t0, np.float64).reshape(M)
    om = np.ascontiguousarray(omega, np.float64).reshape(M)
    sw = np.ascontiguousarray(s, np.float64).reshape(M)
    xs = np.ascontiguousarray(xs, np.float64).reshape(-1, 2)
    ts = np.ascontiguousarray(np.broadcast_to(np.asarray(ts, np.float64), (xs.shape[0],)))
    out = np.zeros(xs.shape[0], np.float64)
    rc = lib.oracle_u(M, _dp(src), fam.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(amp),
                      _dp(t0), _dp(om), _dp(sw), xs.shape[0], _dp(xs), _dp(ts), int(window),
                      float(delta), float(b), float(Aplus), int(self_mode), int(npp), float(hscale),
                      int(nthreads), _dp(out))
    if rc != 0:
        raise ValueError("oracle_u rejected its arguments")
    return out


def u_workload(w, target_idx, times, **kw):
    """Oracle u for a :class:`wfp_workloads.Workload` at targets x times (outer product).

    Returns an array of shape (len(target_idx), len(times)).
    """
    target_idx = np.asarray(target_idx)
    times = np.asarray(times, np.float64)
    xs = np.repeat(w.tgt[target_idx], len(times), axis=0)
    ts = np.tile(times, len(target_idx))
    out = u_direct(w.src, w.family, w.amp, w.t0, w.omega, w.s, xs, ts, **kw)
    return out.reshape(len(target_idx), len(times))


def sig_support(family, amp, t0, omega, s=0.0):
    """(start, end): the oracle takes a signature as exactly zero for t <= start and t >= end."""
    lib = _load()
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.oracle_sig_support(int(family), float(amp), float(t0), float(omega), float(s),
                           ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def phi(t, delta, b):
    """(phi(t), phi'(t)) of eq. KBblending."""
    lib = _load()
    t = np.ascontiguousarray(t, np.float64)
    p = np.zeros_like(t)
    dp = np.zeros_like(t)
    lib.oracle_phi(t.size, _dp(t), float(delta), float(b), _dp(p), _dp(dp))
    return p, dp
