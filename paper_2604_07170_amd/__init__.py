"""Python binding of the wfp2d HIP library (gfx950): 2D wave potentials by TK-WFP.

Argument marshalling only: every step of the method runs in the library's HIP
kernels (libwfp2d.so, built in-tree by ``paper_2604_07170_amd.build``).  If the
library is missing this module raises; there is no CPU fallback.

Typical use::

    plan = Wfp2d(src_xy, tgt_xy, dt, W, tol)          # numpy float64 [n][2]
    for n in range(1, nt + 1):
        plan.step(sigma_n)                            # torch float64 cuda [M]
        u = plan.evaluate()                           # torch float64 cuda [Nx], u(t_{n - lookahead})
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwfp2d.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "wfp2d.h")

PREC_FP64, PREC_MIXED = 0, 1
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_DOMAIN", -3: "ERR_INFEASIBLE", -4: "ERR_NOMEM",
          -5: "ERR_DEVICE", -6: "ERR_STATE", -7: "ERR_NONFINITE"}
ERR_NONFINITE = -7


class Wfp2dError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("interp_order", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("Delta", ctypes.c_double), ("a", ctypes.c_double), ("Kf", ctypes.c_double),
                ("b_Delta", ctypes.c_double), ("nufft_tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("spread_tile", ctypes.c_int32),
                ("local_pairs", ctypes.c_int32), ("host_pointers", ctypes.c_int32), ("check_finite", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_double) for n in ("dt", "delta", "b", "A", "Aplus", "a", "dk", "K", "Kf", "Kmax")]
                + [(n, ctypes.c_int64) for n in ("LA", "R", "n_modes", "n_near", "n_far", "n_far_classes", "nf",
                                                 "band", "fft_q", "fft_p")]
                + [("nufft_w", ctypes.c_int32), ("W", ctypes.c_int32), ("p", ctypes.c_int32),
                   ("lookahead", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("level_min", ctypes.c_int32),
                   ("n_subpanels", ctypes.c_int32), ("cheb_degree", ctypes.c_int32)]
                + [(n, ctypes.c_int64) for n in ("M", "Nx", "n_local_pairs", "sigma_depth", "bytes_device",
                                                 "steps_ingested", "step_reported")]
                + [("precision", ctypes.c_int32), ("n_regular_subpanels", ctypes.c_int32),
                   ("spread_tile", ctypes.c_int32), ("local_path", ctypes.c_int32),
                   ("local_pair_bytes", ctypes.c_int64), ("local_pair_words", ctypes.c_int64),
                   ("init_ms", ctypes.c_double * 7)])


_lib = None


def load_library():
    """Load libwfp2d.so (raise if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_07170_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i32, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    lib.wfp2d_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.wfp2d_init.argtypes = [ctypes.POINTER(vp), i64, dp, i64, dp, d, i32, d, ctypes.POINTER(Opts)]
    lib.wfp2d_step.argtypes = [vp, vp]
    lib.wfp2d_evaluate.argtypes = [vp, vp]
    lib.wfp2d_query.argtypes = [vp, ctypes.POINTER(Info)]
    lib.wfp2d_destroy.argtypes = [vp]
    lib.wfp2d_last_error.argtypes = [vp]
    lib.wfp2d_last_error.restype = ctypes.c_char_p
    lib.wfp2d_debug_copy.argtypes = [vp, i32, vp, ctypes.POINTER(i64)]
    lib.wfp2d_host_eval.argtypes = [i32, dp, i64, dp, i64, ctypes.POINTER(i64)]
    lib.wfp2d_set_timing.argtypes = [vp, i32]
    lib.wfp2d_get_timing.argtypes = [vp, dp, ctypes.POINTER(i64), i32]
    lib.wfp2d_graph_capture.argtypes = [vp, vp, vp]
    lib.wfp2d_graph_launch.argtypes = [vp]
    lib.wfp2d_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), i32, vp]
    lib.wfp2d_batch_launch.argtypes = [vp]
    lib.wfp2d_batch_destroy.argtypes = [vp]
    lib.wfp2d_evaluate_dot.argtypes = [vp, vp, vp]
    lib.wfp2d_evaluate_noalloc.argtypes = [vp, vp]
    lib.wfp2d_adjoint_init.argtypes = [ctypes.POINTER(vp), vp]
    lib.wfp2d_state_bytes.argtypes = [vp, ctypes.POINTER(i64)]
    lib.wfp2d_reset.argtypes = [vp]
    lib.wfp2d_save_state.argtypes = [vp, vp, i64]
    lib.wfp2d_load_state.argtypes = [vp, vp, i64]
    lib.wfp2d_spectral_state_bytes.argtypes = [vp, ctypes.POINTER(i64)]
    lib.wfp2d_save_spectral_state.argtypes = [vp, vp, i64]
    lib.wfp2d_load_spectral_state.argtypes = [vp, vp, i64]
    lib.wfp2d_put_sigma.argtypes = [vp, i64, vp]
    lib.wfp2d_set_spread_tile.argtypes = [vp, i32]
    lib.wfp2d_time_spread.argtypes = [vp, i32, i32, dp]
    for f in ("wfp2d_default_opts", "wfp2d_init", "wfp2d_step", "wfp2d_evaluate", "wfp2d_query", "wfp2d_destroy",
              "wfp2d_debug_copy", "wfp2d_host_eval", "wfp2d_set_timing", "wfp2d_get_timing", "wfp2d_graph_capture",
              "wfp2d_graph_launch", "wfp2d_batch_create", "wfp2d_batch_launch", "wfp2d_batch_destroy",
              "wfp2d_set_spread_tile", "wfp2d_time_spread", "wfp2d_evaluate_dot", "wfp2d_adjoint_init",
              "wfp2d_state_bytes", "wfp2d_save_state", "wfp2d_load_state", "wfp2d_reset",
              "wfp2d_evaluate_noalloc", "wfp2d_spectral_state_bytes", "wfp2d_save_spectral_state",
              "wfp2d_load_spectral_state", "wfp2d_put_sigma"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def host_eval(what: int, inputs, n_out: int) -> np.ndarray:
    """Host-only precomputation routines of the plan (see wfp2d_host_eval)."""
    lib = load_library()
    x = np.ascontiguousarray(np.asarray(inputs, np.float64).ravel())
    out = np.zeros(int(n_out), np.float64)
    cnt = ctypes.c_int64(0)
    rc = lib.wfp2d_host_eval(int(what), _dp(x), x.size, _dp(out), out.size, ctypes.byref(cnt))
    if rc != 0:
        raise Wfp2dError(rc, lib.wfp2d_last_error(None).decode())
    return out[: cnt.value]


def derive_params(dt, W, tol, p=20, lookahead=-1, Delta=1.0, a=0.0, Kf=80.0) -> dict:
    v = host_eval(1, [dt, W, tol, p, lookahead, Delta, a, Kf], 12)
    keys = ("delta", "b", "A", "Aplus", "a", "dk", "K", "Kmax", "LA", "R", "lookahead", "N")
    out = dict(zip(keys, v.tolist()))
    for k in ("LA", "R", "lookahead", "N"):
        out[k] = int(round(out[k]))
    return out


@dataclass
class StageNames:
    S_CUR: int = 1
    S_LAG: int = 2
    ALPHA: int = 3
    U_H: int = 4
    U_L: int = 5
    MODES: int = 6
    HANKEL: int = 7


STAGE = StageNames()


class _Handle:
    def __init__(self, h, device, stream):
        self.h, self.device, self.stream = h, device, stream


class Wfp2d:
    """One plan: sources/targets fixed at construction, one step per sample."""

    def __init__(self, src_xy, tgt_xy, dt: float, W: int, tol: float = 1e-7, *, precision: str = "mixed",
                 interp_order: int = 20, lookahead: int = -1, Delta: float = 1.0, a: float = 0.0, Kf: float = 80.0,
                 b_Delta: float = 30.0, nufft_tol: float = 0.0, max_steps: int = 0, device: int = 0, stream=None,
                 spread_tile: int = 0, local_pairs: bool = True, host_pointers: bool = False,
                 check_finite: bool = False):
        import torch
        self._torch = torch
        self.lib = load_library()
        self._graph_keep = None
        if isinstance(src_xy, _Handle):              # adopt a plan made by the library (adjoint)
            self.h, self.device, self.stream = src_xy.h, src_xy.device, src_xy.stream
            self.host_pointers = False
            inf = self.info()
            self.M, self.Nx, self._keep = inf["M"], inf["Nx"], []
            return
        src = np.ascontiguousarray(np.asarray(src_xy, np.float64).reshape(-1, 2))
        tgt = np.ascontiguousarray(np.asarray(tgt_xy, np.float64).reshape(-1, 2))
        o = Opts()
        self.lib.wfp2d_default_opts(ctypes.byref(o))
        o.precision = PREC_MIXED if precision == "mixed" else PREC_FP64
        o.interp_order, o.lookahead = int(interp_order), int(lookahead)
        o.Delta, o.a, o.Kf, o.b_Delta, o.nufft_tol = float(Delta), float(a), float(Kf), float(b_Delta), float(nufft_tol)
        o.max_steps, o.device, o.spread_tile = int(max_steps), int(device), int(spread_tile)
        o.local_pairs = 0 if local_pairs else -1
        o.host_pointers, o.check_finite = int(bool(host_pointers)), int(bool(check_finite))
        self.host_pointers = bool(host_pointers)
        self.device = torch.device("cuda", int(device))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        o.stream = ctypes.c_void_p(int(stream.cuda_stream))
        h = ctypes.c_void_p()
        rc = self.lib.wfp2d_init(ctypes.byref(h), src.shape[0], _dp(src), tgt.shape[0], _dp(tgt), float(dt), int(W),
                                 float(tol), ctypes.byref(o))
        if rc != 0:
            raise Wfp2dError(rc, self.lib.wfp2d_last_error(None).decode())
        self.h = h
        self.M, self.Nx = src.shape[0], tgt.shape[0]
        self._keep = []

    # -- helpers --
    def _check(self, rc):
        if rc != 0:
            raise Wfp2dError(rc, self.lib.wfp2d_last_error(self.h).decode())

    def info(self) -> dict:
        inf = Info()
        self._check(self.lib.wfp2d_query(self.h, ctypes.byref(inf)))
        out = {name: getattr(inf, name) for name, _ in Info._fields_}
        out["init_ms"] = list(out["init_ms"])
        return out

    # -- the hot path --
    def step(self, sigma):
        t = self._torch
        if self.host_pointers:
            a = np.ascontiguousarray(sigma, np.float64)
            if a.size != self.M:
                raise ValueError("sigma must hold M float64 values")
            self._check(self.lib.wfp2d_step(self.h, a.ctypes.data_as(ctypes.c_void_p)))
            return
        if not (isinstance(sigma, t.Tensor) and sigma.is_cuda and sigma.dtype == t.float64 and sigma.numel() == self.M):
            raise ValueError("sigma must be a float64 CUDA tensor with M elements")
        sigma = sigma.contiguous()
        self._keep = [sigma]
        self._check(self.lib.wfp2d_step(self.h, ctypes.c_void_p(sigma.data_ptr())))

    def evaluate(self, out=None):
        t = self._torch
        if self.host_pointers:
            out = np.empty(self.Nx, np.float64) if out is None else out
            if not (isinstance(out, np.ndarray) and out.dtype == np.float64 and out.size == self.Nx
                    and out.flags["C_CONTIGUOUS"]):
                raise ValueError("out must be a contiguous float64 numpy array with Nx elements")
            self._check(self.lib.wfp2d_evaluate(self.h, out.ctypes.data_as(ctypes.c_void_p)))
            return out
        if out is None:
            out = t.empty(self.Nx, dtype=t.float64, device=self.device)
        if not (out.is_cuda and out.dtype == t.float64 and out.numel() == self.Nx and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 CUDA tensor with Nx elements")
        self._check(self.lib.wfp2d_evaluate(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def evaluate_noalloc(self, out):
        """wfp2d_evaluate_noalloc: evaluate into `out` with the library's fixed device workspace."""
        t = self._torch
        if not (isinstance(out, t.Tensor) and out.is_cuda and out.dtype == t.float64 and out.numel() == self.Nx
                and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 CUDA tensor with Nx elements")
        self._check(self.lib.wfp2d_evaluate_noalloc(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def evaluate_dot(self, weights, acc):
        """acc += weights * u(t_m) (both float64 CUDA tensors of Nx elements)."""
        t = self._torch
        for x in (weights, acc):
            if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float64 and x.numel() == self.Nx
                    and x.is_contiguous()):
                raise ValueError("weights and acc must be contiguous float64 CUDA tensors with Nx elements")
        self._keep = [weights, acc]
        self._check(self.lib.wfp2d_evaluate_dot(self.h, ctypes.c_void_p(weights.data_ptr()),
                                                ctypes.c_void_p(acc.data_ptr())))

    def adjoint(self) -> "Wfp2d":
        """The plan of the transposed operator (sources and targets exchanged)."""
        h = ctypes.c_void_p()
        rc = self.lib.wfp2d_adjoint_init(ctypes.byref(h), self.h)
        if rc != 0:
            raise Wfp2dError(rc, self.lib.wfp2d_last_error(None).decode())
        return Wfp2d(_Handle(h, self.device, self.stream), None, 0.0, 0)

    # -- checkpoints --
    def reset(self):
        """Zero initial data again: step count 0, all history cleared."""
        self._check(self.lib.wfp2d_reset(self.h))

    def state_bytes(self) -> int:
        n = ctypes.c_int64(0)
        self._check(self.lib.wfp2d_state_bytes(self.h, ctypes.byref(n)))
        return n.value

    def save_state(self, buf=None):
        """Copy the evolving state into a uint8 CUDA tensor (allocated if not given)."""
        t = self._torch
        n = self.state_bytes()
        if buf is None:
            buf = t.empty(n, dtype=t.uint8, device=self.device)
        if not (buf.is_cuda and buf.dtype == t.uint8 and buf.numel() >= n and buf.is_contiguous()):
            raise ValueError("state buffer must be a contiguous uint8 CUDA tensor of state_bytes() bytes")
        self._check(self.lib.wfp2d_save_state(self.h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))
        return buf

    def load_state(self, buf):
        t = self._torch
        if not (buf.is_cuda and buf.dtype == t.uint8 and buf.is_contiguous()):
            raise ValueError("state buffer must be a contiguous uint8 CUDA tensor")
        self._check(self.lib.wfp2d_load_state(self.h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))

    def spectral_state_bytes(self) -> int:
        n = ctypes.c_int64(0)
        self._check(self.lib.wfp2d_spectral_state_bytes(self.h, ctypes.byref(n)))
        return n.value

    def save_spectral_state(self, buf=None):
        """Copy the state without the sigma history ring into a uint8 CUDA tensor."""
        t = self._torch
        n = self.spectral_state_bytes()
        if buf is None:
            buf = t.empty(n, dtype=t.uint8, device=self.device)
        if not (buf.is_cuda and buf.dtype == t.uint8 and buf.numel() >= n and buf.is_contiguous()):
            raise ValueError("state buffer must be a contiguous uint8 CUDA tensor of spectral_state_bytes() bytes")
        self._check(self.lib.wfp2d_save_spectral_state(self.h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))
        return buf

    def load_spectral_state(self, buf):
        """Restore a spectral checkpoint; then put_sigma(l, ...) for the ring's steps
        max(1, n - sigma_depth + 1)..n (n = info()["steps_ingested"])."""
        t = self._torch
        if not (buf.is_cuda and buf.dtype == t.uint8 and buf.is_contiguous()):
            raise ValueError("state buffer must be a contiguous uint8 CUDA tensor")
        self._check(self.lib.wfp2d_load_spectral_state(self.h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))

    def put_sigma(self, l: int, sigma):
        t = self._torch
        if self.host_pointers:
            a = np.ascontiguousarray(sigma, np.float64)
            if a.size != self.M:
                raise ValueError("sigma must hold M float64 values")
            self._check(self.lib.wfp2d_put_sigma(self.h, int(l), a.ctypes.data_as(ctypes.c_void_p)))
            return
        if not (isinstance(sigma, t.Tensor) and sigma.is_cuda and sigma.dtype == t.float64 and sigma.numel() == self.M):
            raise ValueError("sigma must be a float64 CUDA tensor with M elements")
        sigma = sigma.contiguous()
        self._keep = [sigma]
        self._check(self.lib.wfp2d_put_sigma(self.h, int(l), ctypes.c_void_p(sigma.data_ptr())))

    # -- spreading tile shape (autotuned by paper_2604_07170_amd.autotune) --
    SPREAD_TILES = {1: (8, 8), 2: (16, 8), 3: (16, 16), 4: (32, 16), 5: (32, 32), 6: (16, 16, "mfma")}

    def set_spread_tile(self, code: int):
        self._check(self.lib.wfp2d_set_spread_tile(self.h, int(code)))

    def time_spread(self, code: int, reps: int = 10) -> float:
        """Mean ms of `reps` spreading launches with tile shape `code` (which stays selected)."""
        ms = ctypes.c_double(0.0)
        self._check(self.lib.wfp2d_time_spread(self.h, int(code), int(reps), ctypes.byref(ms)))
        return ms.value

    # -- graph replay --
    def graph_capture(self, sigma, u):
        """Record one step (reading `sigma`) + evaluation (writing `u`) into a graph; the
        tensors are borrowed until the plan is closed or captured again."""
        t = self._torch
        for x, n in ((sigma, self.M), (u, self.Nx)):
            if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float64 and x.numel() == n
                    and x.is_contiguous()):
                raise ValueError("graph buffers must be contiguous float64 CUDA tensors of size M / Nx")
        self._graph_keep = (sigma, u)
        self._check(self.lib.wfp2d_graph_capture(self.h, ctypes.c_void_p(sigma.data_ptr()),
                                                 ctypes.c_void_p(u.data_ptr())))

    def graph_launch(self):
        self._check(self.lib.wfp2d_graph_launch(self.h))

    STAGES = ("ingest", "spread", "fft_rows1", "fft_cols1", "split", "near", "far", "fft_cols2", "fft_rows2",
              "interp", "local", "combine")
    KERNELS = ("k_ingest", "k_spread", "k_rows1", "k_cols1", "k_split", "k_near", "k_far", "k_cols2", "k_rows2",
               "k_interp", "k_local", "k_combine")

    def set_timing(self, enable: bool):
        self._check(self.lib.wfp2d_set_timing(self.h, 1 if enable else 0))

    def get_timing(self) -> dict:
        """{stage: (total ms, launches)} since timing was enabled (synchronises the stream)."""
        n = len(self.STAGES)
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        self._check(self.lib.wfp2d_get_timing(self.h, _dp(ms), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n))
        return {s: (float(ms[i]), int(cnt[i])) for i, s in enumerate(self.STAGES)}

    def debug(self, what: int) -> np.ndarray:
        inf = self.info()
        if what in (STAGE.U_H, STAGE.U_L):
            buf = np.zeros(self.Nx, np.float64)
        elif what == STAGE.MODES:
            buf = np.zeros((inf["n_modes"], 2), np.int32)
        elif what == STAGE.HANKEL:
            buf = np.zeros((inf["n_far_classes"], 641), np.float64)
        else:
            real = np.float32 if inf["precision"] == PREC_MIXED else np.float64
            buf = np.zeros(2 * inf["n_modes"], real)
        nb = ctypes.c_int64(buf.nbytes)
        self._check(self.lib.wfp2d_debug_copy(self.h, int(what), buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nb)))
        if what in (STAGE.S_CUR, STAGE.S_LAG, STAGE.ALPHA):
            return buf[0::2].astype(np.float64) + 1j * buf[1::2].astype(np.float64)
        return buf

    def close(self):
        self._graph_keep = None
        if getattr(self, "h", None):
            self.lib.wfp2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent plans advanced together: one graph launch per step.

    sigma[i] / u[i] are fixed float64 CUDA tensors of plan i (M_i / Nx_i elements);
    the caller fills sigma[i] with sigma_j(t_n) before each launch and reads u[i]
    (u at t_{n - lookahead_i}) after it.  autotune=True first picks each plan's
    spreading tile shape by timing (cached per size class, see autotune)."""

    def __init__(self, plans, sigma, u, n_streams: int = 4, stream=None, autotune: bool = False,
                 tune_cache: str | None = None):
        import torch
        self.lib = load_library()
        self.tuning = []
        if autotune:
            from .autotune import tune_spread
            self.tuning = [tune_spread(p, cache=tune_cache) for p in plans]
        n = len(plans)
        if not (n == len(sigma) == len(u)) or n == 0:
            raise ValueError("plans, sigma and u must be non-empty lists of equal length")
        for p, s, x in zip(plans, sigma, u):
            for tsr, m in ((s, p.M), (x, p.Nx)):
                if not (isinstance(tsr, torch.Tensor) and tsr.is_cuda and tsr.dtype == torch.float64
                        and tsr.numel() == m and tsr.is_contiguous()):
                    raise ValueError("batch buffers must be contiguous float64 CUDA tensors of size M_i / Nx_i")
        if stream is None:
            stream = torch.cuda.current_stream(plans[0].device)
        self.plans, self.sigma, self.u, self.stream = list(plans), list(sigma), list(u), stream
        arr = lambda xs: (ctypes.c_void_p * n)(*[ctypes.c_void_p(x) for x in xs])
        h = ctypes.c_void_p()
        rc = self.lib.wfp2d_batch_create(ctypes.byref(h), n, arr([p.h.value for p in plans]),
                                         arr([s.data_ptr() for s in sigma]), arr([x.data_ptr() for x in u]),
                                         int(n_streams), ctypes.c_void_p(int(stream.cuda_stream)))
        if rc != 0:
            raise Wfp2dError(rc, self.lib.wfp2d_last_error(None).decode())
        self.h = h

    def launch(self):
        rc = self.lib.wfp2d_batch_launch(self.h)
        if rc != 0:
            raise Wfp2dError(rc, self.lib.wfp2d_last_error(None).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.wfp2d_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
