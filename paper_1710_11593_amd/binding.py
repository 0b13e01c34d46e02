"""Python binding of the fracsolve C ABI (include/fracsolve.h).

Argument marshalling only: every step of the solve runs in the HIP library
csrc/libfracsolve.so.  Fields are torch float64 CUDA tensors of shape [N, M]
(time-major, row n-1 = t_n); their device pointers are handed to the library,
which enqueues its work on torch's current stream.  If the library has not
been built this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "csrc", "libfracsolve.so")

FRACSOLVE_OK = 0
STATUS = {0: "OK", -1: "E_ARG", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_NUMERIC", -5: "E_STATE"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2}
EQUATION = {"diffusion": 0, "advection": 1, "diffusion_cn": 2}


class Problem(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("T", ctypes.c_double), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("M", ctypes.c_int64), ("N", ctypes.c_int64)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("crossover", ctypes.c_int32), ("leaf_solver", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("equation", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("crossover", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("kernels", ctypes.c_int32), ("ms_total", ctypes.c_double), ("ms_leaf", ctypes.c_double),
                ("ms_dense", ctypes.c_double), ("ms_fft", ctypes.c_double), ("residual_norm", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("s", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("tasks", ctypes.c_int32), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class GmresOptions(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("precond", ctypes.c_int32), ("use_guess", ctypes.c_int32)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("relres", ctypes.c_double), ("relres_est", ctypes.c_double)]


class CgOptions(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("rtol", ctypes.c_double), ("use_guess", ctypes.c_int32)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("relres", ctypes.c_double),
                ("relres_est", ctypes.c_double)]


KIND_NAMES = {0: "leaf", 1: "dense_f64", 2: "dense_f32", 3: "fft_f64", 4: "fft_f32", 5: "fft_corner"}

EXPORTS = ["fracsolve_create", "fracsolve_weights", "fracsolve_solve", "fracsolve_apply", "fracsolve_adjoint",
           "fracsolve_gmres", "fracsolve_ode_cg", "fracsolve_ode_cg_noalloc", "fracsolve_plan",
           "fracsolve_set_timing", "fracsolve_set_check", "fracsolve_get_stats", "fracsolve_kernel_stats",
           "fracsolve_destroy", "fracsolve_last_error"]

_lib = None


class FracsolveError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("fracsolve HIP library not built: %s is missing (run paper_1710_11593_amd.build.build())" % LIBPATH)
    L = ctypes.CDLL(LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vpp = ctypes.POINTER(ctypes.c_void_p)
    L.fracsolve_create.restype = ctypes.c_int
    L.fracsolve_create.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Options),
                                   ctypes.POINTER(ctypes.c_void_p)]
    L.fracsolve_weights.restype = ctypes.c_int
    L.fracsolve_weights.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [dp] * 7
    L.fracsolve_solve.restype = ctypes.c_int
    L.fracsolve_solve.argtypes = [ctypes.c_void_p, vpp, vpp, vpp, vpp]
    L.fracsolve_apply.restype = ctypes.c_int
    L.fracsolve_apply.argtypes = [ctypes.c_void_p, vpp, vpp]
    L.fracsolve_adjoint.restype = ctypes.c_int
    L.fracsolve_adjoint.argtypes = [ctypes.c_void_p, vpp, vpp, vpp, vpp, vpp, dp]
    L.fracsolve_gmres.restype = ctypes.c_int
    L.fracsolve_gmres.argtypes = [ctypes.c_void_p, vpp, vpp, vpp, vpp, ctypes.POINTER(GmresOptions),
                                  ctypes.POINTER(GmresInfo), dp, ctypes.c_int32]
    L.fracsolve_ode_cg.restype = ctypes.c_int
    L.fracsolve_ode_cg.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(CgOptions), ctypes.POINTER(CgInfo), dp, ctypes.c_int32,
                                   ctypes.c_void_p]
    L.fracsolve_plan.restype = ctypes.c_int
    L.fracsolve_plan.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Options),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32)]
    L.fracsolve_ode_cg_noalloc.restype = ctypes.c_int
    L.fracsolve_ode_cg_noalloc.argtypes = L.fracsolve_ode_cg.argtypes
    L.fracsolve_set_timing.restype = ctypes.c_int
    L.fracsolve_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fracsolve_set_check.restype = ctypes.c_int
    L.fracsolve_set_check.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fracsolve_get_stats.restype = ctypes.c_int
    L.fracsolve_get_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(Stats)]
    L.fracsolve_kernel_stats.restype = ctypes.c_int
    L.fracsolve_kernel_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(KernelStat), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]
    L.fracsolve_destroy.restype = None
    L.fracsolve_destroy.argtypes = [ctypes.c_void_p]
    L.fracsolve_last_error.restype = ctypes.c_char_p
    L.fracsolve_last_error.argtypes = [ctypes.c_void_p]
    _lib = L
    return L


def _ptrs(tensors, required=True, name="field"):
    """Host array of device pointers (None entries -> NULL)."""
    if tensors is None:
        return None
    arr = (ctypes.c_void_p * len(tensors))()
    for k, t in enumerate(tensors):
        if t is None:
            if required:
                raise ValueError("%s[%d] is None" % (name, k))
            arr[k] = None
            continue
        if not t.is_cuda or t.dtype.__str__() != "torch.float64" or not t.is_contiguous():
            raise ValueError("%s[%d] must be a contiguous float64 CUDA tensor" % (name, k))
        arr[k] = t.data_ptr()
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))


PLAN_SOURCE = {0: "options", 1: "cache", 2: "builtin"}


def _problems(problems):
    arr = (Problem * len(problems))()
    for k, p in enumerate(problems):
        arr[k] = Problem(float(p["gamma"]), float(p.get("T", 1.0)), float(p.get("x0", 0.0)),
                         float(p.get("x1", 1.0)), int(p["M"]), int(p["N"]))
    return arr


def plan(problems: Sequence[dict], precision="fp64", leaf=0, crossover=0, leaf_solver=0, equation="diffusion"):
    """(leaf, crossover, source) that fracsolve_create would choose
    (fracsolve_plan; host only, no device needed)."""
    L = lib()
    opts = Options(PRECISION[precision] if isinstance(precision, str) else int(precision), 0, int(leaf),
                   int(crossover), int(leaf_solver), None,
                   EQUATION[equation] if isinstance(equation, str) else int(equation))
    lf, cr, src = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = L.fracsolve_plan(_problems(problems), len(problems), ctypes.byref(opts), ctypes.byref(lf), ctypes.byref(cr),
                          ctypes.byref(src))
    if rc != FRACSOLVE_OK:
        raise FracsolveError(rc, L.fracsolve_last_error(None).decode())
    return lf.value, cr.value, PLAN_SOURCE.get(src.value, src.value)


class Solver:
    """One handle over `len(problems)` instances (see fracsolve_create)."""

    def __init__(self, problems: Sequence[dict], precision="fp64", refine_steps=0, leaf=0, crossover=0,
                 leaf_solver=0, stream=None, equation="diffusion"):
        L = lib()
        self._lib = L
        self.problems = [dict(p) for p in problems]
        arr = _problems(problems)
        if stream is None:
            import torch

            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        opts = Options(PRECISION[precision] if isinstance(precision, str) else int(precision), int(refine_steps),
                       int(leaf), int(crossover), int(leaf_solver), ctypes.c_void_p(stream),
                       EQUATION[equation] if isinstance(equation, str) else int(equation))
        h = ctypes.c_void_p()
        rc = L.fracsolve_create(arr, len(problems), ctypes.byref(opts), ctypes.byref(h))
        if rc != FRACSOLVE_OK:
            raise FracsolveError(rc, L.fracsolve_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != FRACSOLVE_OK:
            raise FracsolveError(rc, self._lib.fracsolve_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._lib.fracsolve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self, inst=0):
        import numpy as np

        N = self.problems[inst]["N"]
        out = {k: np.zeros(N) for k in ("b", "a", "rho", "psi", "da", "drho", "dpsi")}
        dp = ctypes.POINTER(ctypes.c_double)
        args = [out[k].ctypes.data_as(dp) for k in ("b", "a", "rho", "psi", "da", "drho", "dpsi")]
        self._check(self._lib.fracsolve_weights(self.h, inst, *args))
        return out

    def solve(self, f, u0=None, phi=None, out=None):
        """f: list (one per instance) of [N,M] tensors; returns the list of solutions."""
        import torch

        f = list(f)
        if out is None:
            out = [torch.empty_like(x) for x in f]
        u0p = _ptrs(u0, required=False, name="u0") if u0 is not None else None
        php = _ptrs(phi, required=False, name="phi") if phi is not None else None
        self._check(self._lib.fracsolve_solve(self.h, _ptrs(f, name="f"), u0p, php, _ptrs(out, name="u")))
        return out

    def apply(self, u, out=None):
        import torch

        u = list(u)
        if out is None:
            out = [torch.empty_like(x) for x in u]
        self._check(self._lib.fracsolve_apply(self.h, _ptrs(u, name="u"), _ptrs(out, name="y")))
        return out

    def adjoint(self, g, u=None, u0=None, phi=None, out=None, want_gamma=True):
        import torch

        g = list(g)
        if out is None:
            out = [torch.empty_like(x) for x in g]
        dg = (ctypes.c_double * len(g))() if want_gamma else None
        rc = self._lib.fracsolve_adjoint(
            self.h, _ptrs(g, name="g"), _ptrs(u, name="u") if u is not None else None,
            _ptrs(u0, required=False, name="u0") if u0 is not None else None,
            _ptrs(phi, required=False, name="phi") if phi is not None else None, _ptrs(out, name="dL_df"),
            ctypes.cast(dg, ctypes.POINTER(ctypes.c_double)) if want_gamma else None)
        self._check(rc)
        return out, (list(dg) if want_gamma else None)

    def gmres(self, f, u0=None, phi=None, out=None, restart=30, max_iters=1000, rtol=1e-10, precond=0,
              use_guess=False, hist_cap=0):
        """Restarted GMRES(m) on every instance (fracsolve_gmres).

        Returns (list of iterates, list of info dicts, residual history of
        instance 0 as a numpy array of length min(hist_cap, iterations + 1)).
        """
        import numpy as np
        import torch

        f = list(f)
        if out is None:
            out = [torch.empty_like(x) for x in f]
        opts = GmresOptions(int(restart), int(max_iters), float(rtol), int(precond), 1 if use_guess else 0)
        info = (GmresInfo * len(f))()
        hist = np.zeros(max(int(hist_cap), 1))
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.fracsolve_gmres(
            self.h, _ptrs(f, name="f"), _ptrs(u0, required=False, name="u0") if u0 is not None else None,
            _ptrs(phi, required=False, name="phi") if phi is not None else None, _ptrs(out, name="u"),
            ctypes.byref(opts), info, hist.ctypes.data_as(dp) if hist_cap > 0 else None, int(hist_cap))
        self._check(rc)
        infos = [{k: getattr(info[i], k) for k, _ in GmresInfo._fields_ if k != "reserved"} for i in range(len(f))]
        for d in infos:
            d["converged"] = bool(d["converged"])
        nh = min(int(hist_cap), infos[0]["iterations"] + 1) if hist_cap > 0 else 0
        return out, infos, hist[:nh].copy()

    def set_timing(self, on=True):
        self._check(self._lib.fracsolve_set_timing(self.h, 1 if on else 0))

    def kernel_stats(self):
        """Per-(kind, level) launch count, time and algorithmic bytes of the last call (timing level 2)."""
        cap = 256
        arr = (KernelStat * cap)()
        n = ctypes.c_int32(0)
        self._check(self._lib.fracsolve_kernel_stats(self.h, arr, cap, ctypes.byref(n)))
        return [dict(kind=KIND_NAMES[arr[k].kind], s=arr[k].s, launches=arr[k].launches, tasks=arr[k].tasks,
                     ms=arr[k].ms, bytes=arr[k].bytes) for k in range(min(n.value, cap))]

    def set_check(self, on=True):
        """Scan every later call's outputs for NaN / infinities (E_NUMERIC)."""
        self._check(self._lib.fracsolve_set_check(self.h, 1 if on else 0))

    def set_timing_level(self, level):
        self._check(self._lib.fracsolve_set_timing(self.h, int(level)))

    def stats(self):
        s = Stats()
        self._check(self._lib.fracsolve_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}


def ode_cg(gamma, N, f, out=None, max_iters=10000, rtol=1e-10, use_guess=False, hist_cap=0, stream=None,
           noalloc=False):
    """Scheme 1 (the two-sided fractional ODE) by conjugate gradients with the
    FFT operator (fracsolve_ode_cg; noalloc=True: fracsolve_ode_cg_noalloc,
    whose workspace is the library's fixed device array).  f: float64 CUDA
    tensor of the N - 1 values at t_i = i/N.  Returns (u, info dict, residual
    history)."""
    import numpy as np
    import torch

    L = lib()
    if not f.is_cuda or f.dtype != torch.float64 or not f.is_contiguous() or f.numel() != N - 1:
        raise ValueError("f must be a contiguous float64 CUDA tensor of N - 1 values")
    if out is None:
        out = torch.empty_like(f)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    opts = CgOptions(int(max_iters), float(rtol), 1 if use_guess else 0)
    info = CgInfo()
    hist = np.zeros(max(int(hist_cap), 1))
    fn = L.fracsolve_ode_cg_noalloc if noalloc else L.fracsolve_ode_cg
    rc = fn(float(gamma), int(N), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            ctypes.byref(opts), ctypes.byref(info),
            hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if hist_cap > 0 else None,
            int(hist_cap), ctypes.c_void_p(stream))
    if rc != FRACSOLVE_OK:
        raise FracsolveError(rc, L.fracsolve_last_error(None).decode())
    d = {k: getattr(info, k) for k, _ in CgInfo._fields_}
    d["converged"] = bool(d["converged"])
    nh = min(int(hist_cap), d["iterations"] + 1) if hist_cap > 0 else 0
    return out, d, hist[:nh].copy()


_solver_cache = {}


def _cached_solver(gamma, T, x0, x1, M, N, precision, refine_steps):
    key = (float(gamma), T, x0, x1, M, N, precision, refine_steps)
    s = _solver_cache.get(key)
    if s is None:
        if len(_solver_cache) > 8:
            _solver_cache.clear()
        s = Solver([dict(gamma=float(gamma), T=T, x0=x0, x1=x1, M=M, N=N)], precision=precision,
                   refine_steps=refine_steps)
        _solver_cache[key] = s
    return s


def _make_function():
    import torch

    class FracSolve(torch.autograd.Function):
        """u = solve(f; gamma) with u0, phi fixed data.

        forward(f [N,M], gamma (0-dim tensor), u0 [M] or None, phi [M] or None,
                T=1, x0=0, x1=1) -> u [N,M]
        backward: dL/df by the reverse-time adjoint solve, dL/dgamma through
        the gamma-derivatives of the weights (both computed by the library).
        """

        @staticmethod
        def forward(ctx, f, gamma, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0):
            N, M = f.shape
            s = _cached_solver(float(gamma), T, x0, x1, M, N, "fp64", 0)
            f = f.contiguous()
            u = s.solve([f], [u0] if u0 is not None else None, [phi] if phi is not None else None)[0]
            ctx.solver = s
            ctx.gamma_device = gamma.device if isinstance(gamma, torch.Tensor) else None
            ctx.save_for_backward(u, u0 if u0 is not None else None, phi if phi is not None else None)
            ctx.has = (u0 is not None, phi is not None)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            u, u0, phi = ctx.saved_tensors
            s = ctx.solver
            g = grad_u.contiguous()
            lam, dg = s.adjoint([g], [u], [u0] if ctx.has[0] else None, [phi] if ctx.has[1] else None)
            dgamma = None
            if ctx.gamma_device is not None:
                dgamma = torch.tensor(dg[0], dtype=torch.float64, device=ctx.gamma_device)
            return lam[0], dgamma, None, None, None, None, None

    return FracSolve


_fn = None


def frac_solve(f, gamma, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0):
    """Differentiable solve (see FracSolve)."""
    global _fn
    if _fn is None:
        _fn = _make_function()
    return _fn.apply(f, gamma, u0, phi, T, x0, x1)
