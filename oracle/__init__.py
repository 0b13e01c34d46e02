"""CPU FP64 oracle for the L1 time-stepping scheme (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path.

The arithmetic lives in ``oracle.c`` (plain C, FP64, O(M N^2) forward time
stepping -- the paper's "direct method" for the block lower-triangular Toeplitz
system of Scheme 4, section 3); this module only marshals numpy arrays.

Parity status of each function (what pins it, in tests/test_oracle_*.py):
  weights   -- decimal references, invariants, row sums, digamma vs scipy
  solve     -- closed forms, single-mode reduction, dense LU brute force,
               Table 9 and Table 7 of the paper, convergence rates
  apply     -- dense brute force
  adjoint   -- dot test, central differences in f and in gamma
  mode      -- closed form on linear-in-time data, dense brute force
  solve_adv -- Table 5 and Table 7 of the paper, closed forms on data
               linear in x and t, dense brute force
  solve_cn, apply_cn, mode_cn
            -- exactness on (1 + t) sine modes, dense brute force, single-mode
               reduction, the convergence order 3 - gamma in tau
  ode_column, ode_cg
            -- Theorem 1's row identity, Table 1 of the paper, CG finite
               termination and agreement with a Toeplitz solve
  gmres     -- finite termination at the dense solve, least-squares estimates
               equal to recomputed residuals, the one-step minimal-residual
               closed form, exact convergence in N steps with the
               block-diagonal preconditioner, agreement with solve
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    i64, d, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.oracle_digamma.restype = d
    lib.oracle_digamma.argtypes = [d]
    lib.oracle_threads.restype = i32
    lib.oracle_weights.restype = i32
    lib.oracle_weights.argtypes = [d, d, i64] + [_dp] * 8
    lib.oracle_solve.restype = i32
    lib.oracle_solve.argtypes = [d, d, d, d, i64, i64, i64, _dp, _dp, _dp, _dp, i32]
    lib.oracle_solve_rows.restype = i32
    lib.oracle_solve_rows.argtypes = [d, d, d, d, i64, i64, i64, i64, _dp, _dp, _dp, _dp, i32]
    lib.oracle_apply.restype = i32
    lib.oracle_apply.argtypes = [d, d, d, d, i64, i64, _dp, _dp, i32]
    lib.oracle_adjoint.restype = i32
    lib.oracle_adjoint.argtypes = [d, d, d, d, i64, i64, _dp, _dp, _dp, _dp, _dp, _dp, i32]
    lib.oracle_mode.restype = i32
    lib.oracle_mode.argtypes = [d, d, i64, d, _dp, d, d, _dp]
    lib.oracle_solve_adv.restype = i32
    lib.oracle_solve_adv.argtypes = [d, d, d, d, i64, i64, _dp, _dp, _dp, _dp, i32]
    lib.oracle_solve_cn.restype = i32
    lib.oracle_solve_cn.argtypes = [d, d, d, d, i64, i64, _dp, _dp, _dp, _dp, i32]
    lib.oracle_apply_cn.restype = i32
    lib.oracle_apply_cn.argtypes = [d, d, d, d, i64, i64, _dp, _dp, i32]
    lib.oracle_mode_cn.restype = i32
    lib.oracle_mode_cn.argtypes = [d, d, i64, d, _dp, d, d, _dp]
    lib.oracle_ode_column.restype = i32
    lib.oracle_ode_column.argtypes = [d, i64, _dp]
    lib.oracle_ode_cg.restype = i32
    lib.oracle_ode_cg.argtypes = [d, i64, _dp, _dp, i32, d, i32, ctypes.POINTER(i32), _dp, _dp]
    lib.oracle_gmres.restype = i32
    lib.oracle_gmres.argtypes = [d, d, d, d, i64, i64, _dp, _dp, _dp, _dp, i32, i32, d, i32, i32,
                                 ctypes.POINTER(i32), _dp, _dp, i32]
    _lib = lib
    return lib


def _ptr(x):
    if x is None:
        return None
    return x.ctypes.data_as(_dp)


def _f64(x, shape=None):
    if x is None:
        return None
    x = np.ascontiguousarray(x, dtype=np.float64)
    if shape is not None and x.shape != shape:
        x = x.reshape(shape)
    return x


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with status %d" % (what, rc))


def threads() -> int:
    return int(_load().oracle_threads())


def digamma(x: float) -> float:
    return float(_load().oracle_digamma(float(x)))


def weights(gamma: float, T: float, N: int) -> dict:
    """b_k, a_m, rho_n, psi_n and their gamma-derivatives (length N each)."""
    lib = _load()
    out = {k: np.zeros(N) for k in ("b", "a", "rho", "psi", "da", "drho", "dpsi")}
    scal = np.zeros(2)
    rc = lib.oracle_weights(gamma, T, N, *(_ptr(out[k]) for k in ("b", "a", "rho", "psi", "da", "drho", "dpsi")),
                            _ptr(scal))
    _check(rc, "weights")
    out["coef"], out["dcoef"] = float(scal[0]), float(scal[1])
    return out


def solve(gamma, T, x0, x1, M, N, f, u0=None, phi=None, nsteps=None, nthreads=0):
    """Forward time stepping; returns U [N][M] (rows >= nsteps are zero)."""
    lib = _load()
    f = _f64(f, (N, M))
    u0 = _f64(u0, (M,))
    phi = _f64(phi, (M,))
    u = np.zeros((N, M))
    rc = lib.oracle_solve(gamma, T, x0, x1, M, N, N if nsteps is None else nsteps,
                          _ptr(f), _ptr(u0), _ptr(phi), _ptr(u), nthreads)
    _check(rc, "solve")
    return u


def solve_rows(gamma, T, x0, x1, M, N, f, u, nfirst, nsteps, u0=None, phi=None, nthreads=0):
    """Continue a forward run in place: rows nfirst..nsteps-1 of u (float64
    [N][M], C order; rows below nfirst already solved by earlier calls)."""
    lib = _load()
    f = _f64(f, (N, M))
    u0 = _f64(u0, (M,))
    phi = _f64(phi, (M,))
    if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.shape == (N, M) and u.flags.c_contiguous):
        raise ValueError("u must be a C-contiguous float64 array of shape (N, M)")
    rc = lib.oracle_solve_rows(gamma, T, x0, x1, M, N, nfirst, nsteps, _ptr(f), _ptr(u0), _ptr(phi), _ptr(u),
                               nthreads)
    _check(rc, "solve_rows")
    return u


def apply(gamma, T, x0, x1, M, N, u, nthreads=0):
    """y = A u for the block lower-triangular system (without the u0/phi terms)."""
    lib = _load()
    u = _f64(u, (N, M))
    y = np.zeros((N, M))
    _check(lib.oracle_apply(gamma, T, x0, x1, M, N, _ptr(u), _ptr(y), nthreads), "apply")
    return y


def adjoint(gamma, T, x0, x1, M, N, g, u, u0=None, phi=None, nthreads=0):
    """Returns (Lambda = dL/dF [N][M], dL/dgamma) for upstream gradient g = dL/dU."""
    lib = _load()
    g = _f64(g, (N, M))
    u = _f64(u, (N, M))
    u0 = _f64(u0, (M,))
    phi = _f64(phi, (M,))
    lam = np.zeros((N, M))
    dg = ctypes.c_double(0.0)
    rc = lib.oracle_adjoint(gamma, T, x0, x1, M, N, _ptr(g), _ptr(u), _ptr(u0), _ptr(phi),
                            _ptr(lam), ctypes.byref(dg), nthreads)
    _check(rc, "adjoint")
    return lam, float(dg.value)


def mode(gamma, T, N, lam, g, v0=0.0, phihat=0.0):
    """Scalar recurrence of one sine mode with eigenvalue lam (length-N result)."""
    lib = _load()
    g = _f64(g, (N,))
    v = np.zeros(N)
    _check(lib.oracle_mode(gamma, T, N, lam, _ptr(g), v0, phihat, _ptr(v)), "mode")
    return v


def solve_adv(gamma, T, x0, x1, M, N, f, u0=None, phi=None, nthreads=0):
    """Advection equations D^gamma u + u_x = f, inflow u(x0, t) = 0: Scheme 2
    (gamma < 1; f sampled at x_i - h/2, t_n) or Scheme 3 (gamma > 1; f at
    x_i, t_{n-1/2}).  Returns U [N][M]."""
    lib = _load()
    f = _f64(f, (N, M))
    u0 = _f64(u0, (M,))
    phi = _f64(phi, (M,))
    u = np.zeros((N, M))
    _check(lib.oracle_solve_adv(gamma, T, x0, x1, M, N, _ptr(f), _ptr(u0), _ptr(phi), _ptr(u), nthreads),
           "solve_adv")
    return u


def solve_cn(gamma, T, x0, x1, M, N, f, u0=None, phi=None, nthreads=0):
    """Diffusion-wave (1 < gamma < 2) with the spatial term averaged over t_n
    and t_{n-1}; f sampled at t_{n-1/2}.  Returns U [N][M]."""
    lib = _load()
    f = _f64(f, (N, M))
    u0 = _f64(u0, (M,))
    phi = _f64(phi, (M,))
    u = np.zeros((N, M))
    _check(lib.oracle_solve_cn(gamma, T, x0, x1, M, N, _ptr(f), _ptr(u0), _ptr(phi), _ptr(u), nthreads), "solve_cn")
    return u


def apply_cn(gamma, T, x0, x1, M, N, u, nthreads=0):
    """y = A u for the system of solve_cn (without the u0/phi terms)."""
    lib = _load()
    u = _f64(u, (N, M))
    y = np.zeros((N, M))
    _check(lib.oracle_apply_cn(gamma, T, x0, x1, M, N, _ptr(u), _ptr(y), nthreads), "apply_cn")
    return y


def mode_cn(gamma, T, N, lam, g, v0=0.0, phihat=0.0):
    """Scalar recurrence of one sine mode of solve_cn (length-N result)."""
    lib = _load()
    g = _f64(g, (N,))
    v = np.zeros(N)
    _check(lib.oracle_mode_cn(gamma, T, N, lam, _ptr(g), v0, phihat, _ptr(v)), "mode_cn")
    return v


def ode_column(gamma, N):
    """First column of the symmetric Toeplitz matrix of Scheme 1 (N - 1 entries)."""
    c = np.zeros(N - 1)
    _check(_load().oracle_ode_column(gamma, N, _ptr(c)), "ode_column")
    return c


def ode_cg(gamma, N, f, maxit=10000, rtol=1e-10, guess=None):
    """Conjugate gradients for Scheme 1; returns (u [N-1], info)."""
    lib = _load()
    f = _f64(f, (N - 1,))
    u = np.zeros(N - 1) if guess is None else np.array(_f64(guess, (N - 1,)))
    out = (ctypes.c_int * 2)()
    rel = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    rc = lib.oracle_ode_cg(gamma, N, _ptr(f), _ptr(u), maxit, rtol, 0 if guess is None else 1, out,
                           ctypes.byref(rel), _ptr(hist))
    _check(rc, "ode_cg")
    it = int(out[0])
    return u, {"iters": it, "converged": bool(out[1]), "relres": float(rel.value), "hist": hist[: it + 1].copy()}


def gmres(gamma, T, x0, x1, M, N, f, u0=None, phi=None, restart=30, maxit=1000, rtol=1e-10, precond=0,
          guess=None, nthreads=0):
    """Restarted GMRES(m) on the same system (the paper's iterative method).

    Returns (u [N][M], info) with info = {"iters", "cycles", "converged",
    "relres" (recomputed), "hist" (least-squares residuals / ||b||, length
    iters + 1)}.
    """
    lib = _load()
    f = _f64(f, (N, M))
    u0 = _f64(u0, (M,))
    phi = _f64(phi, (M,))
    u = np.zeros((N, M)) if guess is None else np.array(_f64(guess, (N, M)))
    out = (ctypes.c_int * 3)()
    rel = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    rc = lib.oracle_gmres(gamma, T, x0, x1, M, N, _ptr(f), _ptr(u0), _ptr(phi), _ptr(u), restart, maxit, rtol,
                          precond, 0 if guess is None else 1, out, ctypes.byref(rel), _ptr(hist), nthreads)
    _check(rc, "gmres")
    it = int(out[0])
    return u, {"iters": it, "cycles": int(out[1]), "converged": bool(out[2]), "relres": float(rel.value),
               "hist": hist[: it + 1].copy()}


def grid(x0, x1, M, T, N):
    """x_i (i=1..M) and t_n (n=1..N) of the uniform grid used by every routine."""
    h = (x1 - x0) / (M + 1)
    tau = T / N
    return x0 + h * np.arange(1, M + 1), tau * np.arange(1, N + 1), h, tau


def eig_K(M, j, x0=0.0, x1=1.0):
    """Eigenvalue of K = h^-2 tridiag(-1,2,-1) for the sine mode sin(j pi (x-x0)/(x1-x0))."""
    h = (x1 - x0) / (M + 1)
    return 4.0 / (h * h) * np.sin(j * np.pi * h / (2.0 * (x1 - x0))) ** 2
