"""Extended-precision references for the parity tests (test infrastructure).

The same forward time stepping as the oracle (Scheme 4 / eq. e15-e17 time
weights, one Thomas solve per step) carried out in x87 extended precision
(numpy.longdouble, 64-bit significand), with the weights and the constant
tau^-gamma / Gamma(2-gamma) (or Gamma(3-gamma)) evaluated in 40-digit decimal.
It measures how far the float64 oracle itself is from the exact discrete
solution on inputs where float64 rounding is amplified (rough random sources
at large M or gamma near 2), so that a float64 GPU result can be required to
be at least as accurate as the float64 oracle there.

Pinned in tests/test_ext_reference.py (CPU): against the oracle on benign
inputs, against a 40-digit decimal dense solve of the assembled block system,
and the decimal Gamma function against its closed forms.

ext_mode_lib() loads tests/ext_mode.c, the long double single-mode
recurrence, pinned the same way.
"""
import ctypes
import math
import os
import subprocess
from decimal import Decimal, getcontext, localcontext

import numpy as np

FLOOR_ORACLE_MAX = 1e-8   # the float64 oracle must itself be this close to the extended solve


def dec_pi():
    """pi in the current decimal context (Machin: 4 atan(1/5) - atan(1/239))."""
    def atan_inv(x):
        x = Decimal(x)
        x2, term, total, k = x * x, 1 / x, 1 / x, 1
        eps = Decimal(10) ** (-(getcontext().prec + 2))
        while abs(term) > eps:
            term = -term / x2
            total += term / (2 * k + 1)
            k += 1
        return total

    with localcontext() as ctx:
        ctx.prec += 5
        v = 4 * (4 * atan_inv(5) - atan_inv(239))
    return +v


def _bernoulli_even(count):
    """B_2, B_4, ..., B_{2 count} as exact fractions (Akiyama-Tanigawa)."""
    from fractions import Fraction

    n_max = 2 * count
    out = []
    a = [Fraction(0)] * (n_max + 1)
    for m in range(n_max + 1):
        a[m] = Fraction(1, m + 1)
        for j in range(m, 0, -1):
            a[j - 1] = j * (a[j - 1] - a[j])
        if m >= 2 and m % 2 == 0:
            out.append(a[0])
    return out


def dec_gamma(x):
    """Gamma(x) for 0 < x <= 4 in the current decimal context: shift the
    argument up by K (Gamma(x) = Gamma(x+K) / (x (x+1) ... (x+K-1))) and sum
    Stirling's series for log Gamma(x+K)."""
    x = Decimal(x)
    with localcontext() as ctx:
        ctx.prec += 10
        K = 40
        z = x + K
        prod = Decimal(1)
        for k in range(K):
            prod *= x + k
        lg = (z - Decimal("0.5")) * z.ln() - z + (2 * dec_pi()).ln() / 2
        zpow = z
        for k, B in enumerate(_bernoulli_even(12), start=1):
            lg += Decimal(B.numerator) / Decimal(B.denominator) / (2 * k * (2 * k - 1) * zpow)
            zpow *= z * z
        v = lg.exp() / prod
    return +v


def weights(gamma, N, T=1.0):
    getcontext().prec = 40
    tau = Decimal(repr(T)) / Decimal(N)
    # the system of the float64 gamma given: its exact binary value, with the
    # exponent and the Gamma argument formed exactly (1 - gamma in float64 is
    # rounded)
    g = Decimal(float(gamma))
    garg = (2 - g) if gamma < 1 else (3 - g)
    coef = (tau.ln() * (-g)).exp() / dec_gamma(garg)
    pd = (1 - g) if gamma < 1 else (2 - g)

    def b(k):
        if k < 0:
            return Decimal(0)
        hi = (pd * Decimal(k + 1).ln()).exp()
        lo = Decimal(0) if k == 0 else (pd * Decimal(k).ln()).exp()
        return hi - lo

    B = [b(k) for k in range(-2, N + 1)]

    def bb(k):
        return B[k + 2]

    if gamma < 1:
        a = [coef * (bb(m) - bb(m - 1)) for m in range(N)]
        rho = [-coef * bb(n - 1) for n in range(1, N + 1)]
        psi = [Decimal(0)] * N
    else:
        a = [coef * (bb(m - 2) - 2 * bb(m - 1) + bb(m)) for m in range(N)]
        rho = [coef * (bb(n - 2) - bb(n - 1)) for n in range(1, N + 1)]
        psi = [coef * tau * bb(n - 1) for n in range(1, N + 1)]

    def conv(v):
        return np.array([np.longdouble(str(x)) for x in v])

    return conv(a), conv(rho), conv(psi)


def given_weights(w, N):
    """(a, rho, psi) as long double arrays from float64 weights w (a dict or
    triple of arrays of at least N entries)."""
    if isinstance(w, dict):
        w = (w["a"], w["rho"], w["psi"])
    return tuple(np.asarray(x[:N], dtype=np.longdouble) for x in w)


def solve(gamma, M, N, F, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0, weights_given=None):
    """Extended-precision stepping; weights_given: use these float64 weights
    (the system they define) instead of the decimal ones."""
    a, rho, psi = weights(gamma, N, T) if weights_given is None else given_weights(weights_given, N)
    h = (np.longdouble(x1) - np.longdouble(x0)) / np.longdouble(M + 1)
    e = 1 / (h * h)
    d = a[0] + 2 * e
    cp = np.zeros(M, dtype=np.longdouble)
    inv = np.zeros(M, dtype=np.longdouble)
    prev = np.longdouble(0)
    for i in range(M):
        piv = d + e * prev
        inv[i] = 1 / piv
        cp[i] = -e * inv[i]
        prev = cp[i]
    Fl = np.asarray(F, dtype=np.longdouble)
    u0l = np.zeros(M, dtype=np.longdouble) if u0 is None else np.asarray(u0, dtype=np.longdouble)
    phil = None if (phi is None or gamma < 1) else np.asarray(phi, dtype=np.longdouble)
    U = np.zeros((N, M), dtype=np.longdouble)
    for n in range(N):
        r = Fl[n] - rho[n] * u0l
        if phil is not None:
            r = r + psi[n] * phil
        for j in range(n):
            r = r - a[n - j] * U[j]
        x = np.zeros(M, dtype=np.longdouble)
        pv = np.longdouble(0)
        for i in range(M):
            x[i] = (r[i] + e * pv) * inv[i]
            pv = x[i]
        for i in range(M - 2, -1, -1):
            x[i] -= cp[i] * x[i + 1]
        U[n] = x
    return U


def solve_adv(gamma, M, N, F, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0, weights_given=None):
    """The advection time stepping of the oracle (Scheme 2 for gamma < 1,
    Scheme 3 for gamma > 1; inflow value 0) in extended precision."""
    a, rho, psi = weights(gamma, N, T) if weights_given is None else given_weights(weights_given, N)
    h = (np.longdouble(x1) - np.longdouble(x0)) / np.longdouble(M + 1)
    Fl = np.asarray(F, dtype=np.longdouble)
    u0l = np.zeros(M, dtype=np.longdouble) if u0 is None else np.asarray(u0, dtype=np.longdouble)
    phil = None if (phi is None or gamma < 1) else np.asarray(phi, dtype=np.longdouble)

    def shift(v):  # v_{i-1}, with 0 at the inflow
        return np.concatenate(([np.longdouble(0)], v[:-1]))

    U = np.zeros((N, M), dtype=np.longdouble)
    for n in range(N):
        if gamma < 1:
            r = 2 * Fl[n] - rho[n] * (u0l + shift(u0l))
            for j in range(n):
                r = r - a[n - j] * (U[j] + shift(U[j]))
            lo, di = a[0] - 2 / h, a[0] + 2 / h
        else:
            r = Fl[n] - rho[n] * u0l
            if phil is not None:
                r = r + psi[n] * phil
            for j in range(n):
                r = r - a[n - j] * U[j]
            lo, di = -1 / h, a[0] + 1 / h
        pv = np.longdouble(0)
        for i in range(M):
            U[n, i] = (r[i] - lo * pv) / di
            pv = U[n, i]
    return U


def solve_cn(gamma, M, N, F, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0, weights_given=None):
    """The oracle's stepping of the diffusion-wave variant with the spatial
    term averaged over t_n and t_{n-1}, in extended precision."""
    a, rho, psi = weights(gamma, N, T) if weights_given is None else given_weights(weights_given, N)
    h = (np.longdouble(x1) - np.longdouble(x0)) / np.longdouble(M + 1)
    e = 1 / (h * h)
    he = e / 2
    d = a[0] + e
    cp = np.zeros(M, dtype=np.longdouble)
    inv = np.zeros(M, dtype=np.longdouble)
    prev = np.longdouble(0)
    for i in range(M):
        piv = d + he * prev
        inv[i] = 1 / piv
        cp[i] = -he * inv[i]
        prev = cp[i]
    Fl = np.asarray(F, dtype=np.longdouble)
    u0l = np.zeros(M, dtype=np.longdouble) if u0 is None else np.asarray(u0, dtype=np.longdouble)
    phil = np.zeros(M, dtype=np.longdouble) if phi is None else np.asarray(phi, dtype=np.longdouble)

    def K(v):
        left = np.concatenate(([np.longdouble(0)], v[:-1]))
        right = np.concatenate((v[1:], [np.longdouble(0)]))
        return e * (2 * v - left - right)

    U = np.zeros((N, M), dtype=np.longdouble)
    for n in range(N):
        r = Fl[n] - rho[n] * u0l + psi[n] * phil - K(u0l if n == 0 else U[n - 1]) / 2
        for j in range(n):
            r = r - a[n - j] * U[j]
        x = np.zeros(M, dtype=np.longdouble)
        pv = np.longdouble(0)
        for i in range(M):
            x[i] = (r[i] + he * pv) * inv[i]
            pv = x[i]
        for i in range(M - 2, -1, -1):
            x[i] -= cp[i] * x[i + 1]
        U[n] = x
    return U


_lib_lock = __import__("threading").Lock()
_lib = None


def ext_mode_lib():
    """Build (gcc, into _build/) and load tests/ext_mode.c: ext_mode and
    ext_mode_cn, the long double single-mode recurrences (once per process;
    safe to call from several threads)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            _lib = _build_ext_mode()
        return _lib


def _build_ext_mode():
    here = os.path.dirname(os.path.abspath(__file__))
    out = os.path.join(os.path.dirname(here), "_build", "libext_mode.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    src = os.path.join(here, "ext_mode.c")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    lib = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("ext_mode", "ext_mode_cn"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_double, dp,
                       ctypes.c_double, ctypes.c_double, dp]
    lib.ext_mode_residual.restype = ctypes.c_int
    lib.ext_mode_residual.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_double, dp, ctypes.c_double,
                                      ctypes.c_double, dp, ctypes.c_int, dp, dp]
    lib.ext_mode_given.restype = ctypes.c_int
    lib.ext_mode_given.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_double, dp, ctypes.c_double,
                                   ctypes.c_double, dp, ctypes.c_int]
    return lib


def mode(gamma, T, N, lam, g, v0=0.0, phihat=0.0, cn=False):
    """Long double single-mode recurrence (ext_mode.c), returned as float64."""
    lib = ext_mode_lib()
    dp = ctypes.POINTER(ctypes.c_double)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros(N)
    fn = lib.ext_mode_cn if cn else lib.ext_mode
    assert fn(gamma, T, N, lam, g.ctypes.data_as(dp), v0, phihat, out.ctypes.data_as(dp)) == 0
    return out


def mode_given(a, rho, psi, lam, g, v0=0.0, phihat=0.0, cn=False):
    """Long double single-mode recurrence with the float64 weights given
    (ext_mode_given): the exact solution of the system they define."""
    lib = ext_mode_lib()
    dp = ctypes.POINTER(ctypes.c_double)
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, rho, psi, g)]
    N = len(arrs[3])
    assert all(len(x) >= N for x in arrs[:3])
    out = np.zeros(N)
    assert lib.ext_mode_given(N, *(x.ctypes.data_as(dp) for x in arrs[:3]), lam, arrs[3].ctypes.data_as(dp), v0,
                              phihat, out.ctypes.data_as(dp), 1 if cn else 0) == 0
    return out


def mode_residual(a, rho, psi, lam, g, v, v0=0.0, phihat=0.0, cn=False):
    """(r, scale): the long double residual of the single-mode solution v of
    the system the float64 weights define, and per step the sum of the
    absolute values of its terms (ext_mode_residual)."""
    lib = ext_mode_lib()
    dp = ctypes.POINTER(ctypes.c_double)
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, rho, psi, g, v)]
    N = len(arrs[3])
    assert len(arrs[4]) == N and all(len(x) >= N for x in arrs[:3])
    r, sc = np.zeros(N), np.zeros(N)
    rc = lib.ext_mode_residual(N, arrs[0].ctypes.data_as(dp), arrs[1].ctypes.data_as(dp), arrs[2].ctypes.data_as(dp),
                               lam, arrs[3].ctypes.data_as(dp), v0, phihat, arrs[4].ctypes.data_as(dp),
                               1 if cn else 0, r.ctypes.data_as(dp), sc.ctypes.data_as(dp))
    assert rc == 0
    return r, sc


def modal_backward(weights_given, M, N, series, v_by_mode, cn=False, x0=0.0, x1=1.0):
    """Normwise backward error of a sum-of-sine-modes solution, from its modal
    coefficients v_by_mode[j] (the field's projections): the residual of each
    mode's scalar system, combined as max_n sum_j |r_j^n| / max_n sum_j
    scale_j^n (|sin| <= 1 bounds the field's residual by the sum)."""
    a, rho, psi = (weights_given["a"], weights_given["rho"], weights_given["psi"]) \
        if isinstance(weights_given, dict) else weights_given
    h = (x1 - x0) / (M + 1)
    rsum, ssum = np.zeros(N), np.zeros(N)
    for j, (g, v0, ph) in series.items():
        lam = 4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2
        r, sc = mode_residual(a, rho, psi, lam, g, np.asarray(v_by_mode[j], dtype=np.float64), v0, ph, cn)
        rsum += np.abs(r)
        ssum += sc
    return float(np.max(rsum) / np.max(ssum))


def modal_coefficients(u, js, chunk=2048):
    """Sine coefficients of a field u [N][M] (float64 array, or a torch tensor
    on any device) for the modes js, in long double:
    v_j = 2/(M+1) sum_i u_i sin(j pi i/(M+1)) (discrete orthogonality of the
    sine basis on the grid); rows are converted in chunks."""
    N, M = u.shape
    i = np.arange(1, M + 1, dtype=np.longdouble)
    pi = np.longdouble("3.14159265358979323846264338327950288")
    S = np.stack([np.sin(np.longdouble(j) * pi * i / np.longdouble(M + 1)) for j in js], axis=1)
    out = np.zeros((N, len(js)), dtype=np.longdouble)
    for r0 in range(0, N, chunk):
        blk = u[r0:r0 + chunk]
        blk = blk.cpu().numpy() if hasattr(blk, "cpu") else np.asarray(blk)
        out[r0:r0 + chunk] = np.asarray(blk, dtype=np.longdouble) @ S
    out *= 2 / np.longdouble(M + 1)
    return [out[:, k] for k in range(len(js))]


def backward(weights_given, M, N, F, U, u0=None, phi=None, kind="diffusion", x0=0.0, x1=1.0):
    """Normwise backward error of a float64 solution U [N][M] of the block
    system (kind "diffusion" or "cn") with the float64 weights given, in long
    double: max over (n, i) of |r| divided by the max over (n, i) of the sum
    of the absolute values of the terms of r (a bound of ||A|| ||U|| + ||b||
    row by row; a per-entry ratio would weigh entries whose terms nearly
    vanish)."""
    a, rho, psi = given_weights(weights_given, N)
    h = (np.longdouble(x1) - np.longdouble(x0)) / np.longdouble(M + 1)
    e = 1 / (h * h)
    Ul = np.asarray(U, dtype=np.longdouble)
    Fl = np.asarray(F, dtype=np.longdouble)
    u0l = np.zeros(M, dtype=np.longdouble) if u0 is None else np.asarray(u0, dtype=np.longdouble)
    phil = np.zeros(M, dtype=np.longdouble) if phi is None else np.asarray(phi, dtype=np.longdouble)
    cf = np.longdouble(0.5) if kind == "cn" else np.longdouble(1)

    def Kabs(v):  # |e| (2|v_i| + |v_{i-1}| + |v_{i+1}|) and K v
        z = np.zeros(1, dtype=np.longdouble)
        left, right = np.concatenate((z, v[:-1])), np.concatenate((v[1:], z))
        return e * (2 * v - left - right), e * (2 * np.abs(v) + np.abs(left) + np.abs(right))

    rmax, smax = 0.0, 0.0
    for n in range(N):
        kv, ka = Kabs(Ul[n])
        r = Fl[n] - rho[n] * u0l + psi[n] * phil - a[0] * Ul[n] - cf * kv
        sc = np.abs(Fl[n]) + np.abs(rho[n] * u0l) + np.abs(psi[n] * phil) + np.abs(a[0] * Ul[n]) + cf * ka
        if n:
            hist = a[n:0:-1][:, None] * Ul[:n]
            r -= hist.sum(axis=0)
            sc += np.abs(hist).sum(axis=0)
        if kind == "cn":
            kp, kpa = Kabs(u0l if n == 0 else Ul[n - 1])
            r -= cf * kp
            sc += cf * kpa
        rmax = max(rmax, float(np.max(np.abs(r))))
        smax = max(smax, float(np.max(sc)))
    return rmax / smax if smax > 0 else 0.0


def backward_adv(weights_given, gamma, M, N, F, U, u0=None, phi=None, x0=0.0, x1=1.0):
    """Normwise backward error (as backward()) of a float64 solution U of the
    advection schemes (Scheme 2 for gamma < 1 in its twice-scaled row form,
    Scheme 3 for gamma > 1; inflow value 0) with the float64 weights given,
    in long double (the rows solve_adv steps through)."""
    a, rho, psi = given_weights(weights_given, N)
    h = (np.longdouble(x1) - np.longdouble(x0)) / np.longdouble(M + 1)
    Ul = np.asarray(U, dtype=np.longdouble)
    Fl = np.asarray(F, dtype=np.longdouble)
    u0l = np.zeros(M, dtype=np.longdouble) if u0 is None else np.asarray(u0, dtype=np.longdouble)
    phil = np.zeros(M, dtype=np.longdouble) if (phi is None or gamma < 1) else np.asarray(phi, dtype=np.longdouble)

    def shift(v):  # v_{i-1}, with 0 at the inflow
        return np.concatenate(([np.longdouble(0)], v[:-1]))

    rmax, smax = 0.0, 0.0
    for n in range(N):
        if gamma < 1:
            terms = [2 * Fl[n], -rho[n] * (u0l + shift(u0l)), -(a[0] + 2 / h) * Ul[n], -(a[0] - 2 / h) * shift(Ul[n])]
            hist = a[n:0:-1][:, None] * (Ul[:n] + np.concatenate((np.zeros((n, 1), dtype=np.longdouble),
                                                                  Ul[:n, :-1]), axis=1)) if n else None
        else:
            terms = [Fl[n], -rho[n] * u0l, psi[n] * phil, -(a[0] + 1 / h) * Ul[n], (1 / h) * shift(Ul[n])]
            hist = a[n:0:-1][:, None] * Ul[:n] if n else None
        r = sum(terms)
        sc = sum(np.abs(t) for t in terms)
        if hist is not None:
            r = r - hist.sum(axis=0)
            sc = sc + np.abs(hist).sum(axis=0)
        rmax = max(rmax, float(np.max(np.abs(r))))
        smax = max(smax, float(np.max(sc)))
    return rmax / smax if smax > 0 else 0.0


EPS = 2.0 ** -52
FLOOR_FORWARD_MAX = 1e-8   # forward error allowed in the floor regime (both sides)
BACKWARD_ULPS = 8          # backward error allowed there, in units of float64 roundoff


def assert_floor_parity(e, e_gpu, e_orc, eta_gpu, eta_orc, tol):
    """Parity where the float64 oracle itself misses tol against the exact
    discrete solution.  e is the GPU's distance to the oracle; e_gpu, e_orc
    the GPU's and the oracle's distances to the extended-precision solve;
    eta_gpu, eta_orc their normwise backward errors (long double residuals of
    the systems their own float64 weights define).  Required: the extended
    solve agrees with the oracle (e_orc <= 1e-8: the reference is not in
    doubt) and both forward errors stay <= 1e-8; and the GPU is at least as
    close to the exact solution as the oracle up to a factor 2
    (e_gpu <= max(tol, 2 e_orc)) or, where the problem is so ill-conditioned
    that ulp-level rounding decides which of two float64 results lands
    closer (the diffusion-wave recurrence with long histories), backward
    stable like the oracle: eta_gpu <= max(BACKWARD_ULPS ulp, 2 eta_orc)."""
    assert e_orc <= FLOOR_ORACLE_MAX, ("oracle too far from the extended solve", e, e_gpu, e_orc)
    assert e_gpu <= FLOOR_FORWARD_MAX, ("forward error", e, e_gpu, e_orc)
    forward_ok = e_gpu <= max(tol, 2.0 * e_orc)
    backward_ok = eta_gpu <= max(BACKWARD_ULPS * EPS, 2.0 * eta_orc)
    assert forward_ok or backward_ok, ("forward and backward error", e_gpu, e_orc, eta_gpu / EPS, eta_orc / EPS)
