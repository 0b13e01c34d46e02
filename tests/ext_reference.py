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


def solve(gamma, M, N, F, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0):
    a, rho, psi = weights(gamma, N, T)
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


def solve_adv(gamma, M, N, F, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0):
    """The advection time stepping of the oracle (Scheme 2 for gamma < 1,
    Scheme 3 for gamma > 1; inflow value 0) in extended precision."""
    a, rho, psi = weights(gamma, N, T)
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


def solve_cn(gamma, M, N, F, u0=None, phi=None, T=1.0, x0=0.0, x1=1.0):
    """The oracle's stepping of the diffusion-wave variant with the spatial
    term averaged over t_n and t_{n-1}, in extended precision."""
    a, rho, psi = weights(gamma, N, T)
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


def ext_mode_lib():
    """Build (gcc, into _build/) and load tests/ext_mode.c: ext_mode and
    ext_mode_cn, the long double single-mode recurrences."""
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


def assert_within_floor(e, e_gpu, e_orc, tol):
    """Parity where the float64 oracle misses tol: e is the GPU's distance to
    the oracle, e_gpu and e_orc the GPU's and the oracle's distances to the
    extended-precision solve.  The oracle must be close to that solve
    (e_orc <= FLOOR_ORACLE_MAX: the reference is then not in doubt), and the
    GPU at most twice as far from it as the oracle."""
    assert e_orc <= FLOOR_ORACLE_MAX, ("oracle too far from the extended solve", e, e_gpu, e_orc)
    assert e_gpu <= max(tol, 2.0 * e_orc), (e, e_gpu, e_orc)
