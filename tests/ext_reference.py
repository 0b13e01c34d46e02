"""Extended-precision reference for the parity tests (test infrastructure).

The same forward time stepping as the oracle (Scheme 4 / eq. e15-e17 time
weights, one Thomas solve per step) carried out in x87 extended precision
(numpy.longdouble, 64-bit significand), with the weights evaluated in 40-digit
decimal.  It measures how far the float64 oracle itself is from the exact
discrete solution on inputs where float64 rounding is amplified (rough random
sources at large M or gamma near 2), so that a float64 GPU result can be
required to be at least as accurate as the float64 oracle there.
"""
import math
from decimal import Decimal, getcontext

import numpy as np


def weights(gamma, N, T=1.0):
    getcontext().prec = 40
    p = (1 - gamma) if gamma < 1 else (2 - gamma)
    tau = Decimal(repr(T)) / Decimal(N)
    g = Decimal(repr(gamma))
    garg = (2 - gamma) if gamma < 1 else (3 - gamma)
    coef = (tau.ln() * (-g)).exp() / Decimal(repr(math.gamma(garg)))
    pd = Decimal(repr(p))

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
