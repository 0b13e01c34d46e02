"""Pins for the oracle's adjoint (transpose of the block lower-triangular
Toeplitz system of eq. e20/e21 solved backward in time) and dL/dgamma.

Pinned by the dot-product identity <A^-T g, R> = <g, A^-1 R>, by central
differences in f (exact for the quadratic loss up to round-off) and by
central / Richardson differences in gamma with f, u0, phi held fixed.
"""
import numpy as np
import pytest

from paper_1710_11593_amd import workloads as wl


@pytest.mark.parametrize("gamma", [0.3, 0.7, 1.2, 1.8])
def test_dot_identity(orc, gamma):
    M, N = 24, 40
    rng = np.random.default_rng(3)
    R = rng.standard_normal((N, M))
    g = rng.standard_normal((N, M))
    U = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, R)
    lam, _ = orc.adjoint(gamma, 1.0, 0.0, 1.0, M, N, g, U)
    lhs, rhs = np.vdot(lam, R), np.vdot(g, U)
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.vdot(lam, lam) * np.vdot(R, R))
    # A^T lam = g: time reversal maps the transpose onto the lower-triangular
    # operator, which oracle.apply evaluates (pinned by the dense brute force)
    AtL = orc.apply(gamma, 1.0, 0.0, 1.0, M, N, lam[::-1].copy())[::-1]
    assert np.max(np.abs(AtL - g)) <= 1e-11 * np.max(np.abs(g))


def loss(orc, gamma, M, N, f, u0, phi, Uobs):
    U = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    return float(np.sum((U - Uobs) ** 2)), U


@pytest.mark.parametrize("gamma", [0.6, 1.4])
def test_dLdf_central_differences(orc, gamma):
    M, N = 20, 32
    rng = np.random.default_rng(11)
    f = rng.standard_normal((N, M))
    u0 = rng.standard_normal(M)
    phi = rng.standard_normal(M)
    Uobs = rng.standard_normal((N, M))
    L0, U = loss(orc, gamma, M, N, f, u0, phi, Uobs)
    lam, _ = orc.adjoint(gamma, 1.0, 0.0, 1.0, M, N, 2 * (U - Uobs), U, u0, phi)
    eps = 1e-3
    for _ in range(8):
        v = rng.standard_normal((N, M))
        fd = (loss(orc, gamma, M, N, f + eps * v, u0, phi, Uobs)[0]
              - loss(orc, gamma, M, N, f - eps * v, u0, phi, Uobs)[0]) / (2 * eps)
        assert abs(fd - np.vdot(lam, v)) <= 1e-9 * max(1.0, abs(fd))
    for _ in range(16):
        n, i = rng.integers(N), rng.integers(M)
        v = np.zeros((N, M))
        v[n, i] = 1.0
        fd = (loss(orc, gamma, M, N, f + eps * v, u0, phi, Uobs)[0]
              - loss(orc, gamma, M, N, f - eps * v, u0, phi, Uobs)[0]) / (2 * eps)
        assert abs(fd - lam[n, i]) <= 1e-9 * max(1.0, abs(fd))


@pytest.mark.parametrize("gamma", [0.25, 0.6, 0.95, 1.05, 1.5, 1.9])
def test_dLdgamma_differences(orc, gamma):
    M, N = 16, 48
    rng = np.random.default_rng(5)
    ts = wl.sample_times(gamma, N)
    x, _, _, _ = wl.grid(M, N)
    f = np.outer(ts ** 1.3, np.sin(np.pi * x)) + 0.2 * rng.standard_normal((N, M))
    u0 = np.sin(2 * np.pi * x)
    phi = np.cos(np.pi * x) if gamma > 1 else None
    Uobs = 0.5 * rng.standard_normal((N, M))
    L0, U = loss(orc, gamma, M, N, f, u0, phi, Uobs)
    _, dg = orc.adjoint(gamma, 1.0, 0.0, 1.0, M, N, 2 * (U - Uobs), U, u0, phi)

    def Lg(gg):
        return loss(orc, gg, M, N, f, u0, phi, Uobs)[0]

    d = 1e-3
    rich = (8 * (Lg(gamma + d) - Lg(gamma - d)) - (Lg(gamma + 2 * d) - Lg(gamma - 2 * d))) / (12 * d)
    assert abs(rich - dg) <= 1e-8 * abs(dg), (rich, dg)
    d = 1e-6
    cen = (Lg(gamma + d) - Lg(gamma - d)) / (2 * d)
    assert abs(cen - dg) <= 1e-5 * abs(dg), (cen, dg)
