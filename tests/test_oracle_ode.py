"""Pins for the oracle's Scheme 1 (the two-sided fractional ODE, eq. e7):
its symmetric Toeplitz column and its conjugate gradients (section 2.2).

* the column satisfies, row by row, the identity the paper derives in the
  proof of Theorem 1: A_ii - sum_{j != i} |A_ij| = 1 + mu G_{i-1} + mu G_{N-i-1};
* a Toeplitz solve with that column reproduces Table 1 to the printed digits
  (with the forcing recomputed from the exact solution, the printed one
  being garbled);
* CG ends at the Toeplitz solve within n steps, its recurrence residuals
  equal the recomputed ones, and the A-norm of its error decreases.
"""
import math
import os

import numpy as np
import pytest
from scipy.linalg import solve_toeplitz, toeplitz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def left_caputo_t1mt(s, g):
    return s ** (1 - g) / math.gamma(2 - g) - 2 * s ** (2 - g) / math.gamma(3 - g)


def forcing(gamma, N):
    t = np.arange(1, N) / N
    return t, left_caputo_t1mt(t, gamma) + left_caputo_t1mt(1 - t, gamma) + t * (1 - t)


@pytest.mark.parametrize("gamma", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("N", [3, 8, 33])
def test_theorem1_row_identity(orc, gamma, N):
    c = orc.ode_column(gamma, N)
    n = N - 1
    A = toeplitz(c)
    assert np.array_equal(A, A.T)
    w = orc.weights(gamma, 1.0, N)
    mu, G = w["coef"], w["b"]
    for i in range(1, n + 1):
        lhs = A[i - 1, i - 1] - (np.sum(np.abs(A[i - 1])) - abs(A[i - 1, i - 1]))
        rhs = 1.0 + mu * G[i - 1] + mu * G[N - i - 1]
        assert abs(lhs - rhs) <= 1e-12 * rhs, (i, lhs, rhs)
    assert np.all(np.linalg.eigvalsh(A) > 0)


def read_table():
    rows = []
    for line in open(os.path.join(GOLDEN, "table1.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            g, k, p = line.split()
            rows.append((float(g), int(k), p))
    return rows


@pytest.mark.parametrize("row", read_table(), ids=lambda r: "g%.1f-k%d" % (r[0], r[1]))
def test_table1(orc, row):
    gamma, k, printed = row
    N = 2 ** k
    t, f = forcing(gamma, N)
    u = solve_toeplitz(orc.ode_column(gamma, N), f)
    err = math.sqrt(np.sum((u - t * (1 - t)) ** 2) / N)
    target = float(printed)
    e = math.floor(math.log10(target))
    assert abs(err - target) <= 1.0001 * 10 ** (e - 4), (err, printed)


@pytest.mark.parametrize("gamma", [0.2, 0.8])
def test_cg_finite_termination_and_residuals(orc, gamma):
    N = 24
    t, f = forcing(gamma, N)
    c = orc.ode_column(gamma, N)
    A = toeplitz(c)
    ref = solve_toeplitz(c, f)
    u, info = orc.ode_cg(gamma, N, f, maxit=N - 1, rtol=1e-14)
    assert info["iters"] <= N - 1
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))
    # recurrence residuals equal recomputed ones (early steps, before rounding shows)
    for k in (1, 2, 4, 6):
        uk, ik = orc.ode_cg(gamma, N, f, maxit=k, rtol=0.0)
        true = np.linalg.norm(f - A @ uk) / np.linalg.norm(f)
        assert abs(info["hist"][k] - true) <= 1e-9 * true, (k, info["hist"][k], true)


def test_cg_error_decreases_in_the_energy_norm(orc):
    gamma, N = 0.6, 64
    t, f = forcing(gamma, N)
    c = orc.ode_column(gamma, N)
    A = toeplitz(c)
    ref = solve_toeplitz(c, f)
    prev = np.inf
    for k in range(1, 15):
        uk, _ = orc.ode_cg(gamma, N, f, maxit=k, rtol=0.0)
        e = uk - ref
        en = math.sqrt(e @ A @ e)
        assert en < prev
        prev = en


def test_cg_converges_to_the_toeplitz_solve(orc):
    gamma, N = 0.7, 512
    t, f = forcing(gamma, N)
    ref = solve_toeplitz(orc.ode_column(gamma, N), f)
    u, info = orc.ode_cg(gamma, N, f, maxit=5000, rtol=1e-12)
    assert info["converged"] and info["relres"] <= 1e-12
    assert np.max(np.abs(u - ref)) <= 1e-9 * np.max(np.abs(ref))
