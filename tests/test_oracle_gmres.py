"""Pins for the oracle's restarted GMRES(m) (the iterative method of section
3.1: Arnoldi with modified Gram-Schmidt, least squares on the Hessenberg
matrix, restarts).

Each test checks something GMRES itself fixes, against a dense system
assembled independently from its definition:
* finite termination: with m >= M N the Krylov space is the whole space, so
  the iterate is the dense solve;
* the least-squares residual after step k is the residual of the k-th
  iterate (recomputed from the dense matrix), so a wrong rotation or a
  dropped Hessenberg entry shows;
* one step of GMRES(1) is the minimal-residual step along r_0, in closed form;
* with the block-diagonal preconditioner A P^-1 - I is nilpotent of index N,
  so GMRES ends in at most N steps, and in one when N = 1;
* the residual norms never increase, and the converged iterate agrees with
  the direct time stepping to the accuracy rtol allows.
"""
import numpy as np
import pytest

from tests.test_oracle_solve import dense_system

X0, X1, T = 0.0, 1.0, 1.0


def problem(gamma, M, N, seed=3):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((N, M))
    u0 = rng.standard_normal(M)
    phi = rng.standard_normal(M) if gamma > 1 else None
    A, rho, psi = dense_system(gamma, M, N)
    b = F - np.outer(rho, u0) + (np.outer(psi, phi) if phi is not None else 0.0)
    return F, u0, phi, A, b.ravel()


@pytest.mark.parametrize("gamma", [0.3, 1.5])
@pytest.mark.parametrize("precond", [0, 1])
def test_finite_termination_is_the_dense_solve(orc, gamma, precond):
    M, N = 3, 5
    F, u0, phi, A, b = problem(gamma, M, N)
    u, info = orc.gmres(gamma, T, X0, X1, M, N, F, u0, phi, restart=M * N, maxit=M * N, rtol=1e-14,
                        precond=precond)
    ref = np.linalg.solve(A, b)
    assert info["iters"] <= M * N and info["cycles"] == 1
    assert np.max(np.abs(u.ravel() - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("gamma,precond", [(0.6, 0), (1.4, 0), (0.6, 1)])
def test_least_squares_residual_is_the_iterate_residual(orc, gamma, precond):
    M, N = 4, 6
    F, u0, phi, A, b = problem(gamma, M, N, seed=5)
    full = orc.gmres(gamma, T, X0, X1, M, N, F, u0, phi, restart=24, maxit=12, rtol=0.0, precond=precond)[1]
    bn = np.linalg.norm(b)
    assert abs(full["hist"][0] - 1.0) < 1e-15
    for k in (1, 2, 3, 5, 8, 12):
        uk, ik = orc.gmres(gamma, T, X0, X1, M, N, F, u0, phi, restart=24, maxit=k, rtol=0.0, precond=precond)
        assert ik["iters"] == k
        true = np.linalg.norm(b - A @ uk.ravel()) / bn
        # relative agreement, down to the rounding floor of the residual
        assert abs(full["hist"][k] - true) <= 1e-10 * true + 1e-14, (k, full["hist"][k], true)
        assert abs(ik["relres"] - true) <= 1e-12 * true + 1e-15


def test_gmres1_step_is_the_minimal_residual_step(orc):
    M, N = 5, 7
    F, u0, phi, A, b = problem(0.4, M, N, seed=9)
    u, info = orc.gmres(0.4, T, X0, X1, M, N, F, u0, phi, restart=1, maxit=1, rtol=0.0)
    Ar = A @ b  # r_0 = b from a zero start
    alpha = (Ar @ b) / (Ar @ Ar)
    assert info["iters"] == 1 and info["cycles"] == 1
    assert np.max(np.abs(u.ravel() - alpha * b)) <= 1e-13 * np.max(np.abs(alpha * b))


def test_preconditioned_single_step_is_exact(orc):
    M, N = 9, 1
    F, u0, phi, A, b = problem(0.5, M, N)
    u, info = orc.gmres(0.5, T, X0, X1, M, N, F, u0, phi, restart=5, maxit=5, rtol=1e-14, precond=1)
    assert info["iters"] == 1 and info["converged"]
    assert np.max(np.abs(u.ravel() - np.linalg.solve(A, b))) <= 1e-13 * np.max(np.abs(u))


@pytest.mark.parametrize("gamma", [0.2, 1.7])
def test_preconditioned_ends_within_n_steps(orc, gamma):
    M, N = 8, 6
    F, u0, phi, A, b = problem(gamma, M, N)
    u, info = orc.gmres(gamma, T, X0, X1, M, N, F, u0, phi, restart=N, maxit=N, rtol=1e-13, precond=1)
    assert info["iters"] <= N and info["converged"], info
    assert np.max(np.abs(u.ravel() - np.linalg.solve(A, b))) <= 1e-11 * np.max(np.abs(u))


@pytest.mark.parametrize("restart", [3, 10])
def test_residuals_never_increase_across_restarts(orc, restart):
    M, N = 7, 8
    F, u0, phi, A, b = problem(0.7, M, N, seed=11)
    u, info = orc.gmres(0.7, T, X0, X1, M, N, F, u0, phi, restart=restart, maxit=60, rtol=1e-12)
    h = info["hist"]
    assert np.all(np.diff(h) <= 1e-12 * h[:-1] + 1e-300)
    assert info["cycles"] == -(-info["iters"] // restart) or info["converged"]


@pytest.mark.parametrize("gamma,precond", [(0.1, 0), (0.1, 1), (1.5, 1)])
def test_converged_iterate_matches_the_direct_solve(orc, gamma, precond):
    # h = tau = 1/32: the smallest mesh of the paper's timing table for Scheme 4
    M, N = 31, 32
    rng = np.random.default_rng(21)
    F = rng.standard_normal((N, M))
    u0 = rng.standard_normal(M)
    phi = rng.standard_normal(M) if gamma > 1 else None
    ref = orc.solve(gamma, T, X0, X1, M, N, F, u0=u0, phi=phi)
    u, info = orc.gmres(gamma, T, X0, X1, M, N, F, u0, phi, restart=40, maxit=4000, rtol=1e-12, precond=precond)
    assert info["converged"] and info["relres"] <= 1e-12
    # forward error <= cond(A) * relres; cond(A) < 1e4 at this mesh
    assert np.max(np.abs(u - ref)) <= 1e-7 * np.max(np.abs(ref))


def test_exact_guess_takes_no_step_and_zero_rhs_gives_zero(orc):
    M, N = 6, 5
    F, u0, phi, A, b = problem(0.5, M, N)
    ref = np.linalg.solve(A, b).reshape(N, M)
    u, info = orc.gmres(0.5, T, X0, X1, M, N, F, u0, phi, restart=5, maxit=50, rtol=1e-8, guess=ref)
    assert info["iters"] == 0 and info["converged"] and np.array_equal(u, ref)
    z, iz = orc.gmres(0.5, T, X0, X1, M, N, np.zeros((N, M)), restart=5, maxit=50, rtol=1e-8,
                      guess=np.ones((N, M)))
    assert iz["iters"] == 0 and iz["converged"] and not z.any()


def test_stops_at_maxit_without_convergence(orc):
    M, N = 31, 16
    F, u0, phi, A, b = problem(0.5, M, N)
    u, info = orc.gmres(0.5, T, X0, X1, M, N, F, u0, phi, restart=4, maxit=9, rtol=1e-14)
    assert info["iters"] == 9 and info["cycles"] == 3 and not info["converged"]
    true = np.linalg.norm(b - A @ u.ravel()) / np.linalg.norm(b)
    assert abs(info["relres"] - true) <= 1e-12
