"""Pins of the extended-precision references (tests/ext_reference.py and
tests/ext_mode.c) that arbitrate the GPU parity tests where the float64
oracle's own rounding exceeds the 1e-11 bar.

Each reference must (1) solve the same system as the oracle: agreement with
the oracle on benign inputs, where float64 rounding is small; and (2) be more
accurate than float64: agreement with a 40-digit decimal solve far below
float64's unit roundoff, including on inputs where the float64 oracle is
measurably off.  The decimal solves are brute force (Gaussian elimination of
the whole assembled block system, or the scalar lower-triangular Toeplitz
system of one sine mode) with the weights and constants of section 3 written
out from their definitions.
"""
import math
from decimal import Decimal, getcontext, localcontext

import numpy as np
import pytest

from tests import ext_reference as ext

PREC = 40


# ---------------------------------------------------------------- decimal side

def dec_weights(gamma, N, T=1.0):
    """a_m (m < N), rho_n, psi_n (n = 1..N) from their definitions (section 3:
    G_k for 0<gamma<1, M_k and the second difference for 1<gamma<2)."""
    g = Decimal(float(gamma))   # the exact binary value of the float64 order
    tau = Decimal(float(T)) / N
    wave = gamma > 1
    p = (2 - g) if wave else (1 - g)
    coef = (-g * tau.ln()).exp() / ext.dec_gamma((3 - g) if wave else (2 - g))

    def b(k):
        if k < 0:
            return Decimal(0)
        return (p * Decimal(k + 1).ln()).exp() - (Decimal(0) if k == 0 else (p * Decimal(k).ln()).exp())

    if not wave:
        a = [coef * (b(m) - b(m - 1)) for m in range(N)]
        rho = [-coef * b(n - 1) for n in range(1, N + 1)]
        psi = [Decimal(0)] * N
    else:
        a = [coef * (b(m - 2) - 2 * b(m - 1) + b(m)) for m in range(N)]
        rho = [coef * (b(n - 2) - b(n - 1)) for n in range(1, N + 1)]
        psi = [coef * tau * b(n - 1) for n in range(1, N + 1)]
    return a, rho, psi


def dec_gauss(A, r):
    """Gaussian elimination with partial pivoting on lists of Decimals."""
    n = len(r)
    A = [row[:] for row in A]
    r = r[:]
    for k in range(n):
        piv = max(range(k, n), key=lambda i: abs(A[i][k]))
        A[k], A[piv] = A[piv], A[k]
        r[k], r[piv] = r[piv], r[k]
        for i in range(k + 1, n):
            if A[i][k] == 0:
                continue
            m = A[i][k] / A[k][k]
            for j in range(k, n):
                A[i][j] -= m * A[k][j]
            r[i] -= m * r[k]
    x = [Decimal(0)] * n
    for i in range(n - 1, -1, -1):
        s = r[i] - sum(A[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / A[i][i]
    return x


def dec_block_solve(kind, gamma, M, N, F, u0, phi):
    """Assemble the MN x MN block system of the given kind from the component
    equations and solve it in decimal.  kind: "diffusion" (diagonal block
    a_0 I + K), "cn" (a_0 I + K/2, lag-1 block a_1 I + K/2, step 1 carries
    -(K/2) u0), "adv" (Scheme 2 for gamma<1: blocks a_m B with B the average
    of x_i and x_{i-1}, difference (U_i - U_{i-1})/h on the diagonal;
    Scheme 3 for gamma>1: B = I)."""
    with localcontext() as ctx:
        ctx.prec = PREC
        a, rho, psi = dec_weights(gamma, N)
        h = Decimal(1) / (M + 1)
        e = 1 / (h * h)
        D = lambda v: Decimal(float(v))  # noqa: E731 (exact float64 -> decimal)
        Z = Decimal(0)

        def K(i, j):
            return 2 * e if i == j else (-e if abs(i - j) == 1 else Z)

        def B(i, j):
            if kind != "adv" or gamma > 1:
                return Decimal(1) if i == j else Z
            return Decimal("0.5") if (i == j or i == j + 1) else Z

        def Dx(i, j):
            return (1 / h) if i == j else ((-1 / h) if i == j + 1 else Z)

        n_all = M * N
        A = [[Z] * n_all for _ in range(n_all)]
        r = [Z] * n_all
        for n in range(N):
            for i in range(M):
                row = n * M + i
                for jt in range(n + 1):
                    for k in range(M):
                        v = a[n - jt] * B(i, k)
                        if kind == "diffusion" and jt == n:
                            v += K(i, k)
                        if kind == "cn" and jt >= n - 1:
                            v += K(i, k) / 2
                        if kind == "adv" and jt == n:
                            v += Dx(i, k)
                        A[row][jt * M + k] = v
                s = D(F[n][i]) - rho[n] * sum(B(i, k) * D(u0[k]) for k in range(M))
                if gamma > 1 and phi is not None:
                    s += psi[n] * D(phi[i])
                if kind == "cn" and n == 0:
                    s -= sum(K(i, k) * D(u0[k]) for k in range(M)) / 2
                r[row] = s
        x = dec_gauss(A, r)
        return [[x[n * M + i] for i in range(M)] for n in range(N)]


def dec_mode(gamma, N, lam, g, v0, phihat, cn=False):
    """Scalar recurrence of one sine mode, in decimal:
    (a_0 + lam) v^n = g^n - rho_n v0 + psi_n phihat - sum_{j<n} a_{n-j} v^j
    (cn: lam/2 on v^n and on v^{n-1})."""
    with localcontext() as ctx:
        ctx.prec = PREC
        a, rho, psi = dec_weights(gamma, N)
        L = Decimal(float(lam))
        d0 = a[0] + (L / 2 if cn else L)
        v = []
        V0 = Decimal(float(v0))
        for n in range(N):
            s = Decimal(float(g[n])) - rho[n] * V0 + psi[n] * Decimal(float(phihat))
            for j in range(n):
                s -= a[n - j] * v[j]
            if cn:
                s -= L / 2 * (V0 if n == 0 else v[n - 1])
            v.append(s / d0)
        return v


def dec_relerr(x, ref):
    """max |x - ref| / max |ref| with ref in decimal (x float64 or long double)."""
    with localcontext() as ctx:
        ctx.prec = PREC
        flat_r = [v for row in ref for v in row] if isinstance(ref[0], list) else list(ref)
        xs = np.asarray(x, dtype=np.longdouble).ravel()
        # a long double is the exact sum of two float64 values
        num = max(abs(Decimal(float(xv)) + Decimal(float(xv - np.longdouble(float(xv)))) - rv)
                  for xv, rv in zip(xs, flat_r))
        den = max(abs(rv) for rv in flat_r)
        return float(num / den)


def orc_mode(gamma, N, lam, g, v0, ph, cn):
    import oracle

    return (oracle.mode_cn if cn else oracle.mode)(gamma, 1.0, N, lam, g, v0, ph)


def rough_case(gamma, M, N, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((N, M))
    u0 = rng.standard_normal(M)
    phi = rng.standard_normal(M) if gamma > 1 else None
    return F, u0, phi


def relerr(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


# ---------------------------------------------------------------- Gamma

def test_dec_gamma_closed_forms():
    with localcontext() as ctx:
        ctx.prec = PREC
        pi = ext.dec_pi()
        assert abs(pi - Decimal(math.pi)) < Decimal("1e-15")
        assert abs(ext.dec_gamma(Decimal("0.5")) ** 2 - pi) < Decimal("1e-35")      # Gamma(1/2) = sqrt(pi)
        assert abs(ext.dec_gamma(Decimal("1.5")) * 2 - pi.sqrt()) < Decimal("1e-35")
        assert abs(ext.dec_gamma(Decimal(1)) - 1) < Decimal("1e-35")
        assert abs(ext.dec_gamma(Decimal(3)) - 2) < Decimal("1e-35")
        for x in ("0.3", "1.1", "1.7", "2.45"):
            X = Decimal(x)
            assert abs(ext.dec_gamma(X + 1) - X * ext.dec_gamma(X)) < Decimal("1e-34")   # recursion
            assert abs(float(ext.dec_gamma(X)) / math.gamma(float(x)) - 1) <= 4e-16


# ---------------------------------------------------------------- same system as the oracle

@pytest.mark.parametrize("gamma", [0.3, 0.8, 1.2, 1.7])
def test_solve_matches_oracle(orc, gamma):
    M, N = 24, 96
    x = np.arange(1, M + 1) / (M + 1)
    t = np.arange(1, N + 1) / N
    F = np.outer(1 + t ** 2, np.sin(np.pi * x))
    u0 = np.sin(np.pi * x)
    phi = np.sin(2 * np.pi * x) if gamma > 1 else None
    U = ext.solve(gamma, M, N, F, u0, phi)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi)
    assert relerr(U, ref) <= 1e-13


@pytest.mark.parametrize("gamma", [0.4, 1.5])
def test_solve_adv_matches_oracle(orc, gamma):
    M, N = 20, 80
    x = np.arange(1, M + 1) / (M + 1)
    t = np.arange(1, N + 1) / N
    F = np.outer(1 + t, x)
    u0 = x.copy()
    phi = x ** 2 if gamma > 1 else None
    U = ext.solve_adv(gamma, M, N, F, u0, phi)
    ref = orc.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi)
    assert relerr(U, ref) <= 1e-13


@pytest.mark.parametrize("gamma", [1.3, 1.8])
def test_solve_cn_matches_oracle(orc, gamma):
    M, N = 24, 96
    x = np.arange(1, M + 1) / (M + 1)
    t = np.arange(1, N + 1) / N
    F = np.outer(1 + t ** 2, np.sin(np.pi * x))
    u0 = np.sin(np.pi * x)
    phi = np.sin(3 * np.pi * x)
    U = ext.solve_cn(gamma, M, N, F, u0, phi)
    ref = orc.solve_cn(gamma, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi)
    assert relerr(U, ref) <= 1e-13


@pytest.mark.parametrize("cn", [False, True])
@pytest.mark.parametrize("gamma", [0.35, 1.2, 1.45])
def test_ext_mode_matches_oracle(orc, gamma, cn):
    if cn and gamma < 1:
        pytest.skip("the averaged spatial term is a diffusion-wave variant")
    N, lam = 1024, 123.4
    t = np.arange(1, N + 1) / N
    g = 1 + t ** 1.5
    v = ext.mode(gamma, 1.0, N, lam, g, 0.7, 0.3, cn=cn)
    ref = (orc.mode_cn if cn else orc.mode)(gamma, 1.0, N, lam, g, 0.7, 0.3)
    assert relerr(v, ref) <= 1e-13


# ---------------------------------------------------------------- more accurate than float64

@pytest.mark.parametrize("kind,gamma,M,N", [
    ("diffusion", 0.3, 4, 8), ("diffusion", 1.6, 5, 7), ("diffusion", 1.9, 1, 32),
    ("cn", 1.4, 4, 8), ("adv", 0.6, 4, 8), ("adv", 1.7, 5, 6)])
def test_block_solve_vs_decimal_dense(kind, gamma, M, N):
    F, u0, phi = rough_case(gamma, M, N, seed=M * 100 + N)
    fn = {"diffusion": ext.solve, "cn": ext.solve_cn, "adv": ext.solve_adv}[kind]
    U = fn(gamma, M, N, F, u0, phi)
    ref = dec_block_solve(kind, gamma, M, N, F, u0, phi)
    # long double: unit roundoff 5.4e-20, i.e. 2^-11 of float64's
    assert dec_relerr(U, ref) <= 1e-17


@pytest.mark.parametrize("cn", [False, True])
@pytest.mark.parametrize("gamma,lam", [(0.5, 3.0), (1.5, 50.0), (1.95, 2.0e4)])
def test_ext_mode_vs_decimal(orc, gamma, lam, cn):
    if cn and gamma < 1:
        pytest.skip("the averaged spatial term is a diffusion-wave variant")
    N = 128
    t = (np.arange(1, N + 1) - 0.5) / N
    g = np.sin(7 * t) + t ** 2
    v = ext.mode(gamma, 1.0, N, lam, g, 0.4, -0.2, cn=cn)
    ref = dec_mode(gamma, N, lam, g, 0.4, -0.2, cn=cn)
    e_ext = dec_relerr(v, ref)
    e_orc = dec_relerr(orc_mode(gamma, N, lam, g, 0.4, -0.2, cn), ref)
    # ext_mode returns float64 (one rounding at the end): within float64's
    # unit roundoff where the recurrence does not amplify rounding, and far
    # below the float64 recurrence's error where it does
    assert e_ext <= max(2.0 ** -52, e_orc / 100), (e_ext, e_orc)


def test_ext_mode_beats_the_float64_floor(orc):
    """A diffusion-wave mode at gamma = 1.9 whose history sums cancel: the
    recurrence amplifies rounding about 5000-fold at N = 1024.  The float64
    recurrence is 5.5e-13 off the decimal solution, the long double one about
    1e-15, i.e. its unit roundoff times the same factor."""
    gamma, N, lam = 1.9, 1024, 123.4
    t = (np.arange(1, N + 1) - 0.5) / N
    g = 1 + t ** 1.5
    ref = dec_mode(gamma, N, lam, g, 0.7, 0.3)
    e_orc = dec_relerr(orc.mode(gamma, 1.0, N, lam, g, 0.7, 0.3), ref)
    e_ext = dec_relerr(ext.mode(gamma, 1.0, N, lam, g, 0.7, 0.3), ref)
    assert e_ext <= 4e-15
    assert e_orc > 100 * e_ext


def test_ext_solve_beats_the_float64_floor(orc):
    """Extended-precision stepping of a rough diffusion-wave case: at least
    an order of magnitude closer to the decimal solve than the float64
    oracle."""
    gamma, M, N = 1.9, 3, 12
    F, u0, phi = rough_case(gamma, M, N, seed=4)
    F = F * 1e4
    ref = dec_block_solve("diffusion", gamma, M, N, F, u0, phi)
    e_ext = dec_relerr(ext.solve(gamma, M, N, F, u0, phi), ref)
    e_orc = dec_relerr(orc.solve(gamma, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi), ref)
    assert e_ext <= 1e-17
    assert e_ext * 10 <= max(e_orc, 1e-16)


def test_two_extended_references_agree():
    """ext_mode (C, long double, series weights) and ext_reference.solve
    (decimal weights, long double stepping) on a single sine mode."""
    gamma, M, N, j = 1.6, 7, 64, 2
    h = 1.0 / (M + 1)
    x = h * np.arange(1, M + 1)
    s = np.sin(j * np.pi * x)
    lam = 4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2
    t = (np.arange(1, N + 1) - 0.5) / N
    g = 1 + t ** 2.5
    U = ext.solve(gamma, M, N, np.outer(g, s), 0.3 * s, -0.1 * s)
    v = ext.mode(gamma, 1.0, N, lam, g, 0.3, -0.1)
    assert relerr(np.asarray(U, dtype=np.float64), np.outer(v, s)) <= 1e-15


def test_floor_check_rejects_a_wrong_reference():
    """assert_floor_parity: passes with the GPU forward error within twice
    the oracle's, or with its backward error within 8 ulp; refuses a
    reference far from the oracle, a forward error above 1e-8, and a result
    that fails both the forward and the backward condition."""
    eps = ext.EPS
    ext.assert_floor_parity(3e-11, 2e-11, 1.5e-11, 500 * eps, 0.5 * eps, 1e-11)   # forward
    ext.assert_floor_parity(3e-11, 5e-11, 1.5e-11, 3 * eps, 0.5 * eps, 1e-11)     # backward
    ext.assert_floor_parity(3e-11, 5e-11, 1.5e-11, 20 * eps, 12 * eps, 1e-11)
    with pytest.raises(AssertionError):
        ext.assert_floor_parity(3e-11, 0.5, 0.5, eps, eps, 1e-11)          # reference in doubt
    with pytest.raises(AssertionError):
        ext.assert_floor_parity(3e-8, 2e-8, 1e-9, eps, eps, 1e-11)         # forward error too large
    with pytest.raises(AssertionError):
        ext.assert_floor_parity(3e-11, 5e-11, 1.5e-11, 9 * eps, eps, 1e-11)  # both conditions fail


def test_backward_error_measures(orc):
    """The backward-error measures: about half an ulp for the oracle's own
    solutions, and a perturbation of 1e-13 relative shows as hundreds of
    ulp (field, advection and modal forms)."""
    M, N = 9, 60
    rng = np.random.default_rng(2)
    F, u0, phi = rng.standard_normal((N, M)), rng.standard_normal(M), rng.standard_normal(M)
    for gamma in (0.6, 1.6):
        w = orc.weights(gamma, 1.0, N)
        U = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi)
        assert ext.backward(w, M, N, F, U, u0, phi) <= 4 * ext.EPS
        assert ext.backward(w, M, N, F, U * (1 + 1e-13), u0, phi) >= 50 * ext.EPS
        Ua = orc.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi)
        assert ext.backward_adv(w, gamma, M, N, F, Ua, u0, phi) <= 4 * ext.EPS
        assert ext.backward_adv(w, gamma, M, N, F, Ua * (1 + 1e-13), u0, phi) >= 50 * ext.EPS
    w = orc.weights(1.6, 1.0, N)
    Uc = orc.solve_cn(1.6, 1.0, 0.0, 1.0, M, N, F, u0=u0, phi=phi)
    assert ext.backward(w, M, N, F, Uc, u0, phi, kind="cn") <= 4 * ext.EPS
    assert ext.backward(w, M, N, F, Uc * (1 + 1e-13), u0, phi, kind="cn") >= 50 * ext.EPS
    # modal form through projection of the field
    from paper_1710_11593_amd import workloads as wl

    inst = wl.Instance(1.4, 6, 400, modes=[(1, 0.7, 1.5), (2, -0.4, 2.2), (5, 1.1, 1.2)], manufactured=True)
    wl.fill(inst)
    U = orc.solve(1.4, 1.0, 0.0, 1.0, 6, 400, inst.f, u0=inst.u0, phi=inst.phi)
    series = wl.modal_time_series(inst)
    js = sorted(series)
    V = dict(zip(js, ext.modal_coefficients(U, js)))
    w = orc.weights(1.4, 1.0, 400)
    assert ext.modal_backward(w, 6, 400, series, V) <= 4 * ext.EPS
    assert ext.modal_backward(w, 6, 400, series, {j: V[j] * (1 + 1e-13) for j in js}) >= 50 * ext.EPS
