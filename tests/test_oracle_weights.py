"""Pins for the oracle's weights (section 3: G_k, M_k; Lemma 1; eq. e17, e19).

Checked against values the mathematics fixes, not against the oracle itself:
50-digit decimal evaluations of (k+1)^p - k^p and of the differences that
define a_m, the telescoping sum, monotonicity/convexity, the zero row sum of
the L1 operator, scipy's digamma and Richardson differences in gamma.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

EPS = np.finfo(np.float64).eps
getcontext().prec = 50


def dec_b(k, p):
    """(k+1)^p - k^p in 50-digit decimal; b_{-1} = b_{-2} = 0."""
    if k < 0:
        return Decimal(0)
    kp1 = (Decimal(p) * Decimal(k + 1).ln()).exp()
    kk = Decimal(0) if k == 0 else (Decimal(p) * Decimal(k).ln()).exp()
    return kp1 - kk


SAMPLE_K = list(range(0, 300)) + [511, 1000, 1023, 4095, 12345, 32767, 65535, 65536, 131071]


@pytest.mark.parametrize("gamma", [0.1, 0.3, 0.5, 0.6, 0.7, 0.9, 1.1, 1.5, 1.9])
def test_b_against_decimal(orc, gamma):
    N = 131072
    w = orc.weights(gamma, 1.0, N)
    p = (1.0 - gamma) if gamma < 1 else (2.0 - gamma)
    worst = 0.0
    for k in SAMPLE_K:
        if k >= N:
            continue
        ref = dec_b(k, Decimal(repr(p)))
        rel = abs((Decimal(repr(float(w["b"][k]))) - ref) / ref)
        worst = max(worst, float(rel))
    assert worst <= 4.0 * EPS, worst


@pytest.mark.parametrize("gamma", [0.1, 0.3, 0.5, 0.7, 0.9, 1.1, 1.5, 1.9])
def test_a_relative_against_decimal(orc, gamma):
    """a_m to a few ulps RELATIVE to a_m itself, at every sampled m (the
    differences are formed without cancellation)."""
    N = 131072
    w = orc.weights(gamma, 1.0, N)
    coef = w["coef"]
    pd = Decimal(repr((1.0 - gamma) if gamma < 1 else (2.0 - gamma)))
    worst = 0.0
    for m in SAMPLE_K:
        if m >= N:
            continue
        if gamma < 1:
            d = dec_b(m, pd) - (dec_b(m - 1, pd) if m >= 1 else Decimal(0))
        else:
            d = dec_b(m - 2, pd) - 2 * dec_b(m - 1, pd) + dec_b(m, pd)
        rel = abs((Decimal(repr(float(w["a"][m]))) - Decimal(repr(coef)) * d) / (Decimal(repr(coef)) * d))
        worst = max(worst, float(rel))
        if gamma > 1 and m >= 1:
            # rho_{m+1} = c (M_{m-1} - M_m)
            dr = dec_b(m - 1, pd) - dec_b(m, pd)
            relr = abs((Decimal(repr(float(w["rho"][m]))) - Decimal(repr(coef)) * dr) / (Decimal(repr(coef)) * dr))
            worst = max(worst, float(relr))
    assert worst <= 64 * EPS, worst


@pytest.mark.parametrize("gamma", [0.1, 0.5, 0.9, 1.1, 1.5, 1.9])
def test_a_against_decimal(orc, gamma):
    """a_m = coef * (first or second difference of b), to a few eps of b."""
    N = 131072
    T = 1.0
    w = orc.weights(gamma, T, N)
    tau = T / N
    coef = w["coef"]
    ref_coef = tau ** (-gamma) / math.gamma((2.0 if gamma < 1 else 3.0) - gamma)
    assert abs(coef - ref_coef) <= 8 * EPS * ref_coef
    pd = Decimal(repr((1.0 - gamma) if gamma < 1 else (2.0 - gamma)))
    for m in SAMPLE_K:
        if m >= N:
            continue
        if gamma < 1:
            d = dec_b(m, pd) - (dec_b(m - 1, pd) if m >= 1 else Decimal(0))
            scale = float(dec_b(max(m - 1, 0), pd))
        else:
            d = dec_b(m - 2, pd) - 2 * dec_b(m - 1, pd) + dec_b(m, pd)
            scale = float(dec_b(max(m - 2, 0), pd))
        err = abs(w["a"][m] / coef - float(d))
        assert err <= 6 * EPS * scale, (m, err, scale)


@pytest.mark.parametrize("gamma", [0.2, 0.5, 0.8, 1.2, 1.5, 1.8])
def test_weight_invariants(orc, gamma):
    N = 65536
    w = orc.weights(gamma, 1.0, N)
    b = w["b"]
    p = (1.0 - gamma) if gamma < 1 else (2.0 - gamma)
    assert b[0] == 1.0
    assert np.all(b > 0)
    assert np.all(np.diff(b) < 0), "b_k must decrease strictly (Lemma 1 printed the inequality reversed)"
    assert np.all(b[:-2] - 2 * b[1:-1] + b[2:] > 0), "b_k is convex"
    for n in (1, 2, 7, 100, 4096, 65536):
        tele = math.fsum(b[:n])
        assert abs(tele - n ** p) <= 1e-14 * n ** p
    k = N - 1
    assert abs(b[k] * k ** (1.0 - p) / p - 1.0) < 1e-4


@pytest.mark.parametrize("gamma", [0.1, 0.5, 0.9, 1.1, 1.5, 1.9])
def test_row_sums_vanish(orc, gamma):
    """sum_{m<n} a_m + rho_n = 0: the discrete operator kills constants."""
    N = 4096
    w = orc.weights(gamma, 1.0, N)
    for n in (1, 2, 3, 10, 1000, N):
        s = math.fsum(list(w["a"][:n]) + [w["rho"][n - 1]])
        assert abs(s) <= 1e-13 * w["coef"], (n, s)
    if gamma < 1:
        assert np.all(w["psi"] == 0)
        assert np.allclose(w["rho"], -w["coef"] * w["b"], rtol=1e-15, atol=0)
    else:
        assert w["rho"][0] == -w["coef"]
        assert np.allclose(w["psi"], w["coef"] * (1.0 / N) * w["b"], rtol=1e-15, atol=0)


@pytest.mark.parametrize("x", [0.1, 0.5, 1.0, 1.1, 1.4, 1.5, 1.9, 2.0, 2.3, 3.7, 12.5])
def test_digamma_against_scipy(orc, x):
    scipy_special = pytest.importorskip("scipy.special")
    ref = float(scipy_special.digamma(x))
    assert abs(orc.digamma(x) - ref) <= 4e-15 * max(1.0, abs(ref))


@pytest.mark.parametrize("gamma", [0.3, 0.6, 1.3, 1.7])
def test_weight_derivatives_richardson(orc, gamma):
    """d/dgamma of coef, a_m, rho_n, psi_n vs 4th-order Richardson differences."""
    N = 2048
    d = 1e-3
    w = orc.weights(gamma, 1.0, N)
    wp, wm = orc.weights(gamma + d, 1.0, N), orc.weights(gamma - d, 1.0, N)
    wp2, wm2 = orc.weights(gamma + 2 * d, 1.0, N), orc.weights(gamma - 2 * d, 1.0, N)

    def rich(key):
        return (8 * (wp[key] - wm[key]) - (wp2[key] - wm2[key])) / (12 * d)

    assert abs(rich("coef") - w["dcoef"]) <= 1e-9 * abs(w["dcoef"])
    for key, dkey in (("a", "da"), ("rho", "drho"), ("psi", "dpsi")):
        fd = rich(key)
        scale = np.max(np.abs(fd)) + 1e-300
        assert np.max(np.abs(fd - w[dkey])) <= 1e-8 * scale, key
