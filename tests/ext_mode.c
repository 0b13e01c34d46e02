/*
 * Extended-precision (x87 long double, 64-bit significand) single-mode
 * recurrence -- test infrastructure only.
 *
 * The same definition as the oracle's scalar recurrence of one sine mode
 * (weights of section 3, time stepping of the block system restricted to an
 * eigenvector of K), evaluated in long double with the Toeplitz differences
 * summed from the binomial expansion.  Used to measure the float64 rounding
 * floor of full-size diffusion-wave runs, where the history sum cancels
 * several times the size of the result at every step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef long double ld;

static ld bk(int64_t k, ld p)
{
    if (k < 0) return 0.0L;
    if (k == 0) return 1.0L;
    ld kd = (ld)k;
    return powl(kd, p) * expm1l(p * log1pl(1.0L / kd));
}

/* sum_j c_j (m + j)^p for the second (order 2) or third (order 3) difference */
static ld dser(int64_t m, ld p, int order)
{
    const ld j2[3] = {1, 0, -1}, c2[3] = {1, -2, 1};
    const ld j3[4] = {1, 0, -1, -2}, c3[4] = {1, -3, 3, -1};
    const ld *jj = order == 2 ? j2 : j3, *cc = order == 2 ? c2 : c3;
    int nj = order == 2 ? 3 : 4;
    ld x = 1.0L / (ld)m, binom = 1.0L, sum = 0.0L, jk[4] = {1, 1, 1, 1};
    for (int k = 1; k <= 300; ++k) {
        binom *= (p - (ld)(k - 1)) / (ld)k * x;
        ld inner = 0.0L;
        for (int q = 0; q < nj; ++q) {
            jk[q] *= jj[q];
            inner += cc[q] * jk[q];
        }
        sum += binom * inner;
        if (k > order && fabsl(binom) * 8.0L * powl(2.0L, (ld)k) <= 1e-22L * fabsl(sum)) break;
    }
    return powl((ld)m, p) * sum;
}

/* v[n-1], n = 1..N: (a_0 + lam) v^n = g^n - rho_n v0 + psi_n phihat - sum_{j<n} a_{n-j} v^j
 * (cn: (a_0 + lam/2) v^n = ... - (lam/2) v^{n-1}, v^0 = v0) */
static int ext_mode_any(double gamma, double T, int64_t N, double lam, const double *g, double v0, double phihat,
                        double *vout, int cn)
{
    int wave = gamma > 1.0;
    ld G = (ld)gamma, p = wave ? 2.0L - G : 1.0L - G;
    ld tau = (ld)T / (ld)N;
    ld coef = powl(tau, -G) / tgammal(wave ? 3.0L - G : 2.0L - G);
    ld *a = malloc(sizeof(ld) * (size_t)N), *rho = malloc(sizeof(ld) * (size_t)N), *psi = malloc(sizeof(ld) * (size_t)N);
    ld *v = malloc(sizeof(ld) * (size_t)N);
    if (!a || !rho || !psi || !v) return -2;
    for (int64_t m = 0; m < N; ++m) {
        ld d;
        if (!wave) d = (m >= 4) ? dser(m, p, 2) : bk(m, p) - bk(m - 1, p);
        else d = (m >= 4) ? dser(m, p, 3) : bk(m - 2, p) - 2.0L * bk(m - 1, p) + bk(m, p);
        a[m] = coef * d;
    }
    for (int64_t n = 1; n <= N; ++n) {
        if (!wave) {
            rho[n - 1] = -coef * bk(n - 1, p);
            psi[n - 1] = 0.0L;
        } else {
            rho[n - 1] = (n - 1 >= 4) ? -coef * dser(n - 1, p, 2) : coef * (bk(n - 2, p) - bk(n - 1, p));
            psi[n - 1] = coef * tau * bk(n - 1, p);
        }
    }
    /* cn: the spatial term averaged over t_n and t_{n-1} (lam/2 on both) */
    ld d0 = a[0] + (cn ? 0.5L : 1.0L) * (ld)lam;
    for (int64_t n = 1; n <= N; ++n) {
        ld s = (ld)g[n - 1] - rho[n - 1] * (ld)v0 + psi[n - 1] * (ld)phihat;
        for (int64_t j = 1; j < n; ++j) s -= a[n - j] * v[j - 1];
        if (cn) s -= 0.5L * (ld)lam * (n == 1 ? (ld)v0 : v[n - 2]);
        v[n - 1] = s / d0;
        vout[n - 1] = (double)v[n - 1];
    }
    free(a); free(rho); free(psi); free(v);
    return 0;
}

int ext_mode(double gamma, double T, int64_t N, double lam, const double *g, double v0, double phihat, double *vout)
{
    return ext_mode_any(gamma, T, N, lam, g, v0, phihat, vout, 0);
}

int ext_mode_cn(double gamma, double T, int64_t N, double lam, const double *g, double v0, double phihat,
                double *vout)
{
    return ext_mode_any(gamma, T, N, lam, g, v0, phihat, vout, 1);
}

/* The same recurrence in long double with the float64 weights given (a[m],
 * rho[n-1], psi[n-1], m, n-1 < N): the exact solution of the system those
 * float64 weights define, so that an implementation's solver rounding can be
 * measured apart from the rounding of its weights. */
int ext_mode_given(int64_t N, const double *a, const double *rho, const double *psi, double lam, const double *g,
                   double v0, double phihat, double *vout, int cn)
{
    ld *v = malloc(sizeof(ld) * (size_t)N);
    if (!v) return -2;
    ld d0 = (ld)a[0] + (cn ? 0.5L : 1.0L) * (ld)lam;
    for (int64_t n = 1; n <= N; ++n) {
        ld s = (ld)g[n - 1] - (ld)rho[n - 1] * (ld)v0 + (ld)psi[n - 1] * (ld)phihat;
        for (int64_t j = 1; j < n; ++j) s -= (ld)a[n - j] * v[j - 1];
        if (cn) s -= 0.5L * (ld)lam * (n == 1 ? (ld)v0 : v[n - 2]);
        v[n - 1] = s / d0;
        vout[n - 1] = (double)v[n - 1];
    }
    free(v);
    return 0;
}

/* Residual of a single-mode solution v (float64, as a solver returned it) of
 * the system defined by the float64 weights given, in long double: for every
 * step n
 *   r^n = g^n - rho_n v0 + psi_n phihat - (a_0 + lam) v^n - sum_{m=1}^{n-1} a_m v^{n-m}
 * (cn: lam/2 on v^n and on v^{n-1}, v^0 = v0) into rout[n-1], and the sum of
 * the absolute values of the same terms into sout[n-1]. */
int ext_mode_residual(int64_t N, const double *a, const double *rho, const double *psi, double lam, const double *g,
                      double v0, double phihat, const double *v, int cn, double *rout, double *sout)
{
    const ld L = (ld)lam;
    for (int64_t n = 1; n <= N; ++n) {
        ld terms[4] = {(ld)g[n - 1], -(ld)rho[n - 1] * (ld)v0, (ld)psi[n - 1] * (ld)phihat,
                       -((ld)a[0] + (cn ? 0.5L : 1.0L) * L) * (ld)v[n - 1]};
        ld r = 0.0L, sc = 0.0L;
        for (int k = 0; k < 4; ++k) {
            r += terms[k];
            sc += fabsl(terms[k]);
        }
        for (int64_t j = 1; j < n; ++j) {
            const ld t = (ld)a[n - j] * (ld)v[j - 1];
            r -= t;
            sc += fabsl(t);
        }
        if (cn) {
            const ld t = 0.5L * L * (n == 1 ? (ld)v0 : (ld)v[n - 2]);
            r -= t;
            sc += fabsl(t);
        }
        rout[n - 1] = (double)r;
        sout[n - 1] = (double)sc;
    }
    return 0;
}
