/*
 * oracle.c -- plain CPU FP64 reference for the L1 time-stepping scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) shares no code with it and never calls it.
 *
 * What it computes (Liu, Cheng, Li, Wang, "Fast procedures for Caputo
 * fractional ordinary and partial differential equations"):
 *
 *   Time-fractional diffusion, 0<gamma<1 (Scheme 4, eq. e19/e20):
 *     mu = tau^-gamma / Gamma(2-gamma),  b_k = G_k = (k+1)^(1-gamma) - k^(1-gamma)
 *     a_0 = mu,  a_m = mu (b_m - b_{m-1}),  rho_n = -mu b_{n-1},  psi_n = 0,
 *     F^n = f(x_i, t_n).
 *     The u^0 term of e19 is read as the telescoping L1 term -mu b_{n-1} u^0
 *     (the printed "+G_n u^0" would make the Caputo derivative of a constant
 *     non-zero).
 *
 *   Diffusion-wave, 1<gamma<2 (time part of Scheme 3, eq. e15-e17, and the
 *   Toeplitz matrix of the "new procedure" for Scheme 3):
 *     c = tau^-gamma / Gamma(3-gamma),  b_k = M_k = (k+1)^(2-gamma) - k^(2-gamma),
 *     b_{-1} = b_{-2} = 0,
 *     a_m = c (b_{m-2} - 2 b_{m-1} + b_m),  rho_n = c (b_{n-2} - b_{n-1}),
 *     psi_n = c tau b_{n-1},  F^n = f(x_i, t_{n-1/2});
 *     the spatial term is taken at t_n, as in e16/e17.  That timing is a
 *     reading (the paper prints no diffusion-wave scheme with a second-order
 *     space operator): parity unpinned beyond the observed convergence rate;
 *     the time weights themselves are pinned by Table 7.
 *
 *   Both regimes give, for n = 1..N, with K = h^-2 tridiag(-1,2,-1):
 *     (a_0 I + K) U^n + sum_{j=1}^{n-1} a_{n-j} U^j = F^n - rho_n u^0 + psi_n phi
 *   and this file solves it by plain forward time stepping (the paper's
 *   "direct method" of section 3, O(M N^2) work), one Thomas solve per step.
 *   It also solves it by restarted GMRES(m) (the paper's iterative method
 *   for Scheme 4, section 3.1), with the operator products evaluated from
 *   their definition.
 *
 *   Scheme 1 (the two-sided fractional ODE, eq. e7) has its symmetric
 *   Toeplitz column in oracle_ode_column and conjugate gradients in
 *   oracle_ode_cg.
 *
 *   Advection equations D_t^gamma u + u_x = f (Schemes 2 and 3, eq. e11-e17)
 *   are stepped by oracle_solve_adv, and the diffusion-wave variant with the
 *   spatial term averaged over t_n and t_{n-1} by oracle_solve_cn (see
 *   there).
 *
 * Layout: time-major [N][M] row-major, entry (n-1)*M + (i-1) is (x_i, t_n),
 * h = (x1-x0)/(M+1), x_i = x0 + i h, tau = T/N.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EARG (-1)
#define ORACLE_ENOMEM (-2)

/* Digamma from the asymptotic (Stirling-type) series, Abramowitz & Stegun
 * 6.3.18, after shifting the argument above 10 with psi(x) = psi(x+1) - 1/x
 * (A&S 6.3.5).  Used for d(mu)/d(gamma) = mu (-ln tau + psi(2-gamma)). */
double oracle_digamma(double x)
{
    double acc = 0.0;
    while (x < 10.0) {
        acc -= 1.0 / x;
        x += 1.0;
    }
    double r = 1.0 / x, r2 = r * r;
    /* Bernoulli-number terms B_2k / (2k x^2k), k = 1..7 */
    double series = r2 * (1.0 / 12.0
                  - r2 * (1.0 / 120.0
                  - r2 * (1.0 / 252.0
                  - r2 * (1.0 / 240.0
                  - r2 * (1.0 / 132.0
                  - r2 * (691.0 / 32760.0
                  - r2 * (1.0 / 12.0)))))));
    return acc + log(x) - 0.5 * r - series;
}

static int regime_of(double gamma)
{
    if (gamma > 0.0 && gamma < 1.0) return 0;   /* diffusion */
    if (gamma > 1.0 && gamma < 2.0) return 1;   /* diffusion-wave */
    return -1;
}

/* b_k = (k+1)^p - k^p evaluated without cancellation:
 * (k+1)^p - k^p = k^p ((1+1/k)^p - 1) = k^p expm1(p log1p(1/k)). */
static double bk(int64_t k, double p)
{
    if (k < 0) return 0.0;
    if (k == 0) return 1.0;
    double kd = (double)k;
    return pow(kd, p) * expm1(p * log1p(1.0 / kd));
}

/* d b_k / d p = ln(k+1)(k+1)^p - ln(k) k^p = ln(k) b_k + log1p(1/k) (k+1)^p,
 * a sum of two non-negative terms. */
static double dbk_dp(int64_t k, double p)
{
    if (k <= 0) return 0.0;
    double kd = (double)k;
    return log(kd) * bk(k, p) + log1p(1.0 / kd) * pow(kd + 1.0, p);
}

/*
 * The Toeplitz column is a finite difference of k^p: for m >= 1
 *   0<gamma<1:  b_m - b_{m-1}             = (m+1)^p - 2 m^p + (m-1)^p
 *   1<gamma<2:  b_{m-2} - 2 b_{m-1} + b_m = (m+1)^p - 3 m^p + 3 (m-1)^p - (m-2)^p
 * (section 3: G_k - G_{k-1}, and W_j = M_{j-2} - 2 M_{j-1} + M_j).  Formed as
 * differences of rounded b_k these lose about m (resp. m^2) in relative
 * accuracy.  For large m they are summed instead from the binomial expansion
 * of (1 + j/m)^p, an exact identity: with x = 1/m and C(p,k) the binomial
 * coefficients,
 *   sum_j c_j (1 + j x)^p = sum_{k>=0} C(p,k) x^k sum_j c_j j^k,
 * where the inner sums vanish for k < order of the difference.
 */
static double diff_series(int64_t m, double p, int order)
{
    /* offsets j and coefficients c_j of the difference operator */
    const double j2[3] = {1.0, 0.0, -1.0}, c2[3] = {1.0, -2.0, 1.0};
    const double j3[4] = {1.0, 0.0, -1.0, -2.0}, c3[4] = {1.0, -3.0, 3.0, -1.0};
    const double *jj = (order == 2) ? j2 : j3, *cc = (order == 2) ? c2 : c3;
    int nj = (order == 2) ? 3 : 4;
    double x = 1.0 / (double)m;
    double binom = 1.0; /* C(p,k) x^k */
    double sum = 0.0;
    double jk[4] = {1.0, 1.0, 1.0, 1.0}; /* j^k, updated by one product per k */
    for (int k = 1; k <= 200; ++k) {
        binom *= (p - (double)(k - 1)) / (double)k * x;
        double inner = 0.0;
        for (int q = 0; q < nj; ++q) {
            jk[q] *= jj[q];
            inner += cc[q] * jk[q];
        }
        double term = binom * inner;
        sum += term;
        /* |inner| <= sum_j |c_j| |j|^k <= 8 * 2^k; stop once that bound on the
         * remaining terms is negligible (single terms can vanish exactly) */
        if (k > order && fabs(binom) * 8.0 * pow(2.0, (double)k) <= 1e-18 * fabs(sum)) break;
    }
    return pow((double)m, p) * sum;
}

/*
 * Weights of the discrete system for gamma in (0,1) or (1,2).
 * Arrays have length N; index m holds a_m (m = 0..N-1), index n-1 holds
 * rho_n and psi_n (n = 1..N), index k holds b_k.  Derivative arrays (d/dgamma)
 * may be NULL.  scal[0] = mu or c, scal[1] = its gamma derivative.
 */
int oracle_weights(double gamma, double T, int64_t N,
                   double *b, double *a, double *rho, double *psi,
                   double *da, double *drho, double *dpsi, double *scal)
{
    int reg = regime_of(gamma);
    if (reg < 0 || !(T > 0.0) || N < 1) return ORACLE_EARG;
    double tau = T / (double)N;
    double p = (reg == 0) ? 1.0 - gamma : 2.0 - gamma;
    double g = (reg == 0) ? 2.0 - gamma : 3.0 - gamma;     /* Gamma argument */
    double coef = pow(tau, -gamma) / tgamma(g);
    double dcoef = coef * (-log(tau) + oracle_digamma(g));
    if (scal) { scal[0] = coef; scal[1] = dcoef; }

    /* b_k for k = -2..N (shifted by 2) and d b_k / d gamma = -d b_k / d p */
    double *B = (double *)malloc(sizeof(double) * (size_t)(N + 3));
    double *dB = (double *)malloc(sizeof(double) * (size_t)(N + 3));
    if (!B || !dB) { free(B); free(dB); return ORACLE_ENOMEM; }
    for (int64_t k = -2; k <= N; ++k) {
        B[k + 2] = bk(k, p);
        dB[k + 2] = -dbk_dp(k, p);
    }
#define BB(k) B[(k) + 2]
#define DB(k) dB[(k) + 2]
    for (int64_t k = 0; k < N; ++k)
        if (b) b[k] = BB(k);
    for (int64_t m = 0; m < N; ++m) {
        double am, dam;
        if (reg == 0) {
            /* a_0 = mu G_0, a_m = mu (G_m - G_{m-1}) */
            double d1 = (m >= 4) ? diff_series(m, p, 2) : BB(m) - BB(m - 1);
            double dd1 = DB(m) - DB(m - 1);
            am = coef * d1;
            dam = dcoef * d1 + coef * dd1;
        } else {
            /* a_m = c W_m, W_m = M_{m-2} - 2 M_{m-1} + M_m (W_0 = 1, W_1 = M_1 - 2) */
            double d2 = (m >= 4) ? diff_series(m, p, 3) : BB(m - 2) - 2.0 * BB(m - 1) + BB(m);
            double dd2 = DB(m - 2) - 2.0 * DB(m - 1) + DB(m);
            am = coef * d2;
            dam = dcoef * d2 + coef * dd2;
        }
        if (a) a[m] = am;
        if (da) da[m] = dam;
    }
    for (int64_t n = 1; n <= N; ++n) {
        double r, dr, s, ds;
        if (reg == 0) {
            r = -coef * BB(n - 1);
            dr = -dcoef * BB(n - 1) - coef * DB(n - 1);
            s = 0.0;
            ds = 0.0;
        } else {
            /* rho_n = c (M_{n-2} - M_{n-1}) = -c ((n)^p - 2 (n-1)^p + (n-2)^p) */
            r = (n - 1 >= 4) ? -coef * diff_series(n - 1, p, 2) : coef * (BB(n - 2) - BB(n - 1));
            dr = dcoef * (BB(n - 2) - BB(n - 1)) + coef * (DB(n - 2) - DB(n - 1));
            s = coef * tau * BB(n - 1);
            ds = tau * (dcoef * BB(n - 1) + coef * DB(n - 1));
        }
        if (rho) rho[n - 1] = r;
        if (drho) drho[n - 1] = dr;
        if (psi) psi[n - 1] = s;
        if (dpsi) dpsi[n - 1] = ds;
    }
#undef BB
#undef DB
    free(B);
    free(dB);
    return ORACLE_OK;
}

/* Factor the constant tridiagonal block A0 = a0 I + K once (Thomas, no
 * pivoting; A0 is symmetric and strictly diagonally dominant because a0 > 0).
 * cp[i] = modified super-diagonal, inv[i] = 1/pivot. */
static void thomas_factor(int64_t M, double diag, double off, double *cp, double *inv)
{
    double prev = 0.0;
    for (int64_t i = 0; i < M; ++i) {
        double piv = diag - off * prev;
        inv[i] = 1.0 / piv;
        cp[i] = off * inv[i];
        prev = cp[i];
    }
}

/* Solve A0 x = r in place (r overwritten by x). */
static void thomas_solve(int64_t M, double off, const double *cp, const double *inv, double *r)
{
    for (int64_t i = 0; i < M; ++i) {
        double prev = (i > 0) ? r[i - 1] : 0.0;
        r[i] = (r[i] - off * prev) * inv[i];
    }
    for (int64_t i = M - 2; i >= 0; --i)
        r[i] -= cp[i] * r[i + 1];
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Forward time stepping for n = nfirst+1..nsteps (0 <= nfirst <= nsteps <= N;
 * the grid and the weights are those of the full N-step problem).  Rows
 * below nfirst must already hold the solution (from an earlier call with the
 * same arguments): each step reads only earlier rows, so a run split into
 * consecutive ranges computes exactly what one call does.
 *   f   [N][M]  source sampled at t_n (gamma<1) or t_{n-1/2} (gamma>1)
 *   u0  [M]     initial value (NULL = 0)
 *   phi [M]     initial velocity, used for gamma>1 only (NULL = 0)
 *   u   [N][M]  output; rows outside nfirst..nsteps-1 are left untouched
 */
int oracle_solve_rows(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                      int64_t nfirst, int64_t nsteps, const double *f, const double *u0, const double *phi,
                      double *u, int nthreads)
{
    if (regime_of(gamma) < 0 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !f || !u)
        return ORACLE_EARG;
    if (nsteps < 0 || nsteps > N || nfirst < 0 || nfirst > nsteps) return ORACLE_EARG;
    set_threads(nthreads);
    double h = (x1 - x0) / (double)(M + 1);
    double e = 1.0 / (h * h);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi = (double *)malloc(sizeof(double) * (size_t)N);
    double *cp = (double *)malloc(sizeof(double) * (size_t)M);
    double *inv = (double *)malloc(sizeof(double) * (size_t)M);
    if (!a || !rho || !psi || !cp || !inv) {
        free(a); free(rho); free(psi); free(cp); free(inv);
        return ORACLE_ENOMEM;
    }
    oracle_weights(gamma, T, N, NULL, a, rho, psi, NULL, NULL, NULL, NULL);
    thomas_factor(M, a[0] + 2.0 * e, -e, cp, inv);

    for (int64_t n = nfirst + 1; n <= nsteps; ++n) {
        double *r = u + (size_t)(n - 1) * (size_t)M;
        const double *fn = f + (size_t)(n - 1) * (size_t)M;
        /* right-hand side: F^n - rho_n u^0 + psi_n phi - sum_j a_{n-j} U^j */
        /* blocks of 256 points; each block runs over all earlier rows j in
         * order, so rows are read contiguously */
        #pragma omp parallel for schedule(static)
        for (int64_t i0 = 0; i0 < M; i0 += 256) {
            int64_t i1 = (i0 + 256 < M) ? i0 + 256 : M;
            for (int64_t i = i0; i < i1; ++i) {
                double s = fn[i];
                if (u0) s -= rho[n - 1] * u0[i];
                if (phi) s += psi[n - 1] * phi[i];
                r[i] = s;
            }
            for (int64_t j = 1; j < n; ++j) {
                const double *uj = u + (size_t)(j - 1) * (size_t)M;
                double w = a[n - j];
                for (int64_t i = i0; i < i1; ++i) r[i] -= w * uj[i];
            }
        }
        thomas_solve(M, -e, cp, inv, r);
    }
    free(a); free(rho); free(psi); free(cp); free(inv);
    return ORACLE_OK;
}

/* The whole run n = 1..nsteps (rows >= nsteps are left untouched). */
int oracle_solve(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                 int64_t nsteps, const double *f, const double *u0, const double *phi,
                 double *u, int nthreads)
{
    return oracle_solve_rows(gamma, T, x0, x1, M, N, 0, nsteps, f, u0, phi, u, nthreads);
}

/* y = A u for the Toeplitz column a and e = 1/h^2 (the definition, row by
 * row: the tridiagonal block on U^n plus the history sum). */
static void apply_rows(int64_t M, int64_t N, const double *a, double e, const double *u, double *y)
{
    for (int64_t n = 1; n <= N; ++n) {
        const double *un = u + (size_t)(n - 1) * (size_t)M;
        double *yn = y + (size_t)(n - 1) * (size_t)M;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            double left = (i > 0) ? un[i - 1] : 0.0;
            double right = (i + 1 < M) ? un[i + 1] : 0.0;
            double s = (a[0] + 2.0 * e) * un[i] - e * (left + right);
            for (int64_t j = 1; j < n; ++j)
                s += a[n - j] * u[(size_t)(j - 1) * (size_t)M + (size_t)i];
            yn[i] = s;
        }
    }
}

/*
 * Operator apply y = A u of the whole block lower-triangular system:
 *   y^n = (a_0 I + K) U^n + sum_{j=1}^{n-1} a_{n-j} U^j.
 */
int oracle_apply(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                 const double *u, double *y, int nthreads)
{
    if (regime_of(gamma) < 0 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !u || !y)
        return ORACLE_EARG;
    set_threads(nthreads);
    double h = (x1 - x0) / (double)(M + 1);
    double e = 1.0 / (h * h);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    if (!a) return ORACLE_ENOMEM;
    oracle_weights(gamma, T, N, NULL, a, NULL, NULL, NULL, NULL, NULL, NULL);
    apply_rows(M, N, a, e, u, y);
    free(a);
    return ORACLE_OK;
}

/*
 * Adjoint of the solve.  Given G = dL/dU [N][M] and the forward solution
 * U [N][M], computes Lambda = A^{-T} G (= dL/dF, since F enters the
 * right-hand side with identity) by backward time stepping
 *   (a_0 I + K) Lambda^n = G^n - sum_{j=n+1}^{N} a_{j-n} Lambda^j,  n = N..1,
 * and dL/dgamma = sum_n <Lambda^n, -rho'_n u^0 + psi'_n phi>
 *               - sum_n sum_{j<=n} a'_{n-j} <Lambda^n, U^j>,
 * with f, u^0 and phi held fixed.
 */
int oracle_adjoint(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                   const double *g, const double *u, const double *u0, const double *phi,
                   double *lam, double *dLdgamma, int nthreads)
{
    if (regime_of(gamma) < 0 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !g || !u || !lam)
        return ORACLE_EARG;
    set_threads(nthreads);
    double h = (x1 - x0) / (double)(M + 1);
    double e = 1.0 / (h * h);
    size_t NN = (size_t)N;
    double *a = (double *)malloc(sizeof(double) * NN);
    double *da = (double *)malloc(sizeof(double) * NN);
    double *drho = (double *)malloc(sizeof(double) * NN);
    double *dpsi = (double *)malloc(sizeof(double) * NN);
    double *cp = (double *)malloc(sizeof(double) * (size_t)M);
    double *inv = (double *)malloc(sizeof(double) * (size_t)M);
    if (!a || !da || !drho || !dpsi || !cp || !inv) {
        free(a); free(da); free(drho); free(dpsi); free(cp); free(inv);
        return ORACLE_ENOMEM;
    }
    oracle_weights(gamma, T, N, NULL, a, NULL, NULL, da, drho, dpsi, NULL);
    thomas_factor(M, a[0] + 2.0 * e, -e, cp, inv);

    for (int64_t n = N; n >= 1; --n) {
        double *r = lam + (size_t)(n - 1) * (size_t)M;
        const double *gn = g + (size_t)(n - 1) * (size_t)M;
        #pragma omp parallel for schedule(static)
        for (int64_t i0 = 0; i0 < M; i0 += 256) {
            int64_t i1 = (i0 + 256 < M) ? i0 + 256 : M;
            for (int64_t i = i0; i < i1; ++i) r[i] = gn[i];
            for (int64_t j = n + 1; j <= N; ++j) {
                const double *lj = lam + (size_t)(j - 1) * (size_t)M;
                double w = a[j - n];
                for (int64_t i = i0; i < i1; ++i) r[i] -= w * lj[i];
            }
        }
        thomas_solve(M, -e, cp, inv, r);
    }

    if (dLdgamma) {
        double total = 0.0;
        for (int64_t n = 1; n <= N; ++n) {
            const double *ln = lam + (size_t)(n - 1) * (size_t)M;
            double acc = 0.0;
            #pragma omp parallel for schedule(static) reduction(+:acc)
            for (int64_t i = 0; i < M; ++i) {
                double s = 0.0;
                if (u0) s -= drho[n - 1] * u0[i];
                if (phi) s += dpsi[n - 1] * phi[i];
                for (int64_t j = 1; j <= n; ++j)
                    s -= da[n - j] * u[(size_t)(j - 1) * (size_t)M + (size_t)i];
                acc += ln[i] * s;
            }
            total += acc;
        }
        *dLdgamma = total;
    }
    free(a); free(da); free(drho); free(dpsi); free(cp); free(inv);
    return ORACLE_OK;
}

/*
 * Scalar recurrence of one spatial sine mode.  If the source is g(t) s_j and
 * the initial data are v0 s_j, phihat s_j, with s_j(i) = sin(j pi x_i) an exact
 * eigenvector of K with eigenvalue lam, the discrete solution is v^n s_j with
 *   (a_0 + lam) v^n = g^n - rho_n v0 + psi_n phihat - sum_{j<n} a_{n-j} v^j.
 */
int oracle_mode(double gamma, double T, int64_t N, double lam, const double *g,
                double v0, double phihat, double *v)
{
    if (regime_of(gamma) < 0 || !(T > 0.0) || N < 1 || !g || !v) return ORACLE_EARG;
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi = (double *)malloc(sizeof(double) * (size_t)N);
    if (!a || !rho || !psi) { free(a); free(rho); free(psi); return ORACLE_ENOMEM; }
    oracle_weights(gamma, T, N, NULL, a, rho, psi, NULL, NULL, NULL, NULL);
    double d = a[0] + lam;
    for (int64_t n = 1; n <= N; ++n) {
        double s = g[n - 1] - rho[n - 1] * v0 + psi[n - 1] * phihat;
        for (int64_t j = 1; j < n; ++j) s -= a[n - j] * v[j - 1];
        v[n - 1] = s / d;
    }
    free(a); free(rho); free(psi);
    return ORACLE_OK;
}

/*
 * Diffusion-wave equation (1<gamma<2) with the spatial term averaged over
 * t_n and t_{n-1} (Crank-Nicolson in the spatial term, the form of the
 * Sun-Wu scheme cited with eq. e15): for n = 1..N, with U^0 = u0,
 *   a_0 U^n + sum_{j=1}^{n-1} a_{n-j} U^j + (1/2) K (U^n + U^{n-1})
 *     = f(x_i, t_{n-1/2}) - rho_n u0 + psi_n phi,
 * the weights being those of oracle_weights.  Stepped with one Thomas solve
 * of a_0 I + K/2 per step.
 */
int oracle_solve_cn(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                    const double *f, const double *u0, const double *phi, double *u, int nthreads)
{
    if (regime_of(gamma) != 1 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !f || !u) return ORACLE_EARG;
    set_threads(nthreads);
    const double h = (x1 - x0) / (double)(M + 1);
    const double e = 1.0 / (h * h);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi = (double *)malloc(sizeof(double) * (size_t)N);
    double *cp = (double *)malloc(sizeof(double) * (size_t)M);
    double *inv = (double *)malloc(sizeof(double) * (size_t)M);
    double *zero = (double *)calloc((size_t)M, sizeof(double));
    if (!a || !rho || !psi || !cp || !inv || !zero) {
        free(a); free(rho); free(psi); free(cp); free(inv); free(zero);
        return ORACLE_ENOMEM;
    }
    oracle_weights(gamma, T, N, NULL, a, rho, psi, NULL, NULL, NULL, NULL);
    thomas_factor(M, a[0] + e, -0.5 * e, cp, inv);
    for (int64_t n = 1; n <= N; ++n) {
        double *r = u + (size_t)(n - 1) * (size_t)M;
        const double *fn = f + (size_t)(n - 1) * (size_t)M;
        const double *prev = (n == 1) ? (u0 ? u0 : zero) : u + (size_t)(n - 2) * (size_t)M;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            double s = fn[i];
            if (u0) s -= rho[n - 1] * u0[i];
            if (phi) s += psi[n - 1] * phi[i];
            for (int64_t j = 1; j < n; ++j) s -= a[n - j] * u[(size_t)(j - 1) * (size_t)M + (size_t)i];
            /* (1/2) K U^{n-1} */
            double left = (i > 0) ? prev[i - 1] : 0.0;
            double right = (i + 1 < M) ? prev[i + 1] : 0.0;
            s -= 0.5 * e * (2.0 * prev[i] - left - right);
            r[i] = s;
        }
        thomas_solve(M, -0.5 * e, cp, inv, r);
    }
    free(a); free(rho); free(psi); free(cp); free(inv); free(zero);
    return ORACLE_OK;
}

/* y = A u for the system of oracle_solve_cn (no u0 / phi terms):
 *   y^n = a_0 U^n + sum_{j<n} a_{n-j} U^j + (1/2) K U^n + (1/2) K U^{n-1} [n >= 2]. */
int oracle_apply_cn(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                    const double *u, double *y, int nthreads)
{
    if (regime_of(gamma) != 1 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !u || !y) return ORACLE_EARG;
    set_threads(nthreads);
    const double h = (x1 - x0) / (double)(M + 1);
    const double e = 1.0 / (h * h);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    if (!a) return ORACLE_ENOMEM;
    oracle_weights(gamma, T, N, NULL, a, NULL, NULL, NULL, NULL, NULL, NULL);
    for (int64_t n = 1; n <= N; ++n) {
        const double *un = u + (size_t)(n - 1) * (size_t)M;
        const double *up = (n >= 2) ? u + (size_t)(n - 2) * (size_t)M : NULL;
        double *yn = y + (size_t)(n - 1) * (size_t)M;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            double left = (i > 0) ? un[i - 1] : 0.0;
            double right = (i + 1 < M) ? un[i + 1] : 0.0;
            double s = a[0] * un[i] + 0.5 * e * (2.0 * un[i] - left - right);
            if (up) {
                double pl = (i > 0) ? up[i - 1] : 0.0;
                double pr = (i + 1 < M) ? up[i + 1] : 0.0;
                s += 0.5 * e * (2.0 * up[i] - pl - pr);
            }
            for (int64_t j = 1; j < n; ++j) s += a[n - j] * u[(size_t)(j - 1) * (size_t)M + (size_t)i];
            yn[i] = s;
        }
    }
    free(a);
    return ORACLE_OK;
}

/* One sine mode of oracle_solve_cn (eigenvalue lam of K, v^0 = v0):
 *   (a_0 + lam/2) v^n = g^n - rho_n v0 + psi_n phihat - sum_{j<n} a_{n-j} v^j - (lam/2) v^{n-1}. */
int oracle_mode_cn(double gamma, double T, int64_t N, double lam, const double *g, double v0, double phihat,
                   double *v)
{
    if (regime_of(gamma) != 1 || !(T > 0.0) || N < 1 || !g || !v) return ORACLE_EARG;
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi = (double *)malloc(sizeof(double) * (size_t)N);
    if (!a || !rho || !psi) { free(a); free(rho); free(psi); return ORACLE_ENOMEM; }
    oracle_weights(gamma, T, N, NULL, a, rho, psi, NULL, NULL, NULL, NULL);
    const double d = a[0] + 0.5 * lam;
    for (int64_t n = 1; n <= N; ++n) {
        double s = g[n - 1] - rho[n - 1] * v0 + psi[n - 1] * phihat;
        for (int64_t j = 1; j < n; ++j) s -= a[n - j] * v[j - 1];
        s -= 0.5 * lam * (n == 1 ? v0 : v[n - 2]);
        v[n - 1] = s / d;
    }
    free(a); free(rho); free(psi);
    return ORACLE_OK;
}

/*
 * Advection equations D_t^gamma u + u_x = f on (x0, x1) (a = 1), inflow value
 * u(x0, t) = 0, by time stepping; the unknowns are x_i = x0 + i h, i = 1..M,
 * h = (x1 - x0)/(M + 1), and U_0 = 0.
 *   0<gamma<1, Scheme 2 (eq. e12, e13): the L1 formula of Scheme 4 (weights
 *     a_m, rho_n of the diffusion case) averaged over x_i and x_{i-1}, and
 *     the difference (U_i - U_{i-1})/h, at the midpoint x_{i-1/2}:
 *       (1/2)[a_0 (U_i^n + U_{i-1}^n) + sum_{j<n} a_{n-j} (U_i^j + U_{i-1}^j)
 *             + rho_n (u0_i + u0_{i-1})] + (U_i^n - U_{i-1}^n)/h = f(x_{i-1/2}, t_n);
 *     the u0 term is read as for Scheme 4 (telescoping, rho_n = -mu b_{n-1}).
 *   1<gamma<2, Scheme 3 (eq. e15-e17): the diffusion-wave weights with the
 *     backward difference at x_i:
 *       a_0 U_i^n + sum_{j<n} a_{n-j} U_i^j + (U_i^n - U_{i-1}^n)/h
 *         = f(x_i, t_{n-1/2}) - rho_n u0_i + psi_n phi_i.
 *   Each step is a forward sweep in i.  f[n-1][i-1] holds the source where
 *   the scheme samples it (x_i - h/2 for Scheme 2, x_i for Scheme 3); u0[i-1]
 *   is u0(x_i) (u0(x0) = 0 by the inflow condition).
 */
int oracle_solve_adv(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                     const double *f, const double *u0, const double *phi, double *u, int nthreads)
{
    int reg = regime_of(gamma);
    if (reg < 0 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !f || !u) return ORACLE_EARG;
    set_threads(nthreads);
    const double h = (x1 - x0) / (double)(M + 1);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi = (double *)malloc(sizeof(double) * (size_t)N);
    double *r = (double *)malloc(sizeof(double) * (size_t)M);
    if (!a || !rho || !psi || !r) {
        free(a); free(rho); free(psi); free(r);
        return ORACLE_ENOMEM;
    }
    oracle_weights(gamma, T, N, NULL, a, rho, psi, NULL, NULL, NULL, NULL);
    for (int64_t n = 1; n <= N; ++n) {
        const double *fn = f + (size_t)(n - 1) * (size_t)M;
        double *un = u + (size_t)(n - 1) * (size_t)M;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            double s;
            if (reg == 0) {
                double w0 = u0 ? u0[i] + (i > 0 ? u0[i - 1] : 0.0) : 0.0;
                s = 2.0 * fn[i] - rho[n - 1] * w0;
                for (int64_t j = 1; j < n; ++j) {
                    const double *uj = u + (size_t)(j - 1) * (size_t)M;
                    s -= a[n - j] * (uj[i] + (i > 0 ? uj[i - 1] : 0.0));
                }
            } else {
                s = fn[i];
                if (u0) s -= rho[n - 1] * u0[i];
                if (phi) s += psi[n - 1] * phi[i];
                for (int64_t j = 1; j < n; ++j) s -= a[n - j] * u[(size_t)(j - 1) * (size_t)M + (size_t)i];
            }
            r[i] = s;
        }
        /* forward sweep in i */
        double prev = 0.0;
        for (int64_t i = 0; i < M; ++i) {
            if (reg == 0)
                un[i] = (r[i] - (a[0] - 2.0 / h) * prev) / (a[0] + 2.0 / h);
            else
                un[i] = (r[i] + prev / h) / (a[0] + 1.0 / h);
            prev = un[i];
        }
    }
    free(a); free(rho); free(psi); free(r);
    return ORACLE_OK;
}

static double vdot(int64_t n, const double *x, const double *y);

/*
 * Scheme 1 (eq. e7): the two-sided fractional ODE
 *   D_t^gamma u + tD_1^gamma u + u = f on (0, 1), u(0) = u(1) = 0, 0<gamma<1,
 * with the L1 formula from the left at t_i and its mirror from the right
 * (eq. e4, e5), tau = 1/N, unknowns u_1 .. u_{N-1}.  The matrix is
 * symmetric Toeplitz (Theorem 1): diagonal 1 + 2 mu G_0, and at distance k
 * the weight mu (G_k - G_{k-1}) = a_k of the diffusion case.
 * oracle_ode_column writes that first column c[0..N-2].
 */
int oracle_ode_column(double gamma, int64_t N, double *c)
{
    if (regime_of(gamma) != 0 || N < 2 || !c) return ORACLE_EARG;
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    if (!a) return ORACLE_ENOMEM;
    oracle_weights(gamma, 1.0, N, NULL, a, NULL, NULL, NULL, NULL, NULL, NULL);
    c[0] = 1.0 + 2.0 * a[0];
    for (int64_t k = 1; k < N - 1; ++k) c[k] = a[k];
    free(a);
    return ORACLE_OK;
}

/*
 * Conjugate gradients for Scheme 1 as listed in section 2.2: r_0 = f - A u_0,
 * w_1 = r_0; each step takes the step length |r|^2 / <w, A w>, updates u and
 * r, and the next direction r + (|r_new|^2 / |r_old|^2) w.  The products A w
 * are the symmetric Toeplitz matrix from its definition (O(n^2)); the paper
 * makes them fast by a circulant embedding (e10).  Reading: the iteration
 * stops once |r| <= rtol |f| (the listing leaves the test open).
 *   f, u [N-1]: u holds the initial guess when use_guess != 0
 *   out[0] = steps, out[1] = 1 if converged; *relres = |f - A u| / |f|
 *   recomputed; hist (NULL or maxit + 1) = |r_k| / |f| from the recurrence.
 */
int oracle_ode_cg(double gamma, int64_t N, const double *f, double *u, int maxit, double rtol, int use_guess,
                  int *out, double *relres, double *hist)
{
    if (regime_of(gamma) != 0 || N < 2 || !f || !u || !out || !relres || maxit < 0 || !(rtol >= 0.0))
        return ORACLE_EARG;
    const int64_t n = N - 1;
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *Aw = (double *)malloc(sizeof(double) * (size_t)n);
    if (!c || !r || !w || !Aw) {
        free(c); free(r); free(w); free(Aw);
        return ORACLE_ENOMEM;
    }
    oracle_ode_column(gamma, N, c);
    if (!use_guess)
        for (int64_t i = 0; i < n; ++i) u[i] = 0.0;
#define TOEP_MV(x, y)                                                   \
    for (int64_t i = 0; i < n; ++i) {                                   \
        double s = 0.0;                                                 \
        for (int64_t j = 0; j < n; ++j) s += c[i > j ? i - j : j - i] * (x)[j]; \
        (y)[i] = s;                                                     \
    }
    TOEP_MV(u, Aw)
    for (int64_t i = 0; i < n; ++i) r[i] = f[i] - Aw[i];
    const double fn = sqrt(vdot(n, f, f));
    double rr = vdot(n, r, r);
    out[0] = 0;
    out[1] = 0;
    if (hist) hist[0] = fn > 0.0 ? sqrt(rr) / fn : 0.0;
    for (int64_t i = 0; i < n; ++i) w[i] = r[i];
    int it = 0;
    while (it < maxit && sqrt(rr) > rtol * fn) {
        TOEP_MV(w, Aw)
        const double kap = rr / vdot(n, w, Aw);
        for (int64_t i = 0; i < n; ++i) u[i] += kap * w[i];
        for (int64_t i = 0; i < n; ++i) r[i] -= kap * Aw[i];
        const double rn = vdot(n, r, r);
        ++it;
        if (hist) hist[it] = fn > 0.0 ? sqrt(rn) / fn : 0.0;
        const double bet = rn / rr;
        for (int64_t i = 0; i < n; ++i) w[i] = r[i] + bet * w[i];
        rr = rn;
    }
    TOEP_MV(u, Aw)
#undef TOEP_MV
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (f[i] - Aw[i]) * (f[i] - Aw[i]);
    out[0] = it;
    *relres = fn > 0.0 ? sqrt(s) / fn : 0.0;
    out[1] = *relres <= rtol * (1.0 + 1e-6) || sqrt(rr) <= rtol * fn;
    free(c); free(r); free(w); free(Aw);
    return ORACLE_OK;
}

static double vdot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/*
 * Restarted GMRES(m) for the same block system: the fast iterative method
 * the paper uses for Scheme 4 (section 3.1): an Arnoldi process with
 * modified Gram-Schmidt builds an orthonormal basis V of the Krylov space of
 * the residual, and the update V y minimises || beta e_1 - H y ||_2 over the
 * (j+1) x j Hessenberg matrix H; the method restarts after m steps.  The
 * operator products here are the plain O(M N^2) definition, not the
 * circulant-embedding FFT the paper uses to make them fast (the same
 * products, evaluated slowly).
 *
 * Readings where the paper is silent:
 *   - the least-squares problem is solved by Givens rotations applied as the
 *     columns of H arrive, so |g_{j+1}| is the residual norm of the current
 *     iterate after every step; the cycle stops early once it is at most
 *     rtol ||b||, and the method stops when the residual recomputed from
 *     its definition after a cycle is at most rtol ||b||;
 *   - precond = 1 applies the block-diagonal matrix P = diag(a_0 I + K) on
 *     the right (GMRES on A P^-1; the update is P^-1 V y).  The paper uses
 *     no preconditioner (precond = 0).
 *
 *   f, u0, phi   as in oracle_solve; b = F - rho_n u0 + psi_n phi
 *   u [N][M]     in: initial guess when use_guess != 0; out: the iterate
 *   restart      m >= 1;  maxit: total Arnoldi steps >= 0
 *   hist         NULL or maxit + 1 doubles: hist[0] = ||r_0|| / ||b||,
 *                hist[k] = the least-squares residual after step k, / ||b||
 *   out[0] = steps taken, out[1] = cycles, out[2] = 1 if converged;
 *   *relres = ||b - A u|| / ||b|| recomputed at the end (0 when b = 0).
 */
int oracle_gmres(double gamma, double T, double x0, double x1, int64_t M, int64_t N,
                 const double *f, const double *u0, const double *phi, double *u,
                 int restart, int maxit, double rtol, int precond, int use_guess,
                 int *out, double *relres, double *hist, int nthreads)
{
    if (regime_of(gamma) < 0 || !(T > 0.0) || !(x1 > x0) || M < 1 || N < 1 || !f || !u || !out || !relres)
        return ORACLE_EARG;
    if (restart < 1 || maxit < 0 || !(rtol >= 0.0) || precond < 0 || precond > 1) return ORACLE_EARG;
    set_threads(nthreads);
    const int64_t n = M * N;
    const int m = restart;
    double h = (x1 - x0) / (double)(M + 1);
    double e = 1.0 / (h * h);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi = (double *)malloc(sizeof(double) * (size_t)N);
    double *cp = (double *)malloc(sizeof(double) * (size_t)M);
    double *inv = (double *)malloc(sizeof(double) * (size_t)M);
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(m + 1));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    int rc = ORACLE_OK;
    if (!a || !rho || !psi || !cp || !inv || !b || !w || !z || !V || !H || !cs || !sn || !g || !y) {
        rc = ORACLE_ENOMEM;
        goto done;
    }
    oracle_weights(gamma, T, N, NULL, a, rho, psi, NULL, NULL, NULL, NULL);
    thomas_factor(M, a[0] + 2.0 * e, -e, cp, inv);
#define HH(i, j) H[(size_t)(i) * (size_t)m + (size_t)(j)]
    for (int64_t r = 0; r < N; ++r)
        for (int64_t i = 0; i < M; ++i) {
            double s = f[r * M + i];
            if (u0) s -= rho[r] * u0[i];
            if (phi) s += psi[r] * phi[i];
            b[r * M + i] = s;
        }
    if (!use_guess)
        for (int64_t i = 0; i < n; ++i) u[i] = 0.0;
    const double bnorm = sqrt(vdot(n, b, b));
    out[0] = 0;
    out[1] = 0;
    out[2] = 0;
    if (bnorm == 0.0) {
        /* the solution of A u = 0 */
        for (int64_t i = 0; i < n; ++i) u[i] = 0.0;
        out[2] = 1;
        *relres = 0.0;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    /* r = b - A u */
    apply_rows(M, N, a, e, u, w);
    for (int64_t i = 0; i < n; ++i) w[i] = b[i] - w[i];
    double beta = sqrt(vdot(n, w, w));
    if (hist) hist[0] = beta / bnorm;
    int it = 0;
    while (beta > rtol * bnorm && it < maxit) {
        out[1]++;
        for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && it < maxit; ++j) {
            double *vj = V + (size_t)j * (size_t)n;
            /* w = A P^-1 v_j */
            for (int64_t i = 0; i < n; ++i) z[i] = vj[i];
            if (precond)
                for (int64_t r = 0; r < N; ++r) thomas_solve(M, -e, cp, inv, z + r * M);
            apply_rows(M, N, a, e, z, w);
            /* modified Gram-Schmidt against v_0 .. v_j */
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * (size_t)n;
                double hij = vdot(n, w, vi);
                HH(i, j) = hij;
                for (int64_t q = 0; q < n; ++q) w[q] -= hij * vi[q];
            }
            double hn = sqrt(vdot(n, w, w));
            HH(j + 1, j) = hn;
            /* earlier rotations on column j, then the one that zeroes H[j+1][j] */
            for (int i = 0; i < j; ++i) {
                double t0 = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                double t1 = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
                HH(i, j) = t0;
                HH(i + 1, j) = t1;
            }
            double rr = hypot(HH(j, j), hn);
            cs[j] = HH(j, j) / rr;
            sn[j] = hn / rr;
            HH(j, j) = rr;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            if (hist) hist[it] = fabs(g[j + 1]) / bnorm;
            if (hn == 0.0 || fabs(g[j + 1]) <= rtol * bnorm) break;
            double *vn = V + (size_t)(j + 1) * (size_t)n;
            for (int64_t q = 0; q < n; ++q) vn[q] = w[q] / hn;
        }
        /* y = R^-1 g (back substitution), u += P^-1 V y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < k; ++q) s -= HH(i, q) * y[q];
            y[i] = s / HH(i, i);
        }
        for (int64_t q = 0; q < n; ++q) z[q] = 0.0;
        for (int i = 0; i < k; ++i) {
            const double *vi = V + (size_t)i * (size_t)n;
            for (int64_t q = 0; q < n; ++q) z[q] += y[i] * vi[q];
        }
        if (precond)
            for (int64_t r = 0; r < N; ++r) thomas_solve(M, -e, cp, inv, z + r * M);
        for (int64_t q = 0; q < n; ++q) u[q] += z[q];
        /* residual from its definition */
        apply_rows(M, N, a, e, u, w);
        for (int64_t i = 0; i < n; ++i) w[i] = b[i] - w[i];
        beta = sqrt(vdot(n, w, w));
    }
#undef HH
    out[0] = it;
    out[2] = beta <= rtol * bnorm;
    *relres = beta / bnorm;
done:
    free(a); free(rho); free(psi); free(cp); free(inv); free(b); free(w); free(z);
    free(V); free(H); free(cs); free(sn); free(g); free(y);
    return rc;
}
