/* Sanitizer driver for the oracle (test infrastructure): every entry point of
 * oracle/oracle.c on small shapes, with buffers of exactly the documented
 * sizes in separate heap blocks (so an access one past the end is reported),
 * the edge cases M = 1, N = 1, N = 2, both regimes, and argument errors.
 * Built with -fsanitize=address,undefined by tests/test_sanitize_host.py;
 * exits non-zero on the first unexpected return code. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_weights(double, double, int64_t, double *, double *, double *, double *, double *, double *, double *,
                   double *);
int oracle_solve(double, double, double, double, int64_t, int64_t, int64_t, const double *, const double *,
                 const double *, double *, int);
int oracle_apply(double, double, double, double, int64_t, int64_t, const double *, double *, int);
int oracle_adjoint(double, double, double, double, int64_t, int64_t, const double *, const double *, const double *,
                   const double *, double *, double *, int);
int oracle_mode(double, double, int64_t, double, const double *, double, double, double *);
int oracle_solve_cn(double, double, double, double, int64_t, int64_t, const double *, const double *, const double *,
                    double *, int);
int oracle_apply_cn(double, double, double, double, int64_t, int64_t, const double *, double *, int);
int oracle_mode_cn(double, double, int64_t, double, const double *, double, double, double *);
int oracle_solve_adv(double, double, double, double, int64_t, int64_t, const double *, const double *,
                     const double *, double *, int);
int oracle_ode_column(double, int64_t, double *);
int oracle_ode_cg(double, int64_t, const double *, double *, int, double, int, int *, double *, double *);
int oracle_gmres(double, double, double, double, int64_t, int64_t, const double *, const double *, const double *,
                 double *, int, int, double, int, int, int *, double *, double *, int);

static int fails = 0;

static void expect(int got, int want, const char *what, double g, long long M, long long N)
{
    if ((want == 0 && got != 0) || (want != 0 && got == 0)) {
        fprintf(stderr, "%s gamma=%g M=%lld N=%lld: returned %d\n", what, g, M, N, got);
        ++fails;
    }
}

static double *vec(int64_t n, unsigned seed)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        seed = seed * 1664525u + 1013904223u;
        p[i] = (double)(seed >> 8) / 16777216.0 - 0.5;
    }
    return p;
}

static void all_finite(const double *x, int64_t n, const char *what)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) {
            fprintf(stderr, "%s: non-finite output at %lld\n", what, (long long)i);
            ++fails;
            return;
        }
}

int main(void)
{
    const double gammas[] = {0.3, 0.9, 1.2, 1.8};
    const int64_t Ms[] = {1, 2, 5};
    const int64_t Ns[] = {1, 2, 7};
    for (int gi = 0; gi < 4; ++gi) {
        const double g = gammas[gi];
        for (int ni = 0; ni < 3; ++ni) {
            const int64_t N = Ns[ni];
            double *b = vec(N, 1), *a = vec(N, 2), *rho = vec(N, 3), *psi = vec(N, 4);
            double *da = vec(N, 5), *drho = vec(N, 6), *dpsi = vec(N, 7), *scal = vec(2, 8);
            expect(oracle_weights(g, 1.0, N, b, a, rho, psi, da, drho, dpsi, scal), 0, "weights", g, 0, N);
            all_finite(a, N, "weights a");
            free(b), free(a), free(rho), free(psi), free(da), free(drho), free(dpsi), free(scal);
            double *gm = vec(N, 9), *v = vec(N, 10);
            expect(oracle_mode(g, 1.0, N, 3.5, gm, 0.4, 0.2, v), 0, "mode", g, 1, N);
            all_finite(v, N, "mode");
            if (g > 1.0) {
                expect(oracle_mode_cn(g, 1.0, N, 3.5, gm, 0.4, 0.2, v), 0, "mode_cn", g, 1, N);
                all_finite(v, N, "mode_cn");
            }
            free(gm), free(v);
            for (int mi = 0; mi < 3; ++mi) {
                const int64_t M = Ms[mi], MN = M * N;
                double *f = vec(MN, 11), *u0 = vec(M, 12), *phi = vec(M, 13), *u = vec(MN, 14);
                double *y = vec(MN, 15), *lam = vec(MN, 16), dl = 0.0;
                expect(oracle_solve(g, 1.0, 0.0, 1.0, M, N, N, f, u0, phi, u, 1), 0, "solve", g, M, N);
                all_finite(u, MN, "solve");
                expect(oracle_solve(g, 1.0, 0.0, 1.0, M, N, N, f, NULL, NULL, u, 1), 0, "solve no u0", g, M, N);
                expect(oracle_apply(g, 1.0, 0.0, 1.0, M, N, u, y, 1), 0, "apply", g, M, N);
                all_finite(y, MN, "apply");
                expect(oracle_adjoint(g, 1.0, 0.0, 1.0, M, N, f, u, u0, phi, lam, &dl, 1), 0, "adjoint", g, M, N);
                all_finite(lam, MN, "adjoint");
                if (!isfinite(dl)) ++fails;
                if (g > 1.0) {
                    expect(oracle_solve_cn(g, 1.0, 0.0, 1.0, M, N, f, u0, phi, u, 1), 0, "solve_cn", g, M, N);
                    expect(oracle_apply_cn(g, 1.0, 0.0, 1.0, M, N, u, y, 1), 0, "apply_cn", g, M, N);
                    all_finite(y, MN, "apply_cn");
                }
                expect(oracle_solve_adv(g, 1.0, 0.0, 1.0, M, N, f, u0, phi, u, 1), 0, "solve_adv", g, M, N);
                all_finite(u, MN, "solve_adv");
                const int maxit = 12;
                int out[3] = {0, 0, 0};
                double rel = 0.0, *hist = vec(maxit + 1, 17);
                expect(oracle_gmres(g, 1.0, 0.0, 1.0, M, N, f, u0, phi, u, 3, maxit, 1e-10, 0, 0, out, &rel, hist, 1),
                       0, "gmres", g, M, N);
                expect(oracle_gmres(g, 1.0, 0.0, 1.0, M, N, f, u0, phi, u, 2, maxit, 1e-10, 1, 1, out, &rel, hist, 1),
                       0, "gmres precond", g, M, N);
                free(hist);
                free(f), free(u0), free(phi), free(u), free(y), free(lam);
            }
        }
    }
    /* Scheme 1 (0 < gamma < 1, N >= 2: N - 1 unknowns) */
    for (int64_t N = 2; N <= 9; ++N) {
        const int64_t n = N - 1;
        double *c = vec(n, 20), *f = vec(n, 21), *u = vec(n, 22), *hist = vec(31, 23), rel = 0.0;
        int out[2] = {0, 0};
        expect(oracle_ode_column(0.4, N, c), 0, "ode_column", 0.4, 1, N);
        expect(oracle_ode_cg(0.4, N, f, u, 30, 1e-12, 0, out, &rel, hist), 0, "ode_cg", 0.4, 1, N);
        all_finite(u, n, "ode_cg");
        free(c), free(f), free(u), free(hist);
    }
    /* argument errors: each returns an error before touching memory */
    double one = 1.0, z[4] = {0, 0, 0, 0};
    int out[3];
    double rel;
    expect(oracle_weights(1.0, 1.0, 4, z, z, z, z, NULL, NULL, NULL, NULL), -1, "weights gamma=1", 1.0, 0, 4);
    expect(oracle_weights(0.5, 1.0, 0, z, z, z, z, NULL, NULL, NULL, NULL), -1, "weights N=0", 0.5, 0, 0);
    expect(oracle_solve(0.5, 1.0, 0.0, 1.0, 0, 4, 4, z, NULL, NULL, z, 1), -1, "solve M=0", 0.5, 0, 4);
    expect(oracle_solve(0.5, 1.0, 1.0, 0.0, 1, 1, 1, &one, NULL, NULL, z, 1), -1, "solve x1<x0", 0.5, 1, 1);
    expect(oracle_solve(0.5, 1.0, 0.0, 1.0, 1, 1, 1, NULL, NULL, NULL, z, 1), -1, "solve f=NULL", 0.5, 1, 1);
    expect(oracle_solve(2.0, 1.0, 0.0, 1.0, 1, 1, 1, &one, NULL, NULL, z, 1), -1, "solve gamma=2", 2.0, 1, 1);
    expect(oracle_solve_cn(0.5, 1.0, 0.0, 1.0, 1, 1, &one, NULL, NULL, z, 1), -1, "solve_cn gamma<1", 0.5, 1, 1);
    expect(oracle_ode_cg(1.5, 4, z, z, 5, 1e-8, 0, out, &rel, NULL), -1, "ode_cg gamma>1", 1.5, 1, 4);
    expect(oracle_ode_cg(0.5, 1, z, z, 5, 1e-8, 0, out, &rel, NULL), -1, "ode_cg N=1", 0.5, 1, 1);
    expect(oracle_gmres(0.5, 1.0, 0.0, 1.0, 1, 1, &one, NULL, NULL, z, 0, 5, 1e-8, 0, 0, out, &rel, NULL, 1), -1,
           "gmres restart=0", 0.5, 1, 1);
    expect(oracle_gmres(0.5, 1.0, 0.0, 1.0, 1, 1, &one, NULL, NULL, z, 2, 5, 1e-8, 2, 0, out, &rel, NULL, 1), -1,
           "gmres precond=2", 0.5, 1, 1);
    if (fails) {
        fprintf(stderr, "%d failures\n", fails);
        return 1;
    }
    printf("oracle driver: all calls clean\n");
    return 0;
}
