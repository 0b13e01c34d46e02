// L1 weights of section 3 in float64, cancellation-free.
//
//   0<gamma<1 (Scheme 4):  p = 1-gamma, coef = mu = tau^-gamma / Gamma(2-gamma)
//     b_k = G_k = (k+1)^p - k^p,  a_0 = mu,  a_m = mu (b_m - b_{m-1}),
//     rho_n = -mu b_{n-1},  psi_n = 0.
//   1<gamma<2 (eq. e17 and the Toeplitz matrix of Scheme 3's new procedure):
//     q = 2-gamma, coef = c = tau^-gamma / Gamma(3-gamma), b_k = M_k,
//     b_{-1} = b_{-2} = 0, a_m = c (b_{m-2} - 2 b_{m-1} + b_m),
//     rho_n = c (b_{n-2} - b_{n-1}),  psi_n = c tau b_{n-1}.
//
// b_k is formed as k^p expm1(p log1p(1/k)), never as a difference of powers.
// For large m the first and second differences of b are summed from their
// binomial series in x = 1/m, which has no cancellation:
//   (m+1)^p - 2 m^p + (m-1)^p            = 2 m^p sum_{k>=1} C(p,2k) x^{2k}
//   (m+1)^q - 3 m^q + 3 (m-1)^q - (m-2)^q = m^q sum_{k>=3} C(q,k) (1 + 3(-1)^k - (-2)^k) x^k
// Gamma-derivatives use d b_k/dp = ln(k) b_k + log1p(1/k) (k+1)^p (two
// non-negative terms) and d/dgamma = -d/dp.
//
// The first four differences (m < 4), where the series in 1/m does not yet
// converge and the direct differences of b cancel (by up to 7 bits at m = 3
// for orders near 1), are formed once on the host in x87 extended precision
// (64-bit significand) and passed to the kernel, so every a_m, rho_n and
// their derivatives reach float64 within about one rounding.
#include <cmath>

#include "common.hpp"

namespace fs {

__device__ __forceinline__ double wb(int64_t k, double p)
{
    if (k < 0) return 0.0;
    if (k == 0) return 1.0;
    double kd = (double)k;
    return pow(kd, p) * expm1(p * log1p(1.0 / kd));
}

// d b_k / d gamma
__device__ __forceinline__ double wdb(int64_t k, double p)
{
    if (k <= 0) return 0.0;
    double kd = (double)k;
    return -(log(kd) * wb(k, p) + log1p(1.0 / kd) * pow(kd + 1.0, p));
}

// (m+1)^p - 2 m^p + (m-1)^p for m >= 4
__device__ double second_diff_series(int64_t m, double p)
{
    double x = 1.0 / (double)m, x2 = x * x;
    double t = 0.5 * p * (p - 1.0) * x2;  // C(p,2) x^2
    double s = t;
    for (int k = 1; k < 24; ++k) {
        double j = 2.0 * k;
        t *= (p - j) * (p - j - 1.0) / ((j + 1.0) * (j + 2.0)) * x2;
        s += t;
        if (fabs(t) < 1e-19 * fabs(s)) break;
    }
    return 2.0 * pow((double)m, p) * s;
}

// (m+1)^q - 3 m^q + 3 (m-1)^q - (m-2)^q for m >= 4 (the terms fall off like
// (2/m)^k, so the loop reaches the float64 floor within its 64 terms)
__device__ double third_diff_series(int64_t m, double q)
{
    double x = 1.0 / (double)m;
    double u = 1.0;   // C(q,k) x^k
    double s = 0.0;
    double pm = 1.0;  // (-1)^k
    double p2 = 1.0;  // (-2)^k
    for (int k = 1; k < 64; ++k) {
        u *= (q - (double)(k - 1)) / (double)k * x;
        pm = -pm;
        p2 *= -2.0;
        if (k >= 3) {
            double term = u * (1.0 + 3.0 * pm - p2);
            s += term;
            if (fabs(term) < 1e-19 * fabs(s)) break;
        }
    }
    return pow((double)m, q) * s;
}

// a_m, da_m/dgamma, rho_{m+1}, drho_{m+1}/dgamma for m < 4
struct WeightHead {
    double a[4], da[4], rho[4], drho[4];
};

__global__ void k_weights(WeightHead head, int regime, double p, double coef, double dcoef, double tau, int64_t N,
                          double *__restrict__ b, double *__restrict__ a, double *__restrict__ rho,
                          double *__restrict__ psi, double *__restrict__ da, double *__restrict__ drho,
                          double *__restrict__ dpsi)
{
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= N) return;
    double b0 = wb(m, p), b1 = wb(m - 1, p), b2 = wb(m - 2, p);
    double d0 = wdb(m, p), d1 = wdb(m - 1, p), d2 = wdb(m - 2, p);
    if (b) b[m] = b0;
    double am, dam;
    if (regime == 0) {
        // b_m - b_{m-1} = (m+1)^p - 2 m^p + (m-1)^p for m >= 1
        double diff = (m >= 4) ? second_diff_series(m, p) : (b0 - b1);
        am = coef * diff;
        dam = dcoef * diff + coef * (d0 - d1);
    } else {
        // from m = 4 on the series: the direct second difference of b loses
        // about log2(m^2) bits to cancellation (measured up to 1e-14 relative
        // at m = 5..7 against 40-digit decimal)
        double diff = (m >= 4) ? third_diff_series(m, p) : (b2 - 2.0 * b1 + b0);
        am = coef * diff;
        dam = dcoef * diff + coef * (d2 - 2.0 * d1 + d0);
    }
    if (m < 4) {
        am = head.a[m];
        dam = head.da[m];
    }
    if (a) a[m] = am;
    if (da) da[m] = dam;
    // step n = m + 1
    double r, dr, s, ds;
    if (regime == 0) {
        // rho_n = -mu b_{n-1} = -mu b_m
        r = -coef * b0;
        dr = -dcoef * b0 - coef * d0;
        s = 0.0;
        ds = 0.0;
    } else {
        // rho_n = c (b_{n-2} - b_{n-1}) = c (b_{m-1} - b_m) = -c ((m+1)^q - 2 m^q + (m-1)^q),
        // psi_n = c tau b_m
        r = (m >= 4) ? -coef * second_diff_series(m, p) : coef * (b1 - b0);
        dr = dcoef * (b1 - b0) + coef * (d1 - d0);
        s = coef * tau * b0;
        ds = tau * (dcoef * b0 + coef * d0);
    }
    if (m < 4) {
        r = head.rho[m];
        dr = head.drho[m];
    }
    if (rho) rho[m] = r;
    if (drho) drho[m] = dr;
    if (psi) psi[m] = s;
    if (dpsi) dpsi[m] = ds;
}

namespace {

typedef long double xd;

xd xb(int64_t k, xd p)
{
    if (k < 0) return 0.0L;
    if (k == 0) return 1.0L;
    const xd kd = (xd)k;
    return powl(kd, p) * expm1l(p * log1pl(1.0L / kd));
}

// d b_k / d gamma
xd xdb(int64_t k, xd p)
{
    if (k <= 0) return 0.0L;
    const xd kd = (xd)k;
    return -(logl(kd) * xb(k, p) + log1pl(1.0L / kd) * powl(kd + 1.0L, p));
}

WeightHead weight_head(int regime, double p, double coef, double dcoef)
{
    WeightHead h{};
    const xd P = p, C = coef, DC = dcoef;
    for (int m = 0; m < 4; ++m) {
        const xd b0 = xb(m, P), b1 = xb(m - 1, P), b2 = xb(m - 2, P);
        const xd d0 = xdb(m, P), d1 = xdb(m - 1, P), d2 = xdb(m - 2, P);
        xd diff, ddiff, r, dr;
        if (regime == 0) {
            diff = b0 - b1;
            ddiff = d0 - d1;
            r = -C * b0;
            dr = -DC * b0 - C * d0;
        } else {
            diff = b2 - 2.0L * b1 + b0;
            ddiff = d2 - 2.0L * d1 + d0;
            r = C * (b1 - b0);
            dr = DC * (b1 - b0) + C * (d1 - d0);
        }
        h.a[m] = (double)(C * diff);
        h.da[m] = (double)(DC * diff + C * ddiff);
        h.rho[m] = (double)r;
        h.drho[m] = (double)dr;
    }
    return h;
}

}  // namespace

hipError_t launch_weights(hipStream_t st, int regime, double p, double coef, double dcoef, double tau, int64_t N,
                          double *b, double *a, double *rho, double *psi, double *da, double *drho, double *dpsi)
{
    int bs = 256;
    int64_t nb = (N + bs - 1) / bs;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)nb), dim3(bs), 0, st, weight_head(regime, p, coef, dcoef), regime,
                       p, coef, dcoef, tau, N, b, a, rho, psi, da, drho, dpsi);
    return hipGetLastError();
}

}  // namespace fs
