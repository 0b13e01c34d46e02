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

// (m+1)^q - 3 m^q + 3 (m-1)^q - (m-2)^q for m >= 8
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

__global__ void k_weights(int regime, double p, double coef, double dcoef, double tau, int64_t N,
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
        double diff = (m >= 8) ? third_diff_series(m, p) : (b2 - 2.0 * b1 + b0);
        am = coef * diff;
        dam = dcoef * diff + coef * (d2 - 2.0 * d1 + d0);
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
    if (rho) rho[m] = r;
    if (drho) drho[m] = dr;
    if (psi) psi[m] = s;
    if (dpsi) dpsi[m] = ds;
}

hipError_t launch_weights(hipStream_t st, int regime, double p, double coef, double dcoef, double tau, int64_t N,
                          double *b, double *a, double *rho, double *psi, double *da, double *drho, double *dpsi)
{
    int bs = 256;
    int64_t nb = (N + bs - 1) / bs;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)nb), dim3(bs), 0, st, regime, p, coef, dcoef, tau, N, b, a, rho,
                       psi, da, drho, dpsi);
    return hipGetLastError();
}

}  // namespace fs
