// One-dimensional complex FFT of a power-of-two length L (8 <= L <= 2^23)
// and the symmetric-Toeplitz product built on it (Scheme 1, eq. e10): the
// n x n symmetric Toeplitz matrix with first column c is the leading block of
// the L-periodic circulant whose first column is c followed by zeros and by
// c_{n-1} .. c_1 (any L >= 2n - 1), and a circulant is diagonalised by the
// DFT, so A x = first n entries of IDFT( DFT(ĉ) * DFT(x padded with zeros) ).
//
// The transform is the self-sorting (Stockham) formulation: each pass takes
// L/R butterflies of radix R (64 for six bits of log2 L at a time, one pass
// of 2 .. 32 for the rest); butterfly j of a pass whose sub-transforms have
// length Ns reads the R inputs j + r L/R (consecutive threads read consecutive
// elements), twiddles input r by w^(r k) with k = j mod Ns and w the
// (Ns R)-th root of unity, transforms, and writes output r to
// (j - k) R + k + r Ns, so the result comes out in natural order with no
// bit-reversal pass.  The zero padding of x, the product with the circulant's
// spectrum (real, the column being symmetric; pre-divided by L) and the real
// part of the output are fused into the first forward, first inverse and last
// inverse pass, so one product costs the passes of two transforms.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace fs {

namespace {

struct c2 {
    double x, y;
};

__device__ __forceinline__ c2 cadd(c2 a, c2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c2 csub(c2 a, c2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c2 cmul(c2 a, c2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// sgn i z: +i z for sgn > 0, -i z for sgn < 0
__device__ __forceinline__ c2 cmuli(c2 z, double sgn) { return {-sgn * z.y, sgn * z.x}; }

// sum over the 64 lanes of a wavefront (every lane must take part)
__device__ __forceinline__ double wave_sum(double d)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    return d;
}

// X_k = sum_m v_m exp(sgn 2 pi i m k / R), in place, for R = 2, 4, 8
template <int R>
__device__ __forceinline__ void dft_small(c2 *v, double sgn)
{
    if constexpr (R == 2) {
        const c2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const c2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const c2 s13 = cadd(v[1], v[3]), d13 = cmuli(csub(v[1], v[3]), sgn);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else {
        static_assert(R == 8, "radix 2, 4 or 8");
        // even and odd halves by the radix-4 transform, then one radix-2 step
        // with the eighth roots of unity w^k, w = exp(sgn i pi / 4)
        c2 e[4] = {v[0], v[2], v[4], v[6]};
        c2 o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<4>(e, sgn);
        dft_small<4>(o, sgn);
        const double h = 0.70710678118654752440;  // 1/sqrt(2)
        o[1] = {h * (o[1].x - sgn * o[1].y), h * (o[1].y + sgn * o[1].x)};
        o[2] = cmuli(o[2], sgn);
        o[3] = {h * (-o[3].x - sgn * o[3].y), h * (-o[3].y + sgn * o[3].x)};
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
}

// One Stockham pass.  IN_REAL: the input is the real array xr of nx entries,
// zero beyond (first forward pass, Ns = 1).  SCALE: inputs are multiplied by
// the real spectrum S (first inverse pass, Ns = 1).  OUT_REAL: the real parts
// of outputs below nx go to yr and the rest is dropped (last inverse pass);
// with dotp, the workgroup's share of sum_o yr[o] xr[o] goes to
// dotp[blockIdx.x] (xr is then the product's input).  Workgroups are one
// wavefront; lanes past the end stay to the reduction.
template <int R, bool IN_REAL, bool SCALE, bool OUT_REAL>
__global__ void __launch_bounds__(64) k_fft1d_pass(const c2 *__restrict__ in, const double *__restrict__ xr,
                                                    const double *__restrict__ S, c2 *__restrict__ out,
                                                    double *__restrict__ yr, int64_t L, int64_t Ns, int64_t nx,
                                                    double sgn, const int32_t *__restrict__ skip,
                                                    double *__restrict__ dotp)
{
    if (skip && *skip) return;
    const int64_t q = L / R;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = j < q;
    c2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t idx = j + r * q;
        v[r] = {0.0, 0.0};
        if (!live) continue;
        if constexpr (IN_REAL)
            v[r] = {idx < nx ? xr[idx] : 0.0, 0.0};
        else
            v[r] = in[idx];
        if constexpr (SCALE) {
            const double s = S[idx];
            v[r] = {v[r].x * s, v[r].y * s};
        }
    }
    const int64_t k = j & (Ns - 1);
    if (Ns > 1) {
        // angle of w^(r k), in units of pi: sgn 2 r k / (Ns R)
        const double a = sgn * 2.0 * (double)k / (double)(Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            double sn, cs;
            sincospi(a * r, &sn, &cs);
            v[r] = cmul(v[r], c2{cs, sn});
        }
    }
    dft_small<R>(v, sgn);
    const int64_t base = (j - k) * R + k;
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t o = base + r * Ns;
        if (!live) continue;
        if constexpr (OUT_REAL) {
            if (o < nx) {
                yr[o] = v[r].x;
                if (dotp) d += v[r].x * xr[o];
            }
        } else {
            out[o] = v[r];
        }
    }
    if constexpr (OUT_REAL) {
        if (dotp) {
            d = wave_sum(d);
            if (threadIdx.x == 0) dotp[blockIdx.x] = d;
        }
    }
}

// Two-stage pass of radix R = R1 R2 (64 = 8 x 8, 32 = 4 x 8, 16 = 2 x 8):
// eight threads per butterfly, BPW butterflies per workgroup: 8, one
// wavefront (L = 2^18 gives 512 workgroups at radix 64, enough to reach
// every CU of a latency-bound pass), or 16 for the real-array passes at
// large L.  Input r = R2 n1 + n2 goes to thread n2 < R2; a
// radix-R1 transform over n1 gives Y[n2][k1], which is twiddled by
// w_R^(n2 k1), transposed through LDS, and transformed over n2 by thread
// k1 < R1, giving output k1 + R1 k2.
template <int R1, int R2, bool IN_REAL, bool SCALE, bool OUT_REAL, int BPW>
__global__ void __launch_bounds__(8 * BPW) k_fft1d_pass2(const c2 *__restrict__ in, const double *__restrict__ xr,
                                                    const double *__restrict__ S, c2 *__restrict__ out,
                                                    double *__restrict__ yr, int64_t L, int64_t Ns, int64_t nx,
                                                    double sgn, const int32_t *__restrict__ skip,
                                                    double *__restrict__ dotp)
{
    static_assert(R1 <= 8 && R2 <= 8 && R1 * R2 >= 16, "two stages of at most 8 points");
    static_assert(BPW == 8 || (BPW == 16 && !OUT_REAL), "the partial sums assume one wavefront per workgroup");
    constexpr int R = R1 * R2;
    if (skip && *skip) return;
    __shared__ c2 lds[BPW * 72];  // per butterfly 8 rows of 9 (one pad entry against bank conflicts)
    const int t = threadIdx.x & 7, g = threadIdx.x >> 3;
    const int64_t q = L / R;
    const int64_t j = (int64_t)blockIdx.x * BPW + g;
    const bool live = j < q;
    const int64_t k = j & (Ns - 1);
    c2 *row = lds + g * 72;
    if (t < R2) {
        c2 v[R1];
        const double a = sgn * 2.0 * (double)k / (double)(Ns * R);
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) {
            const int r = R2 * n1 + t;
            const int64_t idx = j + r * q;
            c2 x{0.0, 0.0};
            if (live) {
                if constexpr (IN_REAL)
                    x = {idx < nx ? xr[idx] : 0.0, 0.0};
                else
                    x = in[idx];
                if constexpr (SCALE) {
                    const double s = S[idx];
                    x = {x.x * s, x.y * s};
                }
            }
            if (Ns > 1 && r > 0) {
                double sn, cs;
                sincospi(a * r, &sn, &cs);
                x = cmul(x, c2{cs, sn});
            }
            v[n1] = x;
        }
        dft_small<R1>(v, sgn);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            c2 y = v[k1];
            if (t > 0 && k1 > 0) {
                double sn, cs;
                sincospi(sgn * 2.0 * (double)(t * k1) / (double)R, &sn, &cs);
                y = cmul(y, c2{cs, sn});
            }
            row[t * 9 + k1] = y;
        }
    }
    __syncthreads();
    const bool act = t < R1 && live;
    c2 v[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) v[n2] = row[n2 * 9 + t];  // in the row for every t < 8
    dft_small<R2>(v, sgn);
    const int64_t base = (j - k) * R + k;
    double d = 0.0;
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
        const int64_t o = base + (int64_t)(t + R1 * k2) * Ns;
        if (!act) continue;
        if constexpr (OUT_REAL) {
            if (o < nx) {
                yr[o] = v[k2].x;
                if (dotp) d += v[k2].x * xr[o];
            }
        } else {
            out[o] = v[k2];
        }
    }
    if constexpr (OUT_REAL) {
        if (dotp) {
            d = wave_sum(d);
            if (threadIdx.x == 0) dotp[blockIdx.x] = d;
        }
    }
}

// Passes that read a real array (x, or the spectrum) take 16 butterflies per
// workgroup for L >= 2^20, where HBM bounds them: with 8, a wavefront covers
// 64 B of that array, half a cache line, and the line is fetched twice.
template <int R1, int R2, bool IN_REAL, bool SCALE, bool OUT_REAL>
hipError_t pass2_go(hipStream_t st, const c2 *in, const double *xr, const double *S, c2 *out, double *yr, int64_t L,
                    int64_t Ns, int64_t nx, double sgn, const int32_t *skip, double *dotp)
{
    const int64_t q = L / (R1 * R2);
    if constexpr ((IN_REAL || SCALE) && !OUT_REAL) {
        if (L >= (int64_t(1) << 20)) {
            const unsigned g = (unsigned)((q + 15) / 16);
            hipLaunchKernelGGL((k_fft1d_pass2<R1, R2, IN_REAL, SCALE, OUT_REAL, 16>), dim3(g), dim3(128), 0, st, in,
                               xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
            return hipGetLastError();
        }
    }
    const unsigned g = (unsigned)((q + 7) / 8);
    hipLaunchKernelGGL((k_fft1d_pass2<R1, R2, IN_REAL, SCALE, OUT_REAL, 8>), dim3(g), dim3(64), 0, st, in, xr, S, out,
                       yr, L, Ns, nx, sgn, skip, dotp);
    return hipGetLastError();
}

template <int R, bool IN_REAL, bool SCALE, bool OUT_REAL>
hipError_t pass_go(hipStream_t st, const c2 *in, const double *xr, const double *S, c2 *out, double *yr, int64_t L,
                   int64_t Ns, int64_t nx, double sgn, const int32_t *skip, double *dotp)
{
    const int64_t q = L / R;
    const unsigned g = (unsigned)((q + 63) / 64);
    hipLaunchKernelGGL((k_fft1d_pass<R, IN_REAL, SCALE, OUT_REAL>), dim3(g), dim3(64), 0, st, in, xr, S, out, yr,
                       L, Ns, nx, sgn, skip, dotp);
    return hipGetLastError();
}

template <bool IN_REAL, bool SCALE, bool OUT_REAL>
hipError_t pass_radix(int R, hipStream_t st, const c2 *in, const double *xr, const double *S, c2 *out, double *yr,
                      int64_t L, int64_t Ns, int64_t nx, double sgn, const int32_t *skip, double *dotp = nullptr)
{
    switch (R) {
    case 64: return pass2_go<8, 8, IN_REAL, SCALE, OUT_REAL>(st, in, xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
    case 32: return pass2_go<4, 8, IN_REAL, SCALE, OUT_REAL>(st, in, xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
    case 16: return pass2_go<2, 8, IN_REAL, SCALE, OUT_REAL>(st, in, xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
    case 8: return pass_go<8, IN_REAL, SCALE, OUT_REAL>(st, in, xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
    case 4: return pass_go<4, IN_REAL, SCALE, OUT_REAL>(st, in, xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
    default: return pass_go<2, IN_REAL, SCALE, OUT_REAL>(st, in, xr, S, out, yr, L, Ns, nx, sgn, skip, dotp);
    }
}

// radices of the passes: the log2 L mod 6 bits in one pass (radix 2 .. 32),
// then radix-64 passes
int radix_plan(int p, int *rad)
{
    int np = 0;
    if (p % 6) rad[np++] = 1 << (p % 6);
    for (int b = 0; b < p / 6; ++b) rad[np++] = 64;
    return np;
}

// workgroups of a pass of radix R over L points
int64_t pass_blocks(int R, int64_t L)
{
    return R >= 16 ? (L / R + 7) / 8 : (L / R + 63) / 64;
}

// mode 0: forward transform of the real xr (nx entries, zero-padded) into
// dst; mode 1: inverse transform of S .* src (complex), real part of the
// first nx entries into yr, and with dotp the partial sums of
// sum_o yr[o] xr[o] (one per workgroup of the last pass, their count in
// *ndot).  The passes alternate between the two complex buffers a and b; the
// forward result lands in *res.
hipError_t fft1d_run(hipStream_t st, int mode, const double *xr, const double *S, double *yr, c2 *a, c2 *b,
                     int64_t L, int64_t nx, c2 **res, const int32_t *skip, double *dotp = nullptr,
                     int64_t *ndot = nullptr)
{
    int p = 0;
    while ((int64_t(1) << p) < L) ++p;
    int rad[24];
    const int np = radix_plan(p, rad);
    const double sgn = mode == 0 ? -1.0 : 1.0;
    int64_t Ns = 1;
    c2 *src = a, *dst = b;
    hipError_t e = hipSuccess;
    for (int i = 0; i < np && e == hipSuccess; ++i) {
        const bool first = i == 0, last = i == np - 1;
        const int R = rad[i];
        if (mode == 0) {
            if (first)
                e = pass_radix<true, false, false>(R, st, nullptr, xr, nullptr, dst, nullptr, L, Ns, nx, sgn, skip);
            else
                e = pass_radix<false, false, false>(R, st, src, nullptr, nullptr, dst, nullptr, L, Ns, nx, sgn,
                                                    skip);
        } else {
            if (last && ndot) *ndot = pass_blocks(R, L);
            if (first && last)
                e = pass_radix<false, true, true>(R, st, src, xr, S, nullptr, yr, L, Ns, nx, sgn, skip, dotp);
            else if (first)
                e = pass_radix<false, true, false>(R, st, src, nullptr, S, dst, nullptr, L, Ns, nx, sgn, skip);
            else if (last)
                e = pass_radix<false, false, true>(R, st, src, xr, nullptr, nullptr, yr, L, Ns, nx, sgn, skip,
                                                   dotp);
            else
                e = pass_radix<false, false, false>(R, st, src, nullptr, nullptr, dst, nullptr, L, Ns, nx, sgn,
                                                    skip);
        }
        Ns *= R;
        std::swap(src, dst);
    }
    if (res) *res = src;  // the buffer the last pass wrote
    return e;
}

// ĉ: c_0 at 0, c_m and its mirror L - m for 1 <= m < n, zero elsewhere, with
// c_0 = 1 + 2 a_0 and c_m = a_m (A = I + T + T^T, T lower-triangular Toeplitz
// of the weights a)
__global__ void k_circ_column(const double *__restrict__ a, double *__restrict__ ch, int64_t n, int64_t L)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    double v = 0.0;
    if (i == 0)
        v = 1.0 + 2.0 * a[0];
    else if (i < n)
        v = a[i];
    else if (i > L - n)
        v = a[L - i];
    ch[i] = v;
}

// S = Re(z) / L
__global__ void k_spec_real(const c2 *__restrict__ z, double *__restrict__ S, int64_t L)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) S[i] = z[i].x / (double)L;
}

}  // namespace

int64_t circ_length(int64_t n)
{
    int64_t L = 8;
    while (L < 2 * n - 1) L *= 2;
    return L;
}

hipError_t launch_circ_spectrum(hipStream_t st, const double *a, int64_t n, int64_t L, double *S, double *colbuf,
                                void *za, void *zb)
{
    if (L < 8 || (L & (L - 1)) || L < 2 * n - 1 || L > (int64_t(1) << 23)) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((L + 255) / 256);
    hipLaunchKernelGGL(k_circ_column, dim3(g), dim3(256), 0, st, a, colbuf, n, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    c2 *res = nullptr;
    if ((e = fft1d_run(st, 0, colbuf, nullptr, nullptr, (c2 *)za, (c2 *)zb, L, L, &res, nullptr)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_spec_real, dim3(g), dim3(256), 0, st, res, S, L);
    return hipGetLastError();
}

hipError_t launch_circ_apply(hipStream_t st, const double *x, double *y, int64_t n, int64_t L, const double *S,
                             void *za, void *zb, const int32_t *skip, double *dotp, int64_t *ndot)
{
    if (L < 8 || (L & (L - 1)) || L < 2 * n - 1 || L > (int64_t(1) << 23) || x == y) return hipErrorInvalidValue;
    c2 *res = nullptr;
    hipError_t e = fft1d_run(st, 0, x, nullptr, nullptr, (c2 *)za, (c2 *)zb, L, n, &res, skip);
    if (e != hipSuccess) return e;
    c2 *other = res == (c2 *)za ? (c2 *)zb : (c2 *)za;
    return fft1d_run(st, 1, x, S, y, res, other, L, n, nullptr, skip, dotp, ndot);
}

int64_t circ_dot_parts(int64_t L) { return L / 128 + 1; }

int circ_launches(int64_t L)
{
    int p = 0;
    while ((int64_t(1) << p) < L) ++p;
    int rad[24];
    return 2 * radix_plan(p, rad);
}

}  // namespace fs
