// FFT route for the off-diagonal Toeplitz-block products (section 3.1: a
// Toeplitz matrix is embedded in a circulant of twice its size, which the
// DFT diagonalises).  For a level with half-block size s and n = 2s:
//   z = IDFT_n( H_s . DFT_n(x) ),  H_s = DFT_n(w_0..w_{n-1}),
// x = the s rows of X zero-padded to n, and Y[ylo + p] += alpha z[s + p]/n
// for p < s (those outputs see no wrap-around).  Two real columns are packed
// into one complex column (x = X[:,2c] + i X[:,2c+1]); the kernel is real, so
// real and imaginary parts of z belong to the two columns.
//
// Single pass (n <= 8192 in float64, 16384 in float32): persistent
// workgroups (k_fft2u, k_fft3u), each holding CC complex columns and the
// whole length-n transform in LDS at a time.  n = n1 n2 (n3) is split
// Cooley-Tukey style, q = q1 n2 n3 + q2 n3 + q3, k = k1 + n1 k2 + n1 n2 k3;
// each digit transform runs in registers and LDS only transposes between
// digits.  The first stage reads X straight from HBM and skips the zero half
// (q1 >= n1/2); the middle digit does DFT -> multiply by H -> inverse DFT in
// registers; the last stage writes only the outputs q1 >= n1/2 to Y.
//
// Multi-pass (n = N1 * n_in, n_in the single-pass size): pass 1 does the
// N1-point digit from HBM into a column-chunk scratch buffer, pass 2 runs
// the single-pass machinery over the n_in inner points (with the full
// spectrum) in place, pass 3 does the inverse N1-point digit into Y.
#include "common.hpp"

namespace fs {

// ---------------------------------------------------------------- twiddles
// w[j] = exp(-2 pi i j / nmax), j < nmax, in float64 and float32.
__global__ void k_twiddles(int64_t nmax, cplx<double> *w64, cplx<float> *w32)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nmax; j += (int64_t)gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * (double)j / (double)nmax, &sn, &cs);
        w64[j] = {cs, sn};
        if (w32) w32[j] = {(float)cs, (float)sn};
    }
}

hipError_t launch_twiddles(hipStream_t st, int64_t nmax, cplx<double> *w64, cplx<float> *w32)
{
    int64_t nb = (nmax + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_twiddles, dim3((unsigned)nb), dim3(256), 0, st, nmax, w64, w32);
    return hipGetLastError();
}

// ------------------------------------------------------ in-register DFTs
template <int X>
struct lg2 {
    static constexpr int v = 1 + lg2<X / 2>::v;
};
template <>
struct lg2<1> {
    static constexpr int v = 0;
};

__host__ __device__ constexpr int bitrev(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// exp(-2 pi i m / 32), m < 32, from cos and sin of pi k / 16, k < 8 (folded
// to constants when m is known at compile time).
template <typename T>
__device__ __forceinline__ cplx<T> root32(int m)
{
    constexpr double C[8] = {1.0,
                             0.98078528040323044913,
                             0.92387953251128675613,
                             0.83146961230254523708,
                             0.70710678118654752440,
                             0.55557023301960222474,
                             0.38268343236508977173,
                             0.19509032201612826785};
    const int q = m & 7, h = (m >> 3) & 3;
    const double c0 = C[q], s0 = (q == 0) ? 0.0 : C[8 - q];
    // rotate (c0, s0) by h quarter turns
    const double c = (h == 0) ? c0 : (h == 1) ? -s0 : (h == 2) ? -c0 : s0;
    const double s = (h == 0) ? s0 : (h == 1) ? c0 : (h == 2) ? -s0 : -c0;
    return cplx<T>{(T)c, (T)(-s)};
}

// Radix-2 decimation-in-time DFT of length R <= 32 held in registers;
// natural order in and out.  Forward uses exp(-2 pi i jk/R), inverse its
// conjugate (unnormalised).  The twiddles are compile-time constants.
// HALFZERO: inputs R/2..R-1 are zero and are not read.
template <int R, bool INV, bool HALFZERO, typename T>
__device__ __forceinline__ void dft_reg(cplx<T> (&v)[R])
{
    static_assert(R <= 32, "in-register DFTs up to 32 points");
    constexpr int B = lg2<R>::v;
    cplx<T> w[R];
    if (HALFZERO) {
        // first butterfly stage pairs w[2m] with w[2m+1] = x[bitrev(2m)+R/2] = 0
#pragma unroll
        for (int m = 0; m < R / 2; ++m) {
            cplx<T> a = v[bitrev(2 * m, B)];
            w[2 * m] = a;
            w[2 * m + 1] = a;
        }
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) w[i] = v[bitrev(i, B)];
#pragma unroll
        for (int m = 0; m < R / 2; ++m) {
            cplx<T> a = w[2 * m], b = w[2 * m + 1];
            w[2 * m] = cadd(a, b);
            w[2 * m + 1] = csub(a, b);
        }
    }
#pragma unroll
    for (int len = 4; len <= R; len <<= 1) {
        const int half = len / 2;
#pragma unroll
        for (int st = 0; st < R; st += len) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                cplx<T> a = w[st + j], b = w[st + j + half];
                if (j == 0) {
                } else if (4 * j == len) {
                    // multiply by -i (forward) or +i (inverse)
                    b = INV ? cplx<T>{-b.y, b.x} : cplx<T>{b.y, -b.x};
                } else {
                    const cplx<T> t = root32<T>(j * (32 / len));
                    b = INV ? cmulc(b, t) : cmul(b, t);
                }
                w[st + j] = cadd(a, b);
                w[st + j + half] = csub(a, b);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = w[i];
}

// The pointer unchanged, but opaque to the optimiser: loads through it
// inside a loop are not hoisted out of the loop (the persistent kernels
// would otherwise keep every loop-invariant spectrum and twiddle value of
// all stages live in registers at once).
template <typename P>
__device__ __forceinline__ P opaque(P p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// Bases p[j] = W^(e 2^j), j < log2(R), for apply_twiddles_b.
template <int R, typename T>
__device__ __forceinline__ void twiddle_bases(cplx<T> (&p)[lg2<R>::v], const cplx<T> *__restrict__ tw, int64_t e)
{
#pragma unroll
    for (int j = 0; j < lg2<R>::v; ++j) p[j] = tw[e << j];
}

// v[k] *= W^(k e) (conjugated for INV), k = 1..R-1, W = exp(-2 pi i / nmax),
// from the bases p[j] = W^(e 2^j) in registers: W^(k e) is built as
// W^((k - lowbit k) e) W^(lowbit(k) e), at most log2(R) - 1 products deep.
template <int R, bool INV, typename T>
__device__ __forceinline__ void apply_twiddles_b(cplx<T> (&v)[R], const cplx<T> (&pb)[lg2<R>::v])
{
    constexpr int B = lg2<R>::v;
    cplx<T> p[B];
#pragma unroll
    for (int j = 0; j < B; ++j) p[j] = INV ? cplx<T>{pb[j].x, -pb[j].y} : pb[j];
    cplx<T> w[R];
    w[0] = cplx<T>{(T)1, (T)0};
#pragma unroll
    for (int k = 1; k < R; ++k) {
        const int low = k & -k;
        const int j = __builtin_ctz(k);
        w[k] = (k == low) ? p[j] : cmul(w[k - low], p[j]);
        v[k] = cmul(v[k], w[k]);
    }
}

// Loads of the two packed real columns (one vector access when the pair is
// whole and aligned, i.e. M even and col even); zero beyond M.
template <typename T>
__device__ __forceinline__ cplx<T> load_pair(FS_G const T *__restrict__ row, int64_t col, int64_t M)
{
    if (((M & 1) == 0) && col + 1 < M) return *reinterpret_cast<FS_G const cplx<T> *>(row + col);
    cplx<T> v;
    v.x = (col < M) ? row[col] : (T)0;
    v.y = (col + 1 < M) ? row[col + 1] : (T)0;
    return v;
}

template <typename T>
__device__ __forceinline__ void add_pair(FS_G T *__restrict__ row, int64_t col, int64_t M, cplx<T> v, T scale)
{
    if (((M & 1) == 0) && col + 1 < M) {
        FS_G cplx<T> *p = reinterpret_cast<FS_G cplx<T> *>(row + col);
        cplx<T> o = *p;
        o.x += scale * v.x;
        o.y += scale * v.y;
        *p = o;
        return;
    }
    if (col < M) row[col] += scale * v.x;
    if (col + 1 < M) row[col + 1] += scale * v.y;
}

template <typename T>
__device__ __forceinline__ void store_pair(FS_G T *__restrict__ row, int64_t col, int64_t M, cplx<T> v)
{
    if (((M & 1) == 0) && col + 1 < M) {
        *reinterpret_cast<FS_G cplx<T> *>(row + col) = v;
        return;
    }
    if (col < M) row[col] = v.x;
    if (col + 1 < M) row[col + 1] = v.y;
}

// Near-corner terms of a level product, kept out of the FFT: the entries of
// T_s at distance d = s + p - q < D0 (only rows p < D0 - 1 have any) carry the
// largest weights (|a_1| is of the size of a_0), and leaving them in the
// spectrum would put an error of order eps * |a_1| * |X| * log n on every
// output.  They are added here exactly:
//   Y[p] += alpha * sum_{d = p+1}^{D0-1} w_d X[s + p - d].
// The band is read from the float64 view xc and added to the float64 view
// yc (in float32 mode the products themselves go to a float32 accumulator,
// but the band's weights are too large to round to float32).
template <typename T>
__device__ __forceinline__ void corner_add(const UpdTask<T> &tk, int p, int64_t col, int64_t M)
{
    const int D0 = corner_width(tk.s);
    double sx = 0.0, sy = 0.0;
    FS_G const double *__restrict__ xb = gptr(tk.xc) + tk.xlo * M;
    for (int d = p + 1; d < D0; ++d) {
        FS_G const double *__restrict__ row = xb + (int64_t)(tk.s + p - d) * M;
        const double wd = gptr(tk.w)[d];
        if (col < M) sx += wd * row[col];
        if (col + 1 < M) sy += wd * row[col + 1];
    }
    FS_G double *__restrict__ yr = gptr(tk.yc) + (tk.ylo + p) * M;
    if (col < M) yr[col] += tk.alpha * sx;
    if (col + 1 < M) yr[col + 1] += tk.alpha * sy;
}

// Multi-pass pass 2 (the single-pass machinery over the inner n points):
// complex scratch Z with layout Z[(k1g * Mc + c) * n + q] (q contiguous),
// full input and full output, spectrum entries spec[k1g + N1g * k].
// Twiddles as in the persistent kernels: per-thread bases W^(e 2^j) loaded
// once per stage, compile-time roots inside the digit DFTs.
enum { MODE_UPDATE = 0, MODE_INNER = 1 };

// ---------------------------------------------------- two-digit kernel
// n = N1 N2, q = q1 N2 + q2, k = k1 + N1 k2.
// LDS layout of element (k1 or q1, q2 or k2, c): k1*(N2*CC+1) + q2*CC + c.
template <typename T, int N1, int N2, int CC>
__global__ __launch_bounds__(256) void k_fft2_inner(const UpdTask<T> *__restrict__ tasks,
                                                    const cplx<T> *__restrict__ tw, int64_t nmax,
                                                    cplx<T> *__restrict__ zs, int64_t Mc, int N1g)
{
    constexpr int n = N1 * N2;
    constexpr int RS = N2 * CC + 1;
    __shared__ cplx<T> sd[N1 * RS];
    FS_G const cplx<T> *__restrict__ spec = gptr(tasks[0].spec);
    const int t = threadIdx.x;
    const int64_t cgrp = (int64_t)blockIdx.x * CC;  // first complex column of this workgroup
    const int64_t tws = nmax / n;
    const int k1g = blockIdx.y;

    // stage A: digit q1 -> k1 (forward), twiddle W_n^{q2 k1}, to LDS
    for (int it = t; it < CC * N2; it += 256) {
        const int c = it % CC, q2 = it / CC;
        cplx<T> v[N1];
        const bool cv = cgrp + c < Mc;
        const cplx<T> *__restrict__ zb = zs + ((int64_t)k1g * Mc + cgrp + c) * n;
#pragma unroll
        for (int q1 = 0; q1 < N1; ++q1) v[q1] = cv ? zb[q1 * N2 + q2] : cplx<T>{0, 0};
        cplx<T> pa[lg2<N1>::v];
        twiddle_bases<N1>(pa, tw, (int64_t)q2 * tws);
        dft_reg<N1, false, false>(v);
        apply_twiddles_b<N1, false>(v, pa);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) sd[k1 * RS + q2 * CC + c] = v[k1];
    }
    __syncthreads();
    // stage B: digit q2 -> k2, multiply by the spectrum, back k2 -> q2
    for (int it = t; it < CC * N1; it += 256) {
        const int c = it % CC, k1 = it / CC;
        cplx<T> v[N2];
#pragma unroll
        for (int q2 = 0; q2 < N2; ++q2) v[q2] = sd[k1 * RS + q2 * CC + c];
        dft_reg<N2, false, false>(v);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) v[k2] = cmul(v[k2], spec[k1g + (int64_t)N1g * (k1 + N1 * k2)]);
        dft_reg<N2, true, false>(v);
#pragma unroll
        for (int q2 = 0; q2 < N2; ++q2) sd[k1 * RS + q2 * CC + c] = v[q2];
    }
    __syncthreads();
    // stage C: conjugate twiddle, digit k1 -> q1 (inverse), out
    for (int it = t; it < CC * N2; it += 256) {
        const int c = it % CC, q2 = it / CC;
        cplx<T> v[N1];
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) v[k1] = sd[k1 * RS + q2 * CC + c];
        cplx<T> pa[lg2<N1>::v];
        twiddle_bases<N1>(pa, tw, (int64_t)q2 * tws);
        apply_twiddles_b<N1, true>(v, pa);
        dft_reg<N1, true, false>(v);
        if (cgrp + c < Mc) {
            cplx<T> *__restrict__ zb = zs + ((int64_t)k1g * Mc + cgrp + c) * n;
#pragma unroll
            for (int q1 = 0; q1 < N1; ++q1) zb[q1 * N2 + q2] = v[q1];
        }
    }
}

// -------------------------------------------------- three-digit kernel
// n = N1 N2 N3, q = q1 N2 N3 + q2 N3 + q3, k = k1 + N1 k2 + N1 N2 k3.
// LDS layout of element (a = k1|q1, b = q2|k2, d = q3|k3, c):
//   (a*N2 + b)*(N3*CC + 1) + d*CC + c.
template <typename T, int N1, int N2, int N3, int CC>
__global__ __launch_bounds__(256) void k_fft3_inner(const UpdTask<T> *__restrict__ tasks,
                                                    const cplx<T> *__restrict__ tw, int64_t nmax,
                                                    cplx<T> *__restrict__ zs, int64_t Mc, int N1g)
{
    constexpr int n = N1 * N2 * N3;
    constexpr int RS = N3 * CC + 1;
    __shared__ cplx<T> sd[N1 * N2 * RS];
    FS_G const cplx<T> *__restrict__ spec = gptr(tasks[0].spec);
    const int t = threadIdx.x;
    const int64_t cgrp = (int64_t)blockIdx.x * CC;
    const int64_t tws = nmax / n;
    const int k1g = blockIdx.y;
    auto at = [&](int a, int b, int d, int c) { return (a * N2 + b) * RS + d * CC + c; };

    // A: q1 -> k1, twiddle by W_n^{(q2 N3 + q3) k1}
    for (int it = t; it < CC * N2 * N3; it += 256) {
        const int c = it % CC, r = it / CC, q3 = r % N3, q2 = r / N3;
        cplx<T> v[N1];
        const bool cv = cgrp + c < Mc;
        const cplx<T> *__restrict__ zb = zs + ((int64_t)k1g * Mc + cgrp + c) * n;
#pragma unroll
        for (int q1 = 0; q1 < N1; ++q1) v[q1] = cv ? zb[q1 * N2 * N3 + r] : cplx<T>{0, 0};
        cplx<T> pa[lg2<N1>::v];
        twiddle_bases<N1>(pa, tw, (int64_t)r * tws);
        dft_reg<N1, false, false>(v);
        apply_twiddles_b<N1, false>(v, pa);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) sd[at(k1, q2, q3, c)] = v[k1];
    }
    __syncthreads();
    // B: q2 -> k2, twiddle by W_{N2 N3}^{q3 k2} = W_n^{q3 k2 N1}
    for (int it = t; it < CC * N1 * N3; it += 256) {
        const int c = it % CC, r = it / CC, q3 = r % N3, k1 = r / N3;
        cplx<T> v[N2];
#pragma unroll
        for (int q2 = 0; q2 < N2; ++q2) v[q2] = sd[at(k1, q2, q3, c)];
        cplx<T> pb[lg2<N2>::v];
        twiddle_bases<N2>(pb, tw, (int64_t)(q3 * N1) * tws);
        dft_reg<N2, false, false>(v);
        apply_twiddles_b<N2, false>(v, pb);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) sd[at(k1, k2, q3, c)] = v[k2];
    }
    __syncthreads();
    // C: q3 -> k3, spectrum, k3 -> q3
    for (int it = t; it < CC * N1 * N2; it += 256) {
        const int c = it % CC, r = it / CC, k2 = r % N2, k1 = r / N2;
        cplx<T> v[N3];
#pragma unroll
        for (int q3 = 0; q3 < N3; ++q3) v[q3] = sd[at(k1, k2, q3, c)];
        cplx<T> hs[N3];
#pragma unroll
        for (int k3 = 0; k3 < N3; ++k3) hs[k3] = spec[k1g + (int64_t)N1g * (k1 + N1 * k2 + N1 * N2 * k3)];
        dft_reg<N3, false, false>(v);
#pragma unroll
        for (int k3 = 0; k3 < N3; ++k3) v[k3] = cmul(v[k3], hs[k3]);
        dft_reg<N3, true, false>(v);
#pragma unroll
        for (int q3 = 0; q3 < N3; ++q3) sd[at(k1, k2, q3, c)] = v[q3];
    }
    __syncthreads();
    // D: conjugate twiddle, k2 -> q2
    for (int it = t; it < CC * N1 * N3; it += 256) {
        const int c = it % CC, r = it / CC, q3 = r % N3, k1 = r / N3;
        cplx<T> v[N2];
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) v[k2] = sd[at(k1, k2, q3, c)];
        cplx<T> pb[lg2<N2>::v];
        twiddle_bases<N2>(pb, tw, (int64_t)(q3 * N1) * tws);
        apply_twiddles_b<N2, true>(v, pb);
        dft_reg<N2, true, false>(v);
#pragma unroll
        for (int q2 = 0; q2 < N2; ++q2) sd[at(k1, q2, q3, c)] = v[q2];
    }
    __syncthreads();
    // E: conjugate twiddle, k1 -> q1, out
    for (int it = t; it < CC * N2 * N3; it += 256) {
        const int c = it % CC, r = it / CC;
        cplx<T> v[N1];
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) v[k1] = sd[at(k1, r / N3, r % N3, c)];
        cplx<T> pa[lg2<N1>::v];
        twiddle_bases<N1>(pa, tw, (int64_t)r * tws);
        apply_twiddles_b<N1, true>(v, pa);
        dft_reg<N1, true, false>(v);
        if (cgrp + c < Mc) {
            cplx<T> *__restrict__ zb = zs + ((int64_t)k1g * Mc + cgrp + c) * n;
#pragma unroll
            for (int q1 = 0; q1 < N1; ++q1) zb[q1 * N2 * N3 + r] = v[q1];
        }
    }
}

// ------------------------------------------- persistent update kernels
// Level products (UPDATE mode) by persistent workgroups: workgroup b takes
// column groups g = slot, slot + G0, ... (slot: XCD-aware order of b, so
// that neighbouring groups, which share cache lines, run on one XCD).  The X
// rows of group g + G0 are loaded into registers while group g is
// transformed, and the Y rows of group g one stage before they are needed.
// Vector-memory loads complete in issue order, so the only loads inside the
// stage loop are the spectrum (middle stage, nothing else in flight), then
// Y, then the next X: the twiddles of every stage are built from per-thread
// bases loaded once, before the loop.  Digits are at most 16 points at the
// first and last stage (32 in the middle), which keeps these buffers in
// registers.  One workgroup per CU fits when the transform needs most of the
// LDS, so this overlap is what hides the HBM latency.
//
// Item (c, r) of stage A / the last stage: complex column c of the group,
// r = q2 N3 + q3; its X rows are q1 R + r (q1 < N1/2, the rest is the zero
// padding) and its Y rows p = (q1 - N1/2) R + r (q1 >= N1/2).
// Pair access: with EVEN (M even, rows 16-byte aligned) every in-range
// pair is one aligned vector access; otherwise the scalar path of
// load_pair/store_pair.  Columns past M read as zero and are not written.
template <bool EVEN, typename T>
__device__ __forceinline__ cplx<T> ld_pair(FS_G const T *__restrict__ row, int64_t col, int64_t M)
{
    if (EVEN) {
        cplx<T> v{0, 0};
        if (col < M) v = *reinterpret_cast<FS_G const cplx<T> *>(row + col);
        return v;
    }
    return load_pair(row, col, M);
}

template <bool EVEN, typename T>
__device__ __forceinline__ void st_pair(FS_G T *__restrict__ row, int64_t col, int64_t M, cplx<T> v)
{
    if (EVEN) {
        if (col < M) *reinterpret_cast<FS_G cplx<T> *>(row + col) = v;
        return;
    }
    store_pair(row, col, M, v);
}

template <typename T, int N1, int R, int CC, int NT, bool EVEN>
struct GroupRows {
    static constexpr int NI = CC * R;
    static constexpr int NA = (NI + NT - 1) / NT;
    static constexpr int H = N1 / 2;
    cplx<T> v[NA][H];

    // X rows q1 R + r, q1 < N1/2
    __device__ __forceinline__ void load_x(FS_G const T *__restrict__ xb, int64_t g, int64_t M)
    {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int it = threadIdx.x + NT * a;
            const bool ok = (NI % NT == 0) || it < NI;
            const int c = it % CC, r = it / CC;
            const int64_t col = 2 * (g * CC + c);
#pragma unroll
            for (int q1 = 0; q1 < H; ++q1)
                v[a][q1] = ok ? ld_pair<EVEN>(xb + (int64_t)(q1 * R + r) * M, col, M) : cplx<T>{0, 0};
        }
    }
    // Y rows p = j R + r, j < N1/2, p < ny
    __device__ __forceinline__ void load_y(FS_G const T *__restrict__ yb, int64_t g, int64_t M, int ny)
    {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int it = threadIdx.x + NT * a;
            const bool ok = (NI % NT == 0) || it < NI;
            const int c = it % CC, r = it / CC;
            const int64_t col = 2 * (g * CC + c);
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const int p = j * R + r;
                v[a][j] = (ok && p < ny) ? ld_pair<EVEN>(yb + (int64_t)p * M, col, M) : cplx<T>{0, 0};
            }
        }
    }
};

// The column groups of all tasks of a launch, numbered task after task:
// task t holds flat indices gbase[t] .. gbase[t+1]-1 (gbase has ntasks + 1
// entries, built on the host from each task's width and the kernel's
// columns per group).  The persistent workgroups walk this flat index
// (workgroup b takes slot(b), slot(b) + P, ...), so tasks of different widths
// share the workgroups in proportion to their groups.
template <typename T>
struct GroupCursor {
    const UpdTask<T> *tasks;
    const int64_t *gbase;
    int ntasks;
    int t;  // task holding the current flat index
    // false once f is past the last group; f never decreases.  Each wave
    // looks at 64 task boundaries per step (one load and a ballot).
    __device__ bool seek(int64_t f)
    {
        if (f >= gbase[ntasks]) return false;
        const int lane = threadIdx.x & 63;
        for (;;) {
            const int i = t + lane;
            const bool le = (i <= ntasks) && gbase[i] <= f;
            const int k = __popcll(__ballot(le));  // gbase is sorted: lanes 0..k-1
            if (k < 64) {
                t += k - 1;
                return true;
            }
            t += 63;
        }
    }
};

// What one column group needs of its task.
template <typename T>
struct GroupView {
    FS_G const T *xb;  // X row 0
    FS_G T *yb;        // Y row 0
    FS_G const cplx<T> *spec;
    int64_t M;
    int64_t g;  // group within the task
    int ny;
    T scale;
    FS_G const double *w;  // Toeplitz column (near-corner band)
    double alpha;
};

template <typename T>
__device__ __forceinline__ GroupView<T> group_view(const GroupCursor<T> &c, int64_t f, int n)
{
    const UpdTask<T> &tk = c.tasks[c.t];
    GroupView<T> v;
    v.M = tk.M;
    v.xb = gptr(tk.x) + tk.xlo * v.M;
    v.yb = gptr(tk.y) + tk.ylo * v.M;
    v.spec = gptr(tk.spec);
    v.g = f - c.gbase[c.t];
    v.ny = tk.ny;
    v.scale = (T)(tk.alpha / (double)n);
    v.w = gptr(tk.w);
    v.alpha = tk.alpha;
    return v;
}

// two digits: n = N1 N2 (stage layout as in k_fft2_inner)
template <typename T, int N1, int N2, int CC, bool EVEN>
__global__ __launch_bounds__(256) void k_fft2u(const UpdTask<T> *__restrict__ tasks, const int64_t *__restrict__ gbase,
                                               int ntasks, const cplx<T> *__restrict__ tw0, int64_t nmax)
{
    constexpr int n = N1 * N2;
    constexpr int RS = N2 * CC + 1;
    using GR = GroupRows<T, N1, N2, CC, 256, EVEN>;
    constexpr int NA = GR::NA, H = GR::H;
    __shared__ cplx<T> sd[N1 * RS];
    const int t = threadIdx.x;
    const int64_t tws = nmax / n;
    const int64_t P = gridDim.x;
    int64_t f = xcd_remap(blockIdx.x, gridDim.x);
    GroupCursor<T> cur{tasks, gbase, ntasks, 0};
    if (!cur.seek(f)) return;  // the whole workgroup: no group for it
    GroupView<T> v = group_view(cur, f, n);

    // twiddle bases of the first/last stage, the same for every group
    cplx<T> pa[NA][lg2<N1>::v];
#pragma unroll
    for (int a = 0; a < NA; ++a) twiddle_bases<N1>(pa[a], tw0, (int64_t)(((t + 256 * a) / CC) % N2) * tws);

    GR xc;  // X rows of the current group (loaded during the previous group)
    xc.load_x(v.xb, v.g, v.M);
    for (;;) {
        const cplx<T> *__restrict__ tw = opaque(tw0);  // per-thread twiddle bases
        FS_G const cplx<T> *__restrict__ spec = v.spec;  // per group: not hoisted
        // this group's Y rows, in flight during stages A and B (issued after
        // this group's X, so waiting for X does not wait for them)
        GR yc;
        yc.load_y(v.yb, v.g, v.M, v.ny);
        // stage A: digit q1 -> k1 (forward, zero upper half), twiddle, to LDS
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int it = t + 256 * a;
            if (it < CC * N2) {
                const int c = it % CC, q2 = it / CC;
                cplx<T> w[N1];
#pragma unroll
                for (int q1 = 0; q1 < H; ++q1) w[q1] = xc.v[a][q1];
                dft_reg<N1, false, true>(w);
                apply_twiddles_b<N1, false>(w, pa[a]);
#pragma unroll
                for (int k1 = 0; k1 < N1; ++k1) sd[k1 * RS + q2 * CC + c] = w[k1];
            }
        }
        __syncthreads();
        // stage B: digit q2 -> k2, spectrum, back
#pragma unroll 1
        for (int it = t; it < CC * N1; it += 256) {
            const int c = it % CC, k1 = it / CC;
            cplx<T> w[N2];
#pragma unroll
            for (int q2 = 0; q2 < N2; ++q2) w[q2] = sd[k1 * RS + q2 * CC + c];
            cplx<T> hs[N2];
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) hs[k2] = spec[k1 + N1 * k2];
            dft_reg<N2, false, false>(w);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) w[k2] = cmul(w[k2], hs[k2]);
            dft_reg<N2, true, false>(w);
#pragma unroll
            for (int q2 = 0; q2 < N2; ++q2) sd[k1 * RS + q2 * CC + c] = w[q2];
        }
        // the next group's X rows (after this group's Y: loads complete in
        // order, so waiting for Y does not wait for them)
        GR xn;
        const int64_t fn = f + P;
        GroupCursor<T> nxt = cur;
        const bool more = nxt.seek(fn);
        GroupView<T> vn = v;
        if (more) {
            vn = group_view(nxt, fn, n);
            xn.load_x(vn.xb, vn.g, vn.M);
        }
        __syncthreads();
        // stage C: conjugate twiddle, digit k1 -> q1 (inverse), Y = Y + scale z
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int it = t + 256 * a;
            if (it < CC * N2) {
                const int c = it % CC, q2 = it / CC;
                cplx<T> w[N1];
#pragma unroll
                for (int k1 = 0; k1 < N1; ++k1) w[k1] = sd[k1 * RS + q2 * CC + c];
                apply_twiddles_b<N1, true>(w, pa[a]);
                dft_reg<N1, true, false>(w);
                const int64_t col = 2 * (v.g * CC + c);
#pragma unroll
                for (int q1 = H; q1 < N1; ++q1) {
                    const int p = (q1 - H) * N2 + q2;
                    if (p < v.ny) {
                        const cplx<T> y0 = yc.v[a][q1 - H];
                        st_pair<EVEN>(v.yb + (int64_t)p * v.M, col, v.M,
                                      cplx<T>{y0.x + v.scale * w[q1].x, y0.y + v.scale * w[q1].y});
                    }
                }
            }
        }
        __syncthreads();
        if (!more) break;
        cur = nxt;
        f = fn;
        v = vn;
        xc = xn;
    }
}

// three digits: n = N1 N2 N3 (stage layout as in k_fft3_inner)
// Y rows: loaded at the top of the group iteration (in flight during
// stages A-D) when the registers allow it (n <= 4096 in float64), else in
// stage D after stage C's spectrum reads.
template <typename T, int N1, int N2, int N3, int CC, int NT, bool EVEN>
__global__ __launch_bounds__(NT) void k_fft3u(const UpdTask<T> *__restrict__ tasks, const int64_t *__restrict__ gbase,
                                               int ntasks, const cplx<T> *__restrict__ tw0, int64_t nmax)
{
    constexpr bool EARLY_Y = N1 * N2 * N3 * sizeof(T) <= 4096 * 8;
    constexpr int n = N1 * N2 * N3;
    constexpr int RS = N3 * CC + 1;
    using GR = GroupRows<T, N1, N2 * N3, CC, NT, EVEN>;
    constexpr int NA = GR::NA, H = GR::H;
    constexpr int NB = (CC * N1 * N3 + NT - 1) / NT;  // items per thread of stages B and D
    __shared__ cplx<T> sd[N1 * N2 * RS];
    // Near-corner band in float64 (the sum of k_corner, added where Y rows
    // 0..30 are stored): stage A keeps the group's raw X rows s-1-k,
    // k < KB, in sB[k][c]; stage C the weights w_0..w_KB in sWb.
    constexpr bool BAND = sizeof(T) == 8;
    constexpr int KB = 31;  // corner_width(s) - 1 for every s of these kernels
    static_assert(!BAND || N2 * N3 >= KB, "the band rows come from the last outer digit");
    __shared__ cplx<T> sB[BAND ? KB * CC : 1];
    __shared__ double sWb[BAND ? KB + 1 : 1];
    const int t = threadIdx.x;
    const int64_t tws = nmax / n;
    const int64_t P = gridDim.x;
    int64_t f = xcd_remap(blockIdx.x, gridDim.x);
    GroupCursor<T> cur{tasks, gbase, ntasks, 0};
    if (!cur.seek(f)) return;  // the whole workgroup: no group for it
    GroupView<T> gv = group_view(cur, f, n);
    auto at = [&](int a, int b, int d, int c) { return (a * N2 + b) * RS + d * CC + c; };
    // exponents of the stage twiddles: A/E use W_n^{r k1}, r = q2 N3 + q3;
    // B/D use W_n^{q3 N1 k2}
    auto ea = [&](int a) { return (int64_t)(((t + NT * a) / CC) % (N2 * N3)) * tws; };
    auto eb = [&](int b) { return (int64_t)((((t + NT * b) / CC) % N3) * N1) * tws; };

    GR xc;  // X rows of the current group (loaded during the previous group)
    xc.load_x(gv.xb, gv.g, gv.M);
    for (;;) {
        const cplx<T> *__restrict__ tw = opaque(tw0);  // per-thread twiddle bases
        FS_G const cplx<T> *__restrict__ spec = gv.spec;  // per group: not hoisted
        GR yc;
        if constexpr (EARLY_Y) yc.load_y(gv.yb, gv.g, gv.M, gv.ny);
        // A: q1 -> k1 (zero upper half), twiddle by W_n^{(q2 N3 + q3) k1}
        {
            cplx<T> pa[NA][lg2<N1>::v];
#pragma unroll
            for (int a = 0; a < NA; ++a) twiddle_bases<N1>(pa[a], tw, ea(a));
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int it = t + NT * a;
                if (it < CC * N2 * N3) {
                    const int c = it % CC, r = it / CC, q3 = r % N3, q2 = r / N3;
                    cplx<T> v[N1];
#pragma unroll
                    for (int q1 = 0; q1 < H; ++q1) v[q1] = xc.v[a][q1];
                    // X row (H-1) R + r = s-1-k with k = R-1-r
                    if constexpr (BAND)
                        if (r >= N2 * N3 - KB) sB[(N2 * N3 - 1 - r) * CC + c] = v[H - 1];
                    dft_reg<N1, false, true>(v);
                    apply_twiddles_b<N1, false>(v, pa[a]);
#pragma unroll
                    for (int k1 = 0; k1 < N1; ++k1) sd[at(k1, q2, q3, c)] = v[k1];
                }
            }
        }
        __syncthreads();
        // B: q2 -> k2, twiddle by W_n^{q3 k2 N1}
        {
            cplx<T> pb[NB][lg2<N2>::v];
#pragma unroll
            for (int b = 0; b < NB; ++b) twiddle_bases<N2>(pb[b], tw, eb(b));
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int it = t + NT * b;
                if (it < CC * N1 * N3) {
                    const int c = it % CC, r = it / CC, q3 = r % N3, k1 = r / N3;
                    cplx<T> v[N2];
#pragma unroll
                    for (int q2 = 0; q2 < N2; ++q2) v[q2] = sd[at(k1, q2, q3, c)];
                    dft_reg<N2, false, false>(v);
                    apply_twiddles_b<N2, false>(v, pb[b]);
#pragma unroll
                    for (int k2 = 0; k2 < N2; ++k2) sd[at(k1, k2, q3, c)] = v[k2];
                }
            }
        }
        __syncthreads();
        // C: q3 -> k3, spectrum, k3 -> q3 (no other loads in flight; the
        // band weights are loaded with the spectrum)
        double wband = 0.0;
        if constexpr (BAND)
            if (t <= KB) wband = gv.w[t];
#pragma unroll 1
        for (int it = t; it < CC * N1 * N2; it += NT) {
            const int c = it % CC, r = it / CC, k2 = r % N2, k1 = r / N2;
            cplx<T> v[N3];
#pragma unroll
            for (int q3 = 0; q3 < N3; ++q3) v[q3] = sd[at(k1, k2, q3, c)];
            cplx<T> hs[N3];
#pragma unroll
            for (int k3 = 0; k3 < N3; ++k3) hs[k3] = spec[k1 + N1 * k2 + N1 * N2 * k3];
            dft_reg<N3, false, false>(v);
#pragma unroll
            for (int k3 = 0; k3 < N3; ++k3) v[k3] = cmul(v[k3], hs[k3]);
            dft_reg<N3, true, false>(v);
#pragma unroll
            for (int q3 = 0; q3 < N3; ++q3) sd[at(k1, k2, q3, c)] = v[q3];
        }
        if constexpr (BAND)
            if (t <= KB) sWb[t] = wband;
        __syncthreads();
        // the next group (possibly of the next task)
        const int64_t fn = f + P;
        GroupCursor<T> nxt = cur;
        GroupView<T> vn = gv;
        bool more = false;
        // Loads complete in issue order: first the twiddle bases of D and E,
        // then this group's Y rows, then the next group's X rows, so that each
        // wait below covers only what it needs.
        cplx<T> pa[NA][lg2<N1>::v];
#pragma unroll
        for (int a = 0; a < NA; ++a) twiddle_bases<N1>(pa[a], tw, ea(a));
        {
            cplx<T> pb[NB][lg2<N2>::v];
#pragma unroll
            for (int b = 0; b < NB; ++b) twiddle_bases<N2>(pb[b], tw, eb(b));
            if constexpr (!EARLY_Y) yc.load_y(gv.yb, gv.g, gv.M, gv.ny);
            GR xn;
            more = nxt.seek(fn);
            if (more) {
                vn = group_view(nxt, fn, n);
                xn.load_x(vn.xb, vn.g, vn.M);
            }
            // D: conjugate twiddle, k2 -> q2
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int it = t + NT * b;
                if (it < CC * N1 * N3) {
                    const int c = it % CC, r = it / CC, q3 = r % N3, k1 = r / N3;
                    cplx<T> v[N2];
#pragma unroll
                    for (int k2 = 0; k2 < N2; ++k2) v[k2] = sd[at(k1, k2, q3, c)];
                    apply_twiddles_b<N2, true>(v, pb[b]);
                    dft_reg<N2, true, false>(v);
#pragma unroll
                    for (int q2 = 0; q2 < N2; ++q2) sd[at(k1, q2, q3, c)] = v[q2];
                }
            }
            __syncthreads();
            // E: conjugate twiddle, k1 -> q1, Y = Y + scale z
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int it = t + NT * a;
                if (it < CC * N2 * N3) {
                    const int c = it % CC, r = it / CC, q3 = r % N3, q2 = r / N3;
                    cplx<T> v[N1];
#pragma unroll
                    for (int k1 = 0; k1 < N1; ++k1) v[k1] = sd[at(k1, q2, q3, c)];
                    apply_twiddles_b<N1, true>(v, pa[a]);
                    dft_reg<N1, true, false>(v);
                    const int64_t col = 2 * (gv.g * CC + c);
                    // band of output row p = r < KB (q1 = H):
                    //   sum_{k <= KB-1-r} w_{r+1+k} X[s-1-k]
                    cplx<T> bnd{0, 0};
                    if constexpr (BAND) {
                        if (r < KB) {
                            for (int k = 0; k < KB - r; ++k) {
                                const double wk = sWb[r + 1 + k];
                                const cplx<T> xk = sB[k * CC + c];
                                bnd.x = fma(wk, xk.x, bnd.x);
                                bnd.y = fma(wk, xk.y, bnd.y);
                            }
                        }
                    }
#pragma unroll
                    for (int q1 = H; q1 < N1; ++q1) {
                        const int p = (q1 - H) * N2 * N3 + r;
                        if (p < gv.ny) {
                            const cplx<T> y0 = yc.v[a][q1 - H];
                            cplx<T> yv{y0.x + gv.scale * v[q1].x, y0.y + gv.scale * v[q1].y};
                            if (BAND && q1 == H) {
                                yv.x = fma((T)gv.alpha, bnd.x, yv.x);
                                yv.y = fma((T)gv.alpha, bnd.y, yv.y);
                            }
                            st_pair<EVEN>(gv.yb + (int64_t)p * gv.M, col, gv.M, yv);
                        }
                    }
                }
            }
            __syncthreads();
            xc = xn;
        }
        if (!more) break;
        cur = nxt;
        f = fn;
        gv = vn;
    }
}

// The near-corner band of a level product (see corner_add), for the
// persistent update kernels.  With k = d - p - 1 the band reads only the
// last D0 - 1 rows of X:
//   Y[p] += alpha sum_{k <= D0-2-p} w_{p+1+k} X[s-1-k],   p < D0 - 1.
// One thread per (output row p = blockIdx.y, column): all its X loads are
// issued together (the rows are shared through the cache by the threads of
// the other p), so a launch costs about two memory round trips.  It runs
// after the transform kernel on the same stream, for the levels whose
// transform kernel does not add the band itself (float32, and the two-digit
// sizes below 512 points).
template <typename T>
__global__ __launch_bounds__(256) void k_corner(const UpdTask<T> *__restrict__ tasks)
{
    constexpr int KMAX = 31;  // corner_width(s) - 1 <= 31
    const UpdTask<T> tk = tasks[blockIdx.z];
    const int64_t M = tk.M;
    const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int K = corner_width(tk.s) - 1;
    const int p = blockIdx.y;
    if (col >= M || p >= K || p >= tk.ny) return;
    FS_G const double *__restrict__ xb = gptr(tk.xc) + (tk.xlo + tk.s - 1) * M + col;
    FS_G const double *__restrict__ w = gptr(tk.w) + p + 1;
    FS_G double *__restrict__ yr = gptr(tk.yc) + (tk.ylo + p) * M + col;
    const int nk = K - p;  // k < nk
    double xr[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) xr[k] = (k < nk) ? xb[-(int64_t)k * M] : 0.0;
    const double y0 = *yr;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < nk) acc += w[k] * xr[k];
    *yr = y0 + tk.alpha * acc;
}

// ------------------------------------------------ multi-pass outer digit
// Pass 1: for complex column c of the chunk and inner index q2 < nin:
//   v[k1] = W_n^{q2 k1} sum_{q1 < N1/2} x[q1 nin + q2] W_N1^{q1 k1}
//   Z[(k1 * Mc + c) * nin + q2] = v[k1]
// Workgroup: 16 complex columns x 16 inner indices; LDS transposes so that
// X reads are row-contiguous and Z writes are q2-contiguous.
template <typename T, int N1>
__global__ __launch_bounds__(256) void k_mp_pass1(const UpdTask<T> *__restrict__ tasks, const cplx<T> *__restrict__ tw,
                                                  int64_t nmax, cplx<T> *__restrict__ zs, int64_t c0, int64_t Mc,
                                                  int nin)
{
    __shared__ cplx<T> sb[N1][16][17];
    const UpdTask<T> tk = tasks[0];
    const int64_t M = tk.M;
    const int64_t n = (int64_t)N1 * nin;
    const int64_t tws = nmax / n;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t cl = (int64_t)blockIdx.x * 16 + tx;  // complex column within chunk
    const int q2 = blockIdx.y * 16 + ty;
    cplx<T> v[N1];
    const int64_t col = 2 * (c0 + cl);
    FS_G const T *__restrict__ xb = gptr(tk.x) + tk.xlo * M;
#pragma unroll
    for (int q1 = 0; q1 < N1 / 2; ++q1)
        v[q1] = (cl < Mc) ? load_pair(xb + ((int64_t)q1 * nin + q2) * M, col, M) : cplx<T>{0, 0};
    cplx<T> pa[lg2<N1>::v];
    twiddle_bases<N1>(pa, tw, (int64_t)q2 * tws);
    dft_reg<N1, false, true>(v);
    apply_twiddles_b<N1, false>(v, pa);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) sb[k1][tx][ty] = v[k1];
    __syncthreads();
    // write: thread (ty -> column, tx -> q2)
    const int64_t cw = (int64_t)blockIdx.x * 16 + ty;
    const int qw = blockIdx.y * 16 + tx;
    if (cw < Mc) {
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) zs[((int64_t)k1 * Mc + cw) * nin + qw] = sb[k1][ty][tx];
    }
}

// Pass 3: v[k1] = Z[(k1 * Mc + c) * nin + q2] conj(W_n^{q2 k1}); inverse N1-point
// DFT over k1; outputs q1 >= N1/2 go to Y row (q1 - N1/2) nin + q2.
template <typename T, int N1>
__global__ __launch_bounds__(256) void k_mp_pass3(const UpdTask<T> *__restrict__ tasks, const cplx<T> *__restrict__ tw,
                                                  int64_t nmax, const cplx<T> *__restrict__ zs, int64_t c0,
                                                  int64_t Mc, int nin)
{
    __shared__ cplx<T> sb[N1][16][17];
    const UpdTask<T> tk = tasks[0];
    const int64_t M = tk.M;
    const int64_t n = (int64_t)N1 * nin;
    const int64_t tws = nmax / n;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    // read: thread (ty -> column, tx -> q2), q2-contiguous
    const int64_t cr = (int64_t)blockIdx.x * 16 + ty;
    const int qr = blockIdx.y * 16 + tx;
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
        sb[k1][ty][tx] = (cr < Mc) ? zs[((int64_t)k1 * Mc + cr) * nin + qr] : cplx<T>{0, 0};
    __syncthreads();
    const int64_t cl = (int64_t)blockIdx.x * 16 + tx;
    const int q2 = blockIdx.y * 16 + ty;
    cplx<T> v[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = sb[k1][tx][ty];
    cplx<T> pa[lg2<N1>::v];
    twiddle_bases<N1>(pa, tw, (int64_t)q2 * tws);
    apply_twiddles_b<N1, true>(v, pa);
    dft_reg<N1, true, false>(v);
    if (cl < Mc) {
        const int64_t col = 2 * (c0 + cl);
        const T scale = (T)(tk.alpha / (double)n);
        FS_G T *__restrict__ yb = gptr(tk.y) + tk.ylo * M;
#pragma unroll
        for (int q1 = N1 / 2; q1 < N1; ++q1) {
            const int64_t p = (int64_t)(q1 - N1 / 2) * nin + q2;
            if (p < tk.ny) {
                add_pair(yb + p * M, col, M, v[q1], scale);
                if (p < corner_width(tk.s) - 1) corner_add(tk, (int)p, col, M);
            }
        }
    }
}

// ------------------------------------------------------ spectra (setup)
// Radix-2 Stockham pass over a global complex buffer of length n:
//   for j < n/2, k = j mod Ns: a = x[j], b = x[j + n/2] W_{2Ns}^k,
//   y[(j/Ns)*2Ns + k] = a + b,  y[(j/Ns)*2Ns + k + Ns] = a - b.
// After log2(n) passes y = DFT_n(x) in natural order.
__global__ void k_stockham_pass(const cplx<double> *__restrict__ x, cplx<double> *__restrict__ y, int64_t n,
                                int64_t Ns, const cplx<double> *__restrict__ tw, int64_t nmax)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n / 2; j += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = j % Ns;
        cplx<double> a = x[j], b = x[j + n / 2];
        if (k) b = cmul(b, tw[k * (nmax / (2 * Ns))]);
        int64_t o = (j / Ns) * 2 * Ns + k;
        y[o] = cadd(a, b);
        y[o + Ns] = csub(a, b);
    }
}

__global__ void k_real_to_cplx(const double *__restrict__ w, int64_t n, int64_t d0, cplx<double> *__restrict__ out)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        out[j] = {j < d0 ? 0.0 : w[j], 0.0};
}

__global__ void k_spec_store(const cplx<double> *__restrict__ in, int64_t n, cplx<double> *__restrict__ s64,
                             cplx<float> *__restrict__ s32)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        cplx<double> v = in[j];
        if (s64) s64[j] = v;
        if (s32) s32[j] = {(float)v.x, (float)v.y};
    }
}

// spec = DFT_{2s}(w'), w'_j = w_j for j >= corner_width(s), 0 below (the
// near-corner terms are added exactly: by the float64 three-digit update
// kernels as they store Y, by the last multipass pass, else by k_corner);
// scratch holds 2*2s complex entries.
hipError_t launch_spectrum(hipStream_t st, const double *w, int s, cplx<double> *spec64, cplx<float> *spec32,
                           const cplx<double> *tw, int64_t nmax, cplx<double> *scratch)
{
    const int64_t n = 2 * (int64_t)s;
    cplx<double> *b0 = scratch, *b1 = scratch + n;
    unsigned nb = (unsigned)((n + 255) / 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_real_to_cplx, dim3(nb), dim3(256), 0, st, w, n, (int64_t)corner_width(s), b0);
    cplx<double> *src = b0, *dst = b1;
    for (int64_t Ns = 1; Ns < n; Ns *= 2) {
        hipLaunchKernelGGL(k_stockham_pass, dim3(nb), dim3(256), 0, st, src, dst, n, Ns, tw, nmax);
        cplx<double> *tmp = src;
        src = dst;
        dst = tmp;
    }
    hipLaunchKernelGGL(k_spec_store, dim3(nb), dim3(256), 0, st, src, n, spec64, spec32);
    return hipGetLastError();
}

// ------------------------------------------------------------ dispatch
// Single-pass factorisations and complex columns per workgroup.
// Workgroups of a persistent launch: as many as fill the chip at the
// kernel's LDS use (160 KiB per CU, 256 CUs, at most 8 per CU), and no more
// than the launch has column groups (at most ntasks x groups of the widest).
static unsigned persistent_groups(size_t lds_bytes, int64_t groups, int ntasks)
{
    int64_t per_cu = (int64_t)((160 * 1024) / (lds_bytes ? lds_bytes : 1));
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 8) per_cu = 8;
    int64_t np = 256 * per_cu;
    if (np > groups * ntasks) np = groups * ntasks;
    if (np < 1) np = 1;
    return (unsigned)np;
}

template <typename T, int MODE, bool EVEN = false>
static hipError_t single_pass(hipStream_t st, const UpdTask<T> *d_tasks, int ntasks, int n, int64_t ncols_c,
                              const cplx<T> *tw, int64_t nmax, cplx<T> *zs, int64_t Mc, int N1g, int nk1,
                              const int64_t *gbase = nullptr)
{
    auto grid = [&](int CC) {
        unsigned gx = (unsigned)((ncols_c + CC - 1) / CC);
        return (MODE == MODE_UPDATE) ? dim3(gx, 1, (unsigned)ntasks) : dim3(gx, (unsigned)nk1, 1);
    };
    auto pgrid = [&](int CC, size_t lds) {
        const int64_t groups = (ncols_c + CC - 1) / CC;
        return dim3(persistent_groups(lds, groups, ntasks), 1, 1);
    };
#define FS_F2(N1_, N2_, CC_)                                                                                     \
    case N1_ * N2_:                                                                                              \
        hipLaunchKernelGGL((k_fft2_inner<T, N1_, N2_, CC_>), grid(CC_), dim3(256), 0, st, d_tasks, tw, nmax, zs,  \
                           Mc, N1g);                                                                             \
        return hipGetLastError();
#define FS_F3(N1_, N2_, N3_, CC_)                                                                                 \
    case N1_ * N2_ * N3_:                                                                                         \
        hipLaunchKernelGGL((k_fft3_inner<T, N1_, N2_, N3_, CC_>), grid(CC_), dim3(256), 0, st, d_tasks, tw, nmax, \
                           zs, Mc, N1g);                                                                          \
        return hipGetLastError();
#define FS_U2(N1_, N2_, CC_)                                                                                   \
    case N1_ * N2_:                                                                                            \
        if (CC_ != fft_update_cc(n, sizeof(T) == 4)) return hipErrorInvalidValue;                             \
        hipLaunchKernelGGL((k_fft2u<T, N1_, N2_, CC_, EVEN>), pgrid(CC_, sizeof(cplx<T>) * N1_ * (N2_ * CC_ + 1)),   \
                           dim3(256), 0, st, d_tasks, gbase, ntasks, tw, nmax);                                       \
        return hipGetLastError();
#define FS_U3(N1_, N2_, N3_, CC_, NT_)                                                                         \
    case N1_ * N2_ * N3_:                                                                                      \
        if (CC_ != fft_update_cc(n, sizeof(T) == 4)) return hipErrorInvalidValue;                             \
        hipLaunchKernelGGL((k_fft3u<T, N1_, N2_, N3_, CC_, NT_, EVEN>),                                              \
                           pgrid(CC_, sizeof(cplx<T>) * N1_ * N2_ * (N3_ * CC_ + 1)), dim3(NT_), 0, st, d_tasks, \
                           gbase, ntasks, tw, nmax);                                                           \
        return hipGetLastError();
    if constexpr (MODE == MODE_UPDATE) {
        if constexpr (sizeof(T) == 8) {
            switch (n) {
                FS_U2(4, 2, 8)
                FS_U2(4, 4, 8)
                FS_U2(8, 4, 8)
                FS_U2(8, 8, 8)
                FS_U2(16, 8, 8)
                FS_U2(16, 16, 8)
                FS_U3(16, 8, 4, 8, 256)
                FS_U3(16, 8, 8, 8, 256)
                FS_U3(16, 16, 8, 4, 256)
                FS_U3(16, 16, 16, 2, 256)
                FS_U3(16, 16, 32, 1, 256)
                default:
                    return hipErrorInvalidValue;
            }
        } else {
            switch (n) {
                FS_U2(4, 2, 8)
                FS_U2(4, 4, 8)
                FS_U2(8, 4, 8)
                FS_U2(8, 8, 8)
                FS_U2(16, 8, 8)
                FS_U2(16, 16, 8)
                FS_U3(16, 8, 4, 8, 256)
                FS_U3(16, 8, 8, 8, 256)
                FS_U3(16, 16, 8, 8, 256)
                FS_U3(16, 16, 16, 4, 256)
                FS_U3(16, 16, 32, 2, 256)
                FS_U3(16, 32, 32, 1, 256)
                default:
                    return hipErrorInvalidValue;
            }
        }
#undef FS_U2
#undef FS_U3
    } else {
    if constexpr (sizeof(T) == 8) {
        switch (n) {
            FS_F2(4, 2, 8)
            FS_F2(4, 4, 8)
            FS_F2(8, 4, 8)
            FS_F2(8, 8, 8)
            FS_F2(16, 8, 8)
            FS_F2(16, 16, 8)
            FS_F2(32, 16, 8)
            FS_F2(32, 32, 8)
            FS_F3(16, 16, 8, 4)
            FS_F3(16, 16, 16, 2)
            FS_F3(32, 16, 16, 1)
            default:
                return hipErrorInvalidValue;
        }
    } else {
        switch (n) {
            FS_F2(4, 2, 8)
            FS_F2(4, 4, 8)
            FS_F2(8, 4, 8)
            FS_F2(8, 8, 8)
            FS_F2(16, 8, 8)
            FS_F2(16, 16, 8)
            FS_F2(32, 16, 8)
            FS_F2(32, 32, 8)
            FS_F3(16, 16, 8, 8)
            FS_F3(16, 16, 16, 4)
            FS_F3(32, 16, 16, 2)
            FS_F3(32, 32, 16, 1)
            default:
                return hipErrorInvalidValue;
        }
    }
    }
#undef FS_F2
#undef FS_F3
}

int fft_max_single_pass(bool fp32) { return fp32 ? 16384 : 8192; }

template <typename T>
static hipError_t multipass(hipStream_t st, const UpdTask<T> *d_task, int n, int64_t M, const cplx<T> *tw,
                            int64_t nmax, cplx<T> *zs, size_t zs_elems)
{
    const int nin = fft_max_single_pass(sizeof(T) == 4);
    const int N1 = n / nin;
    const int64_t Mc_all = (M + 1) / 2;
    int64_t chunk = (int64_t)(zs_elems / (size_t)n);
    if (chunk >= Mc_all) {
        chunk = Mc_all;
    } else {
        chunk = (chunk / 16) * 16;
        if (chunk < 16) return hipErrorInvalidValue;
    }
    for (int64_t c0 = 0; c0 < Mc_all; c0 += chunk) {
        int64_t Mc = (Mc_all - c0 < chunk) ? Mc_all - c0 : chunk;
        dim3 g13((unsigned)((Mc + 15) / 16), (unsigned)(nin / 16));
#define FS_P1(N1_) \
    case N1_: hipLaunchKernelGGL((k_mp_pass1<T, N1_>), g13, dim3(256), 0, st, d_task, tw, nmax, zs, c0, Mc, nin); break;
        switch (N1) {
            FS_P1(2)
            FS_P1(4)
            FS_P1(8)
            FS_P1(16)
            default:
                return hipErrorInvalidValue;
        }
#undef FS_P1
        hipError_t e = single_pass<T, MODE_INNER>(st, d_task, 1, nin, Mc, tw, nmax, zs, Mc, N1, N1);
        if (e != hipSuccess) return e;
#define FS_P3(N1_) \
    case N1_: hipLaunchKernelGGL((k_mp_pass3<T, N1_>), g13, dim3(256), 0, st, d_task, tw, nmax, zs, c0, Mc, nin); break;
        switch (N1) {
            FS_P3(2)
            FS_P3(4)
            FS_P3(8)
            FS_P3(16)
            default:
                return hipErrorInvalidValue;
        }
#undef FS_P3
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Entry: tasks of one level (all with the same s).  Multi-pass levels take
// exactly one task and need the scratch buffer zs (zs_elems complex entries).
// Float64 level products of the three-digit kernels (2s >= 512, single pass)
// add the near-corner band themselves.
bool fft_band_in_update(int s, bool fp32) { return !fp32 && 2 * s >= 512 && 2 * s <= fft_max_single_pass(false); }

template <typename T>
hipError_t launch_fft_corner(hipStream_t st, const UpdTask<T> *d_tasks, int ntasks, int s, int64_t maxM)
{
    if (2 * s > fft_max_single_pass(sizeof(T) == 4) || corner_width(s) < 2 || fft_band_in_update(s, sizeof(T) == 4))
        return hipSuccess;
    hipLaunchKernelGGL((k_corner<T>), dim3((unsigned)((maxM + 255) / 256), (unsigned)(corner_width(s) - 1),
                                           (unsigned)ntasks),
                       dim3(256), 0, st, d_tasks);
    return hipGetLastError();
}

// Complex columns per column group of the single-pass update kernels (the
// CC of the dispatch tables of single_pass, MODE_UPDATE).
int fft_update_cc(int n, bool fp32)
{
    if (n <= 1024) return 8;
    if (!fp32) return n == 2048 ? 4 : (n == 4096 ? 2 : 1);
    return n == 2048 ? 8 : (n == 4096 ? 4 : (n == 8192 ? 2 : 1));
}

template <typename T>
hipError_t launch_fft_update_ex(hipStream_t st, const UpdTask<T> *d_tasks, const int64_t *gbase, int ntasks, int s,
                                int64_t maxM, const cplx<T> *tw, int64_t nmax, cplx<T> *zs, size_t zs_elems,
                                bool even, bool corner)
{
    const int n = 2 * s;
    if (n <= fft_max_single_pass(sizeof(T) == 4)) {
        if (!gbase) return hipErrorInvalidValue;
        hipError_t e = even ? single_pass<T, MODE_UPDATE, true>(st, d_tasks, ntasks, n, (maxM + 1) / 2, tw, nmax,
                                                                nullptr, 0, 1, 1, gbase)
                            : single_pass<T, MODE_UPDATE, false>(st, d_tasks, ntasks, n, (maxM + 1) / 2, tw, nmax,
                                                                 nullptr, 0, 1, 1, gbase);
        if (e != hipSuccess || !corner) return e;
        return launch_fft_corner<T>(st, d_tasks, ntasks, s, maxM);
    }
    if (ntasks != 1) return hipErrorInvalidValue;
    return multipass<T>(st, d_tasks, n, maxM, tw, nmax, zs, zs_elems);
}

template hipError_t launch_fft_update_ex<double>(hipStream_t, const UpdTask<double> *, const int64_t *, int, int,
                                                int64_t, const cplx<double> *, int64_t, cplx<double> *, size_t,
                                                bool, bool);
template hipError_t launch_fft_corner<double>(hipStream_t, const UpdTask<double> *, int, int, int64_t);
template hipError_t launch_fft_corner<float>(hipStream_t, const UpdTask<float> *, int, int, int64_t);
template hipError_t launch_fft_update_ex<float>(hipStream_t, const UpdTask<float> *, const int64_t *, int, int,
                                               int64_t, const cplx<float> *, int64_t, cplx<float> *, size_t, bool,
                                               bool);

}  // namespace fs
