// Leaf of the time recursion, scan form (default leaf solver).
//
// The diagonal block A0 = a_0 I + K, K = e tridiag(-1, 2, -1) with
// Dirichlet ends (the matrix A of eq. e20 with uniform diagonal), has the
// closed-form inverse of a symmetric tridiagonal Toeplitz matrix.  With
// cosh(theta) = 1 + a_0 / (2 e), rho = exp(-theta),
//   alpha_i = 1 - rho^(2 i),  beta_i = 1 - rho^(2 (M+1-i)),
//   K0 = 1 / (e (1/rho - rho) (1 - rho^(2 (M+1)))),
// (A0^-1)_{ij} = K0 rho^|i-j| alpha_min(i,j) beta_max(i,j), so
//   x_i = K0 (beta_i P_i + alpha_i Q_i),
//   P_i = rho P_{i-1} + alpha_i r_i,      Q_i = rho (Q_{i+1} + beta_{i+1} r_{i+1}),
// two first-order recurrences with a common multiplier rho <= 1.  Each thread
// owns PT consecutive rows; the recurrences are folded per thread, combined
// across the workgroup by an inclusive scan (multiplier rho^PT per thread:
// shuffles inside a wave, one LDS exchange of wave totals between waves), and
// unfolded again with the carries.  One barrier per time step; no table per
// row beyond alpha and beta.  theta = log1p(d + sqrt(d (2 + d))), d =
// a_0 / (2 e), keeps a_0 exact even when it is tiny next to 2 e, where
// forming the diagonal a_0 + 2 e in float64 would round a_0 away.
//
// In-leaf history is pushed forward in registers as in the PCR leaf.
#include "common.hpp"

namespace fs {

template <int X>
struct slog2 {
    static constexpr int value = 1 + slog2<X / 2>::value;
};
template <>
struct slog2<1> {
    static constexpr int value = 0;
};

// DPP lane moves of a double (two 32-bit halves); lanes without a source
// receive 0.  CTRL: 0x110+d = row_shr:d, 0x100+d = row_shl:d (inside rows
// of 16 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Table layout (doubles): [0] K0, [1] rho, [8 + s] = rho^(PT 2^s) for
// s < log2(NT) (<= 10), [32 + r] alpha of row r (r < NT*PT), then beta.
constexpr int SCAN_TAB_ALPHA = 32;

template <int NT, int PT>
__global__ __launch_bounds__(NT) void k_scan_factor(int64_t M, double a0, double e, double *__restrict__ tab)
{
    constexpr int S = slog2<NT>::value;
    constexpr int MP = NT * PT;
    const double dlt = a0 / (2.0 * e);
    const double th = log1p(dlt + sqrt(dlt * (2.0 + dlt)));
    const int t = threadIdx.x;
    if (t == 0) {
        double gam = -expm1(-2.0 * (double)(M + 1) * th);
        tab[0] = 1.0 / (e * 2.0 * sinh(th) * gam);
        tab[1] = exp(-th);
        for (int s = 0; s < (S > 7 ? S : 7); ++s) tab[8 + s] = exp(-(double)PT * (double)(1 << s) * th);
    }
    for (int r = t; r < MP; r += NT) {
        double i = (double)(r + 1);
        bool real = r < M;
        tab[SCAN_TAB_ALPHA + r] = real ? -expm1(-2.0 * i * th) : 0.0;
        tab[SCAN_TAB_ALPHA + MP + r] = real ? -expm1(-2.0 * ((double)(M + 1) - i) * th) : 0.0;
    }
}

template <int NT, int PT, int L, bool MIXED>
__global__ __launch_bounds__(NT) void k_leaf_scan(const LeafTask *__restrict__ tasks)
{
    static_assert(PT % 2 == 0, "rows per thread must be even");
    constexpr int S = slog2<NT>::value;
    constexpr int NW = NT / 64;
    constexpr int MP = NT * PT;
    constexpr int UT = PT / 2;  // 16-byte units per thread
    __shared__ double sW[2][2][NW > 1 ? NW : 1];

    const LeafTask tk = tasks[blockIdx.x];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = t >> 6;
    const double *__restrict__ tab = tk.fac;
    const int64_t M = tk.M;
    const int c0 = t * PT;
    const int nrows = tk.nrows;
    double *__restrict__ u = tk.u + tk.lo * M;
    const float *__restrict__ hist = MIXED ? tk.hist + tk.lo * M : nullptr;
    float *__restrict__ x32 = MIXED ? tk.x32 + tk.lo * M : nullptr;
    // the thread's PT rows are whole 16-byte units inside the field
    const bool vec = ((M & 1) == 0) && ((((uintptr_t)tk.u) & 15) == 0) && (c0 + PT <= M);

    // right-hand sides of the leaf's rows: the thread's PT consecutive
    // entries of each row, as 16-byte loads (lanes 32 bytes apart)
    double acc[L][PT];
#pragma unroll
    for (int r = 0; r < L; ++r) {
        const double *row = u + (int64_t)r * M + c0;
        if (r < nrows && vec) {
#pragma unroll
            for (int i = 0; i < UT; ++i) {
                const double2 v = reinterpret_cast<const double2 *>(row)[i];
                acc[r][2 * i] = v.x;
                acc[r][2 * i + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < PT; ++k) acc[r][k] = (r < nrows && c0 + k < M) ? row[k] : 0.0;
        }
        if (MIXED && r < nrows) {
#pragma unroll
            for (int k = 0; k < PT; ++k)
                if (c0 + k < M) acc[r][k] += (double)hist[(int64_t)r * M + c0 + k];
        }
    }

    const double K0 = tab[0];
    const double rho = tab[1];
    double mult[S > 7 ? S : 7];
#pragma unroll
    for (int s = 0; s < (S > 7 ? S : 7); ++s) mult[s] = tab[8 + s];
    double al[PT], be[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        al[k] = tab[SCAN_TAB_ALPHA + c0 + k];
        be[k] = tab[SCAN_TAB_ALPHA + MP + c0 + k];
    }
    // per-lane powers m^(lane mod 16) and m^(15 - lane mod 16), m = rho^PT,
    // and the row/wave strides m^16, m^32, m^48, m^64
    double m_lo = 1.0, m_hi = 1.0;
    {
        const int el = lane & 15, eh = 15 - (lane & 15);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (el & (1 << s)) m_lo *= mult[s];
            if (eh & (1 << s)) m_hi *= mult[s];
        }
    }
    const double m16 = mult[4], m32 = mult[5], m48 = mult[4] * mult[5];
    const double m64 = (S > 6) ? mult[6 < S ? 6 : 0] : 0.0;
    double aw[L];
#pragma unroll
    for (int m = 0; m < L; ++m) aw[m] = (m > 0) ? tk.a[m] : 0.0;

    int par = 0;
    // Rolled step loop: acc[0] holds the current row's right-hand side and
    // acc[j] the row j steps ahead; after a step every row moves down by one.
    // The push below therefore always uses a_j for acc[j].
#pragma unroll 1
    for (int r = 0; r < nrows; ++r) {
        {
            // fold the two recurrences over the thread's rows
            double Tf = 0.0, Tb = 0.0;
#pragma unroll
            for (int k = 0; k < PT; ++k) Tf = rho * Tf + al[k] * acc[0][k];
#pragma unroll
            for (int k = PT - 1; k >= 0; --k) Tb = rho * (Tb + be[k] * acc[0][k]);
            // Row-local (16 lanes) inclusive scans by DPP shifts:
            //   prefix  R_t = sum_{t' <= t in row} m^(t-t') Tf(t')
            //   suffix  S_t = sum_{t' >= t in row} m^(t'-t) Tb(t')
            double Rf = Tf, Rb = Tb;
            Rf += mult[0] * dpp_move<0x111>(Rf);
            Rb += mult[0] * dpp_move<0x101>(Rb);
            Rf += mult[1] * dpp_move<0x112>(Rf);
            Rb += mult[1] * dpp_move<0x102>(Rb);
            Rf += mult[2] * dpp_move<0x114>(Rf);
            Rb += mult[2] * dpp_move<0x104>(Rb);
            Rf += mult[3] * dpp_move<0x118>(Rf);
            Rb += mult[3] * dpp_move<0x108>(Rb);
            // row totals (uniform): forward at lanes 15, 31, 47, 63, backward at 0, 16, 32, 48
            const double f0 = read_lane(Rf, 15), f1 = read_lane(Rf, 31), f2 = read_lane(Rf, 47),
                         f3 = read_lane(Rf, 63);
            const double b0 = read_lane(Rb, 0), b1 = read_lane(Rb, 16), b2 = read_lane(Rb, 32),
                         b3 = read_lane(Rb, 48);
            // wave-level prefix at the end of rows 0..3 and suffix at the start of rows 3..0
            const double W15 = f0, W31 = f1 + m16 * W15, W47 = f2 + m16 * W31, W63 = f3 + m16 * W47;
            const double V48 = b3, V32 = b2 + m16 * V48, V16 = b1 + m16 * V32, V0 = b0 + m16 * V16;
            double Cf = 0.0, Cb = 0.0;  // prefix before this wave, suffix after it
            if (NW > 1) {
                if (lane == 0) {
                    sW[par][0][wv] = W63;
                    sW[par][1][wv] = V0;
                }
                __syncthreads();
                double tf[NW], tb[NW];
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    tf[w] = sW[par][0][w];
                    tb[w] = sW[par][1][w];
                }
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    if (w < wv) Cf = Cf * m64 + tf[w];
#pragma unroll
                for (int w = NW - 1; w >= 0; --w)
                    if (w > wv) Cb = Cb * m64 + tb[w];
                par ^= 1;
            }
            // exclusive carries: prefix up to the row before this thread's
            // rows, suffix from the row after them
            const int rw = lane >> 4;
            const double Gf = (rw == 0) ? Cf
                            : (rw == 1) ? W15 + m16 * Cf
                            : (rw == 2) ? W31 + m32 * Cf
                                        : W47 + m48 * Cf;
            const double Gb = (rw == 3) ? Cb
                            : (rw == 2) ? V48 + m16 * Cb
                            : (rw == 1) ? V32 + m32 * Cb
                                        : V16 + m48 * Cb;
            const double cf = dpp_move<0x111>(Rf) + m_lo * Gf;
            const double cb = dpp_move<0x101>(Rb) + m_hi * Gb;
            // unfold with the carries: P forward, Q backward
            double x[PT];
            double P = cf;
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                P = rho * P + al[k] * acc[0][k];
                x[k] = be[k] * P;
            }
            double Q = cb;
#pragma unroll
            for (int k = PT - 1; k >= 0; --k) {
                x[k] = K0 * (x[k] + al[k] * Q);
                Q = rho * (Q + be[k] * acc[0][k]);
            }
            double *row = u + (int64_t)r * M + c0;
            if (vec) {
#pragma unroll
                for (int i = 0; i < UT; ++i)
                    reinterpret_cast<double2 *>(row)[i] = double2{x[2 * i], x[2 * i + 1]};
            } else {
#pragma unroll
                for (int k = 0; k < PT; ++k)
                    if (c0 + k < M) row[k] = x[k];
            }
            if (MIXED) {
#pragma unroll
                for (int k = 0; k < PT; ++k)
                    if (c0 + k < M) x32[(int64_t)r * M + c0 + k] = (float)x[k];
            }
#pragma unroll
            for (int j = 1; j < L; ++j) {
#pragma unroll
                for (int k = 0; k < PT; ++k) acc[j - 1][k] = acc[j][k] - aw[j] * x[k];
            }
        }
    }
}

// Up to 512 threads (two waves per SIMD) with 2, 4 or 8 rows per thread: the
// leaf's right-hand sides and accumulators (L x PT doubles per thread) stay
// in registers and each thread's rows are whole 16-byte units.
LeafCfg scan_config(int64_t M)
{
    if (M <= 128) return {64, 2, 6};
    if (M <= 256) return {64, 4, 6};
    if (M <= 512) return {128, 4, 7};
    if (M <= 1024) return {256, 4, 8};
    if (M <= 2048) return {512, 4, 9};
    return {512, 8, 9};
}

size_t scan_table_doubles(const LeafCfg &c) { return (size_t)SCAN_TAB_ALPHA + 2 * (size_t)c.nt * c.pt; }

hipError_t launch_scan_factor(hipStream_t st, const LeafCfg &c, int64_t M, double a0, double e, double *tab)
{
#define FS_SF(NT_, PT_)                                                                                \
    if (c.nt == NT_ && c.pt == PT_) {                                                                  \
        hipLaunchKernelGGL((k_scan_factor<NT_, PT_>), dim3(1), dim3(NT_), 0, st, M, a0, e, tab);       \
        return hipGetLastError();                                                                      \
    }
    FS_SF(64, 2)
    FS_SF(64, 4)
    FS_SF(128, 4)
    FS_SF(256, 4)
    FS_SF(512, 4)
    FS_SF(512, 8)
#undef FS_SF
    return hipErrorInvalidValue;
}

template <int NT, int PT, int L>
static hipError_t scan_go(hipStream_t st, bool mixed, const LeafTask *d_tasks, int ntasks)
{
    if (mixed)
        hipLaunchKernelGGL((k_leaf_scan<NT, PT, L, true>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
    else
        hipLaunchKernelGGL((k_leaf_scan<NT, PT, L, false>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
    return hipGetLastError();
}

template <int NT, int PT>
static hipError_t scan_go16(hipStream_t st, bool mixed, const LeafTask *d_tasks, int ntasks)
{
    if constexpr (PT <= 2)
        return scan_go<NT, PT, 16>(st, mixed, d_tasks, ntasks);
    else
        return hipErrorInvalidValue;
}

hipError_t launch_leaf_scan(hipStream_t st, const LeafCfg &c, int L, const LeafTask *d_tasks, int ntasks,
                            bool mixed)
{
#define FS_SL(NT_, PT_)                                                              \
    if (c.nt == NT_ && c.pt == PT_) {                                                \
        if (L == 4) return scan_go<NT_, PT_, 4>(st, mixed, d_tasks, ntasks);         \
        if (L == 8) return scan_go<NT_, PT_, 8>(st, mixed, d_tasks, ntasks);         \
        if (L == 16 && PT_ <= 2) return scan_go16<NT_, PT_>(st, mixed, d_tasks, ntasks);   \
        return hipErrorInvalidValue;                                                 \
    }
    FS_SL(64, 2)
    FS_SL(64, 4)
    FS_SL(128, 4)
    FS_SL(256, 4)
    FS_SL(512, 4)
    FS_SL(512, 8)
#undef FS_SL
    return hipErrorInvalidValue;
}

}  // namespace fs
