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
//   P_i = sum_{j <= i} rho^(i-j) alpha_j r_j,   Q_i = sum_{j > i} rho^(j-i) beta_j r_j,
// two first-order recurrences with the common multiplier rho <= 1.
// theta = log1p(d + sqrt(d (2 + d))), d = a_0 / (2 e), keeps a_0 exact even
// when it is tiny next to 2 e, where forming the diagonal a_0 + 2 e in
// float64 would round a_0 away; when a_0 >> e instead, K0 and rho are formed
// from d and sinh(theta) = sqrt(d (2 + d)) without theta (whose absolute
// rounding grows with theta).
//
// Work split.  Thread t owns the PT consecutive rows c0+1 .. c0+PT
// (c0 = t PT).  Per time step it forms the local prefix l_k and suffix s_k
// of its rows (carry-free), so that
//   P_{c0+1+k} = l_k + rho^(k+1) P_{c0},
//   Q_{c0+1+k} = rho s_{k+1} + rho^(PT-1-k) Q_{c0+PT},
// and the two carries P_{c0}, Q_{c0+PT} are exclusive scans of the thread
// totals with multiplier m = rho^PT.  The scans run in three levels: DPP
// shifts inside rows of 16 lanes, one LDS exchange of the row totals (the
// only barrier of the step), and a DPP scan of those totals over the first
// lanes of every wave; each lane then fetches its row's carry with a lane
// permute.  The whole leaf (L steps) is unrolled: the in-leaf history
// sum_{j<n} a_{n-j} x_j is pushed into the later rows' right-hand sides in
// registers (the next row at once, the rest together with the store of x_j
// during the following step), touching only rows still in the leaf.  The
// fields are read and written in the internal column order of ColPerm, so
// that each wave's row accesses are contiguous.
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

// Table layout (doubles):
//   [0] K0, [1] rho, [2] e,
//   [8 + s]  m^(2^s), m = rho^PT, s < 16,
//   [24 + k] rho^(k+1), k < 16,
//   [SCAN_TAB_ALPHA + r] sqrt(K0) alpha of row r+1 (r < NT*PT, 0 beyond M),
//   then sqrt(K0) beta: with both scaled, the prefix and suffix sums carry a
//   factor sqrt(K0) each and x = beta' P' + alpha' Q' needs no product with K0.
constexpr int SCAN_TAB_POW = 24;
constexpr int SCAN_TAB_ALPHA = 40;

template <int NT, int PT>
__global__ __launch_bounds__(NT) void k_scan_factor(int64_t M, double a0, double e, double *__restrict__ tab)
{
    constexpr int MP = NT * PT;
    const double dlt = a0 / (2.0 * e);
    const double sh = sqrt(dlt * (2.0 + dlt));  // sinh(theta)
    const double th = log1p(dlt + sh);
    const int t = threadIdx.x;
    // 1/rho - rho = 2 sinh(theta) from sh itself: through theta it would
    // carry theta's absolute rounding (about theta ulp), a systematic error
    // of every leaf solve that the diffusion-wave recurrence amplifies when
    // a_0 >> e (theta of 10 or more)
    const double K0 = 1.0 / (e * 2.0 * sh * -expm1(-2.0 * (double)(M + 1) * th));
    const double sk = sqrt(K0);
    if (t == 0) {
        tab[0] = K0;
        tab[2] = e;  // the coefficient of tridiag(-1, 2, -1) in the block
        if (th < 0.5) {
            // small theta (a_0 << e): exp of the accurately known theta
            tab[1] = exp(-th);
            for (int s = 0; s < 16; ++s) tab[8 + s] = exp(-(double)PT * (double)(1 << s) * th);
            for (int k = 0; k < 16; ++k) tab[SCAN_TAB_POW + k] = exp(-(double)(k + 1) * th);
        } else {
            // large theta: rho = 1 / (cosh + sinh) to a few ulp, its powers
            // by products (rho^k <= e^{-k/2}: the higher ones only couple
            // rows through factors far below the diagonal's)
            const double rho = 1.0 / (1.0 + dlt + sh);
            tab[1] = rho;
            double pk = rho;
            for (int k = 0; k < 16; ++k) {
                tab[SCAN_TAB_POW + k] = pk;
                pk *= rho;
            }
            double m = 1.0;
            for (int k = 0; k < PT; ++k) m *= rho;
            for (int s = 0; s < 16; ++s) {
                tab[8 + s] = m;
                m *= m;
            }
        }
    }
    for (int r = t; r < MP; r += NT) {
        double i = (double)(r + 1);
        bool real = r < M;
        tab[SCAN_TAB_ALPHA + r] = real ? -sk * expm1(-2.0 * i * th) : 0.0;
        tab[SCAN_TAB_ALPHA + MP + r] = real ? -sk * expm1(-2.0 * ((double)(M + 1) - i) * th) : 0.0;
    }
}

// DPP lane move of a double (two 32-bit halves).  Lanes without a source,
// or outside ROWMASK, receive 0.  CTRL: 0x110+d row_shr:d, 0x100+d
// row_shl:d (inside rows of 16 lanes), 0x142 row_bcast:15.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_move(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// v from lane src (any lane of the wave)
__device__ __forceinline__ double lane_fetch(double v, int src)
{
    int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// c^e for 0 <= e < 32 from the powers c^(2^s) in pw[0..4]
__device__ __forceinline__ double pow_bits(const double *pw, int e)
{
    double r = 1.0;
#pragma unroll
    for (int s = 0; s < 5; ++s)
        if (e & (1 << s)) r *= pw[s];
    return r;
}

// Inclusive scans over the 16 lanes of each row with lane multiplier c:
//   fwd: S_l = sum_{l' <= l} c^(l-l') v_l',  bwd: S_l = sum_{l' >= l} c^(l'-l) v_l'.
// cp[s] = c^(2^s).  Only the first NL (power of two <= 16) lanes of a row
// carry data when NL < 16.
template <int NL>
__device__ __forceinline__ void row_scans(double &f, double &b, const double *cp)
{
    f = fma(cp[0], dpp_move<0x111>(f), f);
    b = fma(cp[0], dpp_move<0x101>(b), b);
    if constexpr (NL > 2) {
        f = fma(cp[1], dpp_move<0x112>(f), f);
        b = fma(cp[1], dpp_move<0x102>(b), b);
    }
    if constexpr (NL > 4) {
        f = fma(cp[2], dpp_move<0x114>(f), f);
        b = fma(cp[2], dpp_move<0x104>(b), b);
    }
    if constexpr (NL > 8) {
        f = fma(cp[3], dpp_move<0x118>(f), f);
        b = fma(cp[3], dpp_move<0x108>(b), b);
    }
}

// CN: the lag-1 block is a_1 I + e tridiag(-1, 2, -1) (the spatial term
// averaged over two time levels; the diagonal block is then a_0 I + e
// tridiag(-1, 2, -1) with the same e): pushing x_r into the next row also
// subtracts e (2 x_i - x_{i-1} - x_{i+1}), with the neighbours across
// threads exchanged through LDS (one more barrier per step).
// PAIR: the task covers two leaves (up to 2L rows) and applies between them
// the level product of half-size L (rows L..2L-1 minus the Toeplitz block
// a_{L+p-q} times rows 0..L-1), so one launch replaces leaf, dense level
// product, leaf.  Each thread re-reads its own columns of the first leaf's
// solution rows, which it has just stored.
template <int NT, int PT, int L, bool MIXED, int VEC, bool CN = false, bool PAIR = false>
__global__ __launch_bounds__(NT) void k_leaf_scan(TaskRef<LeafTask> tr)
{
    static_assert(PT % 2 == 0 && PT <= 16, "rows per thread must be even and at most 16");
    constexpr int NR = NT / 16;  // rows of 16 lanes in the workgroup (<= 32)
    static_assert(NR <= 32, "at most 512 threads");
    constexpr int MP = NT * PT;
    constexpr int UT = PT / 2;
    __shared__ double sR[2][2][NR];  // [parity][forward/backward][row]
    __shared__ double sE[CN ? 2 : 1][2][CN ? NT : 1];  // CN: [parity][first/last][thread]

    const LeafTask tk = get_task(tr, blockIdx.x);
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int rl = lane & 15;  // position inside the row
    const int G = t >> 4;      // row index in the workgroup
    FS_G const double *__restrict__ tab = gptr(tk.fac);
    const int64_t M = tk.M;
    const int c0 = t * PT;
    const int nrows_all = tk.nrows;
    FS_G double *__restrict__ u_base = gptr(tk.u) + tk.lo * M;
    FS_G const float *__restrict__ hist_base = MIXED ? gptr(tk.hist) + tk.lo * M : nullptr;
    FS_G float *__restrict__ x32_base = MIXED ? gptr(tk.x32) + tk.lo * M : nullptr;
    // vec: M is a multiple of PT and the field is 16-byte aligned, so a
    // thread's rows are either all inside [0, M) or all outside.  VEC = 2
    // takes it from the task flags (batches mixing both kinds in one launch).
    const bool vec = (VEC == 2) ? ((tk.flags & LEAF_VEC) != 0) : (VEC == 1);
    const bool act = c0 < M;
    // Memory column of the thread's element k.  In the internal column order
    // ((tk.flags & LEAF_PERM)) a full block of 64 PT columns belongs to one wave, and pair
    // j of lane i sits at 128 j + 2 i, so each of the wave's 16-byte
    // accesses covers 1 KB of contiguous memory.
    constexpr int64_t B = 64 * PT;
    const bool pf = (tk.flags & LEAF_PERM) && (int64_t)((t >> 6) + 1) * B <= M;
    const int64_t cw = (int64_t)(t >> 6) * B + 2 * lane;
    auto col = [&](int k) -> int64_t { return pf ? cw + 128 * (k >> 1) + (k & 1) : (int64_t)c0 + k; };

    // per-row coefficients first (their latency overlaps the field loads)
    double al[PT], be[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        al[k] = tab[SCAN_TAB_ALPHA + c0 + k];
        be[k] = tab[SCAN_TAB_ALPHA + MP + c0 + k];
    }
    // uniform constants
    const double rho = tab[1];
    double mp[4];  // m^(1,2,4,8): lane steps inside a row
#pragma unroll
    for (int s = 0; s < 4; ++s) mp[s] = tab[8 + s];
    double cp[5];  // c^(2^s), c = m^16: row steps
#pragma unroll
    for (int s = 0; s < 5; ++s) cp[s] = tab[12 + s];
    double rp[PT];  // rho^(k+1)
#pragma unroll
    for (int k = 0; k < PT; ++k) rp[k] = tab[SCAN_TAB_POW + k];
    double aw[L];
#pragma unroll
    for (int m = 0; m < L; ++m) aw[m] = (m > 0) ? gptr(tk.a)[m] : 0.0;
    // lane multipliers: m^rl and m^(15-rl) (row carries into a thread);
    // c^((lane&15)+1) for the row_bcast:15 step and c^(16-lane) for the
    // backward step of the row scan (both used only on lanes < NR)
    double mpw[5] = {mp[0], mp[1], mp[2], mp[3], 0.0};
    const double m_lo = pow_bits(mpw, rl);
    const double m_hi = pow_bits(mpw, 15 - rl);
    const double c_b15 = pow_bits(cp, (lane & 15) + 1);
    const double c_bk = pow_bits(cp, 16 - (lane & 15));

    constexpr int NH = PAIR ? 2 : 1;
    // PUSH2 (512 x 4, the configuration of batches up to M = 2048): the
    // second leaf's right-hand sides are loaded with the first leaf's, and
    // each solved row x_q of the first leaf is pushed into them,
    //   acc2[p] -= a_{L+p-q} x_q,  p < L,
    // in the deferred phase of the step after its solve (where the second
    // wave of each SIMD fills the gaps), instead of re-reading the first
    // leaf's rows between the halves.  Measured: c4 batch 161.3 -> 157.4 ms;
    // with one wave per SIMD (256 x 8, c3) the pushes lengthen every step
    // (191 -> 221 ms), and 512 x 8 has no registers left for them.
    constexpr bool PUSH2 = PAIR && !MIXED && !CN && NT == 512 && PT == 4;
    constexpr int L2 = PUSH2 ? L : 1;
    double acc2[L2][PT];
    double ax[PUSH2 ? 2 * L : 1];  // a_0 .. a_{2L-1}
    if constexpr (PUSH2) {
#pragma unroll
        for (int m = 0; m < 2 * L; ++m) ax[m] = gptr(tk.a)[m];
    }
#pragma unroll 1
    for (int hf = 0; hf < NH; ++hf) {
    const int nrows = (hf == 0) ? (nrows_all < L ? nrows_all : L) : nrows_all - L;
    if (nrows <= 0) break;  // whole workgroup
    FS_G double *__restrict__ u = u_base + (int64_t)(hf * L) * M;
    FS_G const float *__restrict__ hist = MIXED ? hist_base + (int64_t)(hf * L) * M : nullptr;
    FS_G float *__restrict__ x32 = MIXED ? x32_base + (int64_t)(hf * L) * M : nullptr;
    // right-hand sides of the leaf's rows (row r of the leaf in acc[r])
    double acc[L][PT];
    auto load_rows = [&](double (&dst)[PT], FS_G const double *row, bool in) {
        if (vec) {
            if (in && act) {
#pragma unroll
                for (int i = 0; i < UT; ++i) {
                    const double2 v = *reinterpret_cast<FS_G const double2 *>(row + col(2 * i));
                    dst[2 * i] = v.x;
                    dst[2 * i + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int k = 0; k < PT; ++k) dst[k] = 0.0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < PT; ++k) dst[k] = (in && c0 + k < M) ? row[col(k)] : 0.0;
        }
    };
    if (PUSH2 && hf == 1) {
#pragma unroll
        for (int r = 0; r < L; ++r)
#pragma unroll
            for (int k = 0; k < PT; ++k) acc[r][k] = acc2[PUSH2 ? r : 0][k];
    } else {
#pragma unroll
        for (int r = 0; r < L; ++r) load_rows(acc[r], u + (int64_t)r * M, r < nrows);
        if constexpr (PUSH2) {
            // the second leaf's rows (none past the task's rows)
#pragma unroll
            for (int r = 0; r < L; ++r) load_rows(acc2[r], u + (int64_t)(L + r) * M, L + r < nrows_all);
        }
    }
    // float32 history rows (mixed mode): row r is loaded one step ahead, in
    // step r - 1 (row 0 with the float64 rows), and added when step r starts
    float hv[PT];
    auto load_hist = [&](int r) {
        FS_G const float *hrow = hist + (int64_t)r * M;
        if (vec) {
            // col(2i) is even and M is even: 8-byte aligned pairs
#pragma unroll
            for (int i = 0; i < UT; ++i) {
                float2 v = float2{0.f, 0.f};
                if (r < nrows && act) v = *reinterpret_cast<FS_G const float2 *>(hrow + col(2 * i));
                hv[2 * i] = v.x;
                hv[2 * i + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < PT; ++k) hv[k] = (r < nrows && c0 + k < M) ? hrow[col(k)] : 0.f;
        }
    };
    if constexpr (PAIR && !PUSH2) {
        if (hf == 1) {
            // the level product of half-size L from the first leaf's rows
            // (this thread's own columns, stored by it in the first half)
            auto load_x = [&](int q, double *xq) {
                FS_G const double *xrow = u_base + (int64_t)q * M;
                if (vec) {
#pragma unroll
                    for (int i = 0; i < UT; ++i) {
                        double2 v = double2{0.0, 0.0};
                        if (act) v = *reinterpret_cast<FS_G const double2 *>(xrow + col(2 * i));
                        xq[2 * i] = v.x;
                        xq[2 * i + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < PT; ++k) xq[k] = (c0 + k < M) ? xrow[col(k)] : 0.0;
                }
            };
            // one row of X in registers at a time (more rows spill at 512 x 8)
#pragma unroll 1
            for (int q = 0; q < L; ++q) {
                double xq[PT];
                load_x(q, xq);
#pragma unroll
                for (int p = 0; p < L; ++p) {
                    const double w = gptr(tk.a)[L + p - q];
#pragma unroll
                    for (int k = 0; k < PT; ++k) acc[p][k] = fma(-w, xq[k], acc[p][k]);
                }
                if constexpr (CN) {
                    if (q == L - 1) {
                        // the lag-1 spatial term from the first leaf's last row;
                        // sE[1] has not been read since the last step's barrier
                        sE[1][0][t] = xq[0];
                        sE[1][1][t] = xq[PT - 1];
                        __syncthreads();
                        const double xl = (t > 0) ? sE[1][1][t - 1] : 0.0;
                        const double xr = (t + 1 < NT) ? sE[1][0][t + 1] : 0.0;
                        const double ec = tab[2];
#pragma unroll
                        for (int k = 0; k < PT; ++k) {
                            const double lft = (k > 0) ? xq[k - 1] : xl;
                            const double rgt = (k < PT - 1) ? xq[k + 1] : xr;
                            acc[0][k] = fma(-ec, 2.0 * xq[k] - lft - rgt, acc[0][k]);
                        }
                    }
                }
            }
        }
    }
    if (MIXED) load_hist(0);

    double xp[PT];  // solution of the previous step, pushed and stored during this step
#pragma unroll
    for (int k = 0; k < PT; ++k) xp[k] = 0.0;

#pragma unroll
    for (int r = 0; r <= L; ++r) {
        const bool run = r < L && r < nrows;
        const int par = r & 1;
        double lf[PT], sb[PT];
        double Sf = 0.0, Sb = 0.0;
        if (MIXED && run) {
#pragma unroll
            for (int k = 0; k < PT; ++k) acc[r][k] += (double)hv[k];
            if (r + 1 < L) load_hist(r + 1);
        }
        if (run) {
            // carry-free local prefix l and suffix s of the thread's rows
            lf[0] = al[0] * acc[r][0];
#pragma unroll
            for (int k = 1; k < PT; ++k) lf[k] = fma(rho, lf[k - 1], al[k] * acc[r][k]);
            sb[PT - 1] = be[PT - 1] * acc[r][PT - 1];
#pragma unroll
            for (int k = PT - 2; k >= 0; --k) sb[k] = fma(rho, sb[k + 1], be[k] * acc[r][k]);
            // thread totals and their row scans (multiplier m per lane)
            Sf = lf[PT - 1];
            Sb = rho * sb[0];
            row_scans<16>(Sf, Sb, mp);
            if (rl == 15) sR[par][0][G] = Sf;
            if (rl == 0) sR[par][1][G] = Sb;
        }
        // the step's barrier, then the reads of the row totals
        double vf = 0.0, vb = 0.0;
        if (run) {
            __syncthreads();
            vf = (lane < NR) ? sR[par][0][lane] : 0.0;
            vb = (lane < NR) ? sR[par][1][lane] : 0.0;
        }
        // deferred work of the previous step: store its solution row and
        // push it into the right-hand sides beyond the next row (the next
        // row itself was updated right after the solve).  It sits after the
        // barrier, where it fills the wait for the row totals' reads and
        // scans instead of delaying every wave's arrival at the barrier.
        // The row's 16-byte stores (32 KB per step from this one CU at
        // M = 4096) are spread over this phase of the step, one part at each
        // of four points pinned by scheduling barriers, rather than issued in
        // one burst: measured about 1% faster per leaf pair.
        constexpr int STORE_PARTS = (UT % 4 == 0) ? 4 : 1;
        static_assert(STORE_PARTS == 1 || STORE_PARTS == 4, "parts 1..3 are issued at fixed points below");
        const bool store_row = r > 0 && r - 1 < nrows;
        FS_G double *const srow = u + (int64_t)(r > 0 ? r - 1 : 0) * M;
        auto store_part = [&](int part) {
            if (store_row && vec && act) {
#pragma unroll
                for (int i = part * (UT / STORE_PARTS); i < (part + 1) * (UT / STORE_PARTS); ++i)
                    *reinterpret_cast<FS_G double2 *>(srow + col(2 * i)) = double2{xp[2 * i], xp[2 * i + 1]};
            }
        };
        if (r > 0 && r - 1 < nrows) {
            FS_G double *row = u + (int64_t)(r - 1) * M;
            if (vec) {
                store_part(0);
                if (STORE_PARTS == 1 || !run) {
#pragma unroll
                    for (int part = 1; part < STORE_PARTS; ++part) store_part(part);
                }
            } else {
#pragma unroll
                for (int k = 0; k < PT; ++k)
                    if (c0 + k < M) row[col(k)] = xp[k];
            }
            if (MIXED) {
                FS_G float *xrow = x32 + (int64_t)(r - 1) * M;
                if (vec) {
                    if (act) {
#pragma unroll
                        for (int i = 0; i < UT; ++i)
                            *reinterpret_cast<FS_G float2 *>(xrow + col(2 * i)) =
                                float2{(float)xp[2 * i], (float)xp[2 * i + 1]};
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < PT; ++k)
                        if (c0 + k < M) xrow[col(k)] = (float)xp[k];
                }
            }
#pragma unroll
            for (int j = r + 1; j < L; ++j) {
#pragma unroll
                for (int k = 0; k < PT; ++k) acc[j][k] = fma(-aw[j - r + 1], xp[k], acc[j][k]);
            }
            if constexpr (PUSH2) {
                if (hf == 0) {
                    // x_{r-1} into the second leaf: a_{L+p-(r-1)}
#pragma unroll
                    for (int p = 0; p < L; ++p)
#pragma unroll
                        for (int k = 0; k < PT; ++k)
                            acc2[p][k] = fma(-ax[PUSH2 ? L + p - r + 1 : 0], xp[k], acc2[p][k]);
                }
            }
        }
        if (!run) break;
        if constexpr (STORE_PARTS > 1) __builtin_amdgcn_sched_barrier(0);
        // scan of the NR row totals (multiplier c = m^16 per row) on lanes < NR
        row_scans<(NR < 16 ? NR : 16)>(vf, vb, cp);
        if constexpr (STORE_PARTS > 1) {
            __builtin_amdgcn_sched_barrier(0);
            store_part(1);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (NR > 16) {
            // rows 0-15 -> 16-31: forward by row_bcast:15 into lanes 16..31,
            // backward by the uniform suffix at lane 16 into lanes 0..15
            vf = fma(c_b15, dpp_move<0x142, 0xA>(vf), vf);
            const double s16 = read_lane(vb, 16);
            vb = (lane < 16) ? fma(c_bk, s16, vb) : vb;
        }
        // carries: P at the row before the thread's rows, Q at its last row
        double Cr = lane_fetch(vf, G > 0 ? G - 1 : 0);
        double Dr = lane_fetch(vb, G < NR - 1 ? G + 1 : 0);
        if constexpr (STORE_PARTS > 1) {
            __builtin_amdgcn_sched_barrier(0);
            store_part(2);
            __builtin_amdgcn_sched_barrier(0);
        }
        Cr = (G > 0) ? Cr : 0.0;
        Dr = (G < NR - 1) ? Dr : 0.0;
        const double cf = fma(m_lo, Cr, dpp_move<0x111>(Sf));
        const double cb = fma(m_hi, Dr, dpp_move<0x101>(Sb));
        if constexpr (STORE_PARTS > 1) {
            __builtin_amdgcn_sched_barrier(0);
            store_part(3);
            __builtin_amdgcn_sched_barrier(0);
        }
        // unfold
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const double P = fma(rp[k], cf, lf[k]);
            const double Q = (k < PT - 1) ? fma(rho, sb[k + 1 < PT ? k + 1 : k], rp[PT - 2 - k >= 0 ? PT - 2 - k : 0] * cb)
                                          : cb;
            xp[k] = fma(be[k], P, al[k] * Q);  // al, be carry sqrt(K0)
        }
        // the next row's right-hand side needs x_r now
        if (r + 1 < L) {
#pragma unroll
            for (int k = 0; k < PT; ++k) acc[r + 1][k] = fma(-aw[1], xp[k], acc[r + 1][k]);
            if constexpr (CN) {
                // columns past M hold x = 0 (their alpha and beta are 0), as do the Dirichlet ends
                sE[par][0][t] = xp[0];
                sE[par][1][t] = xp[PT - 1];
                __syncthreads();
                const double xl = (t > 0) ? sE[par][1][t - 1] : 0.0;
                const double xr = (t + 1 < NT) ? sE[par][0][t + 1] : 0.0;
                const double ec = tab[2];
#pragma unroll
                for (int k = 0; k < PT; ++k) {
                    const double lft = (k > 0) ? xp[k - 1] : xl;
                    const double rgt = (k < PT - 1) ? xp[k + 1] : xr;
                    acc[r + 1][k] = fma(-ec, 2.0 * xp[k] - lft - rgt, acc[r + 1][k]);
                }
            }
        }
    }
    }  // halves
}

// ---- leaf of the advection equations (Schemes 2 and 3) ----
//
// The diagonal block is lower bidiagonal, so each time step is one forward
// recurrence in space,
//   U_i = g r_i + kappa U_{i-1},   U_0 = 0 (inflow value),
// Scheme 3: (a_0 + 1/h) U_i - U_{i-1}/h = r_i, g = 1/(a_0 + 1/h), kappa = g/h;
// Scheme 2: (a_0 + 2/h) U_i + (a_0 - 2/h) U_{i-1} = r_i (twice the scheme,
//   in the unknowns W = B U, W_i = U_i + U_{i-1}, which carry the history),
//   g = 1/(a_0 + 2/h), kappa = (2/h - a_0) g.
// It runs as the forward half of the scan leaf: carry-free local prefixes,
// row scans by DPP, one LDS exchange of row totals, carries by lane fetch.
// Table (doubles): [0] g, [1] kappa, [8 + s] m^(2^s) with m = kappa^PT,
// [24 + k] kappa^(k+1).
constexpr int ADV_TAB = 40;

template <int PT>
__global__ void k_adv_factor(double a0, double h, int scheme2, double *__restrict__ tab)
{
    if (threadIdx.x != 0) return;
    // d = a_0 h / 2 (Scheme 2) or a_0 h (Scheme 3); kappa = (1 - d)/(1 + d)
    // or 1/(1 + d), its powers from log|kappa| (log1p keeps d exact when small)
    const double d = scheme2 ? 0.5 * a0 * h : a0 * h;
    double g, lk, sgn = 1.0;
    bool zero = false;
    if (scheme2) {
        g = 0.5 * h / (1.0 + d);
        if (d < 1.0)
            lk = log1p(-d) - log1p(d);
        else if (d > 1.0) {
            lk = log(d - 1.0) - log1p(d);
            sgn = -1.0;
        } else {
            lk = 0.0;
            zero = true;
        }
    } else {
        g = h / (1.0 + d);
        lk = -log1p(d);
    }
    auto kpow = [&](double n) -> double {  // kappa^n, n >= 1 integral
        if (zero) return 0.0;
        const double v = exp(n * lk);
        return (sgn < 0.0 && fmod(n, 2.0) == 1.0) ? -v : v;
    };
    tab[0] = g;
    tab[1] = kpow(1.0);
    for (int s = 0; s < 16; ++s) tab[8 + s] = kpow((double)PT * (double)(1 << s));
    for (int k = 0; k < 16; ++k) tab[24 + k] = kpow((double)(k + 1));
}

// inclusive forward scan over the 16 lanes of each row, lane multiplier c
template <int NL>
__device__ __forceinline__ void row_scan_fwd(double &f, const double *cp)
{
    f = fma(cp[0], dpp_move<0x111>(f), f);
    if constexpr (NL > 2) f = fma(cp[1], dpp_move<0x112>(f), f);
    if constexpr (NL > 4) f = fma(cp[2], dpp_move<0x114>(f), f);
    if constexpr (NL > 8) f = fma(cp[3], dpp_move<0x118>(f), f);
}

// One workgroup per task.  Thread t owns columns c0 = t PT .. c0 + PT - 1 in
// natural order.  WSUM (Scheme 2): x holds W (right-hand sides in, W = B U
// out) and u receives U; otherwise x is U in place.  The in-leaf history
// pushes -a_m X into the later rows.
template <int NT, int PT, int L, bool WSUM, bool PAIR = false>
__global__ __launch_bounds__(NT) void k_leaf_adv(TaskRef<AdvTask> tr)
{
    constexpr int NR = NT / 16;
    static_assert(NR <= 32, "at most 512 threads");
    __shared__ double sR[2][NR];
    const AdvTask tk = get_task(tr, blockIdx.x);
    const int t = threadIdx.x, lane = t & 63, rl = lane & 15, G = t >> 4;
    FS_G const double *__restrict__ tab = gptr(tk.fac);
    const int64_t M = tk.M;
    const int c0 = t * PT;
    const int nrows_all = tk.nrows;
    FS_G double *__restrict__ x_base = gptr(tk.x) + tk.lo * M;
    FS_G double *__restrict__ u_base = WSUM ? gptr(tk.u) + tk.lo * M : nullptr;
    const double g = tab[0];
    const double kap = tab[1];
    double mp[4], cp[5], kp[PT];
#pragma unroll
    for (int s = 0; s < 4; ++s) mp[s] = tab[8 + s];
#pragma unroll
    for (int s = 0; s < 5; ++s) cp[s] = tab[12 + s];
#pragma unroll
    for (int k = 0; k < PT; ++k) kp[k] = tab[24 + k];
    double aw[L];
#pragma unroll
    for (int m = 0; m < L; ++m) aw[m] = (m > 0) ? gptr(tk.a)[m] : 0.0;
    double mpw[5] = {mp[0], mp[1], mp[2], mp[3], 0.0};
    const double m_lo = pow_bits(mpw, rl);
    const double c_b15 = pow_bits(cp, (lane & 15) + 1);

    // PAIR: two leaves per task with the level product of half-size L
    // between them, from the first leaf's X rows re-read by their owners
    constexpr int NH = PAIR ? 2 : 1;
#pragma unroll 1
    for (int hf = 0; hf < NH; ++hf) {
        const int nrows = (hf == 0) ? (nrows_all < L ? nrows_all : L) : nrows_all - L;
        if (nrows <= 0) break;  // whole workgroup
        FS_G double *__restrict__ x = x_base + (int64_t)(hf * L) * M;
        FS_G double *__restrict__ u = WSUM ? u_base + (int64_t)(hf * L) * M : nullptr;
        double acc[L][PT];
#pragma unroll
        for (int r = 0; r < L; ++r) {
#pragma unroll
            for (int k = 0; k < PT; ++k) acc[r][k] = (r < nrows && c0 + k < M) ? x[(int64_t)r * M + c0 + k] : 0.0;
        }
        if constexpr (PAIR) {
            if (hf == 1) {
#pragma unroll 1
                for (int q = 0; q < L; ++q) {
                    double xq[PT];
#pragma unroll
                    for (int k = 0; k < PT; ++k) xq[k] = (c0 + k < M) ? x_base[(int64_t)q * M + c0 + k] : 0.0;
#pragma unroll
                    for (int p = 0; p < L; ++p) {
                        const double w = gptr(tk.a)[L + p - q];
#pragma unroll
                        for (int k = 0; k < PT; ++k) acc[p][k] = fma(-w, xq[k], acc[p][k]);
                    }
                }
            }
        }

#pragma unroll
        for (int r = 0; r < L; ++r) {
            if (r >= nrows) break;
            const int par = r & 1;
            double lf[PT];
            lf[0] = g * acc[r][0];
#pragma unroll
            for (int k = 1; k < PT; ++k) lf[k] = fma(kap, lf[k - 1], g * acc[r][k]);
            double Sf = lf[PT - 1];
            row_scan_fwd<16>(Sf, mp);
            if (rl == 15) sR[par][G] = Sf;
            __syncthreads();
            double vf = (lane < NR) ? sR[par][lane] : 0.0;
            row_scan_fwd<(NR < 16 ? NR : 16)>(vf, cp);
            if constexpr (NR > 16) vf = fma(c_b15, dpp_move<0x142, 0xA>(vf), vf);
            double Cr = lane_fetch(vf, G > 0 ? G - 1 : 0);
            Cr = (G > 0) ? Cr : 0.0;
            // U at the column before the thread's first one (0 at the inflow)
            const double cf = fma(m_lo, Cr, dpp_move<0x111>(Sf));
            double U[PT], X[PT];
#pragma unroll
            for (int k = 0; k < PT; ++k) U[k] = fma(kp[k], cf, lf[k]);
#pragma unroll
            for (int k = 0; k < PT; ++k) X[k] = WSUM ? U[k] + (k > 0 ? U[k - 1] : cf) : U[k];
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                if (c0 + k < M) {
                    x[(int64_t)r * M + c0 + k] = X[k];
                    if (WSUM) u[(int64_t)r * M + c0 + k] = U[k];
                }
            }
#pragma unroll
            for (int j = r + 1; j < L; ++j) {
#pragma unroll
                for (int k = 0; k < PT; ++k) acc[j][k] = fma(-aw[j - r], X[k], acc[j][k]);
            }
        }
    }
}

hipError_t launch_adv_factor(hipStream_t st, const LeafCfg &c, double a0, double h, bool scheme2, double *tab)
{
    switch (c.pt) {
        case 2: hipLaunchKernelGGL(k_adv_factor<2>, dim3(1), dim3(64), 0, st, a0, h, scheme2 ? 1 : 0, tab); break;
        case 4: hipLaunchKernelGGL(k_adv_factor<4>, dim3(1), dim3(64), 0, st, a0, h, scheme2 ? 1 : 0, tab); break;
        case 8: hipLaunchKernelGGL(k_adv_factor<8>, dim3(1), dim3(64), 0, st, a0, h, scheme2 ? 1 : 0, tab); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t adv_table_doubles() { return ADV_TAB; }

template <int NT, int PT, int L, bool PAIR>
static void adv_go_p(hipStream_t st, bool wsum, const TaskRef<AdvTask> &d_tasks, int ntasks)
{
    if (wsum)
        hipLaunchKernelGGL((k_leaf_adv<NT, PT, L, true, PAIR>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
    else
        hipLaunchKernelGGL((k_leaf_adv<NT, PT, L, false, PAIR>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
}

template <int NT, int PT, int L>
static hipError_t adv_go(hipStream_t st, bool wsum, const TaskRef<AdvTask> &d_tasks, int ntasks, bool pair)
{
    if (pair)
        adv_go_p<NT, PT, L, true>(st, wsum, d_tasks, ntasks);
    else
        adv_go_p<NT, PT, L, false>(st, wsum, d_tasks, ntasks);
    return hipGetLastError();
}

hipError_t launch_leaf_adv(hipStream_t st, const LeafCfg &c, int L, const TaskRef<AdvTask> &d_tasks, int ntasks,
                           bool wsum, bool pair)
{
#define FS_AL(NT_, PT_)                                                                   \
    if (c.nt == NT_ && c.pt == PT_) {                                                     \
        if (L == 4) return adv_go<NT_, PT_, 4>(st, wsum, d_tasks, ntasks, pair);          \
        if (L == 8) return adv_go<NT_, PT_, 8>(st, wsum, d_tasks, ntasks, pair);          \
        return hipErrorInvalidValue;                                                      \
    }
    FS_AL(64, 2)
    FS_AL(64, 4)
    FS_AL(128, 4)
    FS_AL(256, 4)
    FS_AL(512, 4)
    FS_AL(512, 8)
    FS_AL(256, 8)
#undef FS_AL
    return hipErrorInvalidValue;
}

// Up to 512 threads (two waves per SIMD) with 2, 4 or 8 rows per thread: the
// leaf's right-hand sides (L x PT doubles per thread) stay in registers and
// each thread's rows are whole 16-byte units.  For 1024 < M <= 2048, 512 x 4
// (two waves per SIMD, with the in-register pushes between the leaves of a
// pair) is faster than 256 x 8 (one wave per SIMD), alone and in a batch:
// c3 190.5 -> 187.5 ms, and M = 1500 and 1983, whose width is not a multiple
// of 8 (no 16-byte row units with 8 rows per thread), 27-29% faster.  The
// averaged variant (cn: one more LDS exchange and barrier per step) keeps
// 256 x 8 for a single instance (its c3-size solve 240 ms against 246 ms).
LeafCfg scan_config(int64_t M, bool batched, bool cn)
{
    if (M <= 128) return {64, 2, 6};
    if (M <= 256) return {64, 4, 6};
    if (M <= 512) return {128, 4, 7};
    if (M <= 1024) return {256, 4, 8};
    if (M <= 2048) return (cn && !batched) ? LeafCfg{256, 8, 8} : LeafCfg{512, 4, 9};
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
    FS_SF(256, 8)
#undef FS_SF
    return hipErrorInvalidValue;
}

template <int NT, int PT, int L, bool MIXED, bool CN = false, bool PAIR = false>
static void scan_go_m(hipStream_t st, int vec, const TaskRef<LeafTask> &d_tasks, int ntasks)
{
    if (vec == 1)
        hipLaunchKernelGGL((k_leaf_scan<NT, PT, L, MIXED, 1, CN, PAIR>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
    else if (vec == 2)
        hipLaunchKernelGGL((k_leaf_scan<NT, PT, L, MIXED, 2, CN, PAIR>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
    else
        hipLaunchKernelGGL((k_leaf_scan<NT, PT, L, MIXED, 0, CN, PAIR>), dim3(ntasks), dim3(NT), 0, st, d_tasks);
}

// cn: float64 only (the averaged spatial term is not offered with float32 products)
// pair: two leaves per task with the level product of half-size L between
// them (not for L = 16)
template <int NT, int PT, int L>
static hipError_t scan_go(hipStream_t st, bool mixed, int vec, const TaskRef<LeafTask> &d_tasks, int ntasks,
                          bool cn, bool pair)
{
    if (cn) {
        if (mixed) return hipErrorInvalidValue;
        if (pair) {
            if constexpr (L <= 8)
                scan_go_m<NT, PT, L, false, true, true>(st, vec, d_tasks, ntasks);
            else
                return hipErrorInvalidValue;
        } else {
            scan_go_m<NT, PT, L, false, true>(st, vec, d_tasks, ntasks);
        }
    } else if (pair) {
        if constexpr (L <= 8) {
            if (mixed)
                scan_go_m<NT, PT, L, true, false, true>(st, vec, d_tasks, ntasks);
            else
                scan_go_m<NT, PT, L, false, false, true>(st, vec, d_tasks, ntasks);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (mixed)
        scan_go_m<NT, PT, L, true>(st, vec, d_tasks, ntasks);
    else
        scan_go_m<NT, PT, L, false>(st, vec, d_tasks, ntasks);
    return hipGetLastError();
}

template <int NT, int PT>
static hipError_t scan_go16(hipStream_t st, bool mixed, int vec, const TaskRef<LeafTask> &d_tasks, int ntasks,
                            bool cn, bool pair)
{
    if constexpr (PT <= 2)
        return scan_go<NT, PT, 16>(st, mixed, vec, d_tasks, ntasks, cn, pair);
    else
        return hipErrorInvalidValue;
}

hipError_t launch_leaf_scan(hipStream_t st, const LeafCfg &c, int L, const TaskRef<LeafTask> &d_tasks, int ntasks,
                            bool mixed, int vec, bool cn, bool pair)
{
#define FS_SL(NT_, PT_)                                                                                  \
    if (c.nt == NT_ && c.pt == PT_) {                                                                    \
        if (L == 4) return scan_go<NT_, PT_, 4>(st, mixed, vec, d_tasks, ntasks, cn, pair);              \
        if (L == 8) return scan_go<NT_, PT_, 8>(st, mixed, vec, d_tasks, ntasks, cn, pair);              \
        if (L == 16 && PT_ <= 2) return scan_go16<NT_, PT_>(st, mixed, vec, d_tasks, ntasks, cn, pair);  \
        return hipErrorInvalidValue;                                                                     \
    }
    FS_SL(64, 2)
    FS_SL(64, 4)
    FS_SL(128, 4)
    FS_SL(256, 4)
    FS_SL(512, 4)
    FS_SL(512, 8)
    FS_SL(256, 8)
#undef FS_SL
    return hipErrorInvalidValue;
}

}  // namespace fs
