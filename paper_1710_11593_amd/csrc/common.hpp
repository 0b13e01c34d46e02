// Shared declarations of the fracsolve HIP library: task descriptors passed
// to the kernels, small complex helpers and the launcher prototypes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fs {

// Global-memory view of a pointer.  The kernels receive their buffers inside
// task descriptors, where the compiler cannot see that they point to global
// memory and would emit flat accesses; flat accesses count against the LDS
// wait counter as well, so every LDS wait or barrier would also wait for
// outstanding HBM traffic.  Kernels convert each descriptor pointer once.
#if defined(__HIP_DEVICE_COMPILE__)
#define FS_G __attribute__((address_space(1)))
#else
#define FS_G
#endif
template <typename T>
__device__ __forceinline__ FS_G T *gptr(T *p)
{
    return (FS_G T *)p;
}

template <typename T>
struct cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// Column order of the solver's internal fields.  The scan leaf gives each
// thread PT consecutive spatial columns; so that a wave's 16-byte accesses
// to them are contiguous in memory, every full block of B = 64 PT columns is
// stored transposed: memory offset o = 128 j + 2 i + e (j < PT/2, i < 64,
// e < 2) holds spatial offset PT i + 2 j + e.  Columns from mfull on, and all
// columns when pt <= 2, keep the natural order.  Only the leaf and the
// tridiagonal part of the operator look at spatial neighbours; the level
// products treat columns independently, so they run unchanged.
struct ColPerm {
    int pt;        // rows per leaf thread (0 or <= 2: natural order)
    int64_t mfull; // columns covered by full blocks
};

__host__ __device__ inline int64_t perm_s2m(int64_t x, ColPerm p)
{
    if (p.pt <= 2 || x >= p.mfull) return x;
    const int64_t B = 64 * (int64_t)p.pt;
    const int64_t blk = x / B;
    const int s = (int)(x - blk * B);
    const int i = s / p.pt, j = (s % p.pt) >> 1, e = s & 1;
    return blk * B + 128 * j + 2 * i + e;
}

__host__ __device__ inline int64_t perm_m2s(int64_t c, ColPerm p)
{
    if (p.pt <= 2 || c >= p.mfull) return c;
    const int64_t B = 64 * (int64_t)p.pt;
    const int64_t blk = c / B;
    const int o = (int)(c - blk * B);
    const int j = o >> 7, i = (o & 127) >> 1, e = o & 1;
    return blk * B + (int64_t)p.pt * i + 2 * j + e;
}

// One leaf of the recursion: rows [lo, lo+nrows) of one instance, solved by
// forward substitution in time with a tridiagonal solve per row.
struct LeafTask {
    double *u;          // field [N][M]: right-hand side in, solution out
    const double *a;    // Toeplitz column a_0..a_{L-1}
    const double *fac;  // factor table of a_0 I + K (see k_leaf.hip)
    const float *hist;  // float32 history accumulator [N][M] or null
    float *x32;         // float32 shadow of solved rows or null
    int64_t M;
    int64_t lo;
    int32_t nrows;
    // scan leaf flags: bit 0 (LEAF_PERM) fields in the transposed column order
    // of ColPerm; bit 1 (LEAF_VEC) whole 16-byte row units (M a multiple of
    // PT, aligned rows)
    int32_t flags;
};
constexpr int32_t LEAF_PERM = 1, LEAF_VEC = 2;

// Leaf of the advection equations (bidiagonal diagonal block, k_leaf_scan.hip)
struct AdvTask {
    double *x;          // field the level products use: right-hand sides in, X out
    double *u;          // solution U [N][M] (Scheme 2: X = B U is not U) or null
    const double *a;    // Toeplitz column a_0..a_{L-1}
    const double *fac;  // factor table (g, kappa and its powers)
    int64_t M;
    int64_t lo;
    int32_t nrows;
    int32_t pad;
};

// One off-diagonal Toeplitz-block product:
//   Y[ylo + p] += alpha * sum_{q<s} w[s + p - q] X[xlo + q],   p < ny <= s,
// for all M columns.  The rows of X and Y are rows of [*][M] arrays.
template <typename T>
struct UpdTask {
    const T *x;
    T *y;
    const double *w;             // Toeplitz column (dense products, corner band)
    const cplx<T> *spec;         // DFT_{2s} of w with the corner band removed (FFT products)
    const double *xc;            // float64 views of X and Y for the corner band of
    double *yc;                  // the FFT route (equal to x, y in float64 mode)
    int64_t M;
    int64_t xlo, ylo;
    int32_t s;
    int32_t ny;
    double alpha;
};

// Task descriptors reach a kernel either inline, for single-task launches
// (the descriptor travels in the kernel arguments, which saves the kernel a
// dependent memory round trip before its first data load), or through a
// device array indexed by a block index.
template <typename TASK>
struct TaskRef {
    const TASK *tasks;  // device array, used when one_valid == 0
    TASK one;           // the only task, used when one_valid != 0
    int32_t one_valid;
};

template <typename TASK>
__device__ __forceinline__ TASK get_task(const TaskRef<TASK> &r, unsigned i)
{
    if (r.one_valid) return r.one;
    return r.tasks[i];
}

// XCD-aware block order.  Workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2), so consecutive block ids land on different
// L2s.  This maps block b to logical block (b mod 8) * (G/8) + b/8, so that
// logical neighbours (adjacent column groups, which share cache lines) run
// on the same XCD at about the same time.  Blocks past the last multiple of
// 8 keep their id.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned G)
{
    const unsigned full = G & ~7u;
    if (b >= full) return b;
    return (b & 7u) * (full >> 3) + (b >> 3);
}

// Width of the near-corner band of a level product that the FFT route adds
// exactly instead of through the spectrum (see k_fft.hip).
__host__ __device__ inline int corner_width(int s) { return s < 32 ? s : 32; }

// Launchers (defined in the .hip files; all enqueue on `st`).
hipError_t launch_weights(hipStream_t st, int regime, double p, double coef, double dcoef, double tau,
                          int64_t N, double *b, double *a, double *rho, double *psi, double *da,
                          double *drho, double *dpsi);
// Lag-1 spatial term of the averaged variant: y_row += coef (2 x_i - x_{i-1}
// - x_{i+1}) over the spatial order (fields in column order perm), one task
// per row pair; and the same over nrows consecutive row pairs.
struct Lag1Task {
    const double *x;  // source row [M]
    double *y;        // destination row [M]
    int64_t M;
    double coef;
    ColPerm perm;
};
hipError_t launch_halfK_tasks(hipStream_t st, const Lag1Task *d_tasks, int ntasks, int64_t maxM);
hipError_t launch_halfK_rows(hipStream_t st, const double *x, double *y, int64_t M, int64_t nrows, double coef,
                             ColPerm perm);
hipError_t launch_rhs_perm(hipStream_t st, const double *f, const double *u0, const double *phi, const double *rho,
                           const double *psi, double *dst, int64_t M, int64_t N, ColPerm perm);
hipError_t launch_rhs_adv2(hipStream_t st, const double *f, const double *u0, const double *rho, double *y,
                           int64_t M, int64_t N);
hipError_t launch_rhs(hipStream_t st, const double *f, const double *u0, const double *phi,
                      const double *rho, const double *psi, double *u, int64_t M, int64_t N);
hipError_t launch_rhs_scale(hipStream_t st, double *y, const double *u0, const double *phi,
                            const double *rho, const double *psi, int64_t M, int64_t N);

// Leaf configuration chosen from M.
struct LeafCfg {
    int nt;       // threads per workgroup
    int pt;       // rows per thread
    int S;        // PCR stages = log2(2 nt)
    int vec = 0;  // scan leaf row access: 0 per element, 1 whole 16-byte units (M % pt == 0,
                  // aligned fields), 2 chosen per task (LeafTask::vec)
};
LeafCfg leaf_config(int64_t M);
size_t leaf_table_doubles(const LeafCfg &c);
hipError_t launch_leaf_factor(hipStream_t st, const LeafCfg &c, int64_t M, double a0, double e, double *fac);
hipError_t launch_leaf(hipStream_t st, const LeafCfg &c, int L, const LeafTask *d_tasks, int ntasks, bool mixed);
// scan-form leaf (closed-form semiseparable inverse of a_0 I + K)
LeafCfg scan_config(int64_t M, bool batched = false, bool cn = false);
size_t scan_table_doubles(const LeafCfg &c);
hipError_t launch_scan_factor(hipStream_t st, const LeafCfg &c, int64_t M, double a0, double e, double *tab);
hipError_t launch_adv_factor(hipStream_t st, const LeafCfg &c, double a0, double h, bool scheme2, double *tab);
size_t adv_table_doubles();
hipError_t launch_leaf_adv(hipStream_t st, const LeafCfg &c, int L, const TaskRef<AdvTask> &d_tasks, int ntasks,
                           bool wsum, bool pair = false);
hipError_t launch_leaf_scan(hipStream_t st, const LeafCfg &c, int L, const TaskRef<LeafTask> &tr, int ntasks,
                            bool mixed, int vec, bool cn = false, bool pair = false);

hipError_t launch_twiddles(hipStream_t st, int64_t nmax, cplx<double> *w64, cplx<float> *w32);

// lead_rows: rows at the start of Y that the next launch (a leaf) reads
// first; with one task their tiles run on the leaf's XCD (0 = no placement)
template <typename T>
hipError_t launch_gemm_update(hipStream_t st, const TaskRef<UpdTask<T>> &tr, int ntasks, int s, int64_t maxM,
                              int lead_rows = 0);
// even: every task has M even and 16-byte aligned rows (one vector access per
// column pair)
// corner: also launch the near-corner band kernel of single-pass levels
// (launch_fft_corner) after the transform
// gbase (single-pass levels, device): ntasks + 1 offsets of each task's
// first column group in the launch's flat group numbering (groups of
// fft_update_cc(2 s, fp32) complex columns)
template <typename T>
hipError_t launch_fft_update_ex(hipStream_t st, const UpdTask<T> *d_tasks, const int64_t *gbase, int ntasks, int s,
                                int64_t maxM, const cplx<T> *tw, int64_t nmax, cplx<T> *zs, size_t zs_elems,
                                bool even, bool corner = true);
int fft_update_cc(int n, bool fp32);
// near-corner band of a single-pass FFT level (no-op for multi-pass levels,
// which add it inside their last pass, and where fft_band_in_update holds:
// the float64 three-digit update kernels add it when they store Y)
template <typename T>
hipError_t launch_fft_corner(hipStream_t st, const UpdTask<T> *d_tasks, int ntasks, int s, int64_t maxM);
bool fft_band_in_update(int s, bool fp32);
hipError_t launch_spectrum(hipStream_t st, const double *w, int s, cplx<double> *spec64, cplx<float> *spec32,
                           const cplx<double> *tw, int64_t nmax, cplx<double> *scratch);
int fft_max_single_pass(bool fp32);

hipError_t launch_diag_apply(hipStream_t st, const double *x, double *y, const double *a, double e, int64_t M,
                             int64_t N, int L, ColPerm perm);
hipError_t launch_copy_reverse(hipStream_t st, const double *src, double *dst, int64_t M, int64_t N);
// dst row n = src row (reverse ? N-1-n : n) with the columns moved from
// natural to internal order (to_internal) or back.  src == dst is allowed
// without reverse.
hipError_t launch_permute(hipStream_t st, const double *src, double *dst, int64_t M, int64_t N, ColPerm perm,
                          bool to_internal, bool reverse);
hipError_t launch_axpy(hipStream_t st, double *y, const double *x, double alpha, int64_t n);
// symmetric Toeplitz product through its circulant embedding (k_fft1d.hip):
// L = circ_length(n) (a power of two >= max(8, 2n - 1), at most 2^23); S
// (L doubles) = the spectrum of the embedded column 1 + 2 a_0, a_1 .. a_{n-1}
// divided by L (colbuf may alias S); za, zb = two complex arrays of L points.
// y = A x for n entries (x != y).
int64_t circ_length(int64_t n);
int circ_launches(int64_t L);
hipError_t launch_circ_spectrum(hipStream_t st, const double *a, int64_t n, int64_t L, double *S, double *colbuf,
                                void *za, void *zb);
// skip (device, may be NULL): every pass returns at once while *skip != 0.
// dotp (device, may be NULL, circ_dot_parts(L) doubles): the last pass also
// writes partial sums of <x, y>, *ndot of them.
hipError_t launch_circ_apply(hipStream_t st, const double *x, double *y, int64_t n, int64_t L, const double *S,
                             void *za, void *zb, const int32_t *skip = nullptr, double *dotp = nullptr,
                             int64_t *ndot = nullptr);
int64_t circ_dot_parts(int64_t L);
// conjugate-gradient state kept in device memory (k_misc.hip)
struct CgState {
    double rr;       // r.r of the current residual
    double kap, bet;  // step length and direction update of the last step
    double rtol_fn;  // stop when |r| <= rtol_fn
    double fn;       // |f|, for the residual history
    double pAp;      // last <p, A p>
    int32_t it, done, maxit, bad;
};
// one CG step after A p is in Ap and the partial sums of <p, A p> in
// pap[0 .. npap) (pap NULL: computed here, into partial): kappa, the u / r update with the new r.r, beta, the stop
// test and p = r + beta p; no-ops once done is set.  hist (device, hist_cap
// doubles or NULL) receives |r_k| / |f| at k = it.
hipError_t launch_cg_step_tail(hipStream_t st, CgState *cs, double *u, double *r, double *p, const double *Ap,
                               int64_t n, const double *pap, int64_t npap, double *partial, double *hist,
                               int hist_cap);
hipError_t launch_sub(hipStream_t st, double *r, const double *b, const double *y, int64_t n);
hipError_t launch_to_f32(hipStream_t st, const double *x, float *y, int64_t n);
hipError_t launch_zero(hipStream_t st, void *p, size_t bytes);
hipError_t launch_dot_partial(hipStream_t st, const double *x, const double *y, int64_t n, double *partial,
                              int nblocks);
// Krylov-basis products of GMRES: out[v] = <V_v, w> for v < nv (device
// out, partial holds nv * nb doubles); y = beta y + sum_v c_v V_v with the
// coefficients c[0..nv) on the host (passed by value, LINCOMB_MAX per launch).
constexpr int LINCOMB_MAX = 32;
struct LinCoef {
    double c[LINCOMB_MAX];
};
hipError_t launch_multidot(hipStream_t st, const double *V, int64_t ldv, int nv, const double *w, int64_t n,
                           double *partial, int nb, double *out);
hipError_t launch_lincomb(hipStream_t st, double *y, double beta, const double *V, int64_t ldv, int nv,
                          const double *c, int64_t n);
hipError_t launch_gamma_rhs_terms(hipStream_t st, const double *lam, const double *u0, const double *phi,
                                  const double *drho, const double *dpsi, int64_t M, int64_t N, double *partial,
                                  int nblocks);
hipError_t launch_absmax_partial(hipStream_t st, const double *x, int64_t n, double *partial, int nblocks);
hipError_t launch_nonfinite_partial(hipStream_t st, const double *x, int64_t n, double *partial, int nblocks);

}  // namespace fs
