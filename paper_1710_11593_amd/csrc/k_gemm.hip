// Dense off-diagonal Toeplitz-block product of one recursion level:
//   Y[ylo + p][i] += alpha * sum_{q<s} w[s + p - q] X[xlo + q][i],
// with T_s[p][q] = w[s+p-q] (entries w_1..w_{2s-1}) built on chip from the
// Toeplitz column, never stored.  This is the block product of the history
// sum that section 3 identifies as the O(M N^2) cost of time marching, for
// the small blocks where the FFT route of section 3.1 does not pay.
//
// These products are small (s <= 64 by default: at most a few MB of
// traffic) and sit on the critical path of the recursion, so the kernel is
// organised for latency: every thread owns one column and RB output
// rows; all loads of its X column (a chunk of up to 64 rows) and of
// its Y rows are issued together, the weight window sits in LDS (read as
// wave-uniform broadcasts), and the output rows are spread over the grid so
// that even s = 64 occupies every CU.
#include <algorithm>
#include <cstdlib>

#include "common.hpp"

namespace fs {

constexpr int DENSE_MAXS = 1024;  // largest half-block size for this kernel

// RB: output rows per thread (4; 8 or 16 for launches with many tasks,
// where re-reading the X rows once per row block costs more than the
// parallelism gained); QC: X rows per load batch; s is a multiple of QC
// (both powers of two).
// Loads are unconditional: a thread past the last column reads column M - 1
// (a valid address) and stores nothing, so the loads carry no branches and
// are all in flight together.
// Placement.  Workgroups are dispatched to the XCDs round robin (workgroup b
// on XCD b mod 8), so the leaf of task t in a leaf launch runs on XCD t mod 8.
//  lead > 0 (single task): the tiles of the first `lead` row blocks (the rows
//    the next leaf reads) are put on XCD 0, so that they reach the leaf
//    through that XCD's L2; the other tiles go to XCDs 1..7.  1-D grid, tile
//    order row-block major.
//  lead < 0 (several tasks): every tile of task t runs on XCD t mod 8, next to
//    its leaf: grid (8 gxp, gyp, ceil(ntasks / 8)), task = 8 z + x mod 8.
//  lead = 0: grid (gxp, gyp, ntasks).
template <typename T, int QC, int RB, int NTD>
__global__ __launch_bounds__(NTD) void k_dense_update(TaskRef<UpdTask<T>> tr, int lead, int gxp, int gyp, int ntasks)
{
    constexpr int DENSE_RB = RB;
    __shared__ double sw[DENSE_MAXS + DENSE_RB];
    int bx = blockIdx.x, by = blockIdx.y, task = blockIdx.z;
    if (lead < 0) {
        task = 8 * blockIdx.z + blockIdx.x % 8;
        bx = blockIdx.x / 8;
        if (task >= ntasks) return;  // whole workgroup
    } else if (lead > 0) {
        const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
        const int ne = gxp * lead, nl = gxp * (gyp - lead);
        int tile;
        if (xcd == 0) {
            if (slot >= ne) return;  // whole workgroup
            tile = slot;
        } else {
            const int j = slot * 7 + (xcd - 1);
            if (j >= nl) return;
            tile = ne + j;
        }
        bx = tile % gxp;
        by = tile / gxp;
    }
    const UpdTask<T> tk = get_task(tr, task);
    const int s = tk.s;
    const int64_t M = tk.M;
    const int p0 = by * DENSE_RB;  // first output row of the workgroup
    const int64_t col = (int64_t)bx * NTD + threadIdx.x;
    if (p0 >= tk.ny || (int64_t)bx * NTD >= M) return;  // whole workgroup exits together
    const bool ok = col < M;
    const int64_t cl = ok ? col : M - 1;
    const int np = (tk.ny - p0 < DENSE_RB) ? tk.ny - p0 : DENSE_RB;

    FS_G const T *__restrict__ xp = gptr(tk.x) + tk.xlo * M + cl;
    FS_G T *__restrict__ yp = gptr(tk.y) + (tk.ylo + p0) * M + cl;
    // Loads in the order they are waited for, all before the first wait: the
    // thread's first weight of the window sw[k] = w[p0 + 1 + k],
    // k < s + DENSE_RB - 1 (clamped, so unconditional), the Y rows (rows
    // past ny read row ny - 1 and are not stored), the first batch of X.
    FS_G const double *__restrict__ w = gptr(tk.w) + p0 + 1;
    const int nwin = s + DENSE_RB - 1;
    const double w_first = w[(int)threadIdx.x < nwin ? (int)threadIdx.x : nwin - 1];
    T yv[DENSE_RB];
#pragma unroll
    for (int r = 0; r < DENSE_RB; ++r) yv[r] = yp[(int64_t)(r < np ? r : np - 1) * M];
    T xv[QC];
#pragma unroll
    for (int j = 0; j < QC; ++j) xv[j] = xp[(int64_t)j * M];
    if ((int)threadIdx.x < nwin) sw[threadIdx.x] = w_first;
    for (int k = threadIdx.x + NTD; k < nwin; k += NTD) sw[k] = w[k];  // windows past NTD
    __syncthreads();  // weight window ready

    T acc[DENSE_RB];
#pragma unroll
    for (int r = 0; r < DENSE_RB; ++r) acc[r] = (T)0;
    // w[s + p - q] with p = p0 + r: sw[s - 1 + r - q]
    for (int q0 = 0; q0 < s; q0 += QC) {
        if (q0 > 0) {
            FS_G const T *__restrict__ xq = xp + (int64_t)q0 * M;
#pragma unroll
            for (int j = 0; j < QC; ++j) xv[j] = xq[(int64_t)j * M];
        }
        const double *__restrict__ wq = sw + (s - 1 - q0);
#pragma unroll
        for (int j = 0; j < QC; ++j) {
#pragma unroll
            for (int r = 0; r < DENSE_RB; ++r) acc[r] += (T)wq[r - j] * xv[j];
        }
    }
    if (ok) {
        const T alpha = (T)tk.alpha;
#pragma unroll
        for (int r = 0; r < DENSE_RB; ++r)
            if (r < np) yp[(int64_t)r * M] = yv[r] + alpha * acc[r];
    }
}

template <typename T, int RB, int NTD>
static void dense_go_nt(hipStream_t st, const TaskRef<UpdTask<T>> &d_tasks, int ntasks, int s, int64_t maxM,
                        int lead_rows)
{
    dim3 grid((unsigned)((maxM + NTD - 1) / NTD), (unsigned)((s + RB - 1) / RB), (unsigned)ntasks);
    const int gxp = (int)grid.x, gyp = (int)grid.y;
    // single task: the row blocks the next leaf reads on XCD 0 (see the kernel)
    int lead = 0;
    if (ntasks == 1 && lead_rows > 0) {
        lead = std::min(gyp, (lead_rows + RB - 1) / RB);
        const int ne = gxp * lead, nl = gxp * (gyp - lead);
        grid = dim3((unsigned)(8 * std::max(ne, (nl + 6) / 7)), 1, 1);
    } else if (ntasks > 1 && lead_rows > 0) {
        lead = -1;
        grid = dim3((unsigned)(8 * gxp), (unsigned)gyp, (unsigned)((ntasks + 7) / 8));
    }
    if (s <= 4)
        hipLaunchKernelGGL((k_dense_update<T, 4, RB, NTD>), grid, dim3(NTD), 0, st, d_tasks, lead, gxp, gyp, ntasks);
    else if (s <= 8)
        hipLaunchKernelGGL((k_dense_update<T, 8, RB, NTD>), grid, dim3(NTD), 0, st, d_tasks, lead, gxp, gyp, ntasks);
    else if (s <= 16)
        hipLaunchKernelGGL((k_dense_update<T, 16, RB, NTD>), grid, dim3(NTD), 0, st, d_tasks, lead, gxp, gyp, ntasks);
    else if (s <= 32 || RB > 4)
        hipLaunchKernelGGL((k_dense_update<T, 32, RB, NTD>), grid, dim3(NTD), 0, st, d_tasks, lead, gxp, gyp, ntasks);
    else
        hipLaunchKernelGGL((k_dense_update<T, 64, RB, NTD>), grid, dim3(NTD), 0, st, d_tasks, lead, gxp, gyp, ntasks);
}

// One wave per workgroup: the small products finish sooner when their
// loads are spread over more CUs (measured against 128 and 256 threads:
// c2 139.5 -> 138.9 ms, c3 196.2 -> 191.8 ms, c4 batched 170.0 -> 163.9 ms).
constexpr int DENSE_NT = 64;

template <typename T, int RB>
static void dense_go(hipStream_t st, const TaskRef<UpdTask<T>> &d_tasks, int ntasks, int s, int64_t maxM, int lead_rows)
{
    dense_go_nt<T, RB, DENSE_NT>(st, d_tasks, ntasks, s, maxM, lead_rows);
}

// The same level product on the matrix cores, float64 (v_mfma_f64_16x16x4):
// the Toeplitz-expanded GEMM Y_blk += alpha T_s X_blk, T_s[p][q] = w[s+p-q].
// Workgroup: 4 waves over a slab of 16 columns (one 128-byte line of each
// row) and 64 output rows; the slab's s rows of X and the weight window
// w[p0+1 .. p0+s+63] are staged in LDS, and each wave accumulates one
// 16 x 16 output tile over s/4 MFMAs.  Operand layout of the 16x16x4 f64
// instruction (one double per lane): A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k; D[4 r + l/16][l mod 16] in lane l, register r.
template <int SMAX>
__global__ __launch_bounds__(256) void k_dense_mfma(TaskRef<UpdTask<double>> tr)
{
    typedef double v4d __attribute__((ext_vector_type(4)));
    constexpr int NQ = SMAX / 16;            // X rows staged per thread
    constexpr int NW = (SMAX + 63 + 255) / 256;  // weights staged per thread
    __shared__ double sx[SMAX * 16];
    __shared__ double sw[SMAX + 64];
    const UpdTask<double> tk = get_task(tr, blockIdx.z);
    const int s = tk.s;
    const int64_t M = tk.M;
    const int64_t c0 = (int64_t)blockIdx.x * 16;
    const int p0 = blockIdx.y * 64;
    if (p0 >= tk.ny || c0 >= M) return;  // whole workgroup
    const int t = threadIdx.x;
    const int wv = t >> 6, l = t & 63;
    const int li = l & 15, lk = l >> 4;
    const int pt = p0 + 16 * wv;  // first row of this wave's tile
    // Every global load of the workgroup is issued before the first wait:
    // the lane's four Y entries, its NQ rows of the X slab and its share of
    // the weight window.  Loads are unconditional (indices past the data are
    // clamped to a valid element whose value is then discarded), so no
    // branch serialises them.
    const int64_t col = c0 + li;
    const int64_t colc = col < M ? col : M - 1;
    FS_G double *__restrict__ yb = gptr(tk.y) + tk.ylo * M;
    double yv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = pt + 4 * r + lk;
        yv[r] = yb[(int64_t)(p < tk.ny ? p : tk.ny - 1) * M + colc];
    }
    const int j = t & 15;
    const bool okc = c0 + j < M;
    FS_G const double *__restrict__ xb = gptr(tk.x) + tk.xlo * M + (okc ? c0 + j : M - 1);
    double xv[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = (t >> 4) + 16 * i;
        xv[i] = xb[(int64_t)(q < s ? q : s - 1) * M];
    }
    FS_G const double *__restrict__ w = gptr(tk.w) + p0 + 1;
    const int nw = s + 63;  // window w[p0+1 .. p0+s+63]; w has at least p0 + s + 64 entries
    double wvv[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int k = t + 256 * i;
        wvv[i] = w[k < nw ? k : nw - 1];
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = (t >> 4) + 16 * i;
        if (q < s) sx[q * 16 + j] = okc ? xv[i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int k = t + 256 * i;
        if (k < nw) sw[k] = wvv[i];
    }
    __syncthreads();
    if (pt >= tk.ny) return;  // the whole wave (no barrier follows)
    // A[i][k] = w[s + pt + i - q0 - k] = sw[s + pt + i - q0 - k - p0 - 1];
    // four independent accumulation chains over q, summed at the end
    const double *__restrict__ wa = sw + (s + 16 * wv + li - lk - 1);
    const double *__restrict__ xbk = sx + lk * 16 + li;
    v4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
    if (s % 16 == 0) {
#pragma unroll 2
        for (int q0 = 0; q0 < s; q0 += 16) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int q = q0 + 4 * c;
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[-q], xbk[q * 16], acc[c], 0, 0, 0);
            }
        }
    } else {
        // s = 4 or 8 (chains past s stay zero)
        for (int q0 = 0; q0 < s; q0 += 16) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int q = q0 + 4 * c;
                if (q < s) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[-q], xbk[q * 16], acc[c], 0, 0, 0);
            }
        }
    }
    const v4d accs = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (col < M) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = pt + 4 * r + lk;
            if (p < tk.ny) yb[(int64_t)p * M + col] = yv[r] + tk.alpha * accs[r];
        }
    }
}

// Largest half-size routed to the matrix-core kernel, and the smallest:
// below it the VALU kernel above (organised for latency, with XCD placement
// next to the following leaf) is the faster one.
constexpr int DENSE_MFMA_MAX = 512;

static int dense_mfma_from()
{
    static const int v = [] {
        const char *e = getenv("FRACSOLVE_MFMA_FROM");
        return e ? atoi(e) : 128;
    }();
    return v;
}

hipError_t launch_dense_mfma(hipStream_t st, const TaskRef<UpdTask<double>> &d_tasks, int ntasks, int s, int64_t maxM)
{
    const dim3 grid((unsigned)((maxM + 15) / 16), (unsigned)((s + 63) / 64), (unsigned)ntasks);
    if (s <= 64)
        hipLaunchKernelGGL((k_dense_mfma<64>), grid, dim3(256), 0, st, d_tasks);
    else if (s <= 256)
        hipLaunchKernelGGL((k_dense_mfma<256>), grid, dim3(256), 0, st, d_tasks);
    else
        hipLaunchKernelGGL((k_dense_mfma<512>), grid, dim3(256), 0, st, d_tasks);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_update(hipStream_t st, const TaskRef<UpdTask<T>> &d_tasks, int ntasks, int s, int64_t maxM,
                              int lead_rows)
{
    if (s > DENSE_MAXS || s < 1 || (s & (s - 1)) != 0) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 8) {
        if (s >= 4 && s >= dense_mfma_from() && s <= DENSE_MFMA_MAX)
            return launch_dense_mfma(st, d_tasks, ntasks, s, maxM);
    }
    // tiles of 256 columns at 4 rows per thread; past a few per CU the X re-reads
    // dominate and more rows per thread pay
    const int64_t wg4 = (int64_t)ntasks * ((maxM + 255) / 256) * ((s + 3) / 4);
    if (wg4 > 2048 && s >= 16)
        dense_go<T, 16>(st, d_tasks, ntasks, s, maxM, lead_rows);
    else if (wg4 > 2048 && s >= 8)
        dense_go<T, 8>(st, d_tasks, ntasks, s, maxM, lead_rows);
    else
        dense_go<T, 4>(st, d_tasks, ntasks, s, maxM, lead_rows);
    return hipGetLastError();
}

template hipError_t launch_gemm_update<double>(hipStream_t, const TaskRef<UpdTask<double>> &, int, int, int64_t, int);
template hipError_t launch_gemm_update<float>(hipStream_t, const TaskRef<UpdTask<float>> &, int, int, int64_t, int);

}  // namespace fs
