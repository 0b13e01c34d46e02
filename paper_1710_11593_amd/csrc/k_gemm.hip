// Dense off-diagonal Toeplitz-block product of one recursion level:
//   Y[ylo + p][i] += alpha * sum_{q<s} w[s + p - q] X[xlo + q][i],
// with T_s[p][q] = w[s+p-q] (entries w_1..w_{2s-1}) built on chip from the
// Toeplitz column, never stored.  This is the block product of the history
// sum that section 3 identifies as the O(M N^2) cost of time marching, for
// the small blocks where the FFT route of section 3.1 does not pay.
//
// Workgroup tile: 64 columns (one per lane) x 4 waves x PB output rows.
// Each thread keeps PB accumulators; X values stream from global memory
// (coalesced over the 64 columns), the needed slice of w sits in LDS and is
// read as wave-uniform (broadcast) values.
#include "common.hpp"

namespace fs {

constexpr int GEMM_PB = 16;          // output rows per thread
constexpr int GEMM_ROWS = 4 * GEMM_PB;
constexpr int GEMM_MAXS = 1024;      // largest half-block size for this kernel

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_update(const UpdTask<T> *__restrict__ tasks)
{
    __shared__ double sw[GEMM_ROWS + GEMM_MAXS];
    const UpdTask<T> tk = tasks[blockIdx.z];
    const int s = tk.s;
    const int64_t M = tk.M;
    const int pb = blockIdx.y * GEMM_ROWS;
    const int64_t cb = (int64_t)blockIdx.x * 64;
    if (pb >= tk.ny || cb >= M) return;  // whole workgroup exits together

    // sw[k] = w[pb + 1 + k] for k in [0, s + GEMM_ROWS - 1)
    for (int k = threadIdx.x; k < s + GEMM_ROWS - 1; k += 256) sw[k] = gptr(tk.w)[pb + 1 + k];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t col = cb + lane;
    const int p0 = pb + wv * GEMM_PB;  // first output row of this thread
    // w[s + p - q] = sw[s + p - q - pb - 1]
    const int off = s + (p0 - pb) - 1;
    T acc[GEMM_PB];
#pragma unroll
    for (int r = 0; r < GEMM_PB; ++r) acc[r] = (T)0;
    const bool ok = col < M;
    FS_G const T *__restrict__ xp = gptr(tk.x) + tk.xlo * M + col;
    for (int q = 0; q < s; ++q) {
        T xq = ok ? xp[(int64_t)q * M] : (T)0;
#pragma unroll
        for (int r = 0; r < GEMM_PB; ++r) acc[r] += (T)sw[off + r - q] * xq;
    }
    if (ok) {
        FS_G T *__restrict__ yp = gptr(tk.y) + tk.ylo * M + col;
        const T alpha = (T)tk.alpha;
#pragma unroll
        for (int r = 0; r < GEMM_PB; ++r)
            if (p0 + r < tk.ny) yp[(int64_t)(p0 + r) * M] += alpha * acc[r];
    }
}

template <typename T>
hipError_t launch_gemm_update(hipStream_t st, const UpdTask<T> *d_tasks, int ntasks, int s, int64_t maxM)
{
    if (s > GEMM_MAXS) return hipErrorInvalidValue;
    dim3 grid((unsigned)((maxM + 63) / 64), (unsigned)((s + GEMM_ROWS - 1) / GEMM_ROWS), (unsigned)ntasks);
    hipLaunchKernelGGL((k_gemm_update<T>), grid, dim3(256), 0, st, d_tasks);
    return hipGetLastError();
}

template hipError_t launch_gemm_update<double>(hipStream_t, const UpdTask<double> *, int, int, int64_t);
template hipError_t launch_gemm_update<float>(hipStream_t, const UpdTask<float> *, int, int, int64_t);

}  // namespace fs
