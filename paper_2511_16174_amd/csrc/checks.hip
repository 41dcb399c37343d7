// Input checks shared by the drivers: a non-finite entry in the referenced
// triangle of A makes the call report EVD_ERR_NONFINITE in its device `info`
// (LAPACK leaves such input undefined).
//
// Everything stays on the stream, without a host round trip (the call remains
// asynchronous and graph-capturable):
//   begin:  a flag word is cleared, the `uplo` triangle is scanned, and -- only
//           if the flag was raised -- the matrix is replaced by zeros, so every
//           later kernel of the pipeline works on finite data and ends
//           normally;
//   end:    if the flag was raised, info = EVD_ERR_NONFINITE and the outputs
//           (W, and the eigenvectors in A) are set to NaN; likewise
//           EVD_ERR_TIMEOUT if a wait between workgroups gave up (flag[2]).
#include "common.h"

namespace {

// flag[0] non-finite input, [1] band columns published by SBR (bulge chasing
// beside it), [2] a wait between workgroups gave up, [3] spare
__global__ void nf_clear_kernel(int *flag)
{
    if (blockIdx.x == 0 && threadIdx.x < 4) flag[threadIdx.x] = 0;
}

// Workgroups stride over columns, threads over the rows of the referenced
// part of a column, four loads in flight per thread; the flag is written only
// by workgroups that met a non-finite entry, once each.
__global__ __launch_bounds__(256) void nf_scan_kernel(int64_t n, const double *A, int64_t lda, int upper, int *flag)
{
    int bad = 0;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const double *col = A + j * lda;
        const int64_t i0 = upper ? 0 : j, i1 = upper ? j + 1 : n;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += 4 * blockDim.x) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (i + q * blockDim.x < i1) ? col[i + q * blockDim.x] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) bad |= isfinite(v[q]) ? 0 : 1;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void nf_zero_kernel(int64_t n, double *A, int64_t lda, const int *flag)
{
    if (!flag[0]) return;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) A[i + j * lda] = 0.0;
}

__global__ __launch_bounds__(256) void nf_finish_kernel(int64_t n, const int *flag, double *W, double *A, int64_t lda,
                                                        int vec, int32_t *info)
{
    if (!flag[0] && !flag[2]) return;
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    if (blockIdx.x == 0 && threadIdx.x == 0 && info) info[0] = flag[0] ? EVD_ERR_NONFINITE : EVD_ERR_TIMEOUT;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        W[i] = nan;
    if (vec)
        for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) A[i + j * lda] = nan;
}

dim3 nf_grid(int64_t n) { return dim3((unsigned)(n < 4096 ? (n > 0 ? n : 1) : 4096)); }

}  // namespace

// flag: one device int (256 bytes reserved by the caller's workspace layout)
evd_status_t nonfinite_begin(hipStream_t s, int64_t n, double *A, int64_t lda, char uplo, int *flag)
{
    const int upper = (uplo == 'U' || uplo == 'u') ? 1 : 0;
    hipLaunchKernelGGL(nf_clear_kernel, dim3(1), dim3(64), 0, s, flag);
    hipLaunchKernelGGL(nf_scan_kernel, nf_grid(n), dim3(256), 0, s, n, (const double *)A, lda, upper, flag);
    hipLaunchKernelGGL(nf_zero_kernel, nf_grid(n), dim3(256), 0, s, n, A, lda, (const int *)flag);
    return evd_check_last();
}

evd_status_t nonfinite_end(hipStream_t s, int64_t n, const int *flag, double *W, double *A, int64_t lda, bool vec,
                           int32_t *info)
{
    hipLaunchKernelGGL(nf_finish_kernel, nf_grid(n), dim3(256), 0, s, n, flag, W, A, lda, vec ? 1 : 0, info);
    return evd_check_last();
}
