// FP64 eigenpair refinement of Ogita and Aishima (JJIAM 2018, "RefSyEv"),
// used by the mixed-precision path (not in the paper): from an approximate
// eigenvector matrix X of the symmetric A,
//   R = I - X^T X,  S = X^T A X,  lam_i = s_ii / (1 - r_ii),
//   delta = 2 (||S - diag(lam)||_2 + ||A||_2 ||R||_2),
//   E_ij = (s_ij + lam_j r_ij) / (lam_j - lam_i)   if |lam_i - lam_j| > delta
//          r_ij / 2                                 otherwise,
//   X <- X + X E.
// 2-norms are bounded by Frobenius norms (conservative) and ||A||_2 by
// max |lam_i| (1 + ||R||_F).  All products are FP64 MFMA GEMMs.
#include "common.h"

namespace {

__global__ void oa_eye_kernel(int64_t n, double *M, int64_t ld)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        M[i + j * ld] = (i == j) ? 1.0 : 0.0;
    }
}

__global__ void oa_copy_kernel(int64_t n, const double *src, int64_t lds, double *dst, int64_t ldd)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        dst[i + j * ldd] = src[i + j * lds];
    }
}

// lam_i = s_ii / (1 - r_ii)
__global__ void oa_lambda_kernel(int64_t n, const double *S, const double *R, double *lam)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        lam[i] = S[i + i * n] / (1.0 - R[i + i * n]);
}

// partial sums per block: [0] ||S - diag(lam)||_F^2, [1] ||R||_F^2, [2] max |lam|
__global__ __launch_bounds__(256) void oa_norms_kernel(int64_t n, const double *S, const double *R, const double *lam,
                                                       double *part)
{
    __shared__ double r0[4], r1[4], r2[4];
    double a = 0.0, b = 0.0, c = 0.0;
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const double s = S[idx] - ((i == j) ? lam[i] : 0.0);
        a += s * s;
        b += R[idx] * R[idx];
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c = fmax(c, fabs(lam[i]));
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_max(c);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { r0[w] = a; r1[w] = b; r2[w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = r0[0] + r0[1] + r0[2] + r0[3];
        part[blockIdx.x * 3 + 1] = r1[0] + r1[1] + r1[2] + r1[3];
        part[blockIdx.x * 3 + 2] = fmax(fmax(r2[0], r2[1]), fmax(r2[2], r2[3]));
    }
}

// delta from the per-block partials (one thread; fixed order -> deterministic)
__global__ void oa_delta_kernel(int nblk, const double *part, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int q = 0; q < nblk; ++q) {
        a += part[q * 3 + 0];
        b += part[q * 3 + 1];
        c = fmax(c, part[q * 3 + 2]);
    }
    const double rn = sqrt(b);
    out[0] = 2.0 * (sqrt(a) + c * (1.0 + rn) * rn);  // delta
    out[1] = sqrt(a);
    out[2] = rn;
    out[3] = c;
}

// E (in place of R): E_ij as in RefSyEv
__global__ void oa_e_kernel(int64_t n, const double *S, double *R, const double *lam, const double *dl)
{
    const double delta = dl[0];
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const double r = R[idx];
        const double d = lam[j] - lam[i];
        R[idx] = (i != j && fabs(d) > delta) ? (S[idx] + lam[j] * r) / d : 0.5 * r;
    }
}

// residual partials: ||A X - X diag(lam)||_F^2 (AX given) and ||A||_F^2 (lower stored)
__global__ __launch_bounds__(256) void oa_resid_kernel(int64_t n, const double *AX, const double *X, const double *lam,
                                                       const double *A, int64_t lda, double *part)
{
    __shared__ double r0[4], r1[4];
    double a = 0.0, b = 0.0;
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const double r = AX[idx] - X[idx] * lam[j];
        a += r * r;
        if (i >= j) {
            const double v = A[i + j * lda];
            b += (i == j) ? v * v : 2.0 * v * v;
        }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { r0[w] = a; r1[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2 + 0] = r0[0] + r0[1] + r0[2] + r0[3];
        part[blockIdx.x * 2 + 1] = r1[0] + r1[1] + r1[2] + r1[3];
    }
}

__global__ void oa_resid_final_kernel(int nblk, int64_t n, const double *part, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int q = 0; q < nblk; ++q) { a += part[q * 2]; b += part[q * 2 + 1]; }
    out[0] = (b > 0.0) ? sqrt(a) / ((double)n * sqrt(b)) : sqrt(a);
}

// Rayleigh quotients lam_j = (x_j . (A x_j)) / (x_j . x_j), one wavefront per column
__global__ __launch_bounds__(64) void oa_rayleigh_kernel(int64_t n, const double *AX, const double *X, int64_t ldx,
                                                         double *lam)
{
    const int64_t j = blockIdx.x;
    if (j >= n) return;
    double num = 0.0, den = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 64) {
        const double x = X[i + j * ldx];
        num += x * AX[i + j * n];
        den += x * x;
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if (threadIdx.x == 0) lam[j] = num / den;
}

constexpr int OA_BLOCKS = 1024;

}  // namespace

size_t refine_work_bytes(int64_t n)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return 4 * evd_align256(nn * nn * 8) + evd_align256((size_t)OA_BLOCKS * 3 * 8) + 256 * 8 +
           evd_align256(nn * 8);
}

// One or more RefSyEv sweeps on X (n x n, ldx), A lower-stored FP64.
// lam (n) receives the refined eigenvalue estimates.  stats (device, 8
// doubles): [0] delta, [1] ||S - diag(lam)||_F, [2] ||R||_F, [3] max|lam|,
// [4] residual ||A X - X lam||_F / (n ||A||_F) of the final X, whose
// Rayleigh quotients are returned in lam.
evd_status_t refine_run(hipStream_t s, int64_t n, const double *A, int64_t lda, double *X, int64_t ldx, double *lam,
                        int sweeps, void *work, double *stats)
{
    char *base = (char *)work;
    const size_t nn = (size_t)n;
    const size_t mat = evd_align256(nn * nn * 8);
    double *R = (double *)(base);
    double *AX = (double *)(base + mat);
    double *S = (double *)(base + 2 * mat);
    double *Xn = (double *)(base + 3 * mat);
    double *part = (double *)(base + 4 * mat);
    const dim3 g(OA_BLOCKS), t(256);
    for (int sw = 0; sw < sweeps; ++sw) {
        hipLaunchKernelGGL(oa_eye_kernel, g, t, 0, s, n, R, n);
        EVD_CHECK(gemm_f64(s, OP_T, OP_N, 0, n, n, n, -1.0, X, ldx, X, ldx, 1.0, R, n, nullptr, 0));
        EVD_CHECK(gemm_f64(s, OP_S, OP_N, 0, n, n, n, 1.0, A, lda, X, ldx, 0.0, AX, n, nullptr, 0));
        EVD_CHECK(gemm_f64(s, OP_T, OP_N, 0, n, n, n, 1.0, X, ldx, AX, n, 0.0, S, n, nullptr, 0));
        hipLaunchKernelGGL(oa_lambda_kernel, dim3(64), t, 0, s, n, (const double *)S, (const double *)R, lam);
        hipLaunchKernelGGL(oa_norms_kernel, g, t, 0, s, n, (const double *)S, (const double *)R, (const double *)lam,
                           part);
        hipLaunchKernelGGL(oa_delta_kernel, dim3(1), dim3(64), 0, s, OA_BLOCKS, (const double *)part, stats);
        hipLaunchKernelGGL(oa_e_kernel, g, t, 0, s, n, (const double *)S, R, (const double *)lam,
                           (const double *)stats);
        hipLaunchKernelGGL(oa_copy_kernel, g, t, 0, s, n, (const double *)X, ldx, Xn, n);
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, n, n, n, 1.0, X, ldx, R, n, 1.0, Xn, n, nullptr, 0));
        hipLaunchKernelGGL(oa_copy_kernel, g, t, 0, s, n, (const double *)Xn, n, X, ldx);
    }
    // residual of the final X with its Rayleigh quotients
    EVD_CHECK(gemm_f64(s, OP_S, OP_N, 0, n, n, n, 1.0, A, lda, X, ldx, 0.0, AX, n, nullptr, 0));
    hipLaunchKernelGGL(oa_rayleigh_kernel, dim3((unsigned)n), dim3(64), 0, s, n, (const double *)AX,
                       (const double *)X, ldx, lam);
    hipLaunchKernelGGL(oa_resid_kernel, g, t, 0, s, n, (const double *)AX, (const double *)X, (const double *)lam, A,
                       lda, part);
    hipLaunchKernelGGL(oa_resid_final_kernel, dim3(1), dim3(64), 0, s, OA_BLOCKS, n, (const double *)part, stats + 4);
    return hipGetLastError() == hipSuccess ? EVD_OK : EVD_ERR_HIP;
}
