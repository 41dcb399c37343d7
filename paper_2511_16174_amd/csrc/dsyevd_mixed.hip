// Mixed-precision driver (an extension beside the paper's FP64 path, not in
// the paper): the two-stage pipeline of Sections 2.1 and 3.3 runs in FP32
// with split-BF16x3 matrix-core products, the tridiagonal eigenproblem is
// solved in FP64 (secular equations in FP64), and the eigenpairs are then
// refined in FP64 with Ogita-Aishima sweeps; the FP64 residual of the result
// is reported.
//
//   A (FP64) -> A32 -> SBR32 -> BC32 -> (d, e) FP64 -> D&C FP64 -> Q_d
//   SBR-back32, BC-back32 -> Q_sb32;   X = Q_sb32 * fp32(Q_d)  (split-BF16x3)
//   X (FP64) -> RefSyEv sweeps (FP64 MFMA) -> eigenvectors, Rayleigh quotients
#include "common.h"

size_t dc_work_bytes(char compz, int64_t n);
evd_status_t dc_run(evd_ctx_t ctx, char compz, int64_t n, const double *d, const double *e, double *W, double *Z,
                    int64_t ldz, void *work, int32_t *info);
evd_status_t orgsb_run_f32(evd_ctx_t ctx, int64_t n, int64_t b, const float *A, int64_t lda, const float *T, float *Q,
                           int64_t ldq, void *work);
size_t orgsb_work_bytes(int64_t n, int64_t b);
evd_status_t bcback_run_f32(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const float *V, const float *TAU,
                            float *Q, int64_t ldq);
size_t refine_work_bytes(int64_t n);
evd_status_t nonfinite_begin(hipStream_t s, int64_t n, double *A, int64_t lda, char uplo, int *flag);
evd_status_t nonfinite_end(hipStream_t s, int64_t n, const int *flag, double *W, double *A, int64_t lda, bool vec,
                           int32_t *info);
evd_status_t refine_run(evd_ctx_t ctx, int64_t n, const double *A, int64_t lda, double *X, int64_t ldx, double *lam,
                        int max_sweeps, double target, void *work, double *stats, int *done);

namespace {

// lower triangle of A (FP64) -> full-storage FP32 lower triangle (upper untouched)
__global__ void mx_down_lower_kernel(int64_t n, const double *A, int64_t lda, float *A32, int upper)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        if (i >= j) A32[idx] = (float)(upper ? A[j + i * lda] : A[i + j * lda]);
    }
}

__global__ void mx_mirror_upper_kernel(int64_t n, double *A, int64_t lda)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        if (i > j) A[i + j * lda] = A[j + i * lda];
    }
}

__global__ void mx_down_kernel(int64_t count, const double *src, float *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

__global__ void mx_up_kernel(int64_t count, const float *src, double *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

// ascending order of lam with columns of X permuted alike: rank of every
// entry (ties by index), then a column gather into A
__global__ void mx_rank_kernel(int64_t n, const double *lam, int *pos)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double key = lam[q];
    int64_t c = 0;
    for (int64_t r = 0; r < n; ++r) {
        const double v = lam[r];
        c += (v < key || (v == key && r < q)) ? 1 : 0;
    }
    pos[q] = (int)c;
}

__global__ void mx_scatter_kernel(int64_t n, const double *X, const double *lam, const int *pos, double *A,
                                  int64_t lda, double *W)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const int64_t pj = pos[j];
        A[i + pj * lda] = X[idx];
        if (i == 0) W[pj] = lam[j];
    }
}

// info = EVD_ERR_NOT_CONVERGED when a target was given and the returned pairs
// miss it (residual or orthogonality); an earlier status is kept
__global__ void mx_target_kernel(const double *stats, double target, int32_t *info)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && info && target > 0.0 && info[0] == 0 &&
        !(stats[0] <= target && stats[1] <= target))
        info[0] = EVD_ERR_NOT_CONVERGED;
}

int64_t choose_b_mixed(evd_ctx_t ctx, int64_t n) { return evd_choose_b(ctx, n); }

struct MixWork {
    float *A32, *AB, *T, *V, *TAU, *Qs, *Qd32, *X32;
    double *d, *e, *Qd, *Xd, *lam, *stats;
    int *prog, *pos, *nflag;
    void *sbr, *dc, *orgsb, *ref;
    int64_t b, ldab;
};

size_t mix_layout(int64_t n, int64_t b, char *base, MixWork *w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += evd_align256(bytes > 0 ? bytes : 1);
        return (void *)p;
    };
    MixWork t;
    t.b = b;
    t.ldab = 2 * b + 1;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int64_t p = evd_sbr_num_panels(n, b);
    const int64_t steps = bc_num_steps(n, b);
    t.A32 = (float *)take(nn * nn * 4);
    t.AB = (float *)take((size_t)t.ldab * nn * 4);
    t.T = (float *)take((size_t)(p > 0 ? p : 1) * b * b * 4);
    t.V = (float *)take((size_t)(steps > 0 ? steps : 1) * nn * b * 4);
    t.TAU = (float *)take((size_t)(steps > 0 ? steps : 1) * nn * 4);
    t.Qs = (float *)take(nn * nn * 4);
    t.Qd32 = (float *)take(nn * nn * 4);
    t.X32 = t.A32;  // SBR's FP32 copy of A is dead once SBR-back has consumed its Y's
    t.d = (double *)take(nn * 8);
    t.e = (double *)take(nn * 8);
    t.lam = (double *)take(nn * 8);
    t.stats = (double *)take(64);
    t.prog = (int *)take(nn * 4);
    t.pos = (int *)take(nn * 4);
    t.nflag = (int *)take(256);
    t.sbr = take(sbr_work_bytes_f32(n, b));
    t.orgsb = take(orgsb_work_bytes(n, b));
    t.Xd = (double *)take(nn * nn * 8);
    // Q_d and the D&C scratch are dead after the final product: the
    // refinement reuses the same region
    const size_t dcb = nn * nn * 8 + dc_work_bytes('I', n);
    const size_t rfb = refine_work_bytes(n);
    char *region = (char *)take(dcb > rfb ? dcb : rfb);
    t.Qd = (double *)region;
    t.dc = base ? (void *)(region + evd_align256(nn * nn * 8)) : nullptr;
    t.ref = (void *)region;
    if (w) *w = t;
    return off;
}

}  // namespace

extern "C" {

evd_status_t evd_dsyevd_mixed_work_size(evd_ctx_t ctx, char jobz, char uplo, int64_t n, int64_t lda, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    int bad = 0;
    if (!(jobz == 'V' || jobz == 'v')) bad = 2;
    else if (!(uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) bad = 3;
    else if (n < 0) bad = 4;
    else if (lda < (n > 1 ? n : 1)) bad = 5;
    ctx->last_invalid_arg = bad;
    if (bad) return EVD_ERR_INVALID_ARG;
    *bytes = mix_layout(n, choose_b_mixed(ctx, n), nullptr, nullptr);
    return EVD_OK;
}

evd_status_t evd_dsyevd_mixed(evd_ctx_t ctx, char jobz, char uplo, int64_t n, double *A, int64_t lda, double *W,
                              int32_t max_sweeps, double target_residual, void *work, size_t work_bytes,
                              int32_t *info, double *achieved)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    const int64_t b = choose_b_mixed(ctx, n);
    int bad = 0;
    if (!(jobz == 'V' || jobz == 'v')) bad = 2;
    else if (!(uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) bad = 3;
    else if (n < 0) bad = 4;
    else if (n > 0 && !A) bad = 5;
    else if (lda < (n > 1 ? n : 1)) bad = 6;
    else if (n > 0 && !W) bad = 7;
    else if (max_sweeps < 0 || max_sweeps > 8) bad = 8;
    else if (!(target_residual == target_residual)) bad = 9;
    else if (n > 0 && !work) bad = 10;
    else if (work_bytes < mix_layout(n, b, nullptr, nullptr)) bad = 11;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 11 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    hipStream_t s = ctx->stream;
    if (n < 3) {
        // tiny problems: the FP64 driver's workspace fits in ours
        size_t need = 0;
        EVD_CHECK(evd_dsyevd_work_size(ctx, 'V', uplo, n, lda, &need));
        if (need > work_bytes) return EVD_ERR_WORKSPACE;
        return evd_dsyevd(ctx, 'V', uplo, n, A, lda, W, work, work_bytes, info);
    }
    MixWork w;
    mix_layout(n, b, (char *)work, &w);
    const bool up = (uplo == 'U' || uplo == 'u');
    const bool timing = ctx->timing != 0;
    auto mark = [&](int i) { if (timing) (void)hipEventRecord(ctx->ev[i], s); };
    const dim3 g(2048), t(256);
    const int64_t nn = n * n;

    mark(0);
    EVD_CHECK(nonfinite_begin(s, n, A, lda, uplo, w.nflag));
    hipLaunchKernelGGL(mx_down_lower_kernel, g, t, 0, s, n, (const double *)A, lda, w.A32, up ? 1 : 0);
    // the refinement multiplies by A in full storage (A is overwritten by the
    // eigenvectors at the end): the stored triangle is copied into the other
    if (up) hipLaunchKernelGGL(mx_mirror_upper_kernel, g, t, 0, s, n, A, lda);
    else EVD_CHECK(evd_mirror_lower_f64(s, n, A, lda));
    EVD_CHECK(sbr_run_f32(ctx, 'L', n, b, w.A32, n, w.AB, w.ldab, w.T, w.sbr, w.nflag + 2, nullptr));
    mark(1);
    EVD_CHECK(bc_run_f32(ctx, 'V', n, b, w.AB, w.ldab, w.d, w.e, w.V, w.TAU, w.prog, w.nflag + 2, nullptr));
    mark(2);
    EVD_CHECK(dc_run(ctx, 'I', n, w.d, w.e, w.lam, w.Qd, n, w.dc, info));
    hipLaunchKernelGGL(mx_down_kernel, g, t, 0, s, nn, (const double *)w.Qd, w.Qd32);
    mark(3);
    EVD_CHECK(orgsb_run_f32(ctx, n, b, w.A32, n, w.T, w.Qs, n, w.orgsb));
    mark(4);
    EVD_CHECK(bcback_run_f32(ctx, n, n, b, w.V, w.TAU, w.Qs, n));
    mark(5);
    EVD_CHECK(gemm_f32x3(s, OP_N, OP_N, 0, n, n, n, 1.0f, w.Qs, n, w.Qd32, n, 0.0f, w.X32, n, nullptr, 0));
    hipLaunchKernelGGL(mx_up_kernel, g, t, 0, s, nn, (const float *)w.X32, w.Xd);
    mark(6);
    int done = 0;
    EVD_CHECK(refine_run(ctx, n, A, lda, w.Xd, n, w.lam, max_sweeps, target_residual, w.ref, w.stats, &done));
    hipLaunchKernelGGL(mx_target_kernel, dim3(1), dim3(64), 0, s, (const double *)w.stats, target_residual, info);
    hipLaunchKernelGGL(mx_rank_kernel, dim3((unsigned)evd_ceil_div(n, 256)), t, 0, s, n, (const double *)w.lam, w.pos);
    hipLaunchKernelGGL(mx_scatter_kernel, g, t, 0, s, n, (const double *)w.Xd, (const double *)w.lam,
                       (const int *)w.pos, A, lda, W);
    if (achieved) EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(achieved, w.stats, 8 * sizeof(double),
                                                         hipMemcpyDeviceToDevice, s)));
    EVD_CHECK(nonfinite_end(s, n, w.nflag, W, A, lda, true, info));
    mark(7);
    if (timing) {
        if (hipEventSynchronize(ctx->ev[7]) != hipSuccess) return EVD_ERR_HIP;
        float ms = 0.0f;
        for (int i = 0; i < 7; ++i)
            if (hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]) == hipSuccess) ctx->stage_ms[i] = ms;
        if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[7]) == hipSuccess) ctx->stage_ms[7] = ms;
    }
    return evd_check_last();
}

}  // extern "C"
