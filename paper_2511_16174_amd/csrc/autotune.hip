// Band-width autotuner: times evd_dsyevd for each candidate half-bandwidth b
// on the caller's matrix (restored from A before every trial) with events on
// the context's stream, and records the fastest b for the size bucket
// floor(log2 n) in the context; later calls with the "b" parameter at 0 use it.
#include "common.h"

namespace {
__global__ void at_copy_kernel(int64_t n, const double *A, int64_t lda, double *B)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        B[i + j * n] = A[i + j * lda];
    }
}
const int64_t kCandidates[] = {16, 32, 64};
}  // namespace

extern "C" {

evd_status_t evd_autotune_work_size(evd_ctx_t ctx, char jobz, int64_t n, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    const int64_t saved = ctx->b;
    size_t best = 0;
    for (int64_t b : kCandidates) {
        ctx->b = b;
        size_t w = 0;
        evd_status_t st = evd_dsyevd_work_size(ctx, jobz, 'L', n, n > 1 ? n : 1, &w);
        if (st != EVD_OK) { ctx->b = saved; return st; }
        if (w > best) best = w;
    }
    ctx->b = saved;
    *bytes = best + evd_align256((size_t)(n > 0 ? n : 1) * (n > 0 ? n : 1) * sizeof(double)) +
             evd_align256((size_t)(n > 0 ? n : 1) * sizeof(double)) + 256;
    return EVD_OK;
}

evd_status_t evd_autotune(evd_ctx_t ctx, char jobz, int64_t n, const double *A, int64_t lda, void *work,
                          size_t work_bytes, int64_t *best_b, float *best_ms)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    size_t need = 0;
    int bad = 0;
    if (!(jobz == 'N' || jobz == 'n' || jobz == 'V' || jobz == 'v')) bad = 2;
    else if (n < 1) bad = 3;
    else if (!A) bad = 4;
    else if (lda < n) bad = 5;
    else if (!work) bad = 6;
    if (!bad && evd_autotune_work_size(ctx, jobz, n, &need) != EVD_OK) bad = 3;
    if (!bad && work_bytes < need) bad = 7;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 7 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    char *base = (char *)work;
    double *Acopy = (double *)base;
    double *W = (double *)(base + evd_align256((size_t)n * n * sizeof(double)));
    int32_t *info = (int32_t *)((char *)W + evd_align256((size_t)n * sizeof(double)));
    void *ework = (char *)info + 256;
    const size_t ebytes = work_bytes - (size_t)((char *)ework - base);
    const int64_t saved_b = ctx->b, saved_t = ctx->timing;
    ctx->timing = 0;
    hipStream_t s = ctx->stream;
    float best = 3.4e38f;
    int64_t bestb = 0;
    for (int64_t b : kCandidates) {
        if (b >= n) continue;
        ctx->b = b;
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {  // first call warms up
            hipLaunchKernelGGL(at_copy_kernel, dim3(2048), dim3(256), 0, s, n, A, lda, Acopy);
            if (hipEventRecord(ctx->ev[14], s) != hipSuccess) { ctx->b = saved_b; ctx->timing = saved_t; return EVD_ERR_HIP; }
            evd_status_t st = evd_dsyevd(ctx, jobz, 'L', n, Acopy, n, W, ework, ebytes, info);
            if (st != EVD_OK) { ctx->b = saved_b; ctx->timing = saved_t; return st; }
            if (hipEventRecord(ctx->ev[15], s) != hipSuccess || hipEventSynchronize(ctx->ev[15]) != hipSuccess) {
                ctx->b = saved_b;
                ctx->timing = saved_t;
                return EVD_ERR_HIP;
            }
            (void)hipEventElapsedTime(&ms, ctx->ev[14], ctx->ev[15]);
        }
        if (ms < best) { best = ms; bestb = b; }
    }
    ctx->b = saved_b;
    ctx->timing = saved_t;
    if (bestb > 0) {
        int bucket = 0;
        while (bucket < 63 && ((int64_t)1 << (bucket + 1)) <= n) ++bucket;
        ctx->tuned_b[bucket] = bestb;
    }
    if (best_b) *best_b = bestb;
    if (best_ms) *best_ms = best;
    return EVD_OK;
}

}  // extern "C"
