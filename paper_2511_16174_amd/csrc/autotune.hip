// Autotuner: times evd_dsyevd for each candidate configuration -- half
// bandwidth b, SBR outer block (the double-blocking width of the trailing
// update) and, at b = 64, the BC-back block-reflector width -- on the
// caller's matrix (restored from A before every trial) with events on the
// context's stream, and records the fastest for the size bucket
// floor(log2 n) in the context; later calls with those parameters at 0 use it.
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
struct Config {
    int64_t b, nb, sub;
};
// SBR outer blocks of 4 to 16 panels; at b = 64 both BC-back block widths
const Config kConfigs[] = {{16, 256, 0}, {16, 512, 0}, {32, 256, 0}, {32, 512, 0}, {64, 256, 32}, {64, 320, 32},
                           {64, 512, 32}, {64, 320, 64}};
}  // namespace

extern "C" {

evd_status_t evd_autotune_work_size(evd_ctx_t ctx, char jobz, int64_t n, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    const int64_t saved = ctx->b;
    size_t best = 0;
    for (int64_t b : kCandidates) {   // the workspace does not depend on the outer block or BC-back width
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
    const int64_t saved_b = ctx->b, saved_t = ctx->timing, saved_nb = ctx->sbr_nb, saved_sub = ctx->bcback_sub;
    auto restore = [&] {
        ctx->b = saved_b;
        ctx->timing = saved_t;
        ctx->sbr_nb = saved_nb;
        ctx->bcback_sub = saved_sub;
    };
    ctx->timing = 0;
    hipStream_t s = ctx->stream;
    float best = 3.4e38f;
    Config bestc{0, 0, 0};
    for (const Config &c : kConfigs) {
        if (c.b >= n) continue;
        ctx->b = c.b;
        ctx->sbr_nb = c.nb;
        ctx->bcback_sub = c.sub;
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {  // first call warms up
            hipLaunchKernelGGL(at_copy_kernel, dim3(2048), dim3(256), 0, s, n, A, lda, Acopy);
            if (hipEventRecord(ctx->ev[14], s) != hipSuccess) { restore(); return EVD_ERR_HIP; }
            evd_status_t st = evd_dsyevd(ctx, jobz, 'L', n, Acopy, n, W, ework, ebytes, info);
            if (st != EVD_OK) { restore(); return st; }
            if (hipEventRecord(ctx->ev[15], s) != hipSuccess || hipEventSynchronize(ctx->ev[15]) != hipSuccess) {
                restore();
                return EVD_ERR_HIP;
            }
            (void)hipEventElapsedTime(&ms, ctx->ev[14], ctx->ev[15]);
        }
        if (ms < best) { best = ms; bestc = c; }
    }
    restore();
    if (bestc.b > 0) {
        const int bucket = evd_size_bucket(n);
        ctx->tuned_b[bucket] = bestc.b;
        ctx->tuned_nb[bucket] = bestc.nb;
        ctx->tuned_sub[bucket] = bestc.sub;
    }
    ctx->last_tuned_nb = bestc.nb;
    ctx->last_tuned_sub = bestc.sub;
    if (best_b) *best_b = bestc.b;
    if (best_ms) *best_ms = best;
    return EVD_OK;
}

}  // extern "C"
