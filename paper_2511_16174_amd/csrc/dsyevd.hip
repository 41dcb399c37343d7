// dsyevd-style driver: the two-stage pipeline of the paper, with the back
// transformation in either stage order of Section 3.3.
//
//   SBR (A -> band B, panel reflectors)      stage 1   (Section 2.1.1, Eq. 1)
//   BC  (B -> T = tridiag(e, d, e), U)       stage 2   (Section 2.1.1)
//   D&C (T -> Lambda, Q_d)                   stage 3   (independent of 4a/4b)
//   SBR-back (Q_s on the identity)           stage 4a  (Section 2.1.2)
//   BC-back  (Q_sb = Q_s H_1 ... H_m)        stage 4b  (Section 4.3)
//   final GEMM Q = Q_sb Q_d                  stage 5   (Section 3.3)
// That is the reordered order ("order" = 0).  The default ("order" = 1) is
// the conventional order Q = Q_s (H_1 ... H_m Q_d), which needs no final GEMM
// (fewer flops when the stages run one after the other on one device).
// Eigenvalues only: SBR -> BC (no reflectors kept) -> bisection.
#include <chrono>
#include <thread>
#include <vector>

#include "common.h"

size_t dc_work_bytes(char compz, int64_t n);
evd_status_t dc_run(evd_ctx_t ctx, char compz, int64_t n, const double *d, const double *e, double *W, double *Z,
                    int64_t ldz, void *work, int32_t *info);
evd_status_t orgsb_run(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T, double *Q,
                       int64_t ldq, void *work);
size_t orgsb_work_bytes(int64_t n, int64_t b);
evd_status_t bcback_run(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, const double *TAU,
                        double *Q, int64_t ldq);
evd_status_t bcback_run_rev(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, const double *TAU,
                            double *Q, int64_t ldq);
evd_status_t ormsb_run(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T, double *C,
                       int64_t ldc, void *work);
evd_status_t transpose_run(hipStream_t s, int64_t n, const double *A, int64_t lda, double *B, int64_t ldb);
int host_dc_run(char compz, int64_t n, const double *d, const double *e, double *W, double *Z, int64_t ldz,
                int threads, int maxit);
evd_status_t nonfinite_begin(hipStream_t s, int64_t n, double *A, int64_t lda, char uplo, int *flag);
evd_status_t nonfinite_end(hipStream_t s, int64_t n, const int *flag, double *W, double *A, int64_t lda, bool vec,
                           int32_t *info);

namespace {

int64_t choose_b(evd_ctx_t ctx, int64_t n) { return evd_choose_b(ctx, n); }

struct EvdWork {
    double *AB, *T, *d, *e, *V, *TAU, *Qs, *Qd, *Tg;
    int *prog, *nflag;
    void *sbr, *dc, *orgsb;
    int64_t b, ldab;
};

size_t evd_layout(int64_t n, int64_t b, bool vec, char *base, EvdWork *w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += evd_align256(bytes > 0 ? bytes : 1);
        return (void *)p;
    };
    EvdWork t;
    t.b = b;
    t.ldab = 2 * b + 1;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int64_t p = evd_sbr_num_panels(n, b);
    const int64_t steps = bc_num_steps(n, b);
    t.AB = (double *)take((size_t)t.ldab * nn * 8);
    t.T = (double *)take((size_t)(p > 0 ? p : 1) * b * b * 8);
    t.d = (double *)take(nn * 8);
    t.e = (double *)take(nn * 8);
    t.prog = (int *)take(nn * 4);
    t.nflag = (int *)take(256);
    t.sbr = take(sbr_work_bytes(n, b));
    if (vec) {
        t.V = (double *)take((size_t)(steps > 0 ? steps : 1) * nn * b * 8);
        t.TAU = (double *)take((size_t)(steps > 0 ? steps : 1) * nn * 8);
        t.Qs = (double *)take(nn * nn * 8);
        t.Qd = (double *)take(nn * nn * 8);
        t.dc = take(dc_work_bytes('I', n));
        t.orgsb = take(orgsb_work_bytes(n, b));
        const size_t tge = bcback_mfma_t_elems(n, b);
        t.Tg = tge ? (double *)take(tge * 8) : nullptr;
    } else {
        t.V = t.TAU = t.Qs = t.Qd = t.Tg = nullptr;
        t.dc = take(dc_work_bytes('N', n));
        t.orgsb = nullptr;
    }
    if (w) *w = t;
    return off;
}

__global__ void copy_kernel(int64_t n, const double *src, int64_t lds, double *dst, int64_t ldd)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x)
        dst[(idx % n) + (idx / n) * ldd] = src[(idx % n) + (idx / n) * lds];
}

// Bulge chasing started beside SBR (SbrOverlap::launch): on the auxiliary
// stream, after the band storage and BC's scratch are reset on the main one.
struct BesideArg {
    evd_ctx_t ctx;
    char jobz;
    int64_t n, b;
    EvdWork *w;
};
evd_status_t launch_bc_beside(void *p)
{
    BesideArg *a = (BesideArg *)p;
    EvdWork &w = *a->w;
    EVD_CHECK(bc_launch_beside(a->ctx, a->jobz, a->n, a->b, w.AB, w.ldab, w.V, w.TAU, w.prog, w.nflag + 2,
                               w.nflag + 1, a->ctx->astream));
    return evd_hip(a->ctx, hipEventRecord(a->ctx->ev[11], a->ctx->astream));
}

__global__ void trivial_kernel(int64_t n, double *A, double *W, int vec, int32_t *info)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const bool finite = n != 1 || isfinite(A[0]);
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        if (n == 1) {
            W[0] = finite ? A[0] : nan;
            if (vec) A[0] = finite ? 1.0 : nan;
        }
        if (info) info[0] = finite ? 0 : EVD_ERR_NONFINITE;
    }
}

}  // namespace

// Workspace of evd_dsyevd(jobz = 'V') for any band width the drivers may pick.
size_t dsyevd_work_bytes_any_b(int64_t n)
{
    size_t m = 0;
    for (int64_t b = 1; b <= 64; b *= 2) {
        const size_t w = evd_layout(n, b, true, nullptr, nullptr);
        if (w > m) m = w;
    }
    return m;
}

extern "C" {

evd_status_t evd_dsyevd_work_size(evd_ctx_t ctx, char jobz, char uplo, int64_t n, int64_t lda, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    const bool vec = (jobz == 'V' || jobz == 'v');
    int bad = 0;
    if (!(vec || jobz == 'N' || jobz == 'n')) bad = 2;
    else if (!(uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) bad = 3;
    else if (n < 0 || n > EVD_MAX_N) bad = 4;
    else if (lda < (n > 1 ? n : 1) || lda > EVD_MAX_N) bad = 5;
    ctx->last_invalid_arg = bad;
    if (bad) return EVD_ERR_INVALID_ARG;
    *bytes = evd_layout(n, choose_b(ctx, n), vec, nullptr, nullptr);
    return EVD_OK;
}

evd_status_t evd_dsyevd(evd_ctx_t ctx, char jobz, char uplo, int64_t n, double *A, int64_t lda, double *W, void *work,
                        size_t work_bytes, int32_t *info)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    const bool vec = (jobz == 'V' || jobz == 'v');
    const int64_t b = choose_b(ctx, n);
    int bad = 0;
    if (!(vec || jobz == 'N' || jobz == 'n')) bad = 2;
    else if (!(uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) bad = 3;
    else if (n < 0 || n > EVD_MAX_N) bad = 4;
    else if (n > 0 && !A) bad = 5;
    else if (lda < (n > 1 ? n : 1) || lda > EVD_MAX_N) bad = 6;
    else if (n > 0 && !W) bad = 7;
    else if (n > 0 && !work) bad = 8;
    else if (work_bytes < evd_layout(n, b, vec, nullptr, nullptr)) bad = 9;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 9 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    hipStream_t s = ctx->stream;
    const bool timing = ctx->timing != 0;
    for (int i = 0; i < 8; ++i) ctx->stage_ms[i] = 0.0f;
    if (n == 1) {
        hipLaunchKernelGGL(trivial_kernel, dim3(1), dim3(64), 0, s, n, A, W, vec ? 1 : 0, info);
        return evd_hip(ctx, hipGetLastError());
    }
    EvdWork w;
    evd_layout(n, b, vec, (char *)work, &w);
    auto mark = [&](int i) { if (timing) (void)hipEventRecord(ctx->ev[i], s); };

    mark(0);
    // w.nflag: [0] non-finite input, [1] band columns published by SBR, [2] timeout
    EVD_CHECK(nonfinite_begin(s, n, A, lda, uplo, w.nflag));
    const bool beside = ctx->bc_overlap && ctx->astream && !ctx->in_batch && n > 2;
    if (beside) {
        // bulge chasing beside SBR (Section 2.1.1, Alg. 1): launched once SBR
        // has reset the band, each step gated by the published band columns
        BesideArg arg{ctx, vec ? 'V' : 'N', n, b, &w};
        const SbrOverlap ov{w.nflag + 1, launch_bc_beside, &arg};
        ctx->plain_panels = 1;
        const evd_status_t st = sbr_run(ctx, uplo, n, b, A, lda, w.AB, w.ldab, w.T, w.sbr, w.nflag + 2, &ov);
        ctx->plain_panels = 0;
        EVD_CHECK(st);
        mark(1);
        EVD_CHECK(evd_hip(ctx, hipStreamWaitEvent(s, ctx->ev[11], 0)));
        EVD_CHECK(bc_finish(ctx, n, w.AB, w.ldab, w.d, w.e));
    } else {
        EVD_CHECK(sbr_run(ctx, uplo, n, b, A, lda, w.AB, w.ldab, w.T, w.sbr, w.nflag + 2, nullptr));
        mark(1);
        // "debug_gate": wait for band columns nobody publishes (tests of the timeout path)
        EVD_CHECK(bc_run(ctx, vec ? 'V' : 'N', n, b, w.AB, w.ldab, w.d, w.e, w.V, w.TAU, w.prog, w.nflag + 2,
                         ctx->debug_gate ? w.nflag + 1 : nullptr));
    }
    mark(2);
    if (!vec) {
        EVD_CHECK(dc_run(ctx, 'N', n, w.d, w.e, W, nullptr, 1, w.dc, info));
        mark(3);
    } else {
        if (ctx->dc_host && !ctx->in_batch) {
            // the paper's placement (Algorithm 1, Section 3.3): D&C in a host
            // thread on the tridiagonal copied to host memory, while the GPU
            // forms Q_sb = Q_s H_1 ... H_m (reordered stages, independent of
            // D&C); then Q_d is copied to the device and Q = Q_sb Q_d.
            // Stage times: [2] host D&C (host clock, beside [3] and [4]),
            // [3] SBR-back, [4] BC-back, [5] wait for the host, copy of Q_d
            // and W, final GEMM.
            const size_t nn = (size_t)n;
            std::vector<double> hd(nn), he(nn), hw(nn), hz(nn * nn);
            if (!ctx->astream) return EVD_ERR_HIP;
            EVD_CHECK(evd_hip(ctx, hipEventRecord(ctx->ev[12], s)));
            EVD_CHECK(evd_hip(ctx, hipStreamWaitEvent(ctx->astream, ctx->ev[12], 0)));
            EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(hd.data(), w.d, nn * 8, hipMemcpyDeviceToHost, ctx->astream)));
            EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(he.data(), w.e, (nn - 1) * 8, hipMemcpyDeviceToHost, ctx->astream)));
            EVD_CHECK(evd_hip(ctx, hipEventRecord(ctx->ev[13], ctx->astream)));
            int hst = 0;
            float host_ms = 0.0f;
            hipError_t herr = hipSuccess;
            const int maxit = (ctx->dc_max_iter > 0 && ctx->dc_max_iter < 200) ? (int)ctx->dc_max_iter : 200;
            std::thread worker([&] {
                herr = hipEventSynchronize(ctx->ev[13]);
                if (herr != hipSuccess) return;
                const auto t0 = std::chrono::steady_clock::now();
                hst = host_dc_run('I', n, hd.data(), he.data(), hw.data(), hz.data(), n, (int)ctx->dc_host_threads,
                                  maxit);
                host_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
            });
            evd_status_t st = orgsb_run(ctx, n, b, A, lda, w.T, w.Qs, n, w.orgsb);
            mark(3);
            const bool blocked = w.Tg && ctx->bcback_valu == 0 && bcback_mfma_fits(n);
            if (st == EVD_OK && blocked) st = bcback_mfma_prepare(ctx, n, b, w.V, w.TAU, w.Tg, false);
            if (st == EVD_OK)
                st = blocked ? bcback_mfma_apply(ctx, n, n, b, w.V, w.Qs, n, w.Tg, false)
                             : bcback_run(ctx, n, n, b, w.V, w.TAU, w.Qs, n);
            mark(4);
            worker.join();
            EVD_CHECK(st);
            EVD_CHECK(evd_hip(ctx, herr));
            ctx->host_status = hst;
            EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(w.Qd, hz.data(), nn * nn * 8, hipMemcpyHostToDevice, s)));
            EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(W, hw.data(), nn * 8, hipMemcpyHostToDevice, s)));
            if (info) EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(info, &ctx->host_status, 4, hipMemcpyHostToDevice, s)));
            EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, n, n, n, 1.0, w.Qs, n, w.Qd, n, 0.0, A, lda, nullptr, 0));
            // the host buffers stay alive until the copies have completed
            EVD_CHECK(evd_hip(ctx, hipStreamSynchronize(s)));
            mark(5);
            EVD_CHECK(nonfinite_end(s, n, w.nflag, W, A, lda, vec, info));
            if (timing) {
                if (hipEventSynchronize(ctx->ev[5]) != hipSuccess) return EVD_ERR_HIP;
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->stage_ms[0] = ms;
                if (hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]) == hipSuccess) ctx->stage_ms[1] = ms;
                ctx->stage_ms[2] = host_ms;
                if (hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) ctx->stage_ms[3] = ms;
                if (hipEventElapsedTime(&ms, ctx->ev[3], ctx->ev[4]) == hipSuccess) ctx->stage_ms[4] = ms;
                if (hipEventElapsedTime(&ms, ctx->ev[4], ctx->ev[5]) == hipSuccess) ctx->stage_ms[5] = ms;
                if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[5]) == hipSuccess) ctx->stage_ms[6] = ms;
            }
            return evd_hip(ctx, hipGetLastError());
        }
        // conventional order: the BC-back T factors need only the reflectors,
        // so they are formed on an auxiliary stream while D&C runs (not in
        // the batched driver, whose streams are captured into a graph)
        const bool blocked_c = ctx->order != 0 && w.Tg && ctx->bcback_valu == 0 && bcback_mfma_fits(n);
        const bool ahead = blocked_c && !ctx->in_batch && ctx->astream;
        if (ahead) {
            EVD_CHECK(evd_hip(ctx, hipEventRecord(ctx->ev[8], s)));
            EVD_CHECK(evd_hip(ctx, hipStreamWaitEvent(ctx->astream, ctx->ev[8], 0)));
            ctx->stream = ctx->astream;
            const evd_status_t st = bcback_mfma_prepare(ctx, n, b, w.V, w.TAU, w.Tg, true);
            ctx->stream = s;
            EVD_CHECK(st);
            EVD_CHECK(evd_hip(ctx, hipEventRecord(ctx->ev[9], ctx->astream)));
        }
        EVD_CHECK(dc_run(ctx, 'I', n, w.d, w.e, W, w.Qd, n, w.dc, info));
        mark(3);
        if (ctx->order == 0) {
            // reordered stages (Section 3.3): Q_sb = Q_s H_1 ... H_m, then Q = Q_sb Q_d
            EVD_CHECK(orgsb_run(ctx, n, b, A, lda, w.T, w.Qs, n, w.orgsb));
            const bool blocked = w.Tg && ctx->bcback_valu == 0 && bcback_mfma_fits(n);
            if (blocked) EVD_CHECK(bcback_mfma_prepare(ctx, n, b, w.V, w.TAU, w.Tg, false));
            mark(4);
            if (blocked)
                EVD_CHECK(bcback_mfma_apply(ctx, n, n, b, w.V, w.Qs, n, w.Tg, false));
            else
                EVD_CHECK(bcback_run(ctx, n, n, b, w.V, w.TAU, w.Qs, n));
            mark(5);
            EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, n, n, n, 1.0, w.Qs, n, w.Qd, n, 0.0, A, lda, nullptr, 0));
            mark(6);
        } else {
            // conventional order: Z = H_1 ... H_m Q_d as rows of Z^T = Q_d^T H_m ... H_1,
            // then Q = Q_s Z (the panel reflectors still live in A's panel columns)
            // stage times: [3] transpose (+ group T factors), [4] BC-back alone,
            // [5] transpose + SBR-back + copy
            EVD_CHECK(transpose_run(s, n, w.Qd, n, w.Qs, n));
            const bool blocked = blocked_c;
            if (ahead) EVD_CHECK(evd_hip(ctx, hipStreamWaitEvent(s, ctx->ev[9], 0)));
            else if (blocked) EVD_CHECK(bcback_mfma_prepare(ctx, n, b, w.V, w.TAU, w.Tg, true));
            mark(4);
            if (blocked)
                EVD_CHECK(bcback_mfma_apply(ctx, n, n, b, w.V, w.Qs, n, w.Tg, true));
            else
                EVD_CHECK(bcback_run_rev(ctx, n, n, b, w.V, w.TAU, w.Qs, n));
            mark(5);
            EVD_CHECK(transpose_run(s, n, w.Qs, n, w.Qd, n));
            EVD_CHECK(ormsb_run(ctx, n, b, A, lda, w.T, w.Qd, n, w.orgsb));
            hipLaunchKernelGGL(copy_kernel, dim3(4096), dim3(256), 0, s, n, (const double *)w.Qd, n, A, lda);
            mark(6);
        }
    }
    EVD_CHECK(nonfinite_end(s, n, w.nflag, W, A, lda, vec, info));
    if (timing) {
        if (hipEventSynchronize(ctx->ev[vec ? 6 : 3]) != hipSuccess) return EVD_ERR_HIP;
        float ms = 0.0f;
        const int last = vec ? 6 : 3;
        for (int i = 0; i < last; ++i) {
            if (hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]) == hipSuccess) ctx->stage_ms[i] = ms;
        }
        if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[last]) == hipSuccess) ctx->stage_ms[6] = ms;
    }
    return evd_hip(ctx, hipGetLastError());
}

}  // extern "C"
