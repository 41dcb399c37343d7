// Batched EVD of many uneven-size symmetric matrices (an extension beside
// the paper's method, not in the paper; the paper names tight-binding models
// as an application, Section 1).
//
// Each matrix runs the full two-stage pipeline of evd_dsyevd.  Matrices are
// ordered by decreasing n^3 and assigned greedily (longest processing time
// first) to several internal streams, each with its own slice of the
// workspace; optionally ("batch_graph" = 1) the whole fork/join sequence is
// captured once into a hipGraph and replayed while the batch description
// (sizes and pointers) is unchanged.
// Persistent kernels (panel QR, bulge chasing) launched from concurrent
// streams are capped at (compute units / streams) workgroups each, so that all
// of them fit on the chip at once whatever the interleaving.
// Device timestamps (wall_clock64, 100 MHz) bracket every matrix.
#include <algorithm>
#include <vector>

#include "common.h"

namespace {

__global__ void bt_stamp_kernel(uint64_t *t)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *t = wall_clock64();
}

struct BatchPlan {
    std::vector<int> order;       // processing order (indices into the batch)
    std::vector<int> stream_of;   // stream of matrix i
    std::vector<size_t> ws_off;   // workspace offset of each stream
    std::vector<size_t> ws_size;  // workspace size of each stream
    size_t total = 0;
};

int num_streams(const evd_ctx_s *ctx)
{
    int ns = (int)(ctx->batch_streams > 0 ? ctx->batch_streams : 8);
    return ns > 16 ? 16 : ns;
}

evd_status_t plan_batch(evd_ctx_t ctx, char jobz, int32_t batch, const int64_t *n, const int64_t *lda, BatchPlan *p)
{
    const int ns = num_streams(ctx);
    p->order.resize(batch);
    for (int i = 0; i < batch; ++i) p->order[i] = i;
    std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) { return n[a] > n[b]; });
    std::vector<double> load(ns, 0.0);
    p->stream_of.assign(batch, 0);
    p->ws_size.assign(ns, 0);
    for (int i : p->order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        p->stream_of[i] = k;
        load[k] += (double)n[i] * (double)n[i] * (double)n[i];
        size_t w = 0;
        EVD_CHECK(evd_dsyevd_work_size(ctx, jobz, 'L', n[i], lda[i], &w));
        p->ws_size[k] = std::max(p->ws_size[k], w);
    }
    p->ws_off.assign(ns, 0);
    size_t off = 0;
    for (int k = 0; k < ns; ++k) {
        p->ws_off[k] = off;
        off += evd_align256(p->ws_size[k] > 0 ? p->ws_size[k] : 1);
    }
    p->total = off;
    return EVD_OK;
}

uint64_t mix(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

}  // namespace

extern "C" {

evd_status_t evd_dsyevd_batched_work_size(evd_ctx_t ctx, char jobz, int32_t batch, const int64_t *n,
                                          const int64_t *lda, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    int bad = 0;
    if (!(jobz == 'N' || jobz == 'n' || jobz == 'V' || jobz == 'v')) bad = 2;
    else if (batch < 0) bad = 3;
    else if (batch > 0 && !n) bad = 4;
    else if (batch > 0 && !lda) bad = 5;
    for (int i = 0; !bad && i < batch; ++i) {
        if (n[i] < 0) bad = 4;
        else if (lda[i] < (n[i] > 1 ? n[i] : 1)) bad = 5;
    }
    ctx->last_invalid_arg = bad;
    if (bad) return EVD_ERR_INVALID_ARG;
    BatchPlan p;
    EVD_CHECK(plan_batch(ctx, jobz, batch, n, lda, &p));
    *bytes = p.total;
    return EVD_OK;
}

evd_status_t evd_dsyevd_batched(evd_ctx_t ctx, char jobz, char uplo, int32_t batch, const int64_t *n,
                                double *const *A, const int64_t *lda, double *const *W, void *work, size_t work_bytes,
                                int32_t *info, uint64_t *t_start_end)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    int bad = 0;
    if (!(jobz == 'N' || jobz == 'n' || jobz == 'V' || jobz == 'v')) bad = 2;
    else if (!(uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) bad = 3;
    else if (batch < 0) bad = 4;
    else if (batch > 0 && (!n || !A || !lda || !W)) bad = 5;
    for (int i = 0; !bad && i < batch; ++i) {
        if (n[i] < 0) bad = 5;
        else if (n[i] > 0 && (!A[i] || !W[i])) bad = 6;
        else if (lda[i] < (n[i] > 1 ? n[i] : 1)) bad = 7;
    }
    if (!bad && batch > 0 && !info) bad = 11;
    BatchPlan p;
    if (!bad && plan_batch(ctx, jobz, batch, n, lda, &p) != EVD_OK) bad = 5;
    if (!bad && batch > 0 && !work) bad = 9;
    if (!bad && work_bytes < p.total) bad = 10;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 10 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (batch == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));

    const int ns = num_streams(ctx);
    while (ctx->nbstreams < ns) {
        EVD_CHECK(evd_hip(ctx, hipStreamCreateWithFlags(&ctx->bstreams[ctx->nbstreams], hipStreamNonBlocking)));
        ctx->nbstreams++;
    }
    for (int i = 0; i <= ns; ++i)
        if (!ctx->bev[i]) EVD_CHECK(evd_hip(ctx, hipEventCreateWithFlags(&ctx->bev[i], hipEventDisableTiming)));

    // key of the captured graph: everything the launch sequence depends on
    uint64_t key = mix(0x1234, (uint64_t)batch);
    key = mix(key, (uint64_t)jobz);
    key = mix(key, (uint64_t)uplo);
    key = mix(key, (uint64_t)(uintptr_t)work);
    key = mix(key, (uint64_t)(uintptr_t)info);
    key = mix(key, (uint64_t)(uintptr_t)t_start_end);
    key = mix(key, (uint64_t)(uintptr_t)ctx->stream);
    key = mix(key, (uint64_t)ns);
    for (int i = 0; i < batch; ++i) {
        key = mix(key, (uint64_t)n[i]);
        key = mix(key, (uint64_t)lda[i]);
        key = mix(key, (uint64_t)(uintptr_t)A[i]);
        key = mix(key, (uint64_t)(uintptr_t)W[i]);
        key = mix(key, (uint64_t)evd_choose_b(ctx, n[i]));
        key = mix(key, (uint64_t)evd_choose_nb(ctx, n[i]));
        key = mix(key, (uint64_t)evd_choose_sub(ctx, n[i]));
    }
    if (ctx->batch_graph && ctx->gexec && ctx->gkey == key) {
        ctx->last_graph_used = 1;
        return evd_hip(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
    }

    hipStream_t main = ctx->stream;
    const int64_t saved_bc = ctx->bc_waves, saved_pw = ctx->panel_wgs, saved_t = ctx->timing;
    const int64_t cap = (ctx->num_cus / ns) > 1 ? (ctx->num_cus / ns) : 1;
    // fork from `origin` onto the internal streams, join back into it
    auto enqueue = [&](hipStream_t origin) -> evd_status_t {
        ctx->bc_waves = (saved_bc > 0 && saved_bc < cap) ? saved_bc : cap;
        // panels take the fewest workgroups by default (ceil(m / 512) at b = 64,
        // within the per-stream share for m <= 512 * cap)
        ctx->panel_wgs = (saved_pw > 0 && saved_pw < cap) ? saved_pw : 0;
        ctx->timing = 0;
        ctx->in_batch = 1;
        // "batch_plain": the persistent kernels (panel QR, bulge chasing)
        // launched plainly rather than cooperatively, so that the streams'
        // pipelines run side by side.  Co-residency still holds: each stream
        // has at most one persistent kernel in flight, of at most cap
        // workgroups, each workgroup fits on an empty compute unit, and
        // workgroups go round-robin to the XCDs, so the at most num_cus
        // persistent workgroups leave a compute unit without one on every XCD
        // as long as one of them is still waiting to start; every other kernel
        // finishes on its own.  The waits stay bounded in any case.
        int64_t nmax = 0;
        for (int i = 0; i < batch; ++i) nmax = n[i] > nmax ? n[i] : nmax;
        const bool plain = ctx->batch_plain && nmax <= 512 * cap;  // panels of at most cap workgroups
        ctx->plain_panels = plain ? 1 : 0;
        ctx->plain_bc = plain ? 1 : 0;
        evd_status_t st = EVD_OK;
        st = evd_hip(ctx, hipEventRecord(ctx->bev[ns], origin));
        for (int k = 0; st == EVD_OK && k < ns; ++k) st = evd_hip(ctx, hipStreamWaitEvent(ctx->bstreams[k], ctx->bev[ns], 0));
        for (int idx = 0; st == EVD_OK && idx < batch; ++idx) {
            const int i = p.order[idx];
            const int k = p.stream_of[i];
            ctx->stream = ctx->bstreams[k];
            if (t_start_end) hipLaunchKernelGGL(bt_stamp_kernel, dim3(1), dim3(64), 0, ctx->stream, t_start_end + 2 * i);
            st = evd_dsyevd(ctx, jobz, uplo, n[i], A[i], lda[i], W[i], (char *)work + p.ws_off[k], p.ws_size[k],
                            info + i);
            if (t_start_end) hipLaunchKernelGGL(bt_stamp_kernel, dim3(1), dim3(64), 0, ctx->stream, t_start_end + 2 * i + 1);
        }
        ctx->stream = main;
        for (int k = 0; st == EVD_OK && k < ns; ++k) {
            st = evd_hip(ctx, hipEventRecord(ctx->bev[k], ctx->bstreams[k]));
            if (st == EVD_OK) st = evd_hip(ctx, hipStreamWaitEvent(origin, ctx->bev[k], 0));
        }
        ctx->bc_waves = saved_bc;
        ctx->panel_wgs = saved_pw;
        ctx->timing = saved_t;
        ctx->in_batch = 0;
        ctx->plain_panels = 0;
        ctx->plain_bc = 0;
        return st;
    };

    ctx->last_graph_used = 0;
    ctx->capture_error = 0;
    if (ctx->batch_graph) {
        // capture on an internal stream (the caller's may be the null stream,
        // which cannot be captured) and launch the graph on the caller's
        // stream; if anything in the sequence cannot be captured, fall back to
        // running it directly (reported through "last_graph_used")
        if (!ctx->cstream) EVD_CHECK(evd_hip(ctx, hipStreamCreateWithFlags(&ctx->cstream, hipStreamNonBlocking)));
        hipGraph_t graph = nullptr;
        const hipError_t eb = hipStreamBeginCapture(ctx->cstream, hipStreamCaptureModeThreadLocal);
        if (eb != hipSuccess) {
            (void)hipGetLastError();
            ctx->capture_error = (int64_t)eb;
        } else {
            evd_status_t st = enqueue(ctx->cstream);
            hipError_t ec = hipStreamEndCapture(ctx->cstream, &graph);
            if (st == EVD_OK && ec == hipSuccess && graph) {
                hipGraphExec_t exec = nullptr;
                if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
                    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
                    ctx->gexec = exec;
                    ctx->gkey = key;
                    (void)hipGraphDestroy(graph);
                    ctx->last_graph_used = 1;
                    return evd_hip(ctx, hipGraphLaunch(ctx->gexec, main));
                }
            }
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            ctx->capture_error = ctx->last_hip_error ? ctx->last_hip_error : (int64_t)(ec != hipSuccess ? ec : -1);
            ctx->last_hip_error = 0;
            evd_tls_hip_error = 0;
        }
    }
    return enqueue(main);
}

}  // extern "C"
