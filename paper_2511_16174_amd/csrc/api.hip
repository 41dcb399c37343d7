// C ABI: context management, argument checking and the GEMM entry point.
#include <string.h>
#include <new>

#include "common.h"

extern "C" {

const char *evd_status_string(evd_status_t s)
{
    switch (s) {
    case EVD_OK: return "ok";
    case EVD_ERR_INVALID_ARG: return "invalid argument";
    case EVD_ERR_WORKSPACE: return "workspace too small";
    case EVD_ERR_HIP: return "HIP runtime error";
    case EVD_ERR_NONFINITE: return "non-finite input";
    case EVD_ERR_NOT_CONVERGED: return "not converged";
    case EVD_ERR_NOT_IMPLEMENTED: return "not implemented";
    case EVD_ERR_TIMEOUT: return "wait between workgroups timed out";
    }
    return "unknown status";
}

evd_status_t evd_create(evd_ctx_t *ctx, int device)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    *ctx = nullptr;
    if (device == -1) {  // validation-only context: no HIP call is ever made with it
        evd_ctx_s *c = new (std::nothrow) evd_ctx_s();
        if (!c) return EVD_ERR_HIP;
        memset(c, 0, sizeof(*c));
        c->device = -1;
        c->order = 1;
        *ctx = c;
        return EVD_OK;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return EVD_ERR_INVALID_ARG;
    evd_ctx_s *c = new (std::nothrow) evd_ctx_s();
    if (!c) return EVD_ERR_HIP;
    memset(c, 0, sizeof(*c));
    c->device = device;
    c->stream = nullptr;
    c->batch_graph = 0;   // direct launches: the graph's replay runs the streams' branches one after another
    c->batch_plain = 1;
    c->order = 1;  // conventional stage order: fewest flops when the stages run one after another
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) { delete c; return EVD_ERR_HIP; }
    if (hipSetDevice(device) != hipSuccess) { delete c; return EVD_ERR_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return EVD_ERR_HIP; }
    c->num_cus = prop.multiProcessorCount;
    gemm_set_cu_count(c->num_cus);
    for (int i = 0; i < 16; ++i) {
        if (hipEventCreate(&c->ev[i]) != hipSuccess) { evd_destroy(c); return EVD_ERR_HIP; }
    }
    // auxiliary stream (default priority) for work formed beside D&C; created
    // here so that no compute call creates runtime objects
    if (hipStreamCreateWithFlags(&c->astream, hipStreamNonBlocking) != hipSuccess) {
        c->astream = nullptr;
        evd_destroy(c);
        return EVD_ERR_HIP;
    }
    // device address of the allocation-free entry point's static scratch
    if (noalloc_init_device(device) != EVD_OK) { evd_destroy(c); return EVD_ERR_HIP; }
    (void)hipSetDevice(prev);
    *ctx = c;
    return EVD_OK;
}

evd_status_t evd_destroy(evd_ctx_t ctx)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    if (ctx->device >= 0) {
        // drain the context's own streams before their objects go away
        (void)hipSetDevice(ctx->device);
        for (int i = 0; i < ctx->nbstreams; ++i) (void)hipStreamSynchronize(ctx->bstreams[i]);
        if (ctx->cstream) (void)hipStreamSynchronize(ctx->cstream);
        if (ctx->astream) (void)hipStreamSynchronize(ctx->astream);
    }
    for (int i = 0; i < 16; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    for (int i = 0; i < ctx->nbstreams; ++i) (void)hipStreamDestroy(ctx->bstreams[i]);
    if (ctx->cstream) (void)hipStreamDestroy(ctx->cstream);
    if (ctx->astream) (void)hipStreamDestroy(ctx->astream);
    for (int i = 0; i < 17; ++i)
        if (ctx->bev[i]) (void)hipEventDestroy(ctx->bev[i]);
    delete ctx;
    return EVD_OK;
}

evd_status_t evd_set_stream(evd_ctx_t ctx, void *stream)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)stream;
    return EVD_OK;
}

static int64_t *param_slot(evd_ctx_t ctx, const char *key)
{
    if (!key) return nullptr;
    if (!strcmp(key, "b")) return &ctx->b;
    if (!strcmp(key, "bc_waves")) return &ctx->bc_waves;
    if (!strcmp(key, "bcback_group")) return &ctx->bcback_group;
    if (!strcmp(key, "bcback_rows")) return &ctx->bcback_rows;
    if (!strcmp(key, "order")) return &ctx->order;
    if (!strcmp(key, "timing")) return &ctx->timing;
    if (!strcmp(key, "panel_wgs")) return &ctx->panel_wgs;
    if (!strcmp(key, "panel_generic")) return &ctx->panel_generic;
    if (!strcmp(key, "sbr_nb")) return &ctx->sbr_nb;
    if (!strcmp(key, "bcback_valu")) return &ctx->bcback_valu;
    if (!strcmp(key, "bcback_sub")) return &ctx->bcback_sub;
    if (!strcmp(key, "bcback_rt")) return &ctx->bcback_rt;
    if (!strcmp(key, "bcback_lds2")) return &ctx->bcback_lds2;
    if (!strcmp(key, "gemm_staged")) return &ctx->gemm_staged;
    if (!strcmp(key, "orgsb_nb")) return &ctx->orgsb_nb;
    if (!strcmp(key, "batch_streams")) return &ctx->batch_streams;
    if (!strcmp(key, "batch_graph")) return &ctx->batch_graph;
    if (!strcmp(key, "last_graph_used")) return &ctx->last_graph_used;
    if (!strcmp(key, "last_hip_error")) return &ctx->last_hip_error;
    if (!strcmp(key, "capture_error")) return &ctx->capture_error;
    if (!strcmp(key, "dc_max_iter")) return &ctx->dc_max_iter;
    if (!strcmp(key, "bc_overlap")) return &ctx->bc_overlap;
    if (!strcmp(key, "spin_limit_ms")) return &ctx->spin_limit_ms;
    if (!strcmp(key, "debug_gate")) return &ctx->debug_gate;
    if (!strcmp(key, "batch_plain")) return &ctx->batch_plain;
    if (!strcmp(key, "dc_host")) return &ctx->dc_host;
    if (!strcmp(key, "last_tuned_nb")) return &ctx->last_tuned_nb;
    if (!strcmp(key, "last_tuned_sub")) return &ctx->last_tuned_sub;
    if (!strcmp(key, "dc_host_threads")) return &ctx->dc_host_threads;
    return nullptr;
}

evd_status_t evd_set_param(evd_ctx_t ctx, const char *key, int64_t value)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    int64_t *slot = param_slot(ctx, key);
    if (!slot) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    if (value < 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    if ((slot == &ctx->bcback_group && value != 0 && value != 32 && value != 64) ||
        (slot == &ctx->bcback_rows && value != 0 && value != 64 && value != 128) ||
        (slot == &ctx->bcback_sub && value != 0 && value != 16 && value != 32 && value != 64) ||
        (slot == &ctx->bcback_rt && value > 2) || (slot == &ctx->gemm_staged && value > 1) ||
        (slot == &ctx->bcback_lds2 && value > 1) || (slot == &ctx->panel_generic && value > 1)) {
        ctx->last_invalid_arg = 3;
        return EVD_ERR_INVALID_ARG;
    }
    *slot = value;
    if (slot == &ctx->gemm_staged) gemm_set_staged((int)value);
    if (slot == &ctx->last_hip_error && value == 0) evd_tls_hip_error = 0;
    ctx->last_invalid_arg = 0;
    return EVD_OK;
}

evd_status_t evd_get_param(evd_ctx_t ctx, const char *key, int64_t *value)
{
    if (!ctx || !value) return EVD_ERR_INVALID_ARG;
    int64_t *slot = param_slot(ctx, key);
    if (!slot) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    if (slot == &ctx->last_hip_error && !ctx->last_hip_error) ctx->last_hip_error = evd_tls_hip_error;
    *value = *slot;
    return EVD_OK;
}

int evd_last_invalid_arg(evd_ctx_t ctx) { return ctx ? ctx->last_invalid_arg : 0; }

evd_status_t evd_get_stage_times(evd_ctx_t ctx, float *ms)
{
    if (!ctx || !ms) return EVD_ERR_INVALID_ARG;
    for (int i = 0; i < 8; ++i) ms[i] = ctx->stage_ms[i];
    return EVD_OK;
}

static int op_code(char c, bool allow_s)
{
    if (c == 'N' || c == 'n') return OP_N;
    if (c == 'T' || c == 't' || c == 'C' || c == 'c') return OP_T;
    if (allow_s && (c == 'S' || c == 's')) return OP_S;
    return -1;
}

evd_status_t evd_dgemm_work_size(evd_ctx_t ctx, int64_t m, int64_t n, int64_t k, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (m < 0 || n < 0 || k < 0) return EVD_ERR_INVALID_ARG;
    *bytes = gemm_splitk_ws_elems(m, n, k) * sizeof(double);
    return EVD_OK;
}

evd_status_t evd_dgemm(evd_ctx_t ctx, char opa, char opb, int lower_c, int64_t m, int64_t n, int64_t k,
                       double alpha, const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                       double *C, int64_t ldc, void *work, size_t work_bytes)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    ctx->last_invalid_arg = 0;
    const int oa = op_code(opa, true), ob = op_code(opb, false);
    int bad = 0;
    if (oa < 0) bad = 2;
    else if (ob < 0) bad = 3;
    else if (m < 0) bad = 5;
    else if (n < 0) bad = 6;
    else if (k < 0 || (oa == OP_S && k != m)) bad = 7;
    else if (m > 0 && k > 0 && !A) bad = 9;
    else if (lda < ((oa == OP_N || oa == OP_S) ? (m > 1 ? m : 1) : (k > 1 ? k : 1))) bad = 10;
    else if (n > 0 && k > 0 && !B) bad = 11;
    else if (ldb < ((ob == OP_N) ? (k > 1 ? k : 1) : (n > 1 ? n : 1))) bad = 12;
    else if (m > 0 && n > 0 && !C) bad = 14;
    else if (ldc < (m > 1 ? m : 1)) bad = 15;
    else if (lower_c && m != n) bad = 4;
    else if (lower_c == 2 && (oa != OP_N || ob != OP_T)) bad = 4;
    if (bad) { ctx->last_invalid_arg = bad; return EVD_ERR_INVALID_ARG; }
    if (oa == OP_S && ob == OP_T) { /* supported */ }
    if (oa == OP_S && lower_c) { ctx->last_invalid_arg = 4; return EVD_ERR_INVALID_ARG; }
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    return gemm_f64(ctx->stream, oa, ob, lower_c == 2 ? 2 : (lower_c ? 1 : 0), m, n, k, alpha, A, lda, B, ldb, beta, C,
                    ldc, (double *)work, work ? work_bytes / sizeof(double) : 0);
}

}  // extern "C"
