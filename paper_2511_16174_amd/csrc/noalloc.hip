// evd_dsyevd without a caller workspace, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation).  The pipeline's scratch lives in one file-scope
// device array per GPU, `scratch`, of EVD_NOALLOC_SCRATCH_BYTES; the kernels
// are those of evd_dsyevd and receive the array's device address as their
// workspace pointer.
//
// The array's name is a host-side stand-in in host code, not a device
// address: its per-device address is looked up once per device with
// hipGetSymbolAddress (from evd_create, with that device current) and only
// that address is handed to kernels.
//
// Every call on one GPU shares that GPU's array and finds the previous
// call's contents in it.  The pipeline starts from no assumption about its
// scratch: the progress counters of bulge chasing and the panel records of
// SBR are reset by kernels at the start of each call, every other buffer is
// written before it is read.  Calls that overlap on one GPU (two streams, two
// host threads) race on the array; the caller must serialise them.
#include <mutex>

#include "common.h"

static_assert(EVD_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) char scratch[EVD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];          // device address of `scratch` on each GPU
hipError_t g_err[kMaxDevices];     // lookup status (hipSuccess once g_ptr is set)
bool g_done[kMaxDevices];

}  // namespace

// Called by evd_create with `device` current.
evd_status_t noalloc_init_device(int device)
{
    if (device < 0 || device >= kMaxDevices) return EVD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_done[device]) return g_err[device] == hipSuccess ? EVD_OK : EVD_ERR_HIP;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_done[device] = true;
    g_err[device] = e;
    g_ptr[device] = (e == hipSuccess) ? p : nullptr;
    return e == hipSuccess ? EVD_OK : evd_hip_status(e);
}

static void *noalloc_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_done[device] ? g_ptr[device] : nullptr;
}

extern "C" {

evd_status_t evd_dsyevd_noalloc(evd_ctx_t ctx, char jobz, char uplo, int64_t n, double *A, int64_t lda, double *W,
                                int32_t *info)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    size_t need = 0;
    EVD_CHECK(evd_dsyevd_work_size(ctx, jobz, uplo, n, lda, &need));   // sets last_invalid_arg on bad jobz/uplo/n/lda
    if (need > (size_t)EVD_NOALLOC_SCRATCH_BYTES) {
        ctx->last_invalid_arg = 4;   // n too large for the static scratch
        return EVD_ERR_WORKSPACE;
    }
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    void *ptr = noalloc_ptr(ctx->device);
    if (!ptr) return EVD_ERR_HIP;
    // the host-CPU D&C option keeps its tridiagonal and eigenvectors in host
    // buffers it allocates: not used here
    const int64_t saved = ctx->dc_host;
    ctx->dc_host = 0;
    const evd_status_t st = evd_dsyevd(ctx, jobz, uplo, n, A, lda, W, ptr, (size_t)EVD_NOALLOC_SCRATCH_BYTES, info);
    ctx->dc_host = saved;
    return st;
}

}  // extern "C"
