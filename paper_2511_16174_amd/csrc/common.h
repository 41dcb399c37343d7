// Shared definitions for the gfx950 eigensolver library (device + host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/evd.h"

#define EVD_WAVE 64

typedef double double4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- host errors
#define EVD_HIP_CHECK(expr)                                             \
    do {                                                                \
        hipError_t _e = (expr);                                         \
        if (_e != hipSuccess) return EVD_ERR_HIP;                       \
    } while (0)

#define EVD_CHECK(expr)                                                 \
    do {                                                                \
        evd_status_t _s = (expr);                                       \
        if (_s != EVD_OK) return _s;                                    \
    } while (0)

static inline int64_t evd_ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline size_t evd_align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum for blockDim.x a multiple of 64 (<= 1024).  `red` must hold
// blockDim.x/64 doubles of LDS.  All threads get the result.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// Agent-scope acquire / release on 32/64-bit flags in device memory.
__device__ __forceinline__ int flag_load_acquire(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_store_release(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int flag_add_acq_rel(int *p, int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- context
struct evd_ctx_s {
    int device;
    hipStream_t stream;       // borrowed
    int last_invalid_arg;
    // tunables
    int64_t b;                // band width (0 = auto)
    int64_t bc_waves;         // persistent BC waves (0 = auto)
    int64_t bcback_group;     // sweeps per BC-back group (0 = auto)
    int64_t order;            // 0 = reordered stages (paper), 1 = conventional
    int64_t timing;           // 1 = record per-stage times
    int num_cus;
    int max_coop_blocks_panel;
    hipEvent_t ev[16];
    float stage_ms[8];
};

// ---------------------------------------------------------------- internal API
// GEMM (gemm_f64.hip)
enum { OP_N = 0, OP_T = 1, OP_S = 2 };
evd_status_t gemm_f64(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k,
                      double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                      double beta, double *C, int64_t ldc, double *splitk_ws, size_t splitk_ws_elems);
size_t gemm_splitk_ws_elems(int64_t m, int64_t n, int64_t k);
// Grouped C = A * B (no transposes) with per-problem sizes read on the device.
struct GemmProblem {
    const double *A;
    const double *B;
    double *C;
    int64_t lda, ldb, ldc;
    int64_t m, n, k;
};
evd_status_t gemm_f64_grouped(hipStream_t s, const GemmProblem *probs, int nprob, int64_t max_m, int64_t max_n);
// Steps of bulge-chasing sweep 0 (the longest): s >= 0 with 1 + s b <= n - 1.
extern "C" int64_t evd_sbr_num_panels(int64_t n, int64_t b);
__host__ __device__ inline int64_t bc_num_steps(int64_t n, int64_t b) { return (b <= 0 || n < 3) ? 0 : (n - 2) / b + 1; }
