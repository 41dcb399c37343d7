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

__device__ __forceinline__ float wave_sum(float v)
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
// blockDim.x/64 values of LDS.  All threads get the result.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// Sum over the 4 lanes of each aligned quad (lanes 4q .. 4q+3) with DPP
// quad permutations (no LDS round trip).
__device__ __forceinline__ double quad_sum(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    double w = __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, true),
                                __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, true));  // lane ^ 1
    v += w;
    lo = __double2loint(v);
    hi = __double2hiint(v);
    w = __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, true),
                         __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, true));  // lane ^ 2
    return v + w;
}
__device__ __forceinline__ float quad_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
    return v;
}

// Device-coherent accesses for data shared between workgroups of one launch:
// relaxed agent-scope atomics are emitted as sc1 loads/stores, which are
// coherent across the chip's L2 caches without the whole-cache writeback and
// invalidation that agent-scope release/acquire fences perform.  A producer
// drains its own outstanding memory operations (mem_drain) before publishing
// a flag with st_coh; a consumer issues its data loads only after it has
// observed the flag with ld_coh.
template <typename T>
__device__ __forceinline__ T ld_coh(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void mem_drain()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Grid-wide barrier for a co-resident (cooperative) launch of G workgroups:
// bar[0] = arrival count (returns to 0), bar[1] = generation.  Data exchanged
// across the barrier must be accessed with ld_coh / st_coh.
__device__ __forceinline__ void grid_barrier_coh(int *bar, int G)
{
    mem_drain();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int g = ld_coh(&bar[1]);
        mem_drain();
        const int a = __hip_atomic_fetch_add(&bar[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == G - 1) {
            st_coh(&bar[0], 0);
            mem_drain();
            st_coh(&bar[1], g + 1);
        } else {
            while (ld_coh(&bar[1]) == g) __builtin_amdgcn_s_sleep(1);
        }
        mem_drain();
    }
    __syncthreads();
}

// Bounded wait (one thread) until the device-coherent counter *p reaches
// `need`: false if *err is raised meanwhile or `limit` ticks of the 100 MHz
// wall clock pass (the waiter then raises *err itself, so every other waiter
// of the launch gives up at its next poll instead of waiting its full limit).
__device__ __forceinline__ bool wait_ge(const int *p, int need, int *err, uint64_t limit)
{
    if (ld_coh(p) >= need) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (ld_coh(p) >= need) return true;
        if (ld_coh(err) != 0) return false;
        if (wall_clock64() - t0 > limit) {
            st_coh(err, 1);
            return false;
        }
    }
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
    int64_t bcback_group;     // sweeps per blocked BC-back group (0 = auto: 64 for b = 64, else 32)
    int64_t bcback_rows;      // rows per workgroup of the 64-sweep BC-back kernel (0 = auto, 64, 128)
    int64_t order;            // 0 = reordered stages (paper), 1 = conventional
    int64_t timing;           // 1 = record per-stage times
    int num_cus;
    int max_coop_blocks_panel;
    hipEvent_t ev[16];
    float stage_ms[8];
    // autotuned band width per size bucket (bucket = floor(log2 n)), 0 = none
    int64_t tuned_b[64];
    int64_t tuned_nb[64];     // autotuned SBR outer block per size bucket (0 = none)
    int64_t tuned_sub[64];    // autotuned BC-back block reflector per size bucket (0 = none)
    int64_t last_tuned_nb;    // choices of the last evd_autotune call (read only)
    int64_t last_tuned_sub;
    int64_t panel_wgs;        // panel-QR rows spread over about this many workgroups (0 = fewest)
    int64_t panel_generic;    // 1: b = 64 panels in the generic layout (0 = column layout)
    int64_t sbr_nb;           // SBR outer block in columns (0 = 320; <= b: single blocking)
    int64_t orgsb_nb;         // SBR-back reflector group in columns (0 = 512)
    int64_t bcback_valu;      // 1 = reflector-by-reflector BC-back on the vector ALUs (0 = blocked MFMA)
    int64_t bcback_sub;       // sweeps per block reflector inside a 64-sweep group (0 = 32, 16, 32, 64)
    int64_t bcback_rt;        // 16-row tiles per wavefront of the 64-sweep BC-back (0 = 1, 1, 2)
    int64_t bcback_lds2;      // 1: 64-row BC-back workgroups double-buffered, one per CU (0 = single buffer, two per CU)
    int64_t gemm_staged;      // 1: FP64 GEMM main loop staged through registers everywhere (process-wide; 0 = direct-to-LDS loads for whole tiles)
    int64_t batch_streams;    // streams used by the batched driver (0 = 4)
    int64_t batch_graph;      // 1 = capture the batched launch sequence in a hipGraph
    int64_t last_graph_used;  // 1 if the last batched call ran from a graph
    int64_t last_hip_error;   // first HIP error code seen by a call (0 = none; cleared by evd_set_param)
    int64_t capture_error;    // HIP error that made the last graph capture fall back (0 = none)
    // batched driver state
    hipStream_t bstreams[16];
    hipStream_t cstream;      // origin stream of the batched graph capture
    hipEvent_t bev[17];
    int nbstreams;
    hipGraphExec_t gexec;
    uint64_t gkey;
    int in_batch;             // 1 while the batched driver enqueues its matrices
    hipStream_t astream;      // auxiliary stream: BC-back T factors formed beside D&C
    int64_t dc_max_iter;      // iterations per secular root (0 = 200; lower values force non-convergence)
    int64_t bc_overlap;       // 1 = bulge chasing beside SBR, gated by the published band columns
    int64_t spin_limit_ms;    // longest inter-workgroup wait before EVD_ERR_TIMEOUT (0 = 30000)
    int64_t debug_gate;       // 1 = bulge chasing waits on a band frontier that is never published
    int plain_panels;         // internal: panel QR without a cooperative launch (while BC runs beside SBR)
    int plain_bc;             // internal: bulge chasing without a cooperative launch (batched streams)
    int64_t batch_plain;      // 1 = the batched driver's persistent kernels use plain launches (see batched.hip)
    int64_t dc_host;          // 1 = D&C on the host CPU beside the GPU back transformation (vectors)
    int64_t dc_host_threads;  // host threads of that D&C (0 = OMP_NUM_THREADS, else all)
    int32_t host_status;      // internal: status of the last host D&C (source of an async copy)
};

// Wall-clock ticks (100 MHz) a workgroup may wait for another one.
inline uint64_t evd_spin_ticks(const evd_ctx_s *ctx)
{
    const int64_t ms = ctx->spin_limit_ms > 0 ? ctx->spin_limit_ms : 30000;
    return (uint64_t)ms * 100000ull;
}

// First failing HIP status seen on this host thread (internal helpers without
// a context record here; the context reports it through "last_hip_error").
inline thread_local int64_t evd_tls_hip_error = 0;

inline evd_status_t evd_hip_status(hipError_t e)
{
    if (e == hipSuccess) return EVD_OK;
    if (!evd_tls_hip_error) evd_tls_hip_error = (int64_t)e;
    return EVD_ERR_HIP;
}

// Launch errors of the kernels enqueued so far (consumes hipGetLastError).
inline evd_status_t evd_check_last() { return evd_hip_status(hipGetLastError()); }

// Record the first failing HIP status of a call in the context.
inline evd_status_t evd_hip(evd_ctx_s *ctx, hipError_t e)
{
    if (e == hipSuccess) return EVD_OK;
    if (!ctx->last_hip_error) ctx->last_hip_error = (int64_t)e;
    return evd_hip_status(e);
}

// Band width used by the drivers: explicit parameter, else the autotuned
// value for n's size bucket, else the default (32 up to n = 4096, then 64),
// halved until it is narrower than the matrix.
inline int64_t evd_choose_b(const evd_ctx_s *ctx, int64_t n)
{
    int64_t b = ctx->b;
    if (b <= 0 && n > 1) {
        int bucket = 0;
        while (bucket < 63 && ((int64_t)1 << (bucket + 1)) <= n) ++bucket;
        b = ctx->tuned_b[bucket];
    }
    if (b <= 0) b = (n <= 4096) ? 32 : 64;
    while (b > 1 && b >= n) b >>= 1;
    if (b < 1) b = 1;
    return b;
}

inline int evd_size_bucket(int64_t n)
{
    int bucket = 0;
    while (bucket < 63 && ((int64_t)1 << (bucket + 1)) <= n) ++bucket;
    return bucket;
}
// SBR outer block in columns: the parameter, else the autotuned value, else 0
// (the driver's default)
inline int64_t evd_choose_nb(const evd_ctx_s *ctx, int64_t n)
{
    if (ctx->sbr_nb > 0) return ctx->sbr_nb;
    return n > 1 ? ctx->tuned_nb[evd_size_bucket(n)] : 0;
}
// sweeps per BC-back block reflector inside a 64-sweep group
inline int evd_choose_sub(const evd_ctx_s *ctx, int64_t n)
{
    if (ctx->bcback_sub > 0) return (int)ctx->bcback_sub;
    const int64_t t = n > 1 ? ctx->tuned_sub[evd_size_bucket(n)] : 0;
    return t > 0 ? (int)t : 32;
}

// ---------------------------------------------------------------- internal API
// SBR (sbr.hip).  err: device word raised when a wait between workgroups
// gives up.  ov (optional): bulge chasing runs beside SBR -- SBR publishes
// in *ov->front the number of leading band columns it has finished (panel by
// panel, then n) and calls ov->launch(ov->arg) once the band storage is
// initialised, before the first panel.
struct SbrOverlap {
    int *front;
    evd_status_t (*launch)(void *arg);
    void *arg;
};
evd_status_t sbr_run(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, double *A, int64_t lda, double *AB,
                     int64_t ldab, double *T, void *work, int *err, const SbrOverlap *ov);
evd_status_t sbr_run_f32(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, float *A, int64_t lda, float *AB,
                         int64_t ldab, float *T, void *work, int *err, const SbrOverlap *ov);
size_t sbr_work_bytes(int64_t n, int64_t b);
size_t sbr_work_bytes_f32(int64_t n, int64_t b);
// Bulge chasing (bc.hip).  front (optional): every step first waits until
// *front covers the band columns it touches.  bc_run: the whole stage on the
// context's stream (cooperative launch), then d, e.  bc_launch_beside: the
// scratch is reset on the context's stream, then the persistent kernel is
// launched (plain launch, "bc_waves" workgroups) on stream bs after it;
// bc_finish extracts d, e once the caller has joined bs.
evd_status_t bc_run(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab, double *d, double *e,
                    double *V, double *TAU, int *prog, int *err, const int *front);
evd_status_t bc_run_f32(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, float *AB, int64_t ldab, double *d,
                        double *e, float *V, float *TAU, int *prog, int *err, const int *front);
evd_status_t bc_launch_beside(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab, double *V,
                              double *TAU, int *prog, int *err, const int *front, hipStream_t bs);
evd_status_t bc_finish(evd_ctx_t ctx, int64_t n, const double *AB, int64_t ldab, double *d, double *e);
// device address of the allocation-free entry point's scratch (noalloc.hip)
evd_status_t noalloc_init_device(int device);
// GEMM (gemm_f64.hip)
enum { OP_N = 0, OP_T = 1, OP_S = 2 };
evd_status_t gemm_f64(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k,
                      double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                      double beta, double *C, int64_t ldc, double *splitk_ws, size_t splitk_ws_elems);
size_t gemm_splitk_ws_elems(int64_t m, int64_t n, int64_t k);
// compute units the split-K planner fills (called when a context is created)
void gemm_set_cu_count(int cus);
void gemm_set_staged(int on);
// lower triangle of the m x m matrix A copied into its upper triangle (sbr.hip)
evd_status_t evd_mirror_lower_f64(hipStream_t s, int64_t m, double *A, int64_t lda);
// Row (within a 16 x 16 tile) held by lane group lq = lane/16, element r, of
// the FP32 accumulator of v_mfma_f32_16x16x32_bf16.
#define EVD_F32_MFMA_ROW(lq, r) (4 * (lq) + (r))
// FP32 split-BF16x3 GEMM (gemm_f32x3.hip)
evd_status_t gemm_f32x3(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k, float alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                        float *ws, size_t ws_elems);
size_t gemm_f32x3_ws_elems(int64_t m, int64_t n, int64_t k);
// Grouped C = A * B (no transposes) with per-problem sizes read on the device.
struct GemmProblem {
    const double *A;
    const double *B;
    double *C;
    int64_t lda, ldb, ldc;
    int64_t m, n, k;
};
evd_status_t gemm_f64_grouped(hipStream_t s, const GemmProblem *probs, int nprob, int64_t max_m, int64_t max_n);

// Blocked BC-back on the matrix cores (b in {16, 32, 64}): T factors of the
// reflector groups (bcback_mfma_t_elems doubles, 0 for other b), then
// Q <- Q H_1 ... H_m (rev false) or Q H_m ... H_1 (rev true).
size_t bcback_mfma_t_elems(int64_t n, int64_t b);
// the blocked kernels address 64 window columns (16 k-steps) through one
// buffer descriptor: 64 ldq doubles in a 31-bit byte range
inline bool bcback_mfma_fits(int64_t ldq) { return ldq > 0 && ldq < ((int64_t)1 << 22); }
evd_status_t bcback_mfma_prepare(evd_ctx_t ctx, int64_t n, int64_t b, const double *V, const double *TAU, double *Tg,
                                 bool rev);
evd_status_t bcback_mfma_apply(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, double *Q,
                               int64_t ldq, const double *Tg, bool rev);

// One K-slice of a GEMM operand tile is an LC x LS block in memory (LC
// contiguous elements, lines ld apart).  Thread tid loads elements
// e = tid + r*NT, (c, s) = (e % LC, e / LC) with buffer loads through a
// descriptor based at the (wave-uniform) slice origin: elements outside
// c < cmax, s < smax get an offset past the descriptor's range, which the
// hardware turns into a zero, so edge slices need no branches around the
// loads.  Requires ((LS - 1) ld + LC) sizeof(T) < 2^31 (checked by the host).
constexpr uint32_t EVD_BUF_DWORD3 = 0x00020000u;  // raw buffer, 32-bit data format (gfx9 family)
constexpr uint32_t EVD_BUF_OOB = 0x80000000u;     // offset beyond any range the loaders use
template <typename T, int LC, int LS, int NT>
struct TileSlice {
    static constexpr int E = LC * LS / NT;
    static_assert(E * NT == LC * LS, "slice/thread mismatch");
    static __device__ __forceinline__ int c(int tid, int r) { return (tid + r * NT) % LC; }
    static __device__ __forceinline__ int s(int tid, int r) { return (tid + r * NT) / LC; }
    // full: every element in bounds; else c < cmax and s < smax
    static __device__ __forceinline__ void load(T (&v)[E], const T *__restrict__ base, int ld, int tid,
                                                bool full, int64_t cmax, int64_t smax)
    {
        const uint32_t nrec = ((uint32_t)(LS - 1) * (uint32_t)ld + LC) * (uint32_t)sizeof(T);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)nrec,
                                                                           (int)EVD_BUF_DWORD3);
        const int cm = (int)(cmax < LC ? cmax : LC), sm = (int)(smax < LS ? smax : LS);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int cc = c(tid, r), ss = s(tid, r);
            uint32_t off = (uint32_t)(cc + ss * ld) * (uint32_t)sizeof(T);
            if (!full) off = (cc < cm && ss < sm) ? off : EVD_BUF_OOB;
            if constexpr (sizeof(T) == 8)
                v[r] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
            else
                v[r] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
        }
    }
};
// leading dimensions the slice loaders accept (byte offsets stay below 2^31)
inline bool evd_gemm_ld_ok(int64_t ld) { return ld > 0 && ld <= ((int64_t)1 << 21); }

// Type-dispatched GEMM: FP64 MFMA for double, split-BF16x3 for float.
inline evd_status_t gemm_t(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k, double alpha,
                           const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                           int64_t ldc, double *ws, size_t ws_elems)
{
    return gemm_f64(s, opa, opb, lower_c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_elems);
}
inline evd_status_t gemm_t(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k, float alpha,
                           const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                           float *ws, size_t ws_elems)
{
    return gemm_f32x3(s, opa, opb, lower_c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_elems);
}
template <typename T>
inline size_t gemm_ws_elems_t(int64_t m, int64_t n, int64_t k)
{
    return sizeof(T) == 8 ? gemm_splitk_ws_elems(m, n, k) : gemm_f32x3_ws_elems(m, n, k);
}
// Steps of bulge-chasing sweep 0 (the longest): s >= 0 with 1 + s b <= n - 1.
extern "C" int64_t evd_sbr_num_panels(int64_t n, int64_t b);
__host__ __device__ inline int64_t bc_num_steps(int64_t n, int64_t b) { return (b <= 0 || n < 3) ? 0 : (n - 2) / b + 1; }
