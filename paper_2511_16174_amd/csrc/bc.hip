// Stage 2: bulge chasing (BC), band -> tridiagonal (paper Section 2.1.1; the
// per-sweep / per-step structure the distributed BC of Section 4.2 relies on).
//
// The band B (half-bandwidth b) is kept in lower band storage with room for
// one bulge: AB[(i - j) + j*ldab] = B(i, j) for 0 <= i - j <= 2b.
//
// Sweep c (0 <= c < n-2):
//   step 0:  reflector H_0 from B(c+1 : c+b, c) zeroes that column below its
//            sub-diagonal; H_0 is applied two-sided to the diagonal block
//            D_0 = B(c+1 : c+b, c+1 : c+b).
//   step s:  r = c + 1 + s b.  E = B(r : r+b-1, r-b : r-1) receives H_{s-1}
//            from the right (this creates the bulge), H_s is generated from
//            E's first column and applied from the left to E's other columns,
//            then two-sided to D_s = B(r : r+b-1, r : r+b-1).
// Every access of step (c, s) lies in rows r .. r+b-1 of the stored lower
// triangle, so two steps conflict exactly when their row ranges overlap:
// (c, s) conflicts with (c-1, s) and (c-1, s+1) and, transitively through
// them, with every earlier sweep.  Step (c, s) may therefore run as soon as
// sweep c-1 has finished step s+1 (or all of its steps).
//
// Execution: one persistent launch; a one-wavefront workgroup owns sweeps
// c = g, g+P, g+2P, ... and keeps its E and D windows in LDS (lane p = row p
// of the window).  Band entries are read and written with device-coherent
// (sc1) accesses; progress counters prog[c] (steps finished) are published
// after the wavefront's stores have drained and polled the same way, so no
// step needs a whole-cache writeback or invalidation.
#include "common.h"

namespace {

__global__ void bc_fill_int(int *p, int64_t count, int v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ int64_t bc_steps(int64_t n, int64_t c, int b)
{
    // number of s >= 0 with c + 1 + s b <= n - 1
    const int64_t rem = n - 1 - (c + 1);
    return rem < 0 ? 0 : rem / b + 1;
}

// Householder vector of x[0:m) held one entry per lane (lanes >= m hold 0):
// returns v (v[0] = 1) in the lane's slot, tau and beta.
template <typename T>
__device__ __forceinline__ void bc_house(T x, int lane, int m, T *v, T *tau, T *beta)
{
    const T x0 = __shfl(x, 0, 64);
    const T tail = (lane >= 1 && lane < m) ? x * x : 0.0;
    const T sig = wave_sum(tail);
    if (sig == 0.0 || m <= 1) {
        *tau = 0.0;
        *beta = x0;
        *v = (lane == 0) ? 1.0 : 0.0;
        return;
    }
    const T nrm = sqrt(x0 * x0 + sig);
    const T bt = (x0 >= 0.0) ? -nrm : nrm;
    *tau = (bt - x0) / bt;
    *beta = bt;
    const T scale = 1.0 / (x0 - bt);
    *v = (lane == 0) ? 1.0 : ((lane < m) ? x * scale : 0.0);
}

template <int B, typename T>
__global__ __launch_bounds__(64) void bc_kernel(int64_t n, T *AB, int64_t ldab, T *V, T *TAU,
                                                int *prog, int store_v)
{
    constexpr int LDW = B + 1;
    __shared__ T Es[B * LDW];
    __shared__ T Ds[B * LDW];
    __shared__ T vs[B];
    __shared__ T ws[B];

    const int lane = threadIdx.x;
    const bool act = lane < B;  // lanes that own a window row
    for (int e = lane; e < B * LDW; e += 64) {
        Es[e] = (T)0;
        Ds[e] = (T)0;
    }
    __syncthreads();
    const int64_t P = gridDim.x;
    const int64_t nsweeps = n - 2;

    for (int64_t c = blockIdx.x; c < nsweeps; c += P) {
        const int64_t S = bc_steps(n, c, B);
        const int64_t Sprev = (c > 0) ? bc_steps(n, c - 1, B) : 0;
        T vprev = 0.0, tprev = 0.0;  // previous reflector of this sweep (lane entry)
        for (int64_t s = 0; s < S; ++s) {
            // wait for sweep c-1 to finish step s+1 (or all of its steps)
            if (c > 0) {
                // the acquire load invalidates this CU's caches for the data
                // sweep c-1 published before its release store
                const int need = (int)((s + 2 < Sprev) ? s + 2 : Sprev);
                if (lane == 0)
                    while (ld_coh(&prog[c - 1]) < need) __builtin_amdgcn_s_sleep(1);
                __syncthreads();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
            }
            const int64_t r = c + 1 + s * B;
            const int m = (int)((n - r) < B ? (n - r) : B);
            T v = 0.0, tau = 0.0, beta = 0.0;
            if (s == 0) {
                const T x = (lane < m) ? ld_coh(&AB[(1 + lane) + c * ldab]) : (T)0;
                bc_house(x, lane, m, &v, &tau, &beta);
                if (lane < m) st_coh(&AB[(1 + lane) + c * ldab], (lane == 0) ? beta : (T)0);
            } else {
                const int64_t rp = r - B;
                // E (m x B): rows r.., columns rp..; receives H_{s-1} from the right
                if (act) {
                    for (int q = 0; q < B; ++q)
                        Es[lane * LDW + q] = (lane < m) ? ld_coh(&AB[(B + lane - q) + (rp + q) * ldab]) : (T)0;
                    vs[lane] = vprev;
                }
                __syncthreads();
                if (tprev != 0.0 && lane < m) {
                    T y = 0.0;
                    for (int q = 0; q < B; ++q) y += Es[lane * LDW + q] * vs[q];
                    y *= tprev;
                    for (int q = 0; q < B; ++q) Es[lane * LDW + q] -= y * vs[q];
                }
                __syncthreads();
                // H_s from E's first column, applied from the left to columns 1..B-1
                const T x = (lane < m) ? Es[lane * LDW + 0] : 0.0;
                bc_house(x, lane, m, &v, &tau, &beta);
                if (act) vs[lane] = v;
                __syncthreads();
                if (tau != 0.0 && lane >= 1 && lane < B) {
                    // rows >= m of E and entries >= m of v are zero
                    const int q = lane;
                    T w = 0.0;
#pragma unroll 16
                    for (int p = 0; p < B; ++p) w += vs[p] * Es[p * LDW + q];
                    w *= tau;
#pragma unroll 16
                    for (int p = 0; p < B; ++p) Es[p * LDW + q] -= vs[p] * w;
                }
                __syncthreads();
                if (lane < m) {
                    Es[lane * LDW + 0] = (lane == 0) ? beta : 0.0;
                    for (int q = 0; q < B; ++q) st_coh(&AB[(B + lane - q) + (rp + q) * ldab], Es[lane * LDW + q]);
                }
            }
            // D_s two-sided: D <- H D H
            if (tau != 0.0) {
                if (act) vs[lane] = v;
                // load the lower triangle column by column (coalesced, all loads
                // in flight), then mirror into the full block
                T dcol[B];
#pragma unroll
                for (int q = 0; q < B; ++q)
                    dcol[q] = (q < m && lane < m && lane >= q) ? ld_coh(&AB[(lane - q) + (r + q) * ldab]) : (T)0;
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    if (q < m && lane < m && lane >= q) {
                        Ds[lane * LDW + q] = dcol[q];
                        Ds[q * LDW + lane] = dcol[q];
                    }
                }
                __syncthreads();
                T u = 0.0;
                if (lane < m) {
                    // entries of v beyond m are zero; stale finite D entries meet them
#pragma unroll 16
                    for (int q = 0; q < B; ++q) u += Ds[lane * LDW + q] * vs[q];
                    u *= tau;
                }
                const T alpha = 0.5 * tau * wave_sum(lane < m ? u * v : (T)0);
                const T w = u - alpha * v;
                if (act) ws[lane] = w;
                __syncthreads();
                if (lane < m) {
#pragma unroll
                    for (int q = 0; q < B; ++q) {
                        if (q <= lane) {
                            const T d = Ds[lane * LDW + q] - v * ws[q] - w * vs[q];
                            st_coh(&AB[(lane - q) + (r + q) * ldab], d);
                        }
                    }
                }
            }
            if (store_v) {
                if (act) V[((int64_t)s * n + c) * B + lane] = (lane < m) ? v : 0.0;
                if (lane == 0) TAU[(int64_t)s * n + c] = tau;
            }
            vprev = v;
            tprev = tau;
            // publish: this wavefront's (coherent) stores complete before the
            // counter (one wavefront per workgroup)
            mem_drain();
            __syncthreads();
            if (lane == 0) st_coh(&prog[c], (int)(s + 1));
        }
    }
}

template <typename T>
__global__ void bc_extract_kernel(int64_t n, const T *AB, int64_t ldab, double *d, double *e)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        d[j] = AB[j * ldab];
        if (j + 1 < n) e[j] = AB[1 + j * ldab];
    }
}

template <typename T>
__global__ void bc_zero_v_kernel(T *V, T *TAU, int64_t nv, int64_t nt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        V[i] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x)
        TAU[i] = 0.0;
}

template <int B, typename T>
evd_status_t bc_launch(evd_ctx_t ctx, int64_t n, T *AB, int64_t ldab, T *V, T *TAU, int *prog,
                       int store_v)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bc_kernel<B, T>, 64, 0) != hipSuccess) return EVD_ERR_HIP;
    if (per_cu < 1) per_cu = 1;
    int64_t P = (int64_t)per_cu * ctx->num_cus;
    if (ctx->bc_waves > 0 && ctx->bc_waves < P) P = ctx->bc_waves;
    const int64_t nsweeps = n - 2;
    if (P > nsweeps) P = nsweeps;
    if (P < 1) P = 1;
    void *args[] = {(void *)&n, &AB, (void *)&ldab, &V, &TAU, &prog, &store_v};
    hipError_t e = hipLaunchCooperativeKernel((const void *)bc_kernel<B, T>, dim3((unsigned)P), dim3(64), args, 0,
                                              ctx->stream);
    return e == hipSuccess ? EVD_OK : EVD_ERR_HIP;
}

}  // namespace

// prog: n ints of scratch
namespace {
template <typename T>
evd_status_t bc_run_t(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, T *AB, int64_t ldab, double *d, double *e, T *V,
                      T *TAU, int *prog)
{
    hipStream_t s = ctx->stream;
    const int store_v = (jobz == 'V' || jobz == 'v') ? 1 : 0;
    if (n > 2) {
        hipLaunchKernelGGL(bc_fill_int, dim3((unsigned)(evd_ceil_div(n, 256) < 1024 ? evd_ceil_div(n, 256) : 1024)),
                           dim3(256), 0, s, prog, n, 0);
        if (store_v) {
            const int64_t steps = bc_num_steps(n, b);
            const int64_t nv = steps * n * b, nt = steps * n;
            hipLaunchKernelGGL(bc_zero_v_kernel<T>, dim3(4096), dim3(256), 0, s, V, TAU, nv, nt);
        }
        evd_status_t st;
        switch (b) {
        case 1: st = bc_launch<1, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        case 2: st = bc_launch<2, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        case 4: st = bc_launch<4, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        case 8: st = bc_launch<8, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        case 16: st = bc_launch<16, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        case 32: st = bc_launch<32, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        case 64: st = bc_launch<64, T>(ctx, n, AB, ldab, V, TAU, prog, store_v); break;
        default: return EVD_ERR_INVALID_ARG;
        }
        if (st != EVD_OK) return st;
    }
    hipLaunchKernelGGL(bc_extract_kernel<T>, dim3((unsigned)(evd_ceil_div(n, 256) < 1024 ? evd_ceil_div(n, 256) : 1024)),
                       dim3(256), 0, s, n, (const T *)AB, ldab, d, e);
    return hipGetLastError() == hipSuccess ? EVD_OK : EVD_ERR_HIP;
}

}  // namespace

evd_status_t bc_run(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab, double *d, double *e,
                    double *V, double *TAU, int *prog)
{
    return bc_run_t<double>(ctx, jobz, n, b, AB, ldab, d, e, V, TAU, prog);
}

evd_status_t bc_run_f32(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, float *AB, int64_t ldab, double *d, double *e,
                        float *V, float *TAU, int *prog)
{
    return bc_run_t<float>(ctx, jobz, n, b, AB, ldab, d, e, V, TAU, prog);
}

extern "C" {

int64_t evd_bc_num_steps(int64_t n, int64_t b) { return bc_num_steps(n, b); }

evd_status_t evd_dsb2st_work_size(evd_ctx_t ctx, int64_t n, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    *bytes = evd_align256((size_t)(n > 0 ? n : 1) * sizeof(int));
    return EVD_OK;
}

evd_status_t evd_dsb2st(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab, double *d,
                        double *e, double *V, double *TAU, void *work, size_t work_bytes)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    const bool vec = (jobz == 'V' || jobz == 'v');
    int bad = 0;
    if (!(vec || jobz == 'N' || jobz == 'n')) bad = 2;
    else if (n < 0) bad = 3;
    else if (b < 1 || b > 64 || (64 % b) != 0) bad = 4;
    else if (n > 0 && !AB) bad = 5;
    else if (ldab < 2 * b + 1) bad = 6;
    else if (n > 0 && !d) bad = 7;
    else if (n > 1 && !e) bad = 8;
    else if (vec && n > 2 && !V) bad = 9;
    else if (vec && n > 2 && !TAU) bad = 10;
    else if (n > 0 && !work) bad = 11;
    else if (work_bytes < (size_t)n * sizeof(int)) bad = 12;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 12 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    if (hipSetDevice(ctx->device) != hipSuccess) return EVD_ERR_HIP;
    return bc_run(ctx, jobz, n, b, AB, ldab, d, e, V, TAU, (int *)work);
}

}  // extern "C"
