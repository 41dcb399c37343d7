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
// Execution: one persistent launch; a workgroup of sixteen threads per window
// row owns sweeps c = g, g+P, g+2P, ... and stages each step's E and D windows
// in LDS.  All band loads of a step are issued together (one memory latency
// per step), row and column products are split over the sixteen adjacent
// lanes of a row and reduced with lane shuffles (the step's latency is on the
// critical path of the sweep pipeline, so the work is spread as widely as a
// workgroup allows), and the Householder vector is formed by one wavefront.
// Band entries are read and written with device-coherent (sc1) accesses;
// progress counters prog[c] (steps finished) are published after every
// wavefront's stores have drained and polled the same way, so no step needs a
// whole-cache writeback or invalidation.
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

// Sum over the RT adjacent lanes that share a window row (RT a power of two
// dividing 64); every lane of the group ends with the same bits.
template <int RT, typename T>
__device__ __forceinline__ T row_sum(T v)
{
#pragma unroll
    for (int off = RT / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// sixteen lanes, FP64: DPP within a row of 16 (lane ^ 1, lane ^ 2, half-row
// mirror, row mirror), each step pairing lanes symmetrically
template <int CTRL>
__device__ __forceinline__ double dpp_pair(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true),
                            __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true));
}
template <>
__device__ __forceinline__ double row_sum<16, double>(double v)
{
    v += dpp_pair<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_pair<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_pair<0x141>(v);  // row_half_mirror
    v += dpp_pair<0x140>(v);  // row_mirror
    return v;
}

// Sum over the 64 lanes of a wavefront, the same bits in every lane: DPP
// within rows of 16, then the four row sums read from lanes 0, 16, 32, 48.
__device__ __forceinline__ double bc_wave_sum(double v)
{
    v = row_sum<16, double>(v);
    const double r0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                       __builtin_amdgcn_readlane(__double2loint(v), 0));
    const double r1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16),
                                       __builtin_amdgcn_readlane(__double2loint(v), 16));
    const double r2 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                       __builtin_amdgcn_readlane(__double2loint(v), 32));
    const double r3 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 48),
                                       __builtin_amdgcn_readlane(__double2loint(v), 48));
    return (r0 + r1) + (r2 + r3);
}
__device__ __forceinline__ float bc_wave_sum(float v) { return wave_sum(v); }

// Householder vector of x[0:m) held one entry per lane (lanes >= m hold 0):
// returns v (v[0] = 1) in the lane's slot, tau and beta.
template <typename T>
__device__ __forceinline__ void bc_house(T x, int lane, int m, T *v, T *tau, T *beta)
{
    const T x0 = __shfl(x, 0, 64);
    const T tail = (lane >= 1 && lane < m) ? x * x : 0.0;
    const T sig = bc_wave_sum(tail);
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

// Threads per workgroup: sixteen per window row (at least one wavefront).
__host__ __device__ constexpr int bc_threads(int B) { return 16 * B < 64 ? 64 : 16 * B; }


template <int B, typename T>
__global__ __launch_bounds__(bc_threads(B)) void bc_kernel(int64_t n, T *AB, int64_t ldab, T *V, T *TAU,
                                                           int *prog, int store_v, const int *front, int *err,
                                                           uint64_t limit)
{
    constexpr int NT = bc_threads(B);
    constexpr int NW = NT / 64;
    constexpr int LDW = B + 1;
    constexpr int KL = (B * B + NT - 1) / NT;  // window elements per thread (coalesced column loads)
    __shared__ T Es[B * LDW];
    __shared__ T Ds[B * LDW];
    __shared__ T vs[B];   // current reflector
    __shared__ T vps[B];  // previous reflector of the sweep
    __shared__ T ws[B];
    __shared__ T red[NW];
    __shared__ T sh_tb[2];
    __shared__ int sh_ok;

    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    constexpr int RT = NT / B;          // threads per row in the row (column) phases
    const int p = t / RT, rho = t % RT;  // row (or column) p, part rho
    const bool own = p < B;
    for (int e = t; e < B * LDW; e += NT) {
        Es[e] = (T)0;
        Ds[e] = (T)0;
    }
    if (t < B) vps[t] = (T)0;
    __syncthreads();
    const int64_t P = gridDim.x;
    const int64_t nsweeps = n - 2;

    for (int64_t c = blockIdx.x; c < nsweeps; c += P) {
        const int64_t S = bc_steps(n, c, B);
        const int64_t Sprev = (c > 0) ? bc_steps(n, c - 1, B) : 0;
        T tprev = 0.0;
        for (int64_t s = 0; s < S; ++s) {
            const int64_t r = c + 1 + s * B;
            // wait (bounded) for sweep c-1 to finish step s+1 (or all of its
            // steps) and, with SBR running beside, for the band columns up to
            // r + B - 1 to be published; a wait that gives up raises *err and
            // the whole launch leaves
            if (c > 0 || front) {
                if (t == 0) {
                    bool ok = true;
                    if (front) ok = wait_ge(front, (int)((r + B) < n ? (r + B) : n), err, limit);
                    if (ok && c > 0) ok = wait_ge(&prog[c - 1], (int)((s + 2 < Sprev) ? s + 2 : Sprev), err, limit);
                    sh_ok = ok ? 1 : 0;
                }
                __syncthreads();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (!sh_ok) return;
            }
            const int64_t rp = r - B;
            const int m = (int)((n - r) < B ? (n - r) : B);

            // every window load of the step is issued before any is consumed:
            // element k*NT + t is (row, col) = (idx % B, idx / B), so a
            // wavefront reads whole band columns
            // (E and D share the 32-bit in-window offset (row - col) + col*ldab)
            T x = 0.0;
            T eb[KL], db[KL];
            T *const Eb = AB + rp * ldab + B;
            T *const Db = AB + r * ldab;
            const int ld = (int)ldab;
            if (s == 0 && wv == 0 && lane < m) x = ld_coh(&AB[(1 + lane) + c * ldab]);
#pragma unroll
            for (int k = 0; k < KL; ++k) {
                const int idx = k * NT + t, row = idx % B, col = idx / B;
                const int o = (row - col) + col * ld;
                eb[k] = (s > 0 && col < B && row < m) ? ld_coh(Eb + o) : (T)0;
                db[k] = (col < m && row < m && row >= col) ? ld_coh(Db + o) : (T)0;
            }
#pragma unroll
            for (int k = 0; k < KL; ++k) {
                const int idx = k * NT + t, row = idx % B, col = idx / B;
                if (col < B) {
                    if (s > 0) Es[row * LDW + col] = eb[k];
                    if (row >= col) {
                        Ds[row * LDW + col] = db[k];
                        Ds[col * LDW + row] = db[k];
                    }
                }
            }
            __syncthreads();

            if (s > 0) {
                // E receives H_{s-1} from the right: row p, columns q = rho (mod RT)
                if (tprev != 0.0) {
                    T y = 0.0;
                    if (own)
                        for (int q = rho; q < B; q += RT) y += Es[p * LDW + q] * vps[q];
                    y = row_sum<RT>(y) * tprev;
                    if (own)
                        for (int q = rho; q < B; q += RT) Es[p * LDW + q] -= y * vps[q];
                    __syncthreads();
                }
                if (wv == 0) x = (lane < m) ? Es[lane * LDW + 0] : (T)0;
            }
            // H_s from x (wavefront 0)
            if (wv == 0) {
                T v, tau, beta;
                bc_house(x, lane, m, &v, &tau, &beta);
                if (lane < B) vs[lane] = v;
                if (lane == 0) {
                    sh_tb[0] = tau;
                    sh_tb[1] = beta;
                }
                if (s == 0 && lane < m) st_coh(&AB[(1 + lane) + c * ldab], (lane == 0) ? beta : (T)0);
            }
            __syncthreads();
            const T tau = sh_tb[0], beta = sh_tb[1];

            if (s > 0) {
                // H_s from the left on E's columns 1..B-1: column p, rows i = rho (mod RT)
                if (tau != 0.0) {
                    T w = 0.0;
                    if (own && p >= 1)
                        for (int i = rho; i < B; i += RT) w += vs[i] * Es[i * LDW + p];
                    w = row_sum<RT>(w) * tau;
                    if (own && p >= 1)
                        for (int i = rho; i < B; i += RT) Es[i * LDW + p] -= vs[i] * w;
                    __syncthreads();
                }
#pragma unroll
                for (int k = 0; k < KL; ++k) {
                    const int idx = k * NT + t, row = idx % B, col = idx / B;
                    if (col < B && row < m) {
                        const T val = (col == 0) ? ((row == 0) ? beta : (T)0) : Es[row * LDW + col];
                        st_coh(Eb + ((row - col) + col * ld), val);
                    }
                }
            }
            // D_s two-sided: D <- H D H with u = tau D v, w = u - (tau/2)(u.v) v
            if (tau != 0.0) {
                T u = 0.0;
                if (own)
                    for (int q = rho; q < B; q += RT) u += Ds[p * LDW + q] * vs[q];
                u = row_sum<RT>(u) * tau;
                if (own && rho == 0) ws[p] = (p < m) ? u : (T)0;  // u (rows past m: zero)
                // (tau/2) u.v: the rows of a wavefront combined by lane
                // shuffles, the wavefronts' parts added by every thread in the
                // same order; w = u - al v is then formed where it is used
                T aw = (own && p < m) ? u * vs[p] : (T)0;
#pragma unroll
                for (int off = RT; off < 64; off <<= 1) aw += __shfl_xor(aw, off, 64);
                if (lane == 0) red[wv] = aw;
                __syncthreads();
                T al = 0.0;
#pragma unroll
                for (int k = 0; k < NW; ++k) al += red[k];
                al *= (T)0.5 * tau;
#pragma unroll
                for (int k = 0; k < KL; ++k) {
                    const int idx = k * NT + t, row = idx % B, col = idx / B;
                    if (col < m && row < m && row >= col) {
                        const T wr = ws[row] - al * vs[row], wc = ws[col] - al * vs[col];
                        const T d = Ds[row * LDW + col] - vs[row] * wc - wr * vs[col];
                        st_coh(Db + ((row - col) + col * ld), d);
                    }
                }
            }
            if (t < B) {
                if (store_v) V[((int64_t)s * n + c) * B + t] = vs[t];
                vps[t] = vs[t];
            }
            if (store_v && t == 0) TAU[(int64_t)s * n + c] = tau;
            tprev = tau;
            // publish: every wavefront's (coherent) stores complete before the
            // counter moves
            mem_drain();
            __syncthreads();
            if (t == 0) st_coh(&prog[c], (int)(s + 1));
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

// bs == nullptr: cooperative launch on the context's stream; otherwise a
// plain launch on bs of "bc_waves" workgroups (default: half the compute
// units, leaving the rest to SBR running beside)
template <int B, typename T>
evd_status_t bc_launch(evd_ctx_t ctx, int64_t n, T *AB, int64_t ldab, T *V, T *TAU, int *prog,
                       int store_v, const int *front, int *err, hipStream_t bs)
{
    int per_cu = 0;
    constexpr int NT = bc_threads(B);
    EVD_CHECK(evd_hip(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bc_kernel<B, T>, NT, 0)));
    if (per_cu < 1) per_cu = 1;
    int64_t P = (int64_t)per_cu * ctx->num_cus;
    if (bs && P > ctx->num_cus / 2) P = ctx->num_cus / 2;
    if (ctx->bc_waves > 0 && ctx->bc_waves < P) P = ctx->bc_waves;
    const int64_t nsweeps = n - 2;
    if (P > nsweeps) P = nsweeps;
    if (P < 1) P = 1;
    uint64_t limit = evd_spin_ticks(ctx);
    void *args[] = {(void *)&n, &AB, (void *)&ldab, &V, &TAU, &prog, &store_v, (void *)&front, &err, &limit};
    hipError_t e = bs             ? hipLaunchKernel((const void *)bc_kernel<B, T>, dim3((unsigned)P), dim3(NT), args, 0, bs)
                   : ctx->plain_bc ? hipLaunchKernel((const void *)bc_kernel<B, T>, dim3((unsigned)P), dim3(NT), args, 0,
                                                     ctx->stream)
                                   : hipLaunchCooperativeKernel((const void *)bc_kernel<B, T>, dim3((unsigned)P), dim3(NT),
                                                                args, 0, ctx->stream);
    return evd_hip(ctx, e);
}

}  // namespace

// prog: n ints of scratch
namespace {
template <typename T>
evd_status_t bc_extract_t(evd_ctx_t ctx, int64_t n, const T *AB, int64_t ldab, double *d, double *e)
{
    hipLaunchKernelGGL(bc_extract_kernel<T>, dim3((unsigned)(evd_ceil_div(n, 256) < 1024 ? evd_ceil_div(n, 256) : 1024)),
                       dim3(256), 0, ctx->stream, n, AB, ldab, d, e);
    return evd_check_last();
}

// scratch reset on the context's stream, then the persistent kernel (on bs,
// or cooperatively on the context's stream when bs is null)
template <typename T>
evd_status_t bc_start_t(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, T *AB, int64_t ldab, T *V, T *TAU, int *prog,
                        int *err, const int *front, hipStream_t bs)
{
    hipStream_t s = ctx->stream;
    const int store_v = (jobz == 'V' || jobz == 'v') ? 1 : 0;
    if (n <= 2) return EVD_OK;
    hipLaunchKernelGGL(bc_fill_int, dim3((unsigned)(evd_ceil_div(n, 256) < 1024 ? evd_ceil_div(n, 256) : 1024)),
                       dim3(256), 0, s, prog, n, 0);
    if (store_v) {
        const int64_t steps = bc_num_steps(n, b);
        const int64_t nv = steps * n * b, nt = steps * n;
        hipLaunchKernelGGL(bc_zero_v_kernel<T>, dim3(4096), dim3(256), 0, s, V, TAU, nv, nt);
    }
    if (bs) {
        EVD_CHECK(evd_hip(ctx, hipEventRecord(ctx->ev[10], s)));
        EVD_CHECK(evd_hip(ctx, hipStreamWaitEvent(bs, ctx->ev[10], 0)));
    }
    switch (b) {
    case 1: return bc_launch<1, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    case 2: return bc_launch<2, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    case 4: return bc_launch<4, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    case 8: return bc_launch<8, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    case 16: return bc_launch<16, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    case 32: return bc_launch<32, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    case 64: return bc_launch<64, T>(ctx, n, AB, ldab, V, TAU, prog, store_v, front, err, bs);
    default: return EVD_ERR_INVALID_ARG;
    }
}

}  // namespace

evd_status_t bc_run(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab, double *d, double *e,
                    double *V, double *TAU, int *prog, int *err, const int *front)
{
    EVD_CHECK(bc_start_t<double>(ctx, jobz, n, b, AB, ldab, V, TAU, prog, err, front, nullptr));
    return bc_extract_t<double>(ctx, n, AB, ldab, d, e);
}

evd_status_t bc_run_f32(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, float *AB, int64_t ldab, double *d,
                        double *e, float *V, float *TAU, int *prog, int *err, const int *front)
{
    EVD_CHECK(bc_start_t<float>(ctx, jobz, n, b, AB, ldab, V, TAU, prog, err, front, nullptr));
    return bc_extract_t<float>(ctx, n, AB, ldab, d, e);
}

evd_status_t bc_launch_beside(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab, double *V,
                              double *TAU, int *prog, int *err, const int *front, hipStream_t bs)
{
    return bc_start_t<double>(ctx, jobz, n, b, AB, ldab, V, TAU, prog, err, front, bs);
}

evd_status_t bc_finish(evd_ctx_t ctx, int64_t n, const double *AB, int64_t ldab, double *d, double *e)
{
    return bc_extract_t<double>(ctx, n, AB, ldab, d, e);
}

extern "C" {

int64_t evd_bc_num_steps(int64_t n, int64_t b) { return bc_num_steps(n, b); }

evd_status_t evd_dsb2st_work_size(evd_ctx_t ctx, int64_t n, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    *bytes = evd_align256((size_t)(n > 0 ? n : 1) * sizeof(int)) + 256;  // progress counters + the timeout word
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
    else if (work_bytes < evd_align256((size_t)(n > 0 ? n : 1) * sizeof(int)) + 256) bad = 12;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 12 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    int *err = (int *)((char *)work + evd_align256((size_t)n * sizeof(int)));
    hipLaunchKernelGGL(bc_fill_int, dim3(1), dim3(64), 0, ctx->stream, err, (int64_t)1, 0);
    return bc_run(ctx, jobz, n, b, AB, ldab, d, e, V, TAU, (int *)work, err, nullptr);
}

}  // extern "C"
