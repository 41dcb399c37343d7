// Stage 4: back transformation in the reordered stage order (paper
// Section 3.3): SBR-back forms Q_s by applying the panel reflectors to the
// identity, BC-back right-multiplies Q_s by the bulge-chasing reflectors
// (Section 4.3: a BLAS2 kernel that keeps Q in registers and reuses
// reflector groups from on-chip memory), and one GEMM forms Q = Q_sb Q_d.
//
// BC-back ordering.  Reflector (c, s) of sweep c, step s acts on columns
// r .. r+b-1, r = c+1+s b.  In generation order a reflector must precede a
// later-generated one only if their columns overlap, and an overlap between
// sweeps c < c' always has step(c') <= step(c).  Hence, with sweeps grouped in
// blocks of G consecutive sweeps, "blocks ascending; inside a block steps
// descending; inside a step sweeps ascending" is a valid order.  For a fixed
// block the G reflectors of step s live in a window of G+b-1 consecutive
// columns that slides left by b columns when s decreases, so each row keeps the
// window in registers and streams only b columns in and out per G reflectors.
//
// Register layout: a row of Q is spread over 4 lanes (lane = row + 16 rho);
// lane rho holds window columns 4k + rho, k = 0 .. NW-1.  Reflector jj of the
// group touches window columns jj .. jj+b-1, i.e. slots k = jj/4 .. jj/4 + b/4
// on every lane (out-of-range entries meet zero padding of v).  The four
// partial dot products of a row are combined with two cross-lane shuffles.
#include "common.h"

namespace {

constexpr int BCB_ROWS = 128;                 // rows of Q per workgroup
constexpr int BCB_THREADS = BCB_ROWS * 4;     // 4 lanes per row
constexpr int BCB_G = 64;                     // sweeps per block
constexpr int VPAD = 4;                       // zero padding on each side of v

template <int B>
__global__ __launch_bounds__(BCB_THREADS) void bcback_kernel(int64_t mrows, int64_t n, const double *__restrict__ V,
                                                             const double *__restrict__ TAU, double *__restrict__ Q,
                                                             int64_t ldq)
{
    constexpr int G = BCB_G;
    constexpr int NW = (G + B) / 4;       // slots per lane (window G+B-1 columns, one spare)
    constexpr int SH = B / 4;             // slots shifted per step
    constexpr int LDV = B + 2 * VPAD;
    __shared__ double vs[2][G][LDV];
    __shared__ double ts[2][G];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rho = lane >> 4;                            // residue of this lane
    const int64_t row = (int64_t)blockIdx.x * BCB_ROWS + wave * 16 + (lane & 15);
    const bool rowok = row < mrows;
    double *Qr = Q + row;

    const int64_t nsweeps = n - 2;
    const int64_t nsteps = bc_num_steps(n, B);

    // zero the padding once
    for (int e = tid; e < 2 * G * LDV; e += BCB_THREADS) (&vs[0][0][0])[e] = 0.0;
    __syncthreads();

    auto load_group = [&](int buf, int64_t c0, int64_t s) {
        for (int e = tid; e < G * B; e += BCB_THREADS) {
            const int jj = e / B, i = e % B;
            const int64_t c = c0 + jj;
            vs[buf][jj][VPAD + i] = (c < nsweeps && s < nsteps) ? V[((s * n) + c) * B + i] : 0.0;
        }
        for (int jj = tid; jj < G; jj += BCB_THREADS) {
            const int64_t c = c0 + jj;
            ts[buf][jj] = (c < nsweeps && s < nsteps) ? TAU[s * n + c] : 0.0;
        }
    };

    double x[NW];
    double pre[SH];
    for (int64_t c0 = 0; c0 < nsweeps; c0 += G) {
        // steps of the first sweep of the block bound the block's steps
        const int64_t rem = n - 1 - (c0 + 1);
        const int64_t S = rem < 0 ? 0 : rem / B + 1;
        if (S == 0) continue;
        int64_t base = c0 + 1 + (S - 1) * B;
        // initial window
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t col = base + 4 * k + rho;
            x[k] = (rowok && col < n) ? Qr[col * ldq] : 0.0;
        }
        __syncthreads();
        load_group(0, c0, S - 1);
        __syncthreads();
        int buf = 0;
        for (int64_t s = S - 1; s >= 0; --s) {
            // prefetch the columns entering the window at step s-1, and the
            // next reflector group
            if (s > 0) {
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                    const int64_t col = base - B + 4 * k + rho;
                    pre[k] = (rowok && col < n) ? Qr[col * ldq] : 0.0;
                }
                load_group(buf ^ 1, c0, s - 1);
            }
            // apply the G reflectors of step s, sweeps ascending
#pragma unroll
            for (int jj = 0; jj < G; ++jj) {
                const double tau = ts[buf][jj];
                const double *v = &vs[buf][jj][VPAD + rho - jj];
                constexpr int CNT = B / 4 + 1;
                const int k0 = jj / 4;
                double dot = 0.0;
#pragma unroll
                for (int q = 0; q < CNT; ++q) {
                    const int k = k0 + q;
                    if (k < NW) dot += x[k] * v[4 * k];
                }
                dot += __shfl_xor(dot, 16, 64);
                dot += __shfl_xor(dot, 32, 64);
                const double w = tau * dot;
#pragma unroll
                for (int q = 0; q < CNT; ++q) {
                    const int k = k0 + q;
                    if (k < NW) x[k] -= w * v[4 * k];
                }
            }
            // slide: columns leaving the window go back to memory
            if (s > 0) {
#pragma unroll
                for (int k = NW - SH; k < NW; ++k) {
                    const int64_t col = base + 4 * k + rho;
                    if (rowok && col < n) Qr[col * ldq] = x[k];
                }
#pragma unroll
                for (int k = NW - 1; k >= SH; --k) x[k] = x[k - SH];
#pragma unroll
                for (int k = 0; k < SH; ++k) x[k] = pre[k];
                base -= B;
            }
            __syncthreads();
            buf ^= 1;
        }
        // block done: store the whole window
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t col = base + 4 * k + rho;
            if (rowok && col < n) Qr[col * ldq] = x[k];
        }
    }
}

// Plain version for b < 4 (and any b): one thread per row, reflectors in
// generation order, Q read and written in global memory.
__global__ void bcback_simple_kernel(int64_t mrows, int64_t n, int64_t b, const double *__restrict__ V,
                                     const double *__restrict__ TAU, double *__restrict__ Q, int64_t ldq)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= mrows) return;
    const int64_t nsteps = bc_num_steps(n, b);
    double *Qr = Q + row;
    for (int64_t c = 0; c + 2 < n; ++c) {
        for (int64_t s = 0; s < nsteps; ++s) {
            const int64_t r = c + 1 + s * b;
            if (r >= n) break;
            const double tau = TAU[s * n + c];
            if (tau == 0.0) continue;
            const int64_t m = (n - r) < b ? (n - r) : b;
            const double *v = V + (s * n + c) * b;
            double dot = 0.0;
            for (int64_t i = 0; i < m; ++i) dot += Qr[(r + i) * ldq] * v[i];
            dot *= tau;
            for (int64_t i = 0; i < m; ++i) Qr[(r + i) * ldq] -= dot * v[i];
        }
    }
}

__global__ void eye_kernel(int64_t n, double *Q, int64_t ldq)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        Q[i + j * ldq] = (i == j) ? 1.0 : 0.0;
    }
}

}  // namespace

evd_status_t bcback_run(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, const double *TAU,
                        double *Q, int64_t ldq)
{
    hipStream_t s = ctx->stream;
    if (n < 3 || mrows <= 0) return EVD_OK;
    const dim3 grid((unsigned)evd_ceil_div(mrows, BCB_ROWS));
    switch (b) {
    case 4: hipLaunchKernelGGL(bcback_kernel<4>, grid, dim3(BCB_THREADS), 0, s, mrows, n, V, TAU, Q, ldq); break;
    case 8: hipLaunchKernelGGL(bcback_kernel<8>, grid, dim3(BCB_THREADS), 0, s, mrows, n, V, TAU, Q, ldq); break;
    case 16: hipLaunchKernelGGL(bcback_kernel<16>, grid, dim3(BCB_THREADS), 0, s, mrows, n, V, TAU, Q, ldq); break;
    case 32: hipLaunchKernelGGL(bcback_kernel<32>, grid, dim3(BCB_THREADS), 0, s, mrows, n, V, TAU, Q, ldq); break;
    case 64: hipLaunchKernelGGL(bcback_kernel<64>, grid, dim3(BCB_THREADS), 0, s, mrows, n, V, TAU, Q, ldq); break;
    default:
        hipLaunchKernelGGL(bcback_simple_kernel, dim3((unsigned)evd_ceil_div(mrows, 256)), dim3(256), 0, s, mrows, n,
                           b, V, TAU, Q, ldq);
    }
    return hipGetLastError() == hipSuccess ? EVD_OK : EVD_ERR_HIP;
}

size_t orgsb_work_bytes(int64_t n, int64_t b) { return evd_align256((size_t)2 * b * (n > 0 ? n : 1) * 8); }

// Q_s = H^(0) H^(1) ... H^(p-1), H^(k) = I - Y_k T_k Y_k^T on rows/cols (k+1)b .. n-1,
// accumulated backwards on the identity.
evd_status_t orgsb_run(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T, double *Q,
                       int64_t ldq, void *work)
{
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)(evd_ceil_div(n * n, 256) < 8192 ? evd_ceil_div(n * n, 256) : 8192)),
                       dim3(256), 0, s, n, Q, ldq);
    double *W1 = (double *)work;
    double *W2 = W1 + (size_t)b * n;
    const int64_t p = evd_sbr_num_panels(n, b);
    for (int64_t k = p - 1; k >= 0; --k) {
        const int64_t j0 = k * b, i0 = j0 + b, m = n - i0;
        const double *Y = A + i0 + j0 * lda;
        double *Qs = Q + i0 + i0 * ldq;
        // W1 = Y^T Q_sub (b x m);  W2 = T W1;  Q_sub -= Y W2
        EVD_CHECK(gemm_f64(s, OP_T, OP_N, 0, b, m, m, 1.0, Y, lda, Qs, ldq, 0.0, W1, b, nullptr, 0));
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, b, m, b, 1.0, T + k * b * b, b, W1, b, 0.0, W2, b, nullptr, 0));
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, m, m, b, -1.0, Y, lda, W2, b, 1.0, Qs, ldq, nullptr, 0));
    }
    return hipGetLastError() == hipSuccess ? EVD_OK : EVD_ERR_HIP;
}

extern "C" {

evd_status_t evd_dorgsb_work_size(evd_ctx_t ctx, int64_t n, int64_t b, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    if (b < 1 || b > 64 || (64 % b) != 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    *bytes = orgsb_work_bytes(n, b);
    return EVD_OK;
}

evd_status_t evd_dorgsb(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T, double *Q,
                        int64_t ldq, void *work, size_t work_bytes)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    int bad = 0;
    if (n < 0) bad = 2;
    else if (b < 1 || b > 64 || (64 % b) != 0) bad = 3;
    else if (n > 0 && !A) bad = 4;
    else if (lda < (n > 1 ? n : 1)) bad = 5;
    else if (evd_sbr_num_panels(n, b) > 0 && !T) bad = 6;
    else if (n > 0 && !Q) bad = 7;
    else if (ldq < (n > 1 ? n : 1)) bad = 8;
    else if (n > 0 && !work) bad = 9;
    else if (work_bytes < orgsb_work_bytes(n, b)) bad = 10;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 10 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    if (hipSetDevice(ctx->device) != hipSuccess) return EVD_ERR_HIP;
    return orgsb_run(ctx, n, b, A, lda, T, Q, ldq, work);
}

evd_status_t evd_dbcback(evd_ctx_t ctx, int64_t m_rows, int64_t n, int64_t b, const double *V, const double *TAU,
                         double *Q, int64_t ldq)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    int bad = 0;
    if (m_rows < 0) bad = 2;
    else if (n < 0) bad = 3;
    else if (b < 1 || b > 64 || (64 % b) != 0) bad = 4;
    else if (n > 2 && !V) bad = 5;
    else if (n > 2 && !TAU) bad = 6;
    else if (m_rows > 0 && n > 0 && !Q) bad = 7;
    else if (ldq < (m_rows > 1 ? m_rows : 1)) bad = 8;
    ctx->last_invalid_arg = bad;
    if (bad) return EVD_ERR_INVALID_ARG;
    if (n < 3 || m_rows == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    if (hipSetDevice(ctx->device) != hipSuccess) return EVD_ERR_HIP;
    return bcback_run(ctx, m_rows, n, b, V, TAU, Q, ldq);
}

}  // extern "C"
