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
// Register layout: a row of Q is spread over 4 adjacent lanes (lane =
// 4 row + rho); lane rho holds window columns 4k + rho, k = 0 .. NW-1.
// Reflector jj of the group touches window columns jj .. jj+b-1, i.e. slots
// k = jj/4 .. jj/4 + b/4 on every lane (out-of-range entries meet zero padding
// of v).  The four partial dot products of a row are combined with two DPP
// quad permutations; each partial uses two accumulators to halve the FMA chain.
#include <utility>

#include "common.h"

namespace {

constexpr int BCB_G = 64;                     // sweeps per block
constexpr int VPAD = 4;                       // zero padding on each side of v

// Calls f(integral_constant<jj>) for jj = 0..G-1 (descending if REV), so that
// every window slot index is a compile-time constant.
template <int G, bool REV, typename F, int... J>
__device__ __forceinline__ void for_each_reflector(F &&f, std::integer_sequence<int, J...>)
{
    if constexpr (REV) (f(std::integral_constant<int, G - 1 - J>{}), ...);
    else (f(std::integral_constant<int, J>{}), ...);
}

// REV = false: Q <- Q H_1 ... H_m (generation order, the reordered stages);
// REV = true:  Q <- Q H_m ... H_1 (reverse order, i.e. rows of Q_d^T for the
// conventional order).  The reverse order runs the forward schedule
// backwards: blocks descending, steps ascending, sweeps descending, with the
// register window sliding right.
template <int B, typename T, int ROWS, bool REV>
__global__ __launch_bounds__(ROWS * 4) void bcback_kernel(int64_t mrows, int64_t n, const T *__restrict__ V,
                                                             const T *__restrict__ TAU, T *__restrict__ Q,
                                                             int64_t ldq)
{
    constexpr int G = BCB_G;
    constexpr int BCB_THREADS = ROWS * 4;
    constexpr int NW = (G + B) / 4;       // slots per lane (window G+B-1 columns, one spare)
    constexpr int SH = B / 4;             // slots shifted per step
    constexpr int LDV = B + 2 * VPAD;
    __shared__ T vs[2][G][LDV];
    __shared__ T ts[2][G];

    const int tid = threadIdx.x;
    const int rho = tid & 3;                              // residue of this lane
    const int64_t row = (int64_t)blockIdx.x * ROWS + (tid >> 2);
    const bool rowok = row < mrows;
    T *Qr = Q + row;

    const int64_t nsweeps = n - 2;
    const int64_t nsteps = bc_num_steps(n, B);

    // zero the padding once
    for (int e = tid; e < 2 * G * LDV; e += BCB_THREADS) (&vs[0][0][0])[e] = 0.0;
    __syncthreads();

    // the next group is fetched into registers before the current one is
    // applied and written to LDS after it (the fetch latency overlaps the work)
    constexpr int NV = (G * B + BCB_THREADS - 1) / BCB_THREADS;
    T gv[NV], gt = 0.0;
    auto fetch_group = [&](int64_t c0, int64_t s) {
#pragma unroll
        for (int r = 0; r < NV; ++r) {
            const int e = tid + r * BCB_THREADS, jj = e / B, i = e % B;
            const int64_t c = c0 + jj;
            gv[r] = (e < G * B && c < nsweeps && s < nsteps) ? V[((s * n) + c) * B + i] : (T)0;
        }
        const int64_t c = c0 + tid;
        gt = (tid < G && c < nsweeps && s < nsteps) ? TAU[s * n + c] : (T)0;
    };
    auto store_group = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NV; ++r) {
            const int e = tid + r * BCB_THREADS, jj = e / B, i = e % B;
            if (e < G * B) vs[buf][jj][VPAD + i] = gv[r];
        }
        if (tid < G) ts[buf][tid] = gt;
    };
    // one reflector of the current group applied to the lane's window slots
    auto apply = [&](int buf, T(&x)[NW], auto jjc) {
        constexpr int jj = decltype(jjc)::value;
        const T tau = ts[buf][jj];
        const T *v = &vs[buf][jj][VPAD + rho - jj];
        constexpr int CNT = B / 4 + 1;
        constexpr int k0 = jj / 4;
        T d0 = 0.0, d1 = 0.0;
#pragma clang loop unroll(full)
        for (int q = 0; q < CNT; q += 2) {
            const int k = k0 + q;
            if (k < NW) d0 += x[k] * v[4 * k];
            if (q + 1 < CNT && k + 1 < NW) d1 += x[k + 1] * v[4 * (k + 1)];
        }
        const T w = tau * quad_sum(d0 + d1);
#pragma clang loop unroll(full)
        for (int q = 0; q < CNT; ++q) {
            const int k = k0 + q;
            if (k < NW) x[k] -= w * v[4 * k];
        }
    };

    T x[NW];
    T pre[SH];
    const int64_t c0_first = REV ? ((nsweeps - 1) / G) * G : 0;
    for (int64_t c0 = c0_first; REV ? (c0 >= 0) : (c0 < nsweeps); c0 += REV ? -G : G) {
        // steps of the first sweep of the block bound the block's steps
        const int64_t rem = n - 1 - (c0 + 1);
        const int64_t S = rem < 0 ? 0 : rem / B + 1;
        if (S == 0) continue;
        int64_t base = REV ? c0 + 1 : c0 + 1 + (S - 1) * B;
        // initial window
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t col = base + 4 * k + rho;
            x[k] = (rowok && col < n) ? Qr[col * ldq] : 0.0;
        }
        __syncthreads();
        fetch_group(c0, REV ? 0 : S - 1);
        store_group(0);
        __syncthreads();
        int buf = 0;
        for (int64_t it = 0; it < S; ++it) {
            const int64_t s = REV ? it : S - 1 - it;
            const bool more = it + 1 < S;
            // prefetch the columns entering the window at the next step, and
            // the next reflector group
            if (more) {
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                    const int64_t col = REV ? base + B + 4 * (NW - SH + k) + rho : base - B + 4 * k + rho;
                    pre[k] = (rowok && col < n) ? Qr[col * ldq] : 0.0;
                }
                fetch_group(c0, REV ? s + 1 : s - 1);
            }
            // the G reflectors of step s: sweeps ascending (descending for REV)
            for_each_reflector<G, REV>([&](auto jjc) { apply(buf, x, jjc); }, std::make_integer_sequence<int, G>{});
            // slide: columns leaving the window go back to memory
            if (more) {
                store_group(buf ^ 1);
                if (REV) {
#pragma unroll
                    for (int k = 0; k < SH; ++k) {
                        const int64_t col = base + 4 * k + rho;
                        if (rowok && col < n) Qr[col * ldq] = x[k];
                    }
#pragma unroll
                    for (int k = 0; k < NW - SH; ++k) x[k] = x[k + SH];
#pragma unroll
                    for (int k = 0; k < SH; ++k) x[NW - SH + k] = pre[k];
                    base += B;
                } else {
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
template <typename T>
__global__ void bcback_simple_kernel(int64_t mrows, int64_t n, int64_t b, const T *__restrict__ V,
                                     const T *__restrict__ TAU, T *__restrict__ Q, int64_t ldq, int rev)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= mrows) return;
    const int64_t nsteps = bc_num_steps(n, b);
    T *Qr = Q + row;
    for (int64_t ci = 0; ci + 2 < n; ++ci) {
        const int64_t c = rev ? n - 3 - ci : ci;
        for (int64_t si = 0; si < nsteps; ++si) {
            const int64_t s = rev ? nsteps - 1 - si : si;
            const int64_t r = c + 1 + s * b;
            if (r >= n) continue;
            const T tau = TAU[s * n + c];
            if (tau == 0.0) continue;
            const int64_t m = (n - r) < b ? (n - r) : b;
            const T *v = V + (s * n + c) * b;
            T dot = 0.0;
            for (int64_t i = 0; i < m; ++i) dot += Qr[(r + i) * ldq] * v[i];
            dot *= tau;
            for (int64_t i = 0; i < m; ++i) Qr[(r + i) * ldq] -= dot * v[i];
        }
    }
}

template <typename T>
__global__ void eye_kernel(int64_t n, T *Q, int64_t ldq)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        Q[i + j * ldq] = (i == j) ? 1.0 : 0.0;
    }
}

}  // namespace

namespace {
template <typename T>
evd_status_t bcback_run_t(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const T *V, const T *TAU, T *Q,
                          int64_t ldq, bool rev)
{
    hipStream_t s = ctx->stream;
    if (n < 3 || mrows <= 0) return EVD_OK;
    // the largest row block that still gives every compute unit a workgroup
    // (a row's reflectors are applied in sequence, so rows are the only
    // parallelism; every block re-reads every reflector group)
    const int rows = (mrows >= (int64_t)128 * ctx->num_cus) ? 128 : (mrows >= (int64_t)64 * ctx->num_cus ? 64 : 32);
    const dim3 grid((unsigned)evd_ceil_div(mrows, rows));
    const dim3 blk(rows * 4);
#define EVD_BCB_R(BB, RV)                                                                                        \
    if (rows == 128) hipLaunchKernelGGL((bcback_kernel<BB, T, 128, RV>), grid, blk, 0, s, mrows, n, V, TAU, Q, ldq); \
    else if (rows == 64) hipLaunchKernelGGL((bcback_kernel<BB, T, 64, RV>), grid, blk, 0, s, mrows, n, V, TAU, Q, ldq); \
    else hipLaunchKernelGGL((bcback_kernel<BB, T, 32, RV>), grid, blk, 0, s, mrows, n, V, TAU, Q, ldq);
#define EVD_BCB(BB)                                                                                              \
    if (rev) { EVD_BCB_R(BB, true) } else { EVD_BCB_R(BB, false) }
    switch (b) {
    case 4: EVD_BCB(4) break;
    case 8: EVD_BCB(8) break;
    case 16: EVD_BCB(16) break;
    case 32: EVD_BCB(32) break;
    case 64: EVD_BCB(64) break;
    default:
        hipLaunchKernelGGL(bcback_simple_kernel<T>, dim3((unsigned)evd_ceil_div(mrows, 256)), dim3(256), 0, s, mrows, n,
                           b, V, TAU, Q, ldq, rev ? 1 : 0);
    }
#undef EVD_BCB
#undef EVD_BCB_R
    return evd_check_last();
}

}  // namespace

evd_status_t bcback_run(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, const double *TAU,
                        double *Q, int64_t ldq)
{
    return bcback_run_t<double>(ctx, mrows, n, b, V, TAU, Q, ldq, false);
}

// Q <- Q H_m ... H_1 (the rows of Q_d^T in the conventional stage order)
evd_status_t bcback_run_rev(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, const double *TAU,
                            double *Q, int64_t ldq)
{
    return bcback_run_t<double>(ctx, mrows, n, b, V, TAU, Q, ldq, true);
}

evd_status_t bcback_run_f32(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const float *V, const float *TAU,
                            float *Q, int64_t ldq)
{
    return bcback_run_t<float>(ctx, mrows, n, b, V, TAU, Q, ldq, false);
}

// SBR-back.  Q_s = H^(0) H^(1) ... H^(p-1), H^(k) = I - Y_k T_k Y_k^T acting on
// rows/cols (k+1)b .. n-1, accumulated backwards on the identity.  Panels are
// aggregated ORGSB_NB columns at a time into one block reflector
// I - Y_g T_g Y_g^T (T_g from the recurrence T = [[T1, -T1 Y1^T Y2 T2], [0, T2]]),
// so the two large products of each group have inner dimension ORGSB_NB
// rather than b.
constexpr int64_t ORGSB_NB = 512;  // largest group (columns); "orgsb_nb" may pick a smaller one

namespace {

int64_t orgsb_group_panels(int64_t b) { return (ORGSB_NB / b) > 0 ? ORGSB_NB / b : 1; }

template <typename T>
struct OrgsbWork {
    T *Yg, *S, *Tg, *X1, *W1, *W2, *ws;
    size_t ws_elems;
};

template <typename T>
size_t orgsb_layout(int64_t n, int64_t b, char *base, OrgsbWork<T> *w)
{
    const int64_t nb = orgsb_group_panels(b) * b;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    auto take = [&](size_t elems) {
        char *p = base ? base + off : nullptr;
        off += evd_align256(elems * sizeof(T));
        return (T *)p;
    };
    OrgsbWork<T> t;
    t.Yg = take(nn * nb);
    t.S = take((size_t)nb * nb);
    t.Tg = take((size_t)nb * nb);
    t.X1 = take((size_t)nb * b);
    t.W1 = take((size_t)nb * nn);
    t.W2 = take((size_t)nb * nn);
    t.ws_elems = gemm_ws_elems_t<T>(nb, nb, n);
    t.ws = take(t.ws_elems > 0 ? t.ws_elems : 1);
    if (w) *w = t;
    return off;
}

// Yg(r, c) = Y_{k0 + c/b}(row i0 + r, column c % b), zero above that panel's rows.
template <typename T>
__global__ void orgsb_gather_y_kernel(int64_t m, int64_t nbw, int64_t b, int64_t i0, int64_t k0, const T *A,
                                      int64_t lda, T *Yg)
{
    const int64_t total = m * nbw;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx % m, c = idx / m;
        const int64_t kp = k0 + c / b;
        const int64_t gi = i0 + r;
        Yg[idx] = (gi >= kp * b + b) ? A[gi + (kp * b + c % b) * lda] : (T)0;
    }
}

// Tg <- 0 with the panels' T factors on its diagonal blocks.
template <typename T>
__global__ void orgsb_diag_t_kernel(int64_t nbw, int64_t ldt, int64_t b, int64_t k0, const T *Tf, T *Tg)
{
    const int64_t total = nbw * nbw;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx % nbw, c = idx / nbw;
        const int64_t pr = r / b, pc = c / b;
        Tg[r + c * ldt] = (pr == pc) ? Tf[(k0 + pc) * b * b + (r % b) + (c % b) * b] : (T)0;
    }
}

template <typename T>
evd_status_t orgsb_run_t(evd_ctx_t ctx, int64_t n, int64_t b, const T *A, int64_t lda, const T *Tf, T *Q,
                         int64_t ldq, void *work, bool identity)
{
    // identity: Q <- Q_s (accumulated on I, only Q[i0:, i0:] changes per group);
    // otherwise Q <- Q_s Q for an n x n matrix Q (all columns)
    hipStream_t s = ctx->stream;
    if (identity)
        hipLaunchKernelGGL(eye_kernel<T>, dim3((unsigned)(evd_ceil_div(n * n, 256) < 8192 ? evd_ceil_div(n * n, 256) : 8192)),
                           dim3(256), 0, s, n, Q, ldq);
    OrgsbWork<T> w;
    orgsb_layout<T>(n, b, (char *)work, &w);
    const int64_t p = evd_sbr_num_panels(n, b);
    const int64_t gpmax = orgsb_group_panels(b);
    const int64_t nb = gpmax * b;  // leading dimension of the group buffers
    int64_t gp = (ctx->orgsb_nb > 0) ? ctx->orgsb_nb / b : gpmax;
    if (gp < 1) gp = 1;
    if (gp > gpmax) gp = gpmax;
    const int64_t ngroups = evd_ceil_div(p, gp);
    for (int64_t g = ngroups - 1; g >= 0; --g) {
        const int64_t k0 = g * gp;
        const int64_t np = (k0 + gp <= p) ? gp : p - k0;
        const int64_t nbw = np * b;
        const int64_t i0 = k0 * b + b, m = n - i0;
        const int64_t c0 = identity ? i0 : 0, nc = n - c0;
        T *Qs = Q + i0 + c0 * ldq;
        const int64_t blocks_y = evd_ceil_div(m * nbw, 256) < 8192 ? evd_ceil_div(m * nbw, 256) : 8192;
        hipLaunchKernelGGL(orgsb_gather_y_kernel<T>, dim3((unsigned)blocks_y), dim3(256), 0, s, m, nbw, b, i0, k0, A,
                           lda, w.Yg);
        hipLaunchKernelGGL(orgsb_diag_t_kernel<T>, dim3((unsigned)evd_ceil_div(nbw * nbw, 256)), dim3(256), 0, s, nbw,
                           nb, b, k0, Tf, w.Tg);
        if (np > 1) {
            // S = Yg^T Yg, then the off-diagonal blocks of T_g panel by panel
            EVD_CHECK(gemm_t(s, OP_T, OP_N, 0, nbw, nbw, m, (T)1, w.Yg, m, w.Yg, m, (T)0, w.S, nb, w.ws, w.ws_elems));
            for (int64_t i = 1; i < np; ++i) {
                const int64_t cur = i * b;
                EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, cur, b, cur, (T)1, w.Tg, nb, w.S + cur * nb, nb, (T)0, w.X1, nb,
                                 (T *)nullptr, 0));
                EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, cur, b, b, (T)-1, w.X1, nb, Tf + (k0 + i) * b * b, b, (T)0,
                                 w.Tg + cur * nb, nb, (T *)nullptr, 0));
            }
        }
        // W1 = Yg^T Q_sub;  W2 = T_g W1;  Q_sub -= Yg W2
        EVD_CHECK(gemm_t(s, OP_T, OP_N, 0, nbw, nc, m, (T)1, w.Yg, m, Qs, ldq, (T)0, w.W1, nb, (T *)nullptr, 0));
        EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, nbw, nc, nbw, (T)1, w.Tg, nb, w.W1, nb, (T)0, w.W2, nb, (T *)nullptr, 0));
        EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, m, nc, nbw, (T)-1, w.Yg, m, w.W2, nb, (T)1, Qs, ldq, (T *)nullptr, 0));
    }
    return evd_check_last();
}

}  // namespace

size_t orgsb_work_bytes(int64_t n, int64_t b)
{
    const size_t a = orgsb_layout<double>(n, b, nullptr, nullptr);
    const size_t f = orgsb_layout<float>(n, b, nullptr, nullptr);
    return a > f ? a : f;
}

evd_status_t orgsb_run(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T, double *Q,
                       int64_t ldq, void *work)
{
    return orgsb_run_t<double>(ctx, n, b, A, lda, T, Q, ldq, work, true);
}

// C <- Q_s C for an n x n matrix C (the conventional stage order)
evd_status_t ormsb_run(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T, double *C,
                       int64_t ldc, void *work)
{
    return orgsb_run_t<double>(ctx, n, b, A, lda, T, C, ldc, work, false);
}

// B <- A^T (n x n), 32 x 32 tiles through LDS
__global__ __launch_bounds__(256) void transpose_kernel(int64_t n, const double *__restrict__ A, int64_t lda,
                                                        double *__restrict__ B, int64_t ldb)
{
    __shared__ double tile[32][33];
    const int64_t bi = (int64_t)blockIdx.x * 32, bj = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi + tx, j = bj + r;
        if (i < n && j < n) tile[r][tx] = A[i + j * lda];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bj + tx, j = bi + r;
        if (i < n && j < n) B[i + j * ldb] = tile[tx][r];
    }
}

evd_status_t transpose_run(hipStream_t s, int64_t n, const double *A, int64_t lda, double *B, int64_t ldb)
{
    const dim3 grid((unsigned)evd_ceil_div(n, 32), (unsigned)evd_ceil_div(n, 32));
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, n, A, lda, B, ldb);
    return evd_check_last();
}

evd_status_t orgsb_run_f32(evd_ctx_t ctx, int64_t n, int64_t b, const float *A, int64_t lda, const float *T, float *Q,
                           int64_t ldq, void *work)
{
    return orgsb_run_t<float>(ctx, n, b, A, lda, T, Q, ldq, work, true);
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
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    return orgsb_run(ctx, n, b, A, lda, T, Q, ldq, work);
}

evd_status_t evd_dbcback_work_size(evd_ctx_t ctx, int64_t n, int64_t b, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    if (b < 1 || b > 64 || (64 % b) != 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    *bytes = bcback_mfma_t_elems(n, b) * sizeof(double);
    return EVD_OK;
}

evd_status_t evd_dbcback(evd_ctx_t ctx, char trans, int64_t m_rows, int64_t n, int64_t b, const double *V,
                         const double *TAU, double *Q, int64_t ldq, void *work, size_t work_bytes)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    const bool rev = (trans == 'T' || trans == 't');
    const size_t need = ctx->bcback_valu ? 0 : bcback_mfma_t_elems(n > 0 ? n : 0, b) * sizeof(double);
    int bad = 0;
    if (!(rev || trans == 'N' || trans == 'n')) bad = 2;
    else if (m_rows < 0) bad = 3;
    else if (n < 0) bad = 4;
    else if (b < 1 || b > 64 || (64 % b) != 0) bad = 5;
    else if (n > 2 && !V) bad = 6;
    else if (n > 2 && !TAU) bad = 7;
    else if (m_rows > 0 && n > 0 && !Q) bad = 8;
    else if (ldq < (m_rows > 1 ? m_rows : 1)) bad = 9;
    else if (need && m_rows > 0 && !work) bad = 10;
    else if (m_rows > 0 && work_bytes < need) bad = 11;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 11 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n < 3 || m_rows == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    if (need && bcback_mfma_fits(ldq)) {
        double *Tg = (double *)work;
        EVD_CHECK(bcback_mfma_prepare(ctx, n, b, V, TAU, Tg, rev));
        return bcback_mfma_apply(ctx, m_rows, n, b, V, Q, ldq, Tg, rev);
    }
    return rev ? bcback_run_rev(ctx, m_rows, n, b, V, TAU, Q, ldq) : bcback_run(ctx, m_rows, n, b, V, TAU, Q, ldq);
}

}  // extern "C"
