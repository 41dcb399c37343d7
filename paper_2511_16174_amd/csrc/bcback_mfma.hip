// BC-back on the FP64 matrix cores (stage 4b of Section 4.3, blocked).
//
// The reflectors of BC_G = 32 consecutive sweeps at one step form a group
// whose product is a compact-WY block reflector H_c0 ... H_c0+31 = I - Y T Y^T:
// Y is the staircase of their vectors in a window of W = 32 + b columns
// (column j of Y holds v_j shifted down by j) and T is upper triangular
// (forward column recurrence).  Applying a group to a block of rows of Q is
// three small products on v_mfma_f64_16x16x4:
//   P = Q_w Y (16 x 32),  P2 = P T (P T^T for the reverse order),
//   Q_w <- Q_w - P2 Y^T,
// skipping the zero 16 x 4 blocks of the staircase and of T.  The groups are
// taken in the same order as the reflector-by-reflector kernel (blocks
// ascending, steps descending; everything reversed for the reverse product),
// so Q_w is a window of W columns that slides by b columns per step and stays
// in registers.  Register layout: a wavefront owns 16 rows; lane l holds
// x[kk] = Q_w(l % 16, 4 kk + l / 16), which is both the B-operand layout of
// the first product and the accumulator layout of the third (the products are
// issued transposed: the LDS operand goes first).
//
// T factors are computed for all groups beforehand by bct_kernel (one
// wavefront per group: Gram matrix of the staircase, then the recurrence
// T[0:j, j] = -tau_j T[0:j, 0:j] (Y[:, 0:j]^T v_j), T[j, j] = tau_j).
#include "common.h"

namespace {

constexpr int BC_G = 32;   // sweeps per group

__global__ __launch_bounds__(64) void bct_kernel(int64_t n, int B, const double *__restrict__ V,
                                                 const double *__restrict__ TAU, double *__restrict__ Tg, int64_t nblk)
{
    constexpr int G = BC_G;
    __shared__ double vsh[G][65];
    __shared__ double gsh[G][G + 1];
    __shared__ double tsh[G][G + 1];
    __shared__ double tau[G];
    const int64_t blk = blockIdx.x, s = blockIdx.y;
    const int64_t nsweeps = n - 2, nsteps = bc_num_steps(n, B);
    const int tid = threadIdx.x;
    {
        // groups past the steps of the block's first sweep are never read
        const int64_t rem = n - 1 - (blk * G + 1);
        const int64_t S = rem < 0 ? 0 : rem / B + 1;
        if (s >= S) return;
    }
    for (int e = tid; e < G * B; e += 64) {
        const int j = e / B, i = e % B;
        const int64_t c = blk * G + j;
        vsh[j][i] = (c < nsweeps && s < nsteps) ? V[((s * n) + c) * B + i] : 0.0;
    }
    for (int j = tid; j < G; j += 64) {
        const int64_t c = blk * G + j;
        tau[j] = (c < nsweeps && s < nsteps) ? TAU[s * n + c] : 0.0;
    }
    for (int e = tid; e < G * (G + 1); e += 64) (&tsh[0][0])[e] = 0.0;
    __syncthreads();
    // Gram entries g[i][j], i < j: Y[:, i] . Y[:, j] = sum_t v_i[t + j - i] v_j[t]
    for (int e = tid; e < G * G; e += 64) {
        const int i = e / G, j = e % G;
        if (i < j) {
            const int d = j - i;
            double acc = 0.0;
            for (int t = 0; t + d < B; ++t) acc += vsh[i][t + d] * vsh[j][t];
            gsh[i][j] = acc;
        }
    }
    __syncthreads();
    for (int j = 0; j < G; ++j) {
        if (tid < j) {
            double acc = 0.0;
            for (int k = tid; k < j; ++k) acc += tsh[tid][k] * gsh[k][j];
            tsh[tid][j] = -tau[j] * acc;
        }
        if (tid == 0) tsh[j][j] = tau[j];
        __syncthreads();
    }
    double *T = Tg + (s * nblk + blk) * (int64_t)(G * G);
    for (int e = tid; e < G * G; e += 64) T[e] = tsh[e / G][e % G];  // row-major [k][j]
}

template <int B, bool REV>
__global__ __launch_bounds__(256, 2) void bcback_mfma_kernel(int64_t mrows, int64_t n, const double *__restrict__ V,
                                                             const double *__restrict__ Tg, int64_t nblk,
                                                             double *__restrict__ Q, int64_t ldq)
{
    constexpr int G = BC_G;
    constexpr int W = G + B;      // window columns
    constexpr int KW = W / 4;     // k-steps over the window (4 columns each)
    constexpr int SHK = B / 4;    // k-steps the window slides per step
    constexpr int LDY = G + 1;
    constexpr int LDT = G + 1;
    static_assert(W % 16 == 0, "window must be a whole number of 16-column tiles");
    static_assert((G * B) % 256 == 0 && (G * G) % 256 == 0, "group operands must split evenly over the threads");
    __shared__ double Ys[2][W][LDY];
    __shared__ double Ts[2][G][LDT];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + li;
    const bool rowok = row < mrows;
    double *Qr = Q + row;
    const int64_t nsweeps = n - 2;
    const int64_t nsteps = bc_num_steps(n, B);

    // the staircase keeps its zeros: only band positions are ever written
    for (int e = tid; e < 2 * W * LDY; e += 256) (&Ys[0][0][0])[e] = 0.0;
    __syncthreads();

    // a group's operands are fetched into registers before the current group
    // is applied and written to LDS after it, so the fetch latency overlaps
    // the matrix-core work
    constexpr int NV = G * B / 256, NT = G * G / 256;
    double gv[NV], gt[NT];
    auto fetch_group = [&](int64_t blk, int64_t s) {
        const int64_t c0 = blk * G;
#pragma unroll
        for (int r = 0; r < NV; ++r) {
            const int e = tid + r * 256, j = e / B, i = e % B;
            const int64_t c = c0 + j;
            gv[r] = (c < nsweeps && s < nsteps) ? V[((s * n) + c) * B + i] : 0.0;
        }
        const double *T = Tg + (s * nblk + blk) * (int64_t)(G * G);
#pragma unroll
        for (int r = 0; r < NT; ++r) gt[r] = T[tid + r * 256];
    };
    auto store_group = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NV; ++r) {
            const int e = tid + r * 256, j = e / B, i = e % B;
            Ys[buf][j + i][j] = gv[r];
        }
#pragma unroll
        for (int r = 0; r < NT; ++r) {
            const int e = tid + r * 256;
            Ts[buf][e / G][e % G] = gt[r];
        }
    };

    double x[KW];
    double pre[SHK];
    const int64_t blk_first = REV ? nblk - 1 : 0;
    for (int64_t blk = blk_first; REV ? blk >= 0 : blk < nblk; blk += REV ? -1 : 1) {
        const int64_t c0 = blk * G;
        const int64_t rem = n - 1 - (c0 + 1);
        const int64_t S = rem < 0 ? 0 : rem / B + 1;
        if (S == 0) continue;
        int64_t base = REV ? c0 + 1 : c0 + 1 + (S - 1) * B;
#pragma unroll
        for (int kk = 0; kk < KW; ++kk) {
            const int64_t col = base + 4 * kk + lk;
            x[kk] = (rowok && col < n) ? Qr[col * ldq] : 0.0;
        }
        __syncthreads();
        fetch_group(blk, REV ? 0 : S - 1);
        store_group(0);
        __syncthreads();
        int buf = 0;
        for (int64_t it = 0; it < S; ++it) {
            const int64_t s = REV ? it : S - 1 - it;
            const bool more = it + 1 < S;
            if (more) {
#pragma unroll
                for (int k = 0; k < SHK; ++k) {
                    const int64_t col = REV ? base + B + 4 * (KW - SHK + k) + lk : base - B + 4 * k + lk;
                    pre[k] = (rowok && col < n) ? Qr[col * ldq] : 0.0;
                }
                fetch_group(blk, REV ? s + 1 : s - 1);
            }
            // P = Q_w Y: reflector tile jt meets window k-steps 4 jt .. 4 jt + B/4 + 3
            double4_t P[2];
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) {
                P[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 4 * jt; kk < 4 * jt + SHK + 4; ++kk)
                    if (kk < KW)
                        P[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ys[buf][4 * kk + lk][16 * jt + li], x[kk], P[jt], 0,
                                                                     0, 0);
            }
            // P2 = P T (upper) or P T^T (REV)
            double4_t P2[2];
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) {
                P2[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const bool nz = REV ? (kk >= 4 * jt) : (kk <= 4 * jt + 3);
                    if (nz) {
                        const double a = REV ? Ts[buf][16 * jt + li][4 * kk + lk] : Ts[buf][4 * kk + lk][16 * jt + li];
                        P2[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, P[kk / 4][kk % 4], P2[jt], 0, 0, 0);
                    }
                }
            }
            // Q_w -= P2 Y^T: window tile t meets reflectors 16 t - (B - 1) .. 16 t + 15
#pragma unroll
            for (int t = 0; t < KW / 4; ++t) {
                double4_t acc = (double4_t){x[4 * t], x[4 * t + 1], x[4 * t + 2], x[4 * t + 3]};
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const int jlo = 4 * kk, jhi = 4 * kk + 3;
                    if (jhi >= 16 * t - (B - 1) && jlo <= 16 * t + 15)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Ys[buf][16 * t + li][4 * kk + lk], P2[kk / 4][kk % 4],
                                                                   acc, 0, 0, 0);
                }
                x[4 * t] = acc[0];
                x[4 * t + 1] = acc[1];
                x[4 * t + 2] = acc[2];
                x[4 * t + 3] = acc[3];
            }
            if (more) {
                store_group(buf ^ 1);
                if (REV) {
#pragma unroll
                    for (int kk = 0; kk < SHK; ++kk) {
                        const int64_t col = base + 4 * kk + lk;
                        if (rowok && col < n) Qr[col * ldq] = x[kk];
                    }
#pragma unroll
                    for (int kk = 0; kk < KW - SHK; ++kk) x[kk] = x[kk + SHK];
#pragma unroll
                    for (int k = 0; k < SHK; ++k) x[KW - SHK + k] = pre[k];
                    base += B;
                } else {
#pragma unroll
                    for (int kk = KW - SHK; kk < KW; ++kk) {
                        const int64_t col = base + 4 * kk + lk;
                        if (rowok && col < n) Qr[col * ldq] = x[kk];
                    }
#pragma unroll
                    for (int kk = KW - 1; kk >= SHK; --kk) x[kk] = x[kk - SHK];
#pragma unroll
                    for (int k = 0; k < SHK; ++k) x[k] = pre[k];
                    base -= B;
                }
            }
            __syncthreads();
            buf ^= 1;
        }
#pragma unroll
        for (int kk = 0; kk < KW; ++kk) {
            const int64_t col = base + 4 * kk + lk;
            if (rowok && col < n) Qr[col * ldq] = x[kk];
        }
    }
}

}  // namespace

int64_t bcback_mfma_nblk(int64_t n) { return n > 2 ? evd_ceil_div(n - 2, BC_G) : 0; }

// T workspace of the blocked BC-back (doubles); 0 when the blocked kernel
// does not apply to b.
size_t bcback_mfma_t_elems(int64_t n, int64_t b)
{
    if (!(b == 16 || b == 32 || b == 64) || n < 3) return 0;
    return (size_t)bc_num_steps(n, b) * (size_t)bcback_mfma_nblk(n) * BC_G * BC_G;
}

// Q (mrows x n) <- Q H_1 ... H_m (rev = false) or Q H_m ... H_1 (rev = true);
// Tg holds bcback_mfma_t_elems(n, b) doubles of scratch.
evd_status_t bcback_mfma_run(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, const double *TAU,
                             double *Q, int64_t ldq, double *Tg, bool rev)
{
    hipStream_t s = ctx->stream;
    if (n < 3 || mrows <= 0) return EVD_OK;
    const int64_t nblk = bcback_mfma_nblk(n);
    const int64_t nsteps = bc_num_steps(n, b);
    hipLaunchKernelGGL(bct_kernel, dim3((unsigned)nblk, (unsigned)nsteps), dim3(64), 0, s, n, (int)b, V, TAU, Tg, nblk);
    const dim3 grid((unsigned)evd_ceil_div(mrows, 64)), blk(256);
#define EVD_BCM(BB)                                                                                               \
    if (rev) hipLaunchKernelGGL((bcback_mfma_kernel<BB, true>), grid, blk, 0, s, mrows, n, V, (const double *)Tg,  \
                                nblk, Q, ldq);                                                                     \
    else hipLaunchKernelGGL((bcback_mfma_kernel<BB, false>), grid, blk, 0, s, mrows, n, V, (const double *)Tg, nblk, \
                            Q, ldq);
    switch (b) {
    case 16: EVD_BCM(16) break;
    case 32: EVD_BCM(32) break;
    case 64: EVD_BCM(64) break;
    default: return EVD_ERR_INVALID_ARG;
    }
#undef EVD_BCM
    return evd_check_last();
}
