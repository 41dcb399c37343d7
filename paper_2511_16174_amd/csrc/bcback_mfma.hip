// BC-back on the FP64 matrix cores (stage 4b of Section 4.3, blocked).
//
// The reflectors of BC_G = 32 consecutive sweeps at one step form a group
// whose product is a compact-WY block reflector H_c0 ... H_c0+31 = I - Y T Y^T:
// Y is the staircase of their vectors in a window of W = 32 + b columns
// (column j of Y holds v_j shifted down by j) and T is upper triangular
// (forward column recurrence).  Applying a group to a block of rows of Q is
// three small products on v_mfma_f64_16x16x4:
//   P = Q_w Y (16 x 32),  P2 = P (-T) (P (-T)^T for the reverse order),
//   Q_w <- Q_w + P2 Y^T,
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
// T[0:j, j] = -tau_j T[0:j, 0:j] (Y[:, 0:j]^T v_j), T[j, j] = tau_j) and
// stored negated, so that every product accumulates with a plus sign.
// Global addresses are a wave-uniform 64-bit base plus one 32-bit lane offset,
// and a step whose columns and rows are all in range skips the bounds tests.
#include "common.h"

namespace {

constexpr int BC_G = 32;   // sweeps per group

template <typename P>
__device__ __forceinline__ P &at(P *base, uint32_t byte_off)
{
    return *(P *)((char *)base + byte_off);
}
template <typename P>
__device__ __forceinline__ const P &at(const P *base, uint32_t byte_off)
{
    return *(const P *)((const char *)base + byte_off);
}

// Raw buffer access to nk window k-steps (4 nk columns) starting at p, column
// stride ldq doubles: a wave-uniform descriptor, the lane's row offset in the
// vector offset and the k-step offset in the scalar offset, so no 64-bit
// address is formed per access (requires nk * 4 * ldq * 8 < 2^31).
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t window_rsrc(const double *p, int nk, int64_t ldq4)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)((uint32_t)nk * (uint32_t)ldq4 * 8u),
                                             (int)EVD_BUF_DWORD3);
}
__device__ __forceinline__ double window_load(__amdgpu_buffer_rsrc_t rs, uint32_t loff, int k, int64_t ldq4)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)loff, (int)(k * ldq4 * 8), 0));
}
__device__ __forceinline__ void window_store(__amdgpu_buffer_rsrc_t rs, uint32_t loff, int k, int64_t ldq4, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), rs, (int)loff, (int)(k * ldq4 * 8), 0);
}

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
    for (int e = tid; e < G * G; e += 64) T[e] = -tsh[e / G][e % G];  // -T, row-major [k][j]
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
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: lets row0 live in scalar registers
    const int li = lane & 15, lk = lane >> 4;
    // Addresses: a wave-uniform base (scalar registers, one per k-step) plus
    // one 32-bit lane byte offset (16 rows x 4 columns).
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const bool rows_full = row0 + 16 <= mrows;
    const bool rowok = row0 + li < mrows;
    double *Qw = Q + row0;
    const int64_t ldq4 = 4 * ldq;                                          // doubles per k-step
    const uint32_t loff = ((uint32_t)li + (uint32_t)lk * (uint32_t)ldq) * 8u;  // lane offset in bytes
    const int64_t nsweeps = n - 2;
    const int64_t nsteps = bc_num_steps(n, B);

    // the staircase keeps its zeros: only band positions are ever written
    for (int e = tid; e < 2 * W * LDY; e += 256) (&Ys[0][0][0])[e] = 0.0;
    __syncthreads();

    // a group's operands are fetched into registers before the current group
    // is applied and written to LDS after it, so the fetch latency overlaps
    // the matrix-core work.  The vectors of sweeps c0 .. c0 + G - 1 at step s
    // are G B consecutive doubles of V.
    constexpr int NV = G * B / 256, NT = G * G / 256;
    double gv[NV], gt[NT];
    auto fetch_group = [&](int64_t blk, int64_t s) {
        const int64_t c0 = blk * G;
        const double *Vg = V + (s * n + c0) * B;
        if (c0 + G <= nsweeps && s < nsteps) {
#pragma unroll
            for (int r = 0; r < NV; ++r) gv[r] = Vg[tid + r * 256];
        } else {
#pragma unroll
            for (int r = 0; r < NV; ++r) {
                const int e = tid + r * 256;
                gv[r] = (c0 + e / B < nsweeps && s < nsteps) ? Vg[e] : 0.0;
            }
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
        {
            const double *Qc = Qw + base * ldq;
            if (rows_full && base + W <= n) {
#pragma unroll
                for (int kk = 0; kk < KW; ++kk) x[kk] = at(Qc + kk * ldq4, loff);
            } else {
#pragma unroll
                for (int kk = 0; kk < KW; ++kk) {
                    const int64_t col = base + 4 * kk + lk;
                    x[kk] = (rowok && col < n) ? at(Qc + kk * ldq4, loff) : 0.0;
                }
            }
        }
        __syncthreads();
        fetch_group(blk, REV ? 0 : S - 1);
        store_group(0);
        __syncthreads();
        int buf = 0;
        for (int64_t it = 0; it < S; ++it) {
            const int64_t s = REV ? it : S - 1 - it;
            const bool more = it + 1 < S;
            // every column the step reads, writes or prefetches is below n
            const bool full = rows_full && base + W + B <= n;
            if (more) {
                const int64_t pcol = REV ? base + W : base - B;
                const double *Qc = Qw + pcol * ldq;
                if (full) {
#pragma unroll
                    for (int k = 0; k < SHK; ++k) pre[k] = at(Qc + k * ldq4, loff);
                } else {
#pragma unroll
                    for (int k = 0; k < SHK; ++k) {
                        const int64_t col = pcol + 4 * k + lk;
                        pre[k] = (rowok && col < n) ? at(Qc + k * ldq4, loff) : 0.0;
                    }
                }
                fetch_group(blk, REV ? s + 1 : s - 1);
            }
            // The three products are written k-step outer, output tile inner,
            // so that consecutive matrix-core instructions are independent.
            // P = Q_w Y: reflector tile jt meets window k-steps 4 jt .. 4 jt + B/4 + 3;
            // even and odd k-steps go to separate accumulators.
            double4_t P[2], Po[2];
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) {
                P[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
                Po[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
            }
#pragma unroll
            for (int kk = 0; kk < KW; ++kk) {
#pragma unroll
                for (int jt = 0; jt < 2; ++jt) {
                    if (kk >= 4 * jt && kk < 4 * jt + SHK + 4) {
                        const double a = Ys[buf][4 * kk + lk][16 * jt + li];
                        if (kk & 1) Po[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, x[kk], Po[jt], 0, 0, 0);
                        else P[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, x[kk], P[jt], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) P[jt] += Po[jt];
            // P2 = P (-T) (upper) or P (-T)^T (REV); the stored factors are -T
            double4_t P2[2];
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) P2[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
                for (int jt = 0; jt < 2; ++jt) {
                    const bool nz = REV ? (kk >= 4 * jt) : (kk <= 4 * jt + 3);
                    if (nz) {
                        const double a = REV ? Ts[buf][16 * jt + li][4 * kk + lk] : Ts[buf][4 * kk + lk][16 * jt + li];
                        P2[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, P[kk / 4][kk % 4], P2[jt], 0, 0, 0);
                    }
                }
            }
            // Q_w += P2 Y^T: window tile t meets reflectors 16 t - (B - 1) .. 16 t + 15
            double4_t acc[KW / 4];
#pragma unroll
            for (int t = 0; t < KW / 4; ++t) acc[t] = (double4_t){x[4 * t], x[4 * t + 1], x[4 * t + 2], x[4 * t + 3]};
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
                for (int t = 0; t < KW / 4; ++t) {
                    const int jlo = 4 * kk, jhi = 4 * kk + 3;
                    if (jhi >= 16 * t - (B - 1) && jlo <= 16 * t + 15)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ys[buf][16 * t + li][4 * kk + lk],
                                                                      P2[kk / 4][kk % 4], acc[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < KW / 4; ++t) {
                x[4 * t] = acc[t][0];
                x[4 * t + 1] = acc[t][1];
                x[4 * t + 2] = acc[t][2];
                x[4 * t + 3] = acc[t][3];
            }
            if (more) {
                store_group(buf ^ 1);
                if (REV) {
                    // the first B columns leave the window
                    double *Qc = Qw + base * ldq;
                    if (full) {
#pragma unroll
                        for (int kk = 0; kk < SHK; ++kk) at(Qc + kk * ldq4, loff) = x[kk];
                    } else {
#pragma unroll
                        for (int kk = 0; kk < SHK; ++kk) {
                            const int64_t col = base + 4 * kk + lk;
                            if (rowok && col < n) at(Qc + kk * ldq4, loff) = x[kk];
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < KW - SHK; ++kk) x[kk] = x[kk + SHK];
#pragma unroll
                    for (int k = 0; k < SHK; ++k) x[KW - SHK + k] = pre[k];
                    base += B;
                } else {
                    // the last B columns leave the window
                    double *Qc = Qw + (base + W - B) * ldq;
                    if (full) {
#pragma unroll
                        for (int kk = 0; kk < SHK; ++kk) at(Qc + kk * ldq4, loff) = x[KW - SHK + kk];
                    } else {
#pragma unroll
                        for (int kk = 0; kk < SHK; ++kk) {
                            const int64_t col = base + W - B + 4 * kk + lk;
                            if (rowok && col < n) at(Qc + kk * ldq4, loff) = x[KW - SHK + kk];
                        }
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
        {
            double *Qc = Qw + base * ldq;
            if (rows_full && base + W <= n) {
#pragma unroll
                for (int kk = 0; kk < KW; ++kk) at(Qc + kk * ldq4, loff) = x[kk];
            } else {
#pragma unroll
                for (int kk = 0; kk < KW; ++kk) {
                    const int64_t col = base + 4 * kk + lk;
                    if (rowok && col < n) at(Qc + kk * ldq4, loff) = x[kk];
                }
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Wide groups for b = 64: GW = 64 sweeps per group.  The window slides by b
// columns per step whatever the group size, so the rows of Q streamed through
// HBM per unit of reflector work halve against 32-sweep groups (the 32-sweep
// kernel is bound by exactly that stream).  LDS holds the group's vectors
// packed, one padded row per sweep (16 zeros between rows, so the staircase
// reads Y(r, c) = v_c[r - c] fall on zeros outside 0 <= r - c < b without
// masking), and -T (or -T^T for the reverse order) as its nonzero 16 x 4
// tiles, each stored in the lane order of the matrix-core operand.
constexpr int BC_GW = 64;
constexpr int B_MAX_WIDE = 64;  // band widths the wide-group T kernel accepts

template <int G>
__host__ __device__ constexpr int wide_tiles() { return (G / 16) * (G / 4) - 2 * (G / 16) * (G / 16 - 1); }

// position of tile (jt, kk) among the nonzero tiles of M = -T (upper: kk <= 4 jt + 3)
// or M = -T^T (REV, lower: kk >= 4 jt), jt outer
template <int G, bool REV>
__host__ __device__ constexpr int wide_tile(int jt, int kk)
{
    return REV ? jt * (G / 4) - 2 * jt * (jt - 1) + kk - 4 * jt : 2 * jt * (jt + 1) + kk;
}

// -T (or -T^T) of every wide group in tile order: tile (jt, kk), lane l holds
// M(4 kk + l / 16, 16 jt + l % 16).  One workgroup per group.
template <int G, bool REV>
__global__ __launch_bounds__(256) void bct_wide_kernel(int64_t n, int B, const double *__restrict__ V,
                                                       const double *__restrict__ TAU, double *__restrict__ Tg,
                                                       int64_t nblk)
{
    constexpr int NTT = wide_tiles<G>();
    static_assert(B_MAX_WIDE + 1 >= G + 1, "T shares the vectors' LDS");
    __shared__ double vsh[G][B_MAX_WIDE + 1];  // the vectors, then (after the Gram matrix) T
    __shared__ double gsh[G][G + 1];
    __shared__ double tau[G];
    double (*tsh)[B_MAX_WIDE + 1] = vsh;
    const int64_t blk = blockIdx.x, s = blockIdx.y;
    const int64_t nsweeps = n - 2, nsteps = bc_num_steps(n, B);
    const int tid = threadIdx.x;
    {
        const int64_t rem = n - 1 - (blk * G + 1);
        const int64_t S = rem < 0 ? 0 : rem / B + 1;
        if (s >= S) return;
    }
    for (int e = tid; e < G * B; e += 256) {
        const int j = e / B, i = e % B;
        const int64_t c = blk * G + j;
        vsh[j][i] = (c < nsweeps && s < nsteps) ? V[((s * n) + c) * B + i] : 0.0;
    }
    for (int j = tid; j < G; j += 256) {
        const int64_t c = blk * G + j;
        tau[j] = (c < nsweeps && s < nsteps) ? TAU[s * n + c] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < G * G; e += 256) {
        const int i = e / G, j = e % G;
        if (i < j) {
            const int d = j - i;
            double acc = 0.0;
            for (int t = 0; t + d < B; ++t) acc += vsh[i][t + d] * vsh[j][t];
            gsh[i][j] = acc;
        }
    }
    __syncthreads();
    for (int e = tid; e < G * (B_MAX_WIDE + 1); e += 256) (&tsh[0][0])[e] = 0.0;
    __syncthreads();
    // column j: row p of -tau_j T[0:j, 0:j] g[0:j, j] split over 4 adjacent threads
    for (int j = 0; j < G; ++j) {
        const int p = tid >> 2, u = tid & 3;
        double acc = 0.0;
        if (p < j)
            for (int k = p + u; k < j; k += 4) acc += tsh[p][k] * gsh[k][j];
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (p < j && u == 0) tsh[p][j] = -tau[j] * acc;
        if (tid == 0) tsh[j][j] = tau[j];
        __syncthreads();
    }
    double *T = Tg + (s * nblk + blk) * (int64_t)(NTT * 64);
    for (int jt = 0; jt < G / 16; ++jt) {
        const int k0 = REV ? 4 * jt : 0, k1 = REV ? G / 4 : 4 * jt + 4;
        for (int e = tid; e < (k1 - k0) * 64; e += 256) {
            const int kk = k0 + e / 64, l = e % 64;
            const int r = 4 * kk + l / 16, c = 16 * jt + l % 16;  // M(r, c)
            T[wide_tile<G, REV>(jt, kk) * 64 + l] = REV ? -tsh[c][r] : -tsh[r][c];
        }
    }
}

// SG > 0: the G sweeps of a group are applied as G/SG block reflectors of
// SG consecutive sweeps, one after another (ascending sweeps; descending for
// the reverse product), each with its own T: the diagonal SG x SG block of
// the group's T (the forward recurrence of T restricted to the block's
// columns), so the off-diagonal T blocks are never multiplied.  At B = 64,
// G = 64: SG = 16 issues 176 MFMAs per 16 rows and step, SG = 32 184, the
// whole group (SG = 0) 200, but each block reflector must wait for the
// previous one's update of the window.
//
// RT: tiles of 16 rows per wavefront.  With RT = 2 every LDS operand (a
// fragment of Y or of T) feeds two MFMAs, one per row tile, and a wavefront
// carries two independent accumulation chains, so one wavefront per SIMD
// keeps the matrix core fed without a second wavefront to cover LDS latency
// (and the register file of a SIMD holds the two windows of one wavefront).
template <int B, int G, int NWV, bool REV, int SG, int RT, int NB, int MINB>
__global__ __launch_bounds__(NWV * 64, MINB) void bcback_wide_kernel(int64_t mrows, int64_t n,
                                                                  const double *__restrict__ V,
                                                                  const double *__restrict__ Tg, int64_t nblk,
                                                                  double *__restrict__ Q, int64_t ldq)
{
    static_assert(RT == 1 || SG > 0, "several row tiles per wavefront need block reflectors");
    constexpr int W = G + B;      // window columns
    constexpr int KW = W / 4;     // k-steps over the window
    constexpr int SHK = B / 4;    // k-steps the window slides per step
    constexpr int JT = G / 16;    // reflector tiles
    constexpr int GK = G / 4;     // k-steps over the reflectors
    constexpr int WT = W / 16;    // window tiles
    constexpr int LDV = B + 16;   // padded row of one sweep's vector
    constexpr int VPAD = 16;
    constexpr int VS = VPAD + G * LDV;
    constexpr int NTT = wide_tiles<G>();
    constexpr int TS = NTT * 64;
    constexpr int NTH = NWV * 64;
    constexpr int NV = G * B / NTH, NT = TS / NTH;
    constexpr int RW = 16 * RT;   // rows per wavefront
    static_assert(W % 16 == 0 && (G * B) % NTH == 0 && TS % NTH == 0, "tile shapes");
    static_assert(NB == 1 || NB == 2, "LDS buffers");
    __shared__ double Vs[NB][VS];
    __shared__ double Ts[NB][TS];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // Two wavefronts share a SIMD, and the barrier at the end of every step
    // lines them up, so their load-issue phases would coincide and leave the
    // matrix core idle.  The upper half of the wavefronts issues its loads
    // after the first block reflector instead of at the start of the step,
    // while the lower half is already multiplying.
    const bool late = SG > 0 && NWV >= 8 && (wave & (NWV / 2)) != 0;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * (RW * NWV) + wave * RW;
    const bool rows_full = row0 + RW <= mrows;
    bool rowok[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) rowok[r] = row0 + 16 * r + li < mrows;
    double *Qw = Q + row0;
    const int64_t ldq4 = 4 * ldq;
    const uint32_t loff = ((uint32_t)li + (uint32_t)lk * (uint32_t)ldq) * 8u;
    const int64_t nsweeps = n - 2;

    for (int e = tid; e < NB * VS; e += NTH) (&Vs[0][0])[e] = 0.0;
    __syncthreads();

    double gv[NV], gt[NT];
    // buffer loads over the group's vectors (G x B, the sweeps past the last
    // one of a ragged last group fall outside the descriptor and read as zero)
    // and its T tiles
    auto fetch_group = [&](int64_t blk, int64_t s) {
        const int64_t c0 = blk * G;
        const int64_t nvalid = (c0 + G <= nsweeps) ? G : nsweeps - c0;
        const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(V + (s * n + c0) * B), (short)0, (int)(nvalid * B * 8), (int)EVD_BUF_DWORD3);
        const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(Tg + (s * nblk + blk) * (int64_t)TS), (short)0, (int)(TS * 8), (int)EVD_BUF_DWORD3);
#pragma unroll
        for (int r = 0; r < NV; ++r)
            gv[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, tid * 8, r * NTH * 8, 0));
#pragma unroll
        for (int r = 0; r < NT; ++r)
            gt[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rt, tid * 8, r * NTH * 8, 0));
    };
    auto store_group = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NV; ++r) {
            const int e = tid + r * NTH, j = e / B, i = e % B;
            Vs[buf][VPAD + j * LDV + i] = gv[r];
        }
#pragma unroll
        for (int r = 0; r < NT; ++r) Ts[buf][tid + r * NTH] = gt[r];
    };
    // Y(r, c) of the group in buffer buf: window row r, reflector c
    auto yv = [&](int buf, int r, int c) -> double { return Vs[buf][VPAD + c * LDV + (r - c)]; };

    double x[RT][KW];
    double pre[RT][SHK];
    const int64_t blk_first = REV ? nblk - 1 : 0;
    for (int64_t blk = blk_first; REV ? blk >= 0 : blk < nblk; blk += REV ? -1 : 1) {
        const int64_t c0 = blk * G;
        const int64_t rem = n - 1 - (c0 + 1);
        const int64_t S = rem < 0 ? 0 : rem / B + 1;
        if (S == 0) continue;
        int64_t base = REV ? c0 + 1 : c0 + 1 + (S - 1) * B;
        {
            const bool wfull = rows_full && base + W <= n;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const double *Qc = Qw + 16 * r + base * ldq;
                if (wfull) {
#pragma unroll
                    for (int kk = 0; kk < KW; ++kk, Qc += ldq4) x[r][kk] = at(Qc, loff);
                } else {
#pragma unroll
                    for (int kk = 0; kk < KW; ++kk) {
                        const int64_t col = base + 4 * kk + lk;
                        x[r][kk] = (rowok[r] && col < n) ? at(Qc + kk * ldq4, loff) : 0.0;
                    }
                }
            }
        }
        __syncthreads();
        fetch_group(blk, REV ? 0 : S - 1);
        store_group(0);
        __syncthreads();
        int buf = 0;
        for (int64_t it = 0; it < S; ++it) {
            const int64_t s = REV ? it : S - 1 - it;
            const bool more = it + 1 < S;
            const bool full = rows_full && base + W + B <= n;
            // next window columns (pre) and next group (Y, T) into registers
            auto issue_loads = [&]() {
                if (more) {
                    const int64_t pcol = REV ? base + W : base - B;
#pragma unroll
                    for (int r = 0; r < RT; ++r) {
                        const double *Qc = Qw + 16 * r + pcol * ldq;
                        if (full) {
                            const __amdgpu_buffer_rsrc_t rs = window_rsrc(Qc, SHK, ldq4);
#pragma unroll
                            for (int k = 0; k < SHK; ++k) pre[r][k] = window_load(rs, loff, k, ldq4);
                        } else {
#pragma unroll
                            for (int k = 0; k < SHK; ++k) {
                                const int64_t col = pcol + 4 * k + lk;
                                pre[r][k] = (rowok[r] && col < n) ? at(Qc + k * ldq4, loff) : 0.0;
                            }
                        }
                    }
                }
                if constexpr (SG > 0) {
                    if (more) fetch_group(blk, REV ? s + 1 : s - 1);
                }
            };
            if (!late) issue_loads();
            if constexpr (SG > 0) {
                constexpr int ST = SG / 16;   // reflector tiles per block reflector
#pragma unroll
                for (int ii = 0; ii < G / SG; ++ii) {
                    const int i = REV ? G / SG - 1 - ii : ii;
                    const int j0 = i * ST;   // first reflector tile of the block
                    // P = Q_w Y_i: tile jt meets window k-steps 4 jt .. 4 jt + B/4 + 3
                    // (one tile: two accumulators, so consecutive products are independent)
                    double4_t pa[RT][ST], pb[RT][ST];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int u = 0; u < ST; ++u) pa[r][u] = pb[r][u] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int kk = 4 * j0; kk < 4 * (j0 + ST - 1) + SHK + 4; ++kk) {
#pragma unroll
                        for (int u = 0; u < ST; ++u) {
                            const int jt = j0 + u;
                            if (kk >= 4 * jt && kk < 4 * jt + SHK + 4) {
                                const double ya = yv(buf, 4 * kk + lk, 16 * jt + li);
#pragma unroll
                                for (int r = 0; r < RT; ++r) {
                                    if (ST == 1 && (kk & 1))
                                        pb[r][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya, x[r][kk], pb[r][u], 0, 0, 0);
                                    else
                                        pa[r][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya, x[r][kk], pa[r][u], 0, 0, 0);
                                }
                            }
                        }
                    }
                    double4_t p1[RT][ST];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int u = 0; u < ST; ++u)
                            p1[r][u] = (ST == 1) ? pa[r][u] + pb[r][u] : pa[r][u];  // pb is used only when ST == 1
                    // P M_i, M_i the diagonal block of -T (upper) or -T^T (lower)
                    double4_t qa[RT][ST], qb[RT][ST];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int u = 0; u < ST; ++u) qa[r][u] = qb[r][u] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int kk = 4 * j0; kk < 4 * (j0 + ST); ++kk) {
#pragma unroll
                        for (int u = 0; u < ST; ++u) {
                            const int jt = j0 + u;
                            const bool nz = REV ? (kk >= 4 * jt) : (kk <= 4 * jt + 3);
                            if (nz) {
                                const double m = Ts[buf][wide_tile<G, REV>(jt, kk) * 64 + lane];
#pragma unroll
                                for (int r = 0; r < RT; ++r) {
                                    if (ST == 1 && (kk & 1))
                                        qb[r][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(m, p1[r][kk / 4 - j0][kk % 4],
                                                                                        qb[r][u], 0, 0, 0);
                                    else
                                        qa[r][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(m, p1[r][kk / 4 - j0][kk % 4],
                                                                                        qa[r][u], 0, 0, 0);
                                }
                            }
                        }
                    }
                    double4_t p2[RT][ST];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int u = 0; u < ST; ++u) p2[r][u] = (ST == 1) ? qa[r][u] + qb[r][u] : qa[r][u];
                    // Q_w += (P M_i) Y_i^T: window tile t meets reflectors 16 t - (B - 1) .. 16 t + 15
#pragma unroll
                    for (int kk = 4 * j0; kk < 4 * (j0 + ST); ++kk) {
#pragma unroll
                        for (int t = j0; t < j0 + ST + B / 16; ++t) {
                            if (4 * kk + 3 >= 16 * t - (B - 1) && 4 * kk <= 16 * t + 15) {
                                const double ya = yv(buf, 16 * t + li, 4 * kk + lk);
#pragma unroll
                                for (int r = 0; r < RT; ++r) {
                                    double4_t a = (double4_t){x[r][4 * t], x[r][4 * t + 1], x[r][4 * t + 2], x[r][4 * t + 3]};
                                    a = __builtin_amdgcn_mfma_f64_16x16x4f64(ya, p2[r][kk / 4 - j0][kk % 4], a, 0, 0, 0);
                                    x[r][4 * t] = a[0];
                                    x[r][4 * t + 1] = a[1];
                                    x[r][4 * t + 2] = a[2];
                                    x[r][4 * t + 3] = a[3];
                                }
                            }
                        }
                    }
                    if (late && ii == 0) issue_loads();
                }
            } else {
            // P = Q_w Y: reflector tile jt meets window k-steps 4 jt .. 4 jt + B/4 + 3
            double4_t P[JT];
#pragma unroll
            for (int jt = 0; jt < JT; ++jt) P[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KW; ++kk) {
#pragma unroll
                for (int jt = 0; jt < JT; ++jt) {
                    if (kk >= 4 * jt && kk < 4 * jt + SHK + 4)
                        P[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv(buf, 4 * kk + lk, 16 * jt + li), x[0][kk], P[jt],
                                                                     0, 0, 0);
                }
            }
            // P2 = P M, M = -T (upper) or -T^T (REV), from the stored tiles
            double4_t P2[JT];
#pragma unroll
            for (int jt = 0; jt < JT; ++jt) P2[jt] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < GK; ++kk) {
#pragma unroll
                for (int jt = 0; jt < JT; ++jt) {
                    const bool nz = REV ? (kk >= 4 * jt) : (kk <= 4 * jt + 3);
                    if (nz)
                        P2[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ts[buf][wide_tile<G, REV>(jt, kk) * 64 + lane],
                                                                      P[kk / 4][kk % 4], P2[jt], 0, 0, 0);
                }
            }
            // the next group's operands are fetched once P is dead (register
            // pressure) and land during the third product
            if (more) fetch_group(blk, REV ? s + 1 : s - 1);
            // Q_w += P2 Y^T: window tile t meets reflectors 16 t - (B - 1) .. 16 t + 15
            double4_t acc[WT];
#pragma unroll
            for (int t = 0; t < WT; ++t) acc[t] = (double4_t){x[0][4 * t], x[0][4 * t + 1], x[0][4 * t + 2], x[0][4 * t + 3]};
#pragma unroll
            for (int kk = 0; kk < GK; ++kk) {
#pragma unroll
                for (int t = 0; t < WT; ++t) {
                    if (4 * kk + 3 >= 16 * t - (B - 1) && 4 * kk <= 16 * t + 15)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv(buf, 16 * t + li, 4 * kk + lk),
                                                                      P2[kk / 4][kk % 4], acc[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < WT; ++t) {
                x[0][4 * t] = acc[t][0];
                x[0][4 * t + 1] = acc[t][1];
                x[0][4 * t + 2] = acc[t][2];
                x[0][4 * t + 3] = acc[t][3];
            }
            }  // SG == 0
            if (more) {
                if constexpr (NB == 2) store_group(buf ^ 1);
                if (REV) {
#pragma unroll
                    for (int r = 0; r < RT; ++r) {
                        double *Qc = Qw + 16 * r + base * ldq;
                        if (full) {
                            const __amdgpu_buffer_rsrc_t rs = window_rsrc(Qc, SHK, ldq4);
#pragma unroll
                            for (int kk = 0; kk < SHK; ++kk) window_store(rs, loff, kk, ldq4, x[r][kk]);
                        } else {
#pragma unroll
                            for (int kk = 0; kk < SHK; ++kk) {
                                const int64_t col = base + 4 * kk + lk;
                                if (rowok[r] && col < n) at(Qc + kk * ldq4, loff) = x[r][kk];
                            }
                        }
#pragma unroll
                        for (int kk = 0; kk < KW - SHK; ++kk) x[r][kk] = x[r][kk + SHK];
#pragma unroll
                        for (int k = 0; k < SHK; ++k) x[r][KW - SHK + k] = pre[r][k];
                    }
                    base += B;
                } else {
#pragma unroll
                    for (int r = 0; r < RT; ++r) {
                        double *Qc = Qw + 16 * r + (base + W - B) * ldq;
                        if (full) {
                            const __amdgpu_buffer_rsrc_t rs = window_rsrc(Qc, SHK, ldq4);
#pragma unroll
                            for (int kk = 0; kk < SHK; ++kk) window_store(rs, loff, kk, ldq4, x[r][KW - SHK + kk]);
                        } else {
#pragma unroll
                            for (int kk = 0; kk < SHK; ++kk) {
                                const int64_t col = base + W - B + 4 * kk + lk;
                                if (rowok[r] && col < n) at(Qc + kk * ldq4, loff) = x[r][KW - SHK + kk];
                            }
                        }
#pragma unroll
                        for (int kk = KW - 1; kk >= SHK; --kk) x[r][kk] = x[r][kk - SHK];
#pragma unroll
                        for (int k = 0; k < SHK; ++k) x[r][k] = pre[r][k];
                    }
                    base -= B;
                }
            }
            if constexpr (NB == 1) {
                // one buffer: the next group is stored once every wavefront
                // has finished reading the current one
                if (more) {
                    __syncthreads();
                    store_group(0);
                }
                __syncthreads();
            } else {
                __syncthreads();
                buf ^= 1;
            }
        }
        {
            const bool wfull = rows_full && base + W <= n;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                double *Qc = Qw + 16 * r + base * ldq;
                if (wfull) {
#pragma unroll
                    for (int kk = 0; kk < KW; ++kk, Qc += ldq4) at(Qc, loff) = x[r][kk];
                } else {
#pragma unroll
                    for (int kk = 0; kk < KW; ++kk) {
                        const int64_t col = base + 4 * kk + lk;
                        if (rowok[r] && col < n) at(Qc + kk * ldq4, loff) = x[r][kk];
                    }
                }
            }
        }
    }
}

}  // namespace

namespace {

int64_t group_count(int64_t n, int g) { return n > 2 ? evd_ceil_div(n - 2, (int64_t)g) : 0; }

// sweeps per group: 64 for b = 64 unless "bcback_group" asks for 32
int group_sweeps(evd_ctx_t ctx, int64_t b) { return (b == 64 && ctx->bcback_group != 32) ? BC_GW : BC_G; }

size_t t_elems_for(int64_t n, int64_t b, int g)
{
    const size_t per = (g == BC_GW) ? (size_t)wide_tiles<BC_GW>() * 64 : (size_t)BC_G * BC_G;
    return (size_t)bc_num_steps(n, b) * (size_t)group_count(n, g) * per;
}

}  // namespace

// T workspace of the blocked BC-back (doubles, enough for either group size);
// 0 when the blocked kernels do not apply to b.
size_t bcback_mfma_t_elems(int64_t n, int64_t b)
{
    if (!(b == 16 || b == 32 || b == 64) || n < 3) return 0;
    const size_t t32 = t_elems_for(n, b, BC_G);
    const size_t t64 = (b == 64) ? t_elems_for(n, b, BC_GW) : 0;
    return t32 > t64 ? t32 : t64;
}

// T factors of every group into Tg (bcback_mfma_t_elems(n, b) doubles), laid
// out for the order (rev) that bcback_mfma_apply will use.
evd_status_t bcback_mfma_prepare(evd_ctx_t ctx, int64_t n, int64_t b, const double *V, const double *TAU, double *Tg,
                                 bool rev)
{
    if (n < 3) return EVD_OK;
    const int g = group_sweeps(ctx, b);
    const int64_t nblk = group_count(n, g);
    const int64_t nsteps = bc_num_steps(n, b);
    const dim3 grid((unsigned)nblk, (unsigned)nsteps);
    if (g == BC_GW) {
        if (rev) hipLaunchKernelGGL((bct_wide_kernel<BC_GW, true>), grid, dim3(256), 0, ctx->stream, n, (int)b, V, TAU,
                                    Tg, nblk);
        else hipLaunchKernelGGL((bct_wide_kernel<BC_GW, false>), grid, dim3(256), 0, ctx->stream, n, (int)b, V, TAU,
                                Tg, nblk);
    } else {
        hipLaunchKernelGGL(bct_kernel, grid, dim3(64), 0, ctx->stream, n, (int)b, V, TAU, Tg, nblk);
    }
    return evd_check_last();
}

// Q (mrows x n) <- Q H_1 ... H_m (rev = false) or Q H_m ... H_1 (rev = true),
// with the T factors from bcback_mfma_prepare (same b, rev and group size).
evd_status_t bcback_mfma_apply(evd_ctx_t ctx, int64_t mrows, int64_t n, int64_t b, const double *V, double *Q,
                               int64_t ldq, const double *Tg, bool rev)
{
    hipStream_t s = ctx->stream;
    if (n < 3 || mrows <= 0) return EVD_OK;
    if (!bcback_mfma_fits(ldq)) return EVD_ERR_INVALID_ARG;  // lane offsets are 32-bit byte offsets
    const int g = group_sweeps(ctx, b);
    const int64_t nblk = group_count(n, g);
    if (g == BC_GW) {
        // rows r0 .. r0 + rows - 1 with 128-row (two wavefronts per SIMD) or
        // 64-row workgroups, one workgroup per compute unit at a time
        // block reflectors of 32 sweeps by default (measured at n = 32768:
        // 1722 ms against 1776 ms for whole 64-sweep groups and 1859 ms for
        // 16-sweep blocks)
        const int sub = evd_choose_sub(ctx, n);
        // two 16-row tiles per wavefront (4 wavefronts, 128 rows) when block
        // reflectors are used and "bcback_rt" asks for it
        const bool rt2 = (sub == 16 || sub == 32) && ctx->bcback_rt == 2;
        // 64-row workgroups with one LDS buffer (61 KB), two per compute unit,
        // unless "bcback_lds2" asks for the double-buffered single one
        const bool one_buf = ctx->bcback_lds2 == 0;
        auto launch = [&](bool w8, int64_t r0, int64_t rows) {
            const dim3 grid((unsigned)evd_ceil_div(rows, w8 ? 128 : 64));
            double *Qr = Q + r0;
#define EVD_BCW(NW, RV, SB, R)                                                                                      \
    hipLaunchKernelGGL((bcback_wide_kernel<64, BC_GW, NW, RV, SB, R, 2, 1>), grid, dim3(NW * 64), 0, s, rows, n, V,  \
                       Tg, nblk, Qr, ldq)
#define EVD_BCW1(RV, SB)                                                                                             \
    hipLaunchKernelGGL((bcback_wide_kernel<64, BC_GW, 4, RV, SB, 1, 1, 2>), grid, dim3(256), 0, s, rows, n, V, Tg,   \
                       nblk, Qr, ldq)
#define EVD_BCW_SUB(NW, RV)                                                                                          \
    do {                                                                                                             \
        if (sub == 16) EVD_BCW(NW, RV, 16, 1);                                                                       \
        else if (sub == 32) EVD_BCW(NW, RV, 32, 1);                                                                  \
        else EVD_BCW(NW, RV, 0, 1);                                                                                  \
    } while (0)
#define EVD_BCW_RT2(RV)                                                                                              \
    do {                                                                                                             \
        if (sub == 16) EVD_BCW(4, RV, 16, 2);                                                                        \
        else EVD_BCW(4, RV, 32, 2);                                                                                  \
    } while (0)
            if (w8 && rt2) {
                if (rev) EVD_BCW_RT2(true);
                else EVD_BCW_RT2(false);
            } else if (w8) {
                if (rev) EVD_BCW_SUB(8, true);
                else EVD_BCW_SUB(8, false);
            } else if (one_buf && (sub == 16 || sub == 32)) {
                if (rev) {
                    if (sub == 16) EVD_BCW1(true, 16);
                    else EVD_BCW1(true, 32);
                } else {
                    if (sub == 16) EVD_BCW1(false, 16);
                    else EVD_BCW1(false, 32);
                }
            } else {
                if (rev) EVD_BCW_SUB(4, true);
                else EVD_BCW_SUB(4, false);
            }
#undef EVD_BCW1
#undef EVD_BCW_RT2
#undef EVD_BCW_SUB
#undef EVD_BCW
        };
        if (ctx->bcback_rows) {
            launch(ctx->bcback_rows == 128, 0, mrows);
        } else {
            // A round of 64-row workgroups over every compute unit takes about
            // 0.6 of a round of 128-row ones.  Whole rounds run with 128 rows;
            // a remainder of at most one round of 64-row workgroups runs as
            // such, a larger one as one more (partial) 128-row round.
            const int64_t per8 = (int64_t)128 * ctx->num_cus, per4 = (int64_t)64 * ctx->num_cus;
            const int64_t full = (mrows / per8) * per8, rem = mrows - full;
            if (rem == 0 || rem > per4) {
                launch(true, 0, mrows);
            } else {
                if (full > 0) launch(true, 0, full);
                launch(false, full, rem);
            }
        }
        return evd_check_last();
    }
    const dim3 grid((unsigned)evd_ceil_div(mrows, 64)), blk(256);
#define EVD_BCM(BB)                                                                                                   if (rev) hipLaunchKernelGGL((bcback_mfma_kernel<BB, true>), grid, blk, 0, s, mrows, n, V, (const double *)Tg,                                  nblk, Q, ldq);                                                                         else hipLaunchKernelGGL((bcback_mfma_kernel<BB, false>), grid, blk, 0, s, mrows, n, V, (const double *)Tg, nblk,                             Q, ldq);
    switch (b) {
    case 16: EVD_BCM(16) break;
    case 32: EVD_BCM(32) break;
    case 64: EVD_BCM(64) break;
    default: return EVD_ERR_INVALID_ARG;
    }
#undef EVD_BCM
    return evd_check_last();
}
