// Stage 1: successive band reduction (SBR), paper Section 2.1.1, Fig. 1, Eq. 1.
//
// For panel k (columns j0 = k b .. j0+b-1, rows i0 = j0+b .. n-1, m = n-i0):
//   1. panel QR  P_k = (I - Y T Y^T) R  (cooperative kernel below);
//   2. W = Y T;  X = A_2 W (A_2 kept in full storage, see below);
//      M = W^T X;  Z = X - 1/2 Y M                          (Eq. 1, first line)
//   3. A_2 <- A_2 - Y Z^T - Z Y^T                             (Eq. 1, second line)
// With double blocking (Section 4.1) the update of step 3 is deferred over an
// outer block of q panels: the accumulators hold [Y_0 Z_0 Y_1 Z_1 ...] and
// [Z_0 Y_0 Z_1 Y_1 ...], so any prefix of them is a consistent rank-2jb
// update; each panel's columns are brought up to date just before its QR,
// A_2 W is corrected for the deferred part, and one rank-2qb product per
// outer block updates the trailing matrix: its lower triangle is computed and
// every entry is stored in both triangles (the input is mirrored once at the
// start), so inside the next block every A_2 W reads the same stale full
// matrix with a plain (non-symmetric) product.
//
// Panel QR: the m x b panel is split into row chunks, one workgroup per chunk
// holding its rows in registers for the whole factorization.  Column j needs one
// chip-wide reduction: every workgroup publishes the partial sums
// h_q = sum_{i > j} P(i, j) P(i, q) for all q (its squared norm for q = j,
// the dot products with the remaining columns for q > j and with the finished
// reflectors for q < j), workgroup 0 adds row j; every workgroup waits for all
// records, sums them in the same fixed order (so all hold bitwise identical
// sums), forms the Householder vector and applies it to its rows.  Records
// cross workgroups through device-coherent accesses in a self-validating form
// (each 64-bit word carries the column's epoch, which grows across columns
// and panels; the buffer is cleared once per call), and they are double
// buffered by column parity: a workgroup can only start writing column j+2
// after every workgroup has published column j+1, i.e. has finished reading
// column j.  The T factor (forward, column-wise: T[0:j, j] = -tau_j T[0:j, 0:j]
// (Y[:, 0:j]^T v_j)) is formed at the end by workgroup 0 from the reduced
// Y^T v products.
#include "common.h"

namespace {

constexpr int PANEL_THREADS = 512;
constexpr int PANEL_MAX_WGS = 256;  // workgroups of one panel launch (at most)

// Panel partial-sum records cross workgroups in a self-validating form: every
// 64-bit word carries 32 data bits and the 32-bit epoch of the column it
// belongs to (a double takes two words, a float one), so a reader that sees
// its epoch in every word of an entry has the whole value, without a flag and
// without waiting for the writer's stores to drain.  64-bit device-coherent
// stores and loads are single-copy atomic.
template <typename T>
constexpr int LL_WORDS = sizeof(T) == 8 ? 2 : 1;
constexpr int LL_SPIN_MAX = 1 << 20;  // polls of an unwritten record before giving up (result poisoned)

// uint64 words of the record buffer: two column parities x PANEL_MAX_WGS
// records x 2b entries x (at most) two words
inline size_t panel_part_words(int64_t b) { return (size_t)2 * PANEL_MAX_WGS * 2 * (size_t)b * 2; }

__device__ __forceinline__ uint64_t ll_word(uint32_t bits, uint32_t epoch)
{
    return (uint64_t)bits | ((uint64_t)epoch << 32);
}
__device__ __forceinline__ uint32_t ll_epoch(uint64_t w) { return (uint32_t)(w >> 32); }

template <typename T>
__device__ __forceinline__ void ll_store(uint64_t *p, T v, uint32_t epoch)
{
    if constexpr (sizeof(T) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        st_coh(p, ll_word((uint32_t)b, epoch));
        st_coh(p + 1, ll_word((uint32_t)(b >> 32), epoch));
    } else {
        st_coh(p, ll_word(__builtin_bit_cast(uint32_t, v), epoch));
    }
}

template <typename T>
__device__ __forceinline__ T ll_value(const uint64_t (&w)[LL_WORDS<T>])
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, (uint64_t)(uint32_t)w[0] | ((uint64_t)(uint32_t)w[1] << 32));
    else
        return __builtin_bit_cast(T, (uint32_t)w[0]);
}

// one entry, polled until every word carries `epoch` (NaN, and *err raised,
// if it never does)
template <typename T>
__device__ __forceinline__ T ll_load(const uint64_t *p, uint32_t epoch, int *err)
{
    uint64_t w[LL_WORDS<T>];
#pragma unroll
    for (int q = 0; q < LL_WORDS<T>; ++q) w[q] = ld_coh(p + q);
    for (int it = 0; it < LL_SPIN_MAX; ++it) {
        bool ok = true;
#pragma unroll
        for (int q = 0; q < LL_WORDS<T>; ++q) {
            if (ll_epoch(w[q]) != epoch) {
                ok = false;
                w[q] = ld_coh(p + q);
            }
        }
        if (ok) return ll_value<T>(w);
        __builtin_amdgcn_s_sleep(1);
    }
    st_coh(err, 2);
    return (T)__builtin_nan("");
}

template <typename T>
__global__ void fill_kernel(T *p, int64_t count, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// A(i, j) <- A(j, i) for i > j  (mirror the stored upper triangle into the lower)
// A(j, i) <- A(i, j) for i > j on an m x m block (lower triangle -> upper),
// 32 x 32 tiles through LDS; tiles strictly above the diagonal exit.
template <typename T>
__global__ __launch_bounds__(256) void mirror_lower_kernel(int64_t m, T *A, int64_t lda)
{
    __shared__ T tile[32][33];
    const int64_t bi = (int64_t)blockIdx.x * 32, bj = (int64_t)blockIdx.y * 32;  // tile rows bi.., cols bj..
    if (bi < bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi + tx, j = bj + r;
        if (i < m && j < m && i > j) tile[r][tx] = A[i + j * lda];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bj + tx, j = bi + r;  // destination (i, j) = source (j, i)
        if (i < m && j < m && j > i) A[i + j * lda] = tile[tx][r];
    }
}

template <typename T>
__global__ void mirror_upper_kernel(int64_t n, T *A, int64_t lda)
{
    const int64_t j = blockIdx.y;
    for (int64_t i = j + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        A[i + j * lda] = A[j + i * lda];
}

// Copy the lower part of the diagonal blocks of the band into AB:
// column j of panel block kb = (j / b) b covers rows j .. min(kb + b, n) - 1;
// columns of the final (tail) block extend to row n - 1.
template <typename T>
__global__ void extract_diag_blocks_kernel(int64_t n, int64_t b, int64_t tail0, const T *A, int64_t lda, T *AB,
                                           int64_t ldab)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
    if (j >= n) return;
    int64_t limit = (j >= tail0) ? n : ((j / b) * b + b);
    if (limit > n) limit = n;
    for (int64_t d = threadIdx.x; j + d < limit; d += blockDim.x) AB[d + j * ldab] = A[j + d + j * lda];
}

// Band columns j0 .. j1-1 (their diagonal-block part, as above) copied with
// device-coherent stores by one workgroup, then the count of finished
// leading band columns published in *front for bulge chasing running beside
// SBR (after every store of the workgroup has completed).
template <typename T>
__global__ __launch_bounds__(256) void publish_band_kernel(int64_t n, int64_t b, int64_t j0, int64_t j1, int64_t tail0,
                                                           const T *A, int64_t lda, T *AB, int64_t ldab, int *front,
                                                           int value)
{
    for (int64_t j = j0 + threadIdx.y; j < j1; j += blockDim.y) {
        int64_t limit = (j >= tail0) ? n : ((j / b) * b + b);
        if (limit > n) limit = n;
        for (int64_t d = threadIdx.x; j + d < limit; d += blockDim.x) st_coh(&AB[d + j * ldab], A[j + d + j * lda]);
    }
    mem_drain();
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) st_coh(front, value);
}

// Thread layout of the panel kernel's column phases: column cq gets TPC =
// PANEL_THREADS / B threads; the first L = min(TPC, 64) of them are adjacent
// lanes of one wavefront (their partial sums meet through lane shuffles),
// and for narrow panels (TPC > 64) WPC = TPC / 64 wavefronts share a column.
template <int B>
struct PanelLayout {
    static constexpr int TPC = PANEL_THREADS / B;
    static constexpr int L = TPC < 64 ? TPC : 64;
    static constexpr int WPC = TPC / L;
    static __device__ __forceinline__ int col(int tid)
    {
        return (WPC == 1) ? (tid >> 6) * (64 / L) + (tid & 63) / L : (tid >> 6) / WPC;
    }
    static __device__ __forceinline__ int sub(int tid)
    {
        return (WPC == 1) ? (tid & 63) % L : (tid & 63) + 64 * ((tid >> 6) % WPC);
    }
};

// sum over the L adjacent lanes of a column (xor butterfly: every lane ends
// with the same bits, the additions being commutative pairwise)
template <int L, typename T>
__device__ __forceinline__ T lane_group_sum(T v)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Rows of one workgroup's slice of the panel: R rows per thread, held in
// registers (thread (sub, cq) holds rows sub, sub + TPC, ... of column cq).
template <int B>
struct PanelRows {
    static constexpr int TPC = PanelLayout<B>::TPC;
    static constexpr int CH = (64 * TPC < 2048) ? 64 * TPC : 2048;  // rows per workgroup at most
    static constexpr int R = CH / TPC;
};

template <int B, typename T>
__global__ __launch_bounds__(PANEL_THREADS) void panel_qr_kernel(int64_t m, int chunk, T *P, int64_t lda,
                                                                 T *Y1, T *Y2, int64_t ldy, T *part,
                                                                 T *Sg, T *taus, T *Tout,
                                                                 T *AB, int64_t ldab, int64_t j0, int epoch0,
                                                                 int *err)
{
    // Workgroup g holds rows r0 .. r0 + chunk - 1 of the m x B panel in
    // registers.  Per column j: (1) the owners of column j put it in LDS;
    // every thread forms its partial sums h_q = sum_{rows i > j} P(i, j) P(i, q)
    // for its column q; (2) the partial sums of all workgroups are combined
    // (through records in device memory when G > 1: entry q of record h,
    // LL_WORDS words from ((j & 1) * PANEL_MAX_WGS * 2B + h * 2B + q) *
    // LL_WORDS, holds workgroup h's sum for q < B and, for h = 0, row j of
    // the panel for B <= q < 2B, tagged with column j's epoch; every
    // workgroup sums all records in the same order, so all hold identical
    // sums); (3) every thread forms
    // the Householder scalars of column j and applies H_j to its own rows of
    // its column.  Columns stay unscaled (v_j = scale_j * P(:, j) below row j)
    // until the write-back.
    using LY = PanelLayout<B>;
    constexpr int TPC = LY::TPC, L = LY::L, WPC = LY::WPC;
    constexpr int CH = PanelRows<B>::CH, R = PanelRows<B>::R;
    constexpr int NWV = PANEL_THREADS / 64;
    // pivot column, local rows; two buffers, since the owners of column j + 1
    // write it while other wavefronts may still apply reflector j from column j
    __shared__ T colbuf2[2][CH];
    __shared__ T scr[PANEL_THREADS];    // partial sums being combined
    __shared__ T Ts[B * B];             // T factor (workgroup 0)
    __shared__ T hsh[B];
    __shared__ T topsh[B];
    __shared__ T scales[B];
    __shared__ T betas[B];

    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)g * chunk;
    const int rows = (int)((m - r0) < chunk ? (m - r0) : chunk);
    const int nr = (int)(m < B ? m : B);
    const int cq = LY::col(tid), sub = LY::sub(tid);

    T x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int i = sub + TPC * t;
        x[t] = (i < rows) ? P[(r0 + i) + (int64_t)cq * lda] : (T)0;
    }

    for (int j = 0; j < nr; ++j) {
        const int E = epoch0 + j + 1;
        uint64_t *rec = (uint64_t *)part + (size_t)(j & 1) * PANEL_MAX_WGS * 2 * B * LL_WORDS<T>;
        const int jl = (int)(j - r0);  // local index of row j (meaningful in workgroup 0)
        T *colbuf = colbuf2[j & 1];
        // ---- (1) pivot column to LDS, partial sums of column cq against it
        // (rows past the slice hold zeros in x, and so in colbuf: no row tests)
        if (cq == j) {
#pragma unroll
            for (int t = 0; t < R; ++t) colbuf[sub + TPC * t] = x[t];
        }
        __syncthreads();
        // only the first TB register rows can hold a row <= j (local rows
        // 0 .. B-1 of workgroup 0); the others are below j in every workgroup
        constexpr int TB = (B + TPC - 1) / TPC;
        T acc = 0.0, topv = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int i = sub + TPC * t;
            const T pr = colbuf[i] * x[t];
            if (t < TB) {
                acc += (i > jl) ? pr : (T)0;
                topv = (i == jl) ? x[t] : topv;
            } else {
                acc += pr;
            }
            if ((t & 15) == 15) __builtin_amdgcn_sched_barrier(0);  // bound the LDS reads in flight (registers)
        }
        acc = lane_group_sum<L>(acc);
        if (WPC > 1) {
            if (lane == 0) scr[cq * WPC + w % WPC] = acc;
            __syncthreads();
            acc = 0.0;
#pragma unroll
            for (int u = 0; u < WPC; ++u) acc += scr[cq * WPC + u];
        }
        const bool holds_row_j = (g == 0) && (jl % TPC == sub) && (jl < rows);
        if (G == 1) {
            if (sub == 0) hsh[cq] = acc;
            if (holds_row_j) topsh[cq] = topv;
        } else {
            // records in the self-validating form of ll_store: no flags and
            // no wait for the stores to land before others may read them
            if (sub == 0) ll_store(&rec[((size_t)g * 2 * B + cq) * LL_WORDS<T>], acc, (uint32_t)E);
            if (holds_row_j) ll_store(&rec[((size_t)B + cq) * LL_WORDS<T>], topv, (uint32_t)E);
            if (WPC > 1) __syncthreads();  // scr was just read by the column reduction
            // ---- (2) every record of this column, summed: wavefront w reads
            // records h = w, w + NWV, ... whole (lane q entry q, eight records
            // in flight, those not yet written polled again); the NWV partial
            // sums per entry are added in wavefront order
            if (lane < B) {
                T s2 = 0.0;
                for (int h0 = w; h0 < G; h0 += 8 * NWV) {
                    uint64_t wd[8][LL_WORDS<T>];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int h = h0 + u * NWV;
#pragma unroll
                        for (int q = 0; q < LL_WORDS<T>; ++q)
                            wd[u][q] = (h < G) ? ld_coh(&rec[((size_t)h * 2 * B + lane) * LL_WORDS<T> + q])
                                               : ll_word(0u, (uint32_t)E);
                    }
                    bool ok = false;
                    for (int it = 0; it < LL_SPIN_MAX && !ok; ++it) {
                        ok = true;
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int h = h0 + u * NWV;
#pragma unroll
                            for (int q = 0; q < LL_WORDS<T>; ++q) {
                                if (ll_epoch(wd[u][q]) != (uint32_t)E) {
                                    ok = false;
                                    wd[u][q] = ld_coh(&rec[((size_t)h * 2 * B + lane) * LL_WORDS<T> + q]);
                                }
                            }
                        }
                        if (!ok) __builtin_amdgcn_s_sleep(1);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) s2 += ll_value<T>(wd[u]);
                    if (!ok) {  // never written: poison, report, do not hang
                        s2 = (T)__builtin_nan("");
                        st_coh(err, 2);
                    }
                }
                scr[w * B + lane] = s2;
            }
            if (tid < B) topsh[tid] = ll_load<T>(&rec[((size_t)B + tid) * LL_WORDS<T>], (uint32_t)E, err);
            __syncthreads();
            if (tid < B) {
                T r = 0.0;
#pragma unroll
                for (int u = 0; u < NWV; ++u) r += scr[u * B + tid];
                hsh[tid] = r;
            }
        }
        __syncthreads();
        // ---- (3) Householder vector of column j: v = (x - beta e_j) / (x_j - beta)
        const T x0 = topsh[j], sig = hsh[j];
        T tau = 0.0, beta = x0, scale = 0.0;
        if (sig != 0.0) {
            const T nrm = sqrt(x0 * x0 + sig);
            beta = (x0 >= 0.0) ? -nrm : nrm;
            tau = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        if (tid == 0) {
            scales[j] = scale;
            betas[j] = beta;
            if (g == 0) taus[j] = tau;
        }
        // Y(:, q)^T v_j for q < j, with column q's own scale applied
        if (g == 0 && tid < j) Sg[tid + (int64_t)j * B] = scales[tid] * (topsh[tid] + scale * hsh[tid]);
        if (tau != 0.0 && cq > j) {
            // rows i >= j of column cq: P(i, cq) -= v_i tau (v_j^T P(:, cq))
            const T cf = tau * (topsh[cq] + scale * hsh[cq]);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int i = sub + TPC * t;
                const T v = (t >= TB) ? scale * colbuf[i] : ((i == jl) ? (T)1 : ((i > jl) ? scale * colbuf[i] : (T)0));
                x[t] -= v * cf;
                if ((t & 15) == 15) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    __syncthreads();

    // ---- write back: explicit Y into the panel of A and into the two
    // accumulator slots of the outer block (the row index is recomputed
    // from an opaque copy, so the load's addresses are not kept alive in
    // registers across the column loop)
    int sub2 = sub;
    asm volatile("" : "+v"(sub2));
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int i = sub2 + TPC * t;
        if (i < rows) {
            const int64_t gi = r0 + i;
            T y = 0.0;
            if (cq < nr) y = (gi > cq) ? scales[cq] * x[t] : (gi == cq ? (T)1 : (T)0);
            P[gi + (int64_t)cq * lda] = y;
            Y1[gi + (int64_t)cq * ldy] = y;
            Y2[gi + (int64_t)cq * ldy] = y;
        }
    }
    if (g != 0) return;
    // R (upper trapezoid of the first nr rows) -> band storage
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int p = sub + TPC * t;
        if (p < B && p <= cq) {
            const T v = (p >= nr) ? (T)0 : ((p == cq) ? betas[cq] : x[t]);
            AB[(B + p - cq) + (j0 + cq) * ldab] = v;
        }
    }
    // T factor in LDS, then out
    for (int e = tid; e < B * B; e += PANEL_THREADS) Ts[e] = 0.0;
    __syncthreads();
    // column j: T[0:j, j] = -tau_j T[0:j, 0:j] Sg[0:j, j]; row p of the
    // product is split over the TPC adjacent threads of row p (TPC <= 64)
    for (int j = 0; j < B; ++j) {
        const T tj = (j < nr) ? taus[j] : 0.0;
        if (TPC <= 64) {
            const int pr = tid / TPC, u = tid % TPC;
            T s = 0.0;
            if (pr < j)
                for (int r = pr + u; r < j; r += TPC) s += Ts[pr + r * B] * Sg[r + (int64_t)j * B];
            s = lane_group_sum<(TPC <= 64 ? TPC : 64)>(s);
            if (pr < j && u == 0) Ts[pr + j * B] = -tj * s;
        } else if (tid < j) {
            T s = 0.0;
            for (int r = tid; r < j; ++r) s += Ts[tid + r * B] * Sg[r + (int64_t)j * B];
            Ts[tid + j * B] = -tj * s;
        }
        if (tid == 0) Ts[j + j * B] = tj;
        __syncthreads();
    }
    for (int e = tid; e < B * B; e += PANEL_THREADS) Tout[e] = Ts[e];
}

// B = 64 with a column layout: wavefront w holds columns 8w .. 8w+7 of the
// workgroup's rows, lane l the rows l + 64 t (t < 8).  A wavefront's LDS read
// of the pivot column then touches 64 different rows (the layout above has
// eight lanes of a wavefront read each entry), and the entries a thread reads
// feed the products of its eight columns (and, read once more, their
// update).  A column's sum over the rows is a reduction across the wavefront:
// a reduce-scatter (exchanges with lanes 32, 16 and 8 apart, after which the
// lanes that agree in bits 3..5 hold one column each) and a butterfly over
// the last eight lanes.  The records, the Householder scalars, Y and T are
// formed as in panel_qr_kernel; only the order of the sums differs.
constexpr int P64_CPW = 8;    // columns per wavefront
constexpr int P64_RR = 8;     // rows per lane and column
constexpr int P64_CH = 64 * P64_RR;  // rows per workgroup at most

template <typename T>
__global__ __launch_bounds__(PANEL_THREADS) void panel_qr64_kernel(int64_t m, int chunk, T *P, int64_t lda,
                                                                   T *Y1, T *Y2, int64_t ldy, T *part,
                                                                   T *Sg, T *taus, T *Tout,
                                                                   T *AB, int64_t ldab, int64_t j0, int epoch0,
                                                                   int *err)
{
    constexpr int B = 64, NWV = PANEL_THREADS / 64, CPW = P64_CPW, RR = P64_RR;
    static_assert(NWV * CPW == B, "eight wavefronts of eight columns");
    __shared__ T colbuf2[2][P64_CH];
    __shared__ T scr[NWV * B];
    __shared__ T Ts[B * B];
    __shared__ T hsh[B];
    __shared__ T topsh[B];
    __shared__ T scales[B];
    __shared__ T betas[B];

    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)g * chunk;
    const int rows = (int)((m - r0) < chunk ? (m - r0) : chunk);
    const int nr = (int)(m < B ? m : B);
    // the column whose sum this lane holds after the reduction
    const int cl = 4 * ((lane >> 5) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 3) & 1);

    T x[CPW][RR];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int t = 0; t < RR; ++t) {
            const int i = lane + 64 * t;
            x[c][t] = (i < rows) ? P[(r0 + i) + (int64_t)(CPW * w + c) * lda] : (T)0;
        }

    for (int j = 0; j < nr; ++j) {
        const int E = epoch0 + j + 1;
        uint64_t *rec = (uint64_t *)part + (size_t)(j & 1) * PANEL_MAX_WGS * 2 * B * LL_WORDS<T>;
        const int jl = (int)(j - r0);  // local index of row j (0 .. 63 in workgroup 0, negative elsewhere)
        T *colbuf = colbuf2[j & 1];
        // ---- (1) pivot column to LDS; every thread reads its rows of it
        if (w == j / CPW) {
#pragma unroll
            for (int c = 0; c < CPW; ++c)
                if (c == j % CPW) {
#pragma unroll
                    for (int t = 0; t < RR; ++t) colbuf[lane + 64 * t] = x[c][t];
                }
        }
        __syncthreads();
        T pv[RR];
#pragma unroll
        for (int t = 0; t < RR; ++t) pv[t] = colbuf[lane + 64 * t];
        // rows <= j can only be local rows 0 .. 63 of workgroup 0 (t = 0)
        const T p0 = (lane > jl) ? pv[0] : (T)0;
        T acc[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            T a = p0 * x[c][0];
#pragma unroll
            for (int t = 1; t < RR; ++t) a += pv[t] * x[c][t];
            acc[c] = a;
        }
        // ---- reduce-scatter over the wavefront, then the last eight lanes
        T a4[4], a2[2];
        {
            const bool h = (lane & 32) != 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T send = h ? acc[k] : acc[k + 4];
                a4[k] = (h ? acc[k + 4] : acc[k]) + __shfl_xor(send, 32, 64);
            }
        }
        {
            const bool h = (lane & 16) != 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const T send = h ? a4[k] : a4[k + 2];
                a2[k] = (h ? a4[k + 2] : a4[k]) + __shfl_xor(send, 16, 64);
            }
        }
        T a1;
        {
            const bool h = (lane & 8) != 0;
            const T send = h ? a2[0] : a2[1];
            a1 = (h ? a2[1] : a2[0]) + __shfl_xor(send, 8, 64);
        }
        a1 += __shfl_xor(a1, 4, 64);
        a1 += __shfl_xor(a1, 2, 64);
        a1 += __shfl_xor(a1, 1, 64);
        const int q = CPW * w + cl;
        const bool holds_row_j = (g == 0) && (lane == jl) && (jl < rows);
        if (G == 1) {
            if ((lane & 7) == 0) hsh[q] = a1;
            if (holds_row_j) {
#pragma unroll
                for (int c = 0; c < CPW; ++c) topsh[CPW * w + c] = x[c][0];
            }
        } else {
            if ((lane & 7) == 0) ll_store(&rec[((size_t)g * 2 * B + q) * LL_WORDS<T>], a1, (uint32_t)E);
            if (holds_row_j) {
#pragma unroll
                for (int c = 0; c < CPW; ++c)
                    ll_store(&rec[((size_t)B + CPW * w + c) * LL_WORDS<T>], x[c][0], (uint32_t)E);
            }
            // ---- (2) every record of this column, summed: wavefront w reads
            // records h = w, w + NWV, ... whole (lane q entry q, eight records
            // in flight, those not yet written polled again); the NWV partial
            // sums per entry are added in wavefront order
            T s2 = 0.0;
            for (int h0 = w; h0 < G; h0 += 8 * NWV) {
                uint64_t wd[8][LL_WORDS<T>];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int h = h0 + u * NWV;
#pragma unroll
                    for (int k = 0; k < LL_WORDS<T>; ++k)
                        wd[u][k] = (h < G) ? ld_coh(&rec[((size_t)h * 2 * B + lane) * LL_WORDS<T> + k])
                                           : ll_word(0u, (uint32_t)E);
                }
                bool ok = false;
                for (int it = 0; it < LL_SPIN_MAX && !ok; ++it) {
                    ok = true;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int h = h0 + u * NWV;
#pragma unroll
                        for (int k = 0; k < LL_WORDS<T>; ++k) {
                            if (ll_epoch(wd[u][k]) != (uint32_t)E) {
                                ok = false;
                                wd[u][k] = ld_coh(&rec[((size_t)h * 2 * B + lane) * LL_WORDS<T> + k]);
                            }
                        }
                    }
                    if (!ok) __builtin_amdgcn_s_sleep(1);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s2 += ll_value<T>(wd[u]);
                if (!ok) {  // never written: poison, report, do not hang
                    s2 = (T)__builtin_nan("");
                    st_coh(err, 2);
                }
            }
            scr[w * B + lane] = s2;
            if (tid < B) topsh[tid] = ll_load<T>(&rec[((size_t)B + tid) * LL_WORDS<T>], (uint32_t)E, err);
            __syncthreads();
            if (tid < B) {
                T r = 0.0;
#pragma unroll
                for (int u = 0; u < NWV; ++u) r += scr[u * B + tid];
                hsh[tid] = r;
            }
        }
        __syncthreads();
        // ---- (3) Householder vector of column j: v = (x - beta e_j) / (x_j - beta)
        const T x0 = topsh[j], sig = hsh[j];
        T tau = 0.0, beta = x0, scale = 0.0;
        if (sig != 0.0) {
            const T nrm = sqrt(x0 * x0 + sig);
            beta = (x0 >= 0.0) ? -nrm : nrm;
            tau = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        if (tid == 0) {
            scales[j] = scale;
            betas[j] = beta;
            if (g == 0) taus[j] = tau;
        }
        // Y(:, q)^T v_j for q < j, with column q's own scale applied
        if (g == 0 && tid < j) Sg[tid + (int64_t)j * B] = scales[tid] * (topsh[tid] + scale * hsh[tid]);
        if (tau != 0.0) {
            // rows i >= j of column q > j: P(i, q) -= v_i tau (v_j^T P(:, q));
            // the pivot entries read again (not kept across the exchange:
            // registers)
            T v[RR];
#pragma unroll
            for (int t = 0; t < RR; ++t) v[t] = colbuf[lane + 64 * t];
            v[0] = (lane == jl) ? (T)1 : ((lane > jl) ? scale * v[0] : (T)0);
#pragma unroll
            for (int t = 1; t < RR; ++t) v[t] = scale * v[t];
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                const int qc = CPW * w + c;
                if (qc > j) {
                    const T cf = tau * (topsh[qc] + scale * hsh[qc]);
#pragma unroll
                    for (int t = 0; t < RR; ++t) x[c][t] -= v[t] * cf;
                }
            }
        }
    }
    __syncthreads();

    // ---- write back: explicit Y into the panel of A and into the two
    // accumulator slots of the outer block
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int qc = CPW * w + c;
#pragma unroll
        for (int t = 0; t < RR; ++t) {
            const int i = lane + 64 * t;
            if (i < rows) {
                const int64_t gi = r0 + i;
                T y = 0.0;
                if (qc < nr) y = (gi > qc) ? scales[qc] * x[c][t] : (gi == qc ? (T)1 : (T)0);
                P[gi + (int64_t)qc * lda] = y;
                Y1[gi + (int64_t)qc * ldy] = y;
                Y2[gi + (int64_t)qc * ldy] = y;
            }
        }
    }
    if (g != 0) return;
    // R (upper trapezoid of the first nr rows) -> band storage: row p = lane
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int qc = CPW * w + c;
        if (lane <= qc) {
            const T v = (lane >= nr) ? (T)0 : ((lane == qc) ? betas[qc] : x[c][0]);
            AB[(B + lane - qc) + (j0 + qc) * ldab] = v;
        }
    }
    // T factor in LDS, then out: column j: T[0:j, j] = -tau_j T[0:j, 0:j] Sg[0:j, j];
    // row p of the product split over the TPC adjacent threads of row p
    constexpr int TPC = PANEL_THREADS / B;
    for (int e = tid; e < B * B; e += PANEL_THREADS) Ts[e] = 0.0;
    __syncthreads();
    for (int j = 0; j < B; ++j) {
        const T tj = (j < nr) ? taus[j] : 0.0;
        const int pr = tid / TPC, u = tid % TPC;
        T s = 0.0;
        if (pr < j)
            for (int r = pr + u; r < j; r += TPC) s += Ts[pr + r * B] * Sg[r + (int64_t)j * B];
        s = lane_group_sum<TPC>(s);
        if (pr < j && u == 0) Ts[pr + j * B] = -tj * s;
        if (tid == 0) Ts[j + j * B] = tj;
        __syncthreads();
    }
    for (int e = tid; e < B * B; e += PANEL_THREADS) Tout[e] = Ts[e];
}

template <int B, typename T>
evd_status_t launch_panel(evd_ctx_t ctx, int64_t m, T *P, int64_t lda, T *Y1, T *Y2, int64_t ldy, T *part,
                          T *Sg, T *taus, T *Tout, T *AB, int64_t ldab, int64_t j0, int epoch0, int *err)
{
    // Automatic: as few workgroups as the registers allow (CH rows each):
    // every workgroup reads every record of a column, so the exchange grows
    // with G, and it costs more than the longer per-workgroup loops.  A cap
    // "panel_wgs" spreads the rows over about that many workgroups instead.
    // Workgroup 0 always holds rows 0 .. B-1.
    constexpr int TPC = PanelLayout<B>::TPC;
    constexpr int CH = PanelRows<B>::CH;
    int64_t chunk = CH;
    if (ctx->panel_wgs > 0) {
        chunk = evd_ceil_div(m, ctx->panel_wgs);
        if (chunk < B) chunk = B;
        chunk = evd_ceil_div(chunk, TPC) * TPC;
        if (chunk > CH) chunk = CH;
    }
    const int64_t G = evd_ceil_div(m, chunk);
    if (G > PANEL_MAX_WGS) return EVD_ERR_INVALID_ARG;  // m > PANEL_MAX_WGS * CH rows
    const size_t lds = 0;
    int chunk_i = (int)chunk;
    void *args[] = {&m, &chunk_i, &P, (void *)&lda, &Y1, &Y2, (void *)&ldy, &part, &Sg, &taus, &Tout, &AB,
                    (void *)&ldab, (void *)&j0, &epoch0, &err};
    // while bulge chasing runs beside SBR the panel is a plain launch (its at
    // most PANEL_MAX_WGS workgroups find free compute units: the previous
    // kernels of the stream have finished and bulge chasing holds at most
    // "bc_waves" of them); its record polls are bounded either way
    // B = 64: the column layout (chunk <= 512 rows always holds at B = 64)
    const void *kern = (const void *)panel_qr_kernel<B, T>;
    if constexpr (B == 64)
        if (!ctx->panel_generic && chunk <= P64_CH) kern = (const void *)panel_qr64_kernel<T>;
    hipError_t e = ctx->plain_panels
                       ? hipLaunchKernel(kern, dim3((unsigned)G), dim3(PANEL_THREADS), args, lds, ctx->stream)
                       : hipLaunchCooperativeKernel(kern, dim3((unsigned)G), dim3(PANEL_THREADS), args, (unsigned)lds,
                                                    ctx->stream);
    return evd_hip(ctx, e);
}

template <typename T>
evd_status_t panel_dispatch(evd_ctx_t ctx, int64_t b, int64_t m, T *P, int64_t lda, T *Y1, T *Y2, int64_t ldy, T *part,
                            T *Sg, T *taus, T *Tout, T *AB, int64_t ldab, int64_t j0, int epoch0,
                            int *err)
{
    switch (b) {
    case 1: return launch_panel<1, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    case 2: return launch_panel<2, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    case 4: return launch_panel<4, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    case 8: return launch_panel<8, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    case 16: return launch_panel<16, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    case 32: return launch_panel<32, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    case 64: return launch_panel<64, T>(ctx, m, P, lda, Y1, Y2, ldy, part, Sg, taus, Tout, AB, ldab, j0, epoch0, err);
    default: return EVD_ERR_INVALID_ARG;
    }
}

template <typename T>
struct SbrWork {
    T *YZ;    // [Y_0 Z_0 Y_1 Z_1 ...] of the outer block, n x 2nb
    T *ZY;    // [Z_0 Y_0 Z_1 Y_1 ...], n x 2nb
    T *W;     // n x b
    T *M;     // b x b
    T *U;     // 2nb x b
    T *part;  // partial-sum records of the panel kernel (uint64 words)
    T *Sg;    // b x b
    T *taus;  // b
    T *gemm_ws;
    size_t gemm_ws_elems;
    int64_t q;  // panels per outer block
};

// Outer block of SBR: SBR_NB columns by default (at least one panel); the
// accumulators are sized for up to SBR_NB_MAX ("sbr_nb" may ask for more).
constexpr int64_t SBR_NB = 320;
constexpr int64_t SBR_NB_MAX = 512;

inline int64_t sbr_panels_per_block(int64_t b) { return (SBR_NB_MAX / b) > 0 ? SBR_NB_MAX / b : 1; }

template <typename T>
size_t sbr_layout(int64_t n, int64_t b, char *base, SbrWork<T> *w)
{
    size_t off = 0;
    auto take = [&](size_t elems) {
        char *p = base ? base + off : nullptr;
        off += evd_align256((elems > 0 ? elems : 1) * sizeof(T));
        return (T *)p;
    };
    SbrWork<T> t;
    t.q = sbr_panels_per_block(b);
    const int64_t nb = t.q * b;
    t.YZ = take((size_t)n * 2 * nb);
    t.ZY = take((size_t)n * 2 * nb);
    t.W = take((size_t)n * b);
    t.M = take((size_t)b * b);
    t.U = take((size_t)2 * nb * b);
    t.part = take(panel_part_words(b) * sizeof(uint64_t) / sizeof(T));
    t.Sg = take((size_t)b * b);
    t.taus = take((size_t)b);
    // split-K workspace for the products with K = the trailing size m of each
    // panel (A_2 W, W^T X, [Z_J Y_J]^T W); the split count grows as m falls,
    // so take the largest need over every panel's m
    size_t ws = 0;
    for (int64_t m = n - b; m > 0; m -= b) {
        const size_t c[3] = {gemm_ws_elems_t<T>(m, b, m), gemm_ws_elems_t<T>(b, b, m),
                             gemm_ws_elems_t<T>(2 * nb, b, m)};
        for (size_t v : c) ws = v > ws ? v : ws;
    }
    t.gemm_ws = take(ws);
    t.gemm_ws_elems = ws;
    if (w) *w = t;
    return off;
}

template <typename T>
__global__ void fill2d_kernel(int64_t m, int64_t ncol, T *p, int64_t ld)
{
    const int64_t total = m * ncol;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        p[(i % m) + (i / m) * ld] = (T)0;
}

template <typename T>
__global__ void copy2d_kernel(int64_t m, int64_t ncol, const T *src, int64_t lds, T *dst, int64_t ldd)
{
    const int64_t total = m * ncol;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        dst[(i % m) + (i / m) * ldd] = src[(i % m) + (i / m) * lds];
}

inline dim3 grid_for(int64_t count)
{
    const int64_t g = evd_ceil_div(count, 256);
    return dim3((unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096));
}

// Double-blocked SBR (the paper's two-level blocking): inside an outer block
// of q panels the trailing matrix is not updated; each panel's columns are
// brought up to date just before its QR, its product A_2 W uses the stale
// trailing matrix corrected by the block's accumulated reflectors,
//   A_2 W = A_stale W - Y_J (Z_J^T W) - Z_J (Y_J^T W),
// and one rank-2nb SYR2K per outer block updates the trailing matrix.  With
// q = 1 this is the single-blocked scheme of Eq. 1.
template <typename T>
evd_status_t sbr_run_t(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, T *A, int64_t lda, T *AB, int64_t ldab,
                       T *Tf, void *work, int *err, const SbrOverlap *ov)
{
    hipStream_t s = ctx->stream;
    SbrWork<T> w;
    sbr_layout<T>(n, b, (char *)work, &w);
    if (uplo == 'U' || uplo == 'u') {
        dim3 grid((unsigned)evd_ceil_div(n, 256) < 64 ? (unsigned)evd_ceil_div(n, 256) : 64u, (unsigned)n);
        hipLaunchKernelGGL(mirror_upper_kernel<T>, grid, dim3(256), 0, s, n, A, lda);
    }
    {
        const int64_t cnt = ldab * n;
        hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)(evd_ceil_div(cnt, 256) < 4096 ? evd_ceil_div(cnt, 256) : 4096)),
                           dim3(256), 0, s, AB, cnt, (T)0);
    }
    // panel records start with epoch 0, which no column uses (records of an
    // earlier call carry the same epochs and must not be taken for new ones)
    hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(64), dim3(256), 0, s, (unsigned long long *)w.part,
                       (int64_t)panel_part_words(b), 0ull);
    // the trailing matrix is kept in full (both triangles) at the start of every
    // outer block, so A_2 W is a plain product over the stale matrix
    auto mirror = [&](int64_t i0) {
        const int64_t m = n - i0;
        if (m <= 1) return;
        const dim3 grid((unsigned)evd_ceil_div(m, 32), (unsigned)evd_ceil_div(m, 32));
        hipLaunchKernelGGL(mirror_lower_kernel<T>, grid, dim3(256), 0, s, m, A + i0 + i0 * lda, lda);
    };
    mirror(b);
    const int64_t p = evd_sbr_num_panels(n, b);
    // bulge chasing beside SBR: started once the band storage is zeroed
    if (ov) EVD_CHECK(ov->launch(ov->arg));
    auto publish = [&](int64_t j0, int64_t j1, int64_t value) {
        hipLaunchKernelGGL(publish_band_kernel<T>, dim3(1), dim3(64, 4), 0, s, n, b, j0, j1, p * b, (const T *)A,
                           lda, AB, ldab, ov->front, (int)value);
    };
    const int64_t nbk = evd_choose_nb(ctx, n);
    const int64_t q = (nbk > 0) ? ((nbk / b) > 0 ? nbk / b : 1)
                                        : ((SBR_NB / b) > 0 ? SBR_NB / b : 1);
    const int64_t qmax = w.q < q ? w.q : q;  // the accumulators hold w.q panels
    for (int64_t K0 = 0; K0 < p; K0 += qmax) {
        const int64_t qe = (K0 + qmax <= p) ? qmax : p - K0;
        const int64_t base = K0 * b + b;        // first row held by the accumulators
        const int64_t ldc = n - base;           // their leading dimension
        for (int64_t t = 0; t < qe; ++t) {
            const int64_t k = K0 + t, j0 = k * b, i0 = j0 + b, m = n - i0;
            const int64_t ro = i0 - base, jb = t * b;
            T *Tk = Tf + k * b * b;
            if (t > 0) {
                // bring the panel's columns (rows j0..n-1) up to date with the block so far
                const int64_t rj = j0 - base;
                EVD_CHECK(gemm_t(s, OP_N, OP_T, 0, n - j0, b, 2 * jb, (T)-1, w.YZ + rj, ldc, w.ZY + rj, ldc, (T)1,
                                 A + j0 + j0 * lda, lda, (T *)nullptr, 0));
                // rows of the block above this panel are zero in its Y and Z columns
                hipLaunchKernelGGL(fill2d_kernel<T>, grid_for(ro * 2 * b), dim3(256), 0, s, ro, 2 * b,
                                   w.YZ + 2 * t * b * ldc, ldc);
                hipLaunchKernelGGL(fill2d_kernel<T>, grid_for(ro * 2 * b), dim3(256), 0, s, ro, 2 * b,
                                   w.ZY + 2 * t * b * ldc, ldc);
            }
            T *Y = w.YZ + ro + 2 * t * b * ldc;
            T *Zs = w.YZ + ro + (2 * t + 1) * b * ldc;
            T *P = A + i0 + j0 * lda;
            T *A2 = A + i0 + i0 * lda;
            EVD_CHECK(panel_dispatch<T>(ctx, b, m, P, lda, Y, w.ZY + ro + (2 * t + 1) * b * ldc, ldc, w.part, w.Sg,
                                        w.taus, Tk, AB, ldab, j0, (int)(k * (b + 1)), err));
            // the panel's band columns are final: its diagonal block was brought
            // up to date before the QR, and R is in the band
            if (ov) publish(j0, j0 + b, j0 + b);
            // W = Y T
            EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, m, b, b, (T)1, Y, ldc, Tk, b, (T)0, w.W, m, (T *)nullptr, 0));
            // X = A_2 W (stale A_2 inside the block) into the Z slot
            EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, m, b, m, (T)1, A2, lda, w.W, m, (T)0, Zs, ldc, w.gemm_ws,
                             w.gemm_ws_elems));
            if (t > 0) {
                // X -= [Y_J Z_J] ([Z_J Y_J]^T W)
                EVD_CHECK(gemm_t(s, OP_T, OP_N, 0, 2 * jb, b, m, (T)1, w.ZY + ro, ldc, w.W, m, (T)0, w.U, 2 * jb,
                                 w.gemm_ws, w.gemm_ws_elems));
                EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, m, b, 2 * jb, (T)-1, w.YZ + ro, ldc, w.U, 2 * jb, (T)1, Zs, ldc,
                                 (T *)nullptr, 0));
            }
            // M = W^T X;  Z = X - 1/2 Y M
            EVD_CHECK(gemm_t(s, OP_T, OP_N, 0, b, b, m, (T)1, w.W, m, Zs, ldc, (T)0, w.M, b, w.gemm_ws,
                             w.gemm_ws_elems));
            EVD_CHECK(gemm_t(s, OP_N, OP_N, 0, m, b, b, (T)-0.5, Y, ldc, w.M, b, (T)1, Zs, ldc, (T *)nullptr, 0));
            hipLaunchKernelGGL(copy2d_kernel<T>, grid_for(m * b), dim3(256), 0, s, m, b, (const T *)Zs, ldc,
                               w.ZY + ro + 2 * t * b * ldc, ldc);
        }
        // A_2 <- A_2 - [Y Z ...] [Z Y ...]^T on the lower triangle, rank 2 qe b
        const int64_t iK = (K0 + qe - 1) * b + b, rK = iK - base, mK = n - iK;
        if (mK > 0) {
            // (written into both triangles: the next block's A_2 W reads the full trailing matrix)
            EVD_CHECK(gemm_t(s, OP_N, OP_T, 2, mK, mK, 2 * qe * b, (T)-1, w.YZ + rK, ldc, w.ZY + rK, ldc, (T)1,
                             A + iK + iK * lda, lda, (T *)nullptr, 0));
        }
    }
    if (ov) {
        publish(p * b, n, n);   // the trailing block, final after the last update
    } else {
        dim3 blk(64, 4);
        hipLaunchKernelGGL(extract_diag_blocks_kernel<T>, dim3((unsigned)evd_ceil_div(n, 4)), blk, 0, s, n, b, p * b,
                           (const T *)A, lda, AB, ldab);
    }
    return evd_check_last();
}

}  // namespace

evd_status_t sbr_run(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, double *A, int64_t lda, double *AB,
                     int64_t ldab, double *T, void *work, int *err, const SbrOverlap *ov)
{
    return sbr_run_t<double>(ctx, uplo, n, b, A, lda, AB, ldab, T, work, err, ov);
}

evd_status_t sbr_run_f32(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, float *A, int64_t lda, float *AB,
                         int64_t ldab, float *T, void *work, int *err, const SbrOverlap *ov)
{
    return sbr_run_t<float>(ctx, uplo, n, b, A, lda, AB, ldab, T, work, err, ov);
}

size_t sbr_work_bytes(int64_t n, int64_t b) { return sbr_layout<double>(n, b, nullptr, nullptr); }
size_t sbr_work_bytes_f32(int64_t n, int64_t b) { return sbr_layout<float>(n, b, nullptr, nullptr); }

extern "C" {

int64_t evd_sbr_num_panels(int64_t n, int64_t b)
{
    if (b <= 0 || n < b + 2) return 0;
    return (n - b - 2) / b + 1;
}

evd_status_t evd_dsy2sb_work_size(evd_ctx_t ctx, int64_t n, int64_t b, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (n < 0) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    if (b < 1 || b > 64 || (64 % b) != 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    *bytes = sbr_work_bytes(n, b) + 256;   // + the word a timed-out wait raises
    return EVD_OK;
}

evd_status_t evd_dsy2sb(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, double *A, int64_t lda, double *AB,
                        int64_t ldab, double *T, void *work, size_t work_bytes)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    int bad = 0;
    if (!(uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) bad = 2;
    else if (n < 0) bad = 3;
    else if (b < 1 || b > 64 || (64 % b) != 0) bad = 4;
    else if (n > 0 && !A) bad = 5;
    else if (lda < (n > 1 ? n : 1)) bad = 6;
    else if (n > 0 && !AB) bad = 7;
    else if (ldab < 2 * b + 1) bad = 8;
    else if (evd_sbr_num_panels(n, b) > 0 && !T) bad = 9;
    else if (n > 0 && !work) bad = 10;
    else if (work_bytes < sbr_work_bytes(n, b) + 256) bad = 11;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 11 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    int *err = (int *)((char *)work + sbr_work_bytes(n, b));
    hipLaunchKernelGGL(fill_kernel<int>, dim3(1), dim3(64), 0, ctx->stream, err, (int64_t)1, 0);
    return sbr_run(ctx, uplo, n, b, A, lda, AB, ldab, T, work, err, nullptr);
}

}  // extern "C"

// A(j, i) <- A(i, j) for i > j on the m x m matrix A (lower triangle copied
// into the upper one), on stream s.
evd_status_t evd_mirror_lower_f64(hipStream_t s, int64_t m, double *A, int64_t lda)
{
    if (m <= 1) return EVD_OK;
    const dim3 grid((unsigned)evd_ceil_div(m, 32), (unsigned)evd_ceil_div(m, 32));
    hipLaunchKernelGGL(mirror_lower_kernel<double>, grid, dim3(256), 0, s, m, A, lda);
    return evd_check_last();
}
