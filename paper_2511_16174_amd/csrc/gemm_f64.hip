// FP64 GEMM on gfx950 matrix cores: C = alpha op(A) op(B) + beta C.
//
// Used for every dense product of the method: the panel products of the ZY
// update (paper Eq. 1: A_2 W, W^T (A_2 W), Y M, and the rank-2b SYR2K
// A_2 - Y Z^T - Z Y^T), SBR-back, the divide-and-conquer merge products and
// the final eigenvector GEMM Q = Q_sb Q_d of the reordered stages (Sec. 3.3).
//
// Design: a workgroup computes a BM x BN tile of C with (BM/WM) x (BN/WN)
// wavefronts; each wavefront owns a WM x WN sub-tile made of 16 x 16
// accumulators of v_mfma_f64_16x16x4 (1024 FMAs per instruction).  The large
// tiles use eight wavefronts of 64 x 32 or 32 x 32 (about 120 VGPRs, so two
// workgroups and four wavefronts per SIMD share a CU).  K is staged through
// LDS in slices of 16 with two buffers (one barrier per slice; the global
// loads of slice t+1 are in flight while slice t is multiplied).  Slices are
// fetched with buffer loads whose out-of-range lanes read zero, so edge tiles
// run the same branch-free loop as interior ones.  The MFMA is issued with the B fragment as its first operand,
// so each group of 16 lanes holds 16 consecutive rows of one column of C and
// the stores are coalesced along the column-major C.  (Accumulator layout of
// v_mfma_f64_16x16x4: lane l, element r holds D(l/16 + 4 r, l % 16).)
//
// op(A) can be A, A^T, or the symmetric matrix held in A's lower triangle
// (tiles strictly below the diagonal are read directly, tiles strictly above
// are read transposed from the mirror tile, diagonal tiles element-wise).
//
// Large products (128-row tiles, op N or T) take a second kernel of the same
// tile shapes and MFMA order whose slices are written into LDS by the loads
// themselves (see the direct-to-LDS main loop below); both give the same
// bits, and the staged loop above serves the remaining shapes.
#include "common.h"

namespace {

constexpr int BK = 16;
constexpr int PAD = 1;
int g_gemm_swizzle = 1;  // XCD-aware tile order (gemm_tile); not used for triangular outputs, where it was slower
int g_gemm_cus = 256;    // compute units of the device (set when a context is created)
int g_gemm_dl = 1;       // direct-to-LDS kernel for 128 x 128 tiles (0: main loop staged through registers)
constexpr int GEMM_LOWER_BAND = 4;  // tile rows per band of the triangular grids (1: row-major order)

// waves per SIMD to budget registers for: 8-wavefront tiles (two workgroups
// per CU, four waves per SIMD) fit 128 VGPRs, 4-wavefront tiles 256; the
// symmetric-operand loader needs more
constexpr int gemm_min_waves(int BM, int BN, int WM, int WN, int OPA)
{
    return ((BM / WM) * (BN / WN) >= 8 ? 4 : 2) / (OPA == OP_S ? 2 : 1);
}

// Epilogue of a wavefront's WM x WN sub-tile at (mw, nw): lane holds
// C(mw + i 16 + lane % 16, nw + j 16 + lane / 16 + 4 r), r = 0..3.  Entries
// are stored inside C, at rows >= mlo and columns >= nlo (a tile moved back
// to fit inside C stores only what the tile before it does not), and on or
// below the diagonal for LOWER (LOWER = 2 also stores the transpose).
template <int WM, int WN, int TM, int TN, int LOWER>
__device__ __forceinline__ void gemm_epilogue(const double4_t (&acc)[TM][TN], int64_t m, int64_t n, int64_t mw,
                                              int64_t nw, int64_t mlo, int64_t nlo, double alpha, double beta,
                                              double *__restrict__ C, int64_t ldc, int lane)
{
    const int lr = lane & 15, lq = lane >> 4;
    double *Cw = C + mw + nw * ldc;
    const int ildc = (int)ldc;
    const bool cfull = (mw + WM <= m) && (nw + WN <= n) && mw >= mlo && nw >= nlo && (!LOWER || mw >= nw + WN - 1);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int li = i * 16 + lr;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int lj = j * 16 + lq + 4 * r;
                const int64_t gi = mw + li, gj = nw + lj;
                if (cfull || (gi < m && gj < n && gi >= mlo && gj >= nlo && (!LOWER || gi >= gj))) {
                    double *cp = Cw + (li + lj * ildc);
                    double v = alpha * acc[i][j][r];
                    if (beta != 0.0) v += beta * (*cp);
                    *cp = v;
                    if (LOWER == 2 && gi > gj) C[gj + gi * ldc] = v;  // mirror into the upper triangle
                }
            }
        }
    }
}

template <int BM, int BN, int WM, int WN, int OPA, int OPB, int LOWER>
__device__ __forceinline__ void gemm_body(int64_t m, int64_t n, int64_t k, int64_t kbeg, int64_t kend, int64_t m0,
                                          int64_t n0, double alpha, const double *__restrict__ A, int64_t lda,
                                          const double *__restrict__ B, int64_t ldb, double beta,
                                          double *__restrict__ C, int64_t ldc)
{
    constexpr int NW = (BM / WM) * (BN / WN);
    constexpr int NT = NW * 64;
    constexpr int TM = WM / 16, TN = WN / 16;
    using SAm = TileSlice<double, BM, BK, NT>;  // A slice, contiguous along M (A, or the lower triangle read directly)
    using SAk = TileSlice<double, BK, BM, NT>;  // A slice, contiguous along K (A^T, or the mirrored upper part)
    using SBk = TileSlice<double, BK, BN, NT>;  // B slice, contiguous along K (B)
    using SBn = TileSlice<double, BN, BK, NT>;  // B slice, contiguous along N (B^T)
    constexpr int EA = SAm::E;
    constexpr int EB = SBk::E;

    __shared__ double As[2][BK][BM + PAD];
    __shared__ double Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % (BM / WM), wn = wave / (BM / WM);
    const int ilda = (int)lda, ildb = (int)ldb;
    (void)k;

    double ra[EA], rb[EB];
    int amap = 0;  // 0: A slice contiguous along M, 1: along K

    auto load_a = [&](int64_t kt) {
        const int64_t mrem = m - m0, krem = kend - kt;
        const bool full = mrem >= BM && krem >= BK;
        if (OPA == OP_N) {
            amap = 0;
            SAm::load(ra, A + m0 + kt * lda, ilda, tid, full, mrem, krem);
        } else if (OPA == OP_T) {
            amap = 1;
            SAk::load(ra, A + kt + m0 * lda, ilda, tid, full, krem, mrem);
        } else {  // symmetric, lower triangle stored
            if (m0 >= kt + BK - 1) {  // all rows >= all cols: read directly
                amap = 0;
                SAm::load(ra, A + m0 + kt * lda, ilda, tid, full, mrem, krem);
            } else if (m0 + BM - 1 <= kt) {  // all rows <= all cols: mirror
                amap = 1;
                SAk::load(ra, A + kt + m0 * lda, ilda, tid, full, krem, mrem);
            } else {
                amap = 0;
#pragma unroll
                for (int r = 0; r < EA; ++r) {
                    const int64_t gi = m0 + SAm::c(tid, r), gk = kt + SAm::s(tid, r);
                    double v = 0.0;
                    if (gi < m && gk < kend) v = (gi >= gk) ? A[gi + gk * lda] : A[gk + gi * lda];
                    ra[r] = v;
                }
            }
        }
    };
    auto store_a = [&](int buf) {
        if (amap == 0) {
#pragma unroll
            for (int r = 0; r < EA; ++r) As[buf][SAm::s(tid, r)][SAm::c(tid, r)] = ra[r];
        } else {
#pragma unroll
            for (int r = 0; r < EA; ++r) As[buf][SAk::c(tid, r)][SAk::s(tid, r)] = ra[r];
        }
    };
    auto load_b = [&](int64_t kt) {
        const int64_t nrem = n - n0, krem = kend - kt;
        const bool full = nrem >= BN && krem >= BK;
        if (OPB == OP_N) SBk::load(rb, B + kt + n0 * ldb, ildb, tid, full, krem, nrem);
        else SBn::load(rb, B + n0 + kt * ldb, ildb, tid, full, nrem, krem);
    };
    auto store_b = [&](int buf) {
        if (OPB == OP_N) {
#pragma unroll
            for (int r = 0; r < EB; ++r) Bs[buf][SBk::c(tid, r)][SBk::s(tid, r)] = rb[r];
        } else {
#pragma unroll
            for (int r = 0; r < EB; ++r) Bs[buf][SBn::s(tid, r)][SBn::c(tid, r)] = rb[r];
        }
    };

    double4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

    const int64_t nkt = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
    if (nkt > 0) {
        load_a(kbeg);
        load_b(kbeg);
        store_a(0);
        store_b(0);
        __syncthreads();
        const int lr = lane & 15, lk = lane >> 4;
        for (int64_t t = 0; t < nkt; ++t) {
            const int cur = (int)(t & 1);
            if (t + 1 < nkt) {
                load_a(kbeg + (t + 1) * BK);
                load_b(kbeg + (t + 1) * BK);
            }
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                double fa[TM], fb[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) fa[i] = As[cur][k4 + lk][wm * WM + i * 16 + lr];
#pragma unroll
                for (int j = 0; j < TN; ++j) fb[j] = Bs[cur][k4 + lk][wn * WN + j * 16 + lr];
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j], fa[i], acc[i][j], 0, 0, 0);
            }
            if (t + 1 < nkt) {
                store_a(cur ^ 1);
                store_b(cur ^ 1);
            }
            __syncthreads();
        }
    }

    gemm_epilogue<WM, WN, TM, TN, LOWER>(acc, m, n, m0 + wm * WM, n0 + wn * WN, m0, n0, alpha, beta, C, ldc, lane);
}

// Output tile of this workgroup.  Workgroups are dispatched round-robin over
// the eight XCDs (each with its own L2), so the linear id is first made
// XCD-contiguous (the workgroups resident on one XCD get consecutive ids),
// then ids walk groups of GM tile rows column by column, so the tiles that
// share an XCD's L2 at a time reuse the same few A row strips and B column
// strips.  Both steps are bijections on the grid.
__device__ __forceinline__ void gemm_tile(int swz, int &bx, int &by)
{
    bx = blockIdx.x;
    by = blockIdx.y;
    if (!swz) return;
    constexpr int XCD = 8, GM = 8;
    const int nbx = gridDim.x, nby = gridDim.y, total = nbx * nby;
    int pid = bx + by * nbx;
    const int full = (total / XCD) * XCD;
    if (pid < full) pid = (pid % XCD) * (total / XCD) + pid / XCD;
    const int group = pid / (GM * nby), first = group * GM;
    const int gsz = (nbx - first) < GM ? (nbx - first) : GM;
    const int r = pid - group * GM * nby;
    bx = first + r % gsz;
    by = r / gsz;
}

// Tile (bx >= by) of a lower-triangular grid of T tile rows launched as one
// dimension of T (T + 1) / 2 workgroups: ids made XCD-contiguous as in
// gemm_tile, then taken band by band, a band being G tile rows walked column
// by column (so a tile column's slice of B serves G tiles in a row from L2);
// G = 1 is the row-major order of the lower triangle.
__device__ __forceinline__ void gemm_tile_lower(int &bx, int &by, int G)
{
    constexpr int XCD = 8;
    const int total = gridDim.x;
    int pid = blockIdx.x;
    const int full = (total / XCD) * XCD;
    if (pid < full) pid = (pid % XCD) * (total / XCD) + pid / XCD;
    // tiles before band b (all full): C(b) = G^2 b (b - 1) / 2 + b G (G + 1) / 2
    auto start = [&](int b) { return (G * G * b * (b - 1)) / 2 + b * (G * (G + 1)) / 2; };
    int b = (int)((sqrt(8.0 * (double)pid + 1.0) - 1.0) / (2.0 * G));
    while (b > 0 && start(b) > pid) --b;
    while (start(b + 1) <= pid) ++b;
    int T = (int)((sqrt(8.0 * (double)total + 1.0) - 1.0) * 0.5);
    while (T * (T + 1) / 2 > total) --T;
    while ((T + 1) * (T + 2) / 2 <= total) ++T;
    const int r0 = b * G, h = (T - r0) < G ? (T - r0) : G;
    int o = pid - start(b);
    if (o < h * r0) {  // columns left of the band's diagonal block: h tiles each
        by = o / h;
        bx = r0 + o % h;
        return;
    }
    o -= h * r0;  // the band's diagonal block, column jj holding h - jj tiles
    int jj = 0;
    while (o >= h - jj) {
        o -= h - jj;
        ++jj;
    }
    by = r0 + jj;
    bx = r0 + jj + o;
}

template <int BM, int BN, int WM, int WN, int OPA, int OPB, int LOWER>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, gemm_min_waves(BM, BN, WM, WN, OPA)) void gemm_f64_kernel(
    int64_t m, int64_t n, int64_t k, int64_t kchunk, double alpha, const double *__restrict__ A, int64_t lda,
    const double *__restrict__ B, int64_t ldb, double beta, double *__restrict__ C, int64_t ldc,
    int64_t split_stride, int swz)
{
    int bx, by;
    if (LOWER && BM == BN && swz >= 2) gemm_tile_lower(bx, by, swz - 1);  // triangular grid
    else gemm_tile(swz, bx, by);
    const int64_t m0 = (int64_t)bx * BM, n0 = (int64_t)by * BN;
    if (LOWER && n0 > m0 + BM - 1) return;  // tile strictly above the diagonal
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;
    gemm_body<BM, BN, WM, WN, OPA, OPB, LOWER>(m, n, k, kbeg, kend, m0, n0, alpha, A, lda, B, ldb, beta,
                                               C + (int64_t)blockIdx.z * split_stride, ldc);
}

// ------------------------------------------------ direct-to-LDS main loop
// 128 x 128 and 128 x 64 tiles (op N or T, m >= 128, n >= the tile width)
// are multiplied from K slices that buffer loads write straight into LDS
// (buffer_load_dwordx4 ... lds): no staging registers and no LDS stores, and
// the loads of slice t + 1 are in flight while slice t is multiplied.  One load instruction of a
// wavefront moves 1 KB: lane l's 16 bytes land 16 l bytes after the
// instruction's LDS address, whatever global address the lane reads.  Two
// layouts:
//  * MN, operand contiguous along the tile's M (or N): stage[k][d], one
//    column of 128 per instruction, rows padded to 144 doubles so that the
//    two half-wavefronts of a fragment read (k and k + 1) use different LDS
//    banks;
//  * K, operand contiguous along K: stage[d][16], 8 rows of 16 per
//    instruction; the k-pair p of row d sits in slot p ^ ((d >> 1) & 7) (the
//    lane picks its global address to match), so that the 16 rows a fragment
//    read touches hit 16 different bank pairs.
typedef __attribute__((address_space(3))) void lds_void_t;
constexpr int DL_RS = 144;            // padded MN row (doubles)
constexpr int DL_STAGE = 16 * DL_RS;  // doubles per operand and stage (>= 128 x 16)

// s_waitcnt on the vector-memory count only (gfx9 encoding)
__device__ __forceinline__ void wait_vmcnt0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// workgroup barrier without a memory fence: a fence would also wait for the
// LDS loads still in flight; the empty asm statements keep the compiler from
// moving LDS accesses across it
__device__ __forceinline__ void barrier_nofence()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ __volatile__("" ::: "memory");
}

// slice of 16 along K of one operand of the tile, origin org, into an LDS
// stage, spread over the 8 wavefronts (D: the tile's extent along M or N;
// 128, or 64 with the K layout)
template <bool KLAY, int D>
__device__ __forceinline__ void dl_issue(const double *org, int64_t ld, double *stage, int wave, int lane)
{
    static_assert(D == 128 || (KLAY && D == 64), "direct-load tile extent");
    constexpr int PER = D * 16 / 128 / 8;  // 1 KB instructions per wavefront
    const uint32_t nrec = KLAY ? (uint32_t)(((D - 1) * ld + 16) * 8) : (uint32_t)((15 * ld + 128) * 8);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)org, (short)0, (int)nrec,
                                                                       (int)EVD_BUF_DWORD3);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = PER * wave + q;  // instruction of the slice
        uint32_t off;
        double *dst;
        if (!KLAY) {
            off = (uint32_t)(2 * lane + c * ld) * 8u;
            dst = stage + c * DL_RS;
        } else {
            const int row = lane >> 3, slot = lane & 7, d = 8 * c + row;
            off = (uint32_t)(2 * (slot ^ ((d >> 1) & 7)) + d * ld) * 8u;
            dst = stage + c * 128;
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t *)dst, 16, (int)off, 0, 0, 0);
    }
}

template <bool KLAY>
__device__ __forceinline__ double dl_frag(const double *stage, int d, int k)
{
    if (!KLAY) return stage[k * DL_RS + d];
    return stage[d * 16 + 2 * ((k >> 1) ^ ((d >> 1) & 7)) + (k & 1)];
}

// C tile (m0, n0) of 128 x 128, inside C; K range kbeg .. kend of whole
// slices; 8 wavefronts of 64 x 32 (the same products in the same order as
// gemm_body, so both main loops give identical results)
// Last, partial K slice (krem < 16 columns of K): slots past krem are
// zero-filled.  MN layout: a whole instruction per K column, so invalid
// columns take an offset beyond the descriptor.  K layout: the two columns of
// a k-pair share 16 bytes, so the slice moves as 4-byte words, each with its
// own validity (four instructions per 1 KB).
template <bool KLAY, int D>
__device__ __forceinline__ void dl_issue_tail(const double *org, int64_t ld, double *stage, int wave, int lane,
                                              int krem)
{
    constexpr int PER = D * 16 / 128 / 8;
    const uint32_t nrec = KLAY ? (uint32_t)(((D - 1) * ld + 16) * 8) : (uint32_t)((15 * ld + 128) * 8);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)org, (short)0, (int)nrec,
                                                                       (int)EVD_BUF_DWORD3);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = PER * wave + q;
        if (!KLAY) {
            const uint32_t off = (c < krem) ? (uint32_t)(2 * lane + c * ld) * 8u : EVD_BUF_OOB;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t *)(stage + c * DL_RS), 16, (int)off, 0, 0, 0);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int w = 64 * j + lane;  // word of the 1 KB chunk
                const int row = w >> 5, slot = (w >> 2) & 7, h = w & 3, d = 8 * c + row;
                const int kk = 2 * (slot ^ ((d >> 1) & 7)) + (h >> 1);
                const uint32_t off =
                    (kk < krem) ? (uint32_t)(kk + d * ld) * 8u + 4u * (uint32_t)(h & 1) : EVD_BUF_OOB;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t *)(stage + c * 128 + 32 * j), 4, (int)off,
                                                         0, 0, 0);
            }
        }
    }
}

// One 128 x BN tile of C from K columns kbeg .. kend (a partial last slice is
// zero-filled): tile (mlo, nlo), moved back inside C when it crosses the edge
// (m >= 128, n >= BN), storing only its own entries; smem holds 2 stages.
// The products are those of gemm_body, in the same order, so both main loops
// give the same bits.
template <int OPA, int OPB, int LOWER, int BN>
__device__ __forceinline__ void gemm_dl_tile(int64_t m, int64_t n, int64_t kbeg, int64_t kend, int64_t mlo,
                                             int64_t nlo, double alpha, const double *__restrict__ A, int64_t lda,
                                             const double *__restrict__ B, int64_t ldb, double beta,
                                             double *__restrict__ C, int64_t ldc, double *smem)
{
    constexpr int WM = BN == 128 ? 64 : 32, WN = 32, TM = WM / 16, TN = WN / 16, NWM = 128 / WM;
    constexpr bool AK = (OPA == OP_T), BKL = (OPB == OP_N);
    static_assert(BN == 128 || (BN == 64 && BKL && !LOWER), "64-wide tiles: op(B) = B, full C");
    constexpr int SA = DL_STAGE, SB = BN == 128 ? DL_STAGE : BN * 16, SS = SA + SB;
    const int64_t m0 = (mlo + 128 <= m) ? mlo : m - 128, n0 = (nlo + BN <= n) ? nlo : n - BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % NWM, wn = wave / NWM;
    const int lr = lane & 15, lk = lane >> 4;
    auto a_org = [&](int64_t kt) { return AK ? A + kt + m0 * lda : A + m0 + kt * lda; };
    auto b_org = [&](int64_t kt) { return BKL ? B + kt + n0 * ldb : B + n0 + kt * ldb; };
    auto stage = [&](int st, int op) { return smem + st * SS + op * SA; };
    const int64_t klen = (kend > kbeg) ? kend - kbeg : 0;
    const int64_t nkt = (klen + BK - 1) / BK;
    const int krem = (int)(klen - (nkt - 1) * BK);  // columns of the last slice
    auto issue = [&](int64_t t, int st) {
        if (t + 1 < nkt || krem == BK) {
            dl_issue<AK, 128>(a_org(kbeg + t * BK), lda, stage(st, 0), wave, lane);
            dl_issue<BKL, BN>(b_org(kbeg + t * BK), ldb, stage(st, 1), wave, lane);
        } else {
            dl_issue_tail<AK, 128>(a_org(kbeg + t * BK), lda, stage(st, 0), wave, lane, krem);
            dl_issue_tail<BKL, BN>(b_org(kbeg + t * BK), ldb, stage(st, 1), wave, lane, krem);
        }
    };
    double4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};
    if (nkt > 0) issue(0, 0);
    for (int64_t t = 0; t < nkt; ++t) {
        const int st = (int)(t & 1);
        // this wavefront's loads of slice t have landed; past the barrier all
        // of them have, and no wavefront still reads the other stage
        wait_vmcnt0();
        barrier_nofence();
        if (t + 1 < nkt) issue(t + 1, st ^ 1);
        const double *As = stage(st, 0), *Bs = stage(st, 1);
#pragma unroll
        for (int k4 = 0; k4 < BK; k4 += 4) {
            double fa[TM], fb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) fa[i] = dl_frag<AK>(As, wm * WM + i * 16 + lr, k4 + lk);
#pragma unroll
            for (int j = 0; j < TN; ++j) fb[j] = dl_frag<BKL>(Bs, wn * WN + j * 16 + lr, k4 + lk);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j], fa[i], acc[i][j], 0, 0, 0);
        }
    }
    gemm_epilogue<WM, WN, TM, TN, LOWER>(acc, m, n, m0 + wm * WM, n0 + wn * WN, mlo, nlo, alpha, beta, C, ldc, lane);
}

template <int BN>
constexpr int dl_lds_elems() { return 2 * (DL_STAGE + (BN == 128 ? DL_STAGE : BN * 16)); }

template <int OPA, int OPB, int LOWER, int BN>
__global__ __launch_bounds__(512, gemm_min_waves(128, BN, BN == 128 ? 64 : 32, 32, OPA)) void gemm_f64_dl_kernel(
    int64_t m, int64_t n, int64_t k, int64_t kchunk, double alpha, const double *__restrict__ A, int64_t lda,
    const double *__restrict__ B, int64_t ldb, double beta, double *__restrict__ C, int64_t ldc,
    int64_t split_stride, int swz)
{
    __shared__ double smem[dl_lds_elems<BN>()];
    int bx, by;
    if (LOWER && swz >= 2) gemm_tile_lower(bx, by, swz - 1);
    else gemm_tile(swz, bx, by);
    const int64_t mlo = (int64_t)bx * 128, nlo = (int64_t)by * BN;
    if (LOWER && nlo > mlo + 127) return;  // tile strictly above the diagonal
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;
    gemm_dl_tile<OPA, OPB, LOWER, BN>(m, n, kbeg, kend, mlo, nlo, alpha, A, lda, B, ldb, beta,
                                      C + (int64_t)blockIdx.z * split_stride, ldc, smem);
}

// Grouped products on the direct-load path: problems with m, n >= 128 (the
// others are left to gemm_f64_grouped_kernel, which skips these)
__global__ __launch_bounds__(512, gemm_min_waves(128, 128, 64, 32, OP_N)) void gemm_f64_grouped_dl_kernel(
    const GemmProblem *probs)
{
    __shared__ double smem[dl_lds_elems<128>()];
    const GemmProblem p = probs[blockIdx.z];
    if (p.m < 128 || p.n < 128) return;
    const int64_t mlo = (int64_t)blockIdx.x * 128, nlo = (int64_t)blockIdx.y * 128;
    if (mlo >= p.m || nlo >= p.n) return;
    gemm_dl_tile<OP_N, OP_N, 0, 128>(p.m, p.n, 0, p.k, mlo, nlo, 1.0, p.A, p.lda, p.B, p.ldb, 0.0, p.C, p.ldc, smem);
}

// Grouped product with sizes in device memory: problem blockIdx.z, C = A B
// (op N, N); tiles outside the problem exit.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, gemm_min_waves(BM, BN, WM, WN, OP_N)) void gemm_f64_grouped_kernel(const GemmProblem *probs, int skip_dl)
{
    const GemmProblem p = probs[blockIdx.z];
    if (skip_dl && p.m >= 128 && p.n >= 128) return;  // taken by gemm_f64_grouped_dl_kernel
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    if (m0 >= p.m || n0 >= p.n) return;
    gemm_body<BM, BN, WM, WN, OP_N, OP_N, 0>(p.m, p.n, p.k, 0, p.k, m0, n0, 1.0, p.A, p.lda, p.B, p.ldb, 0.0, p.C,
                                             p.ldc);
}

__global__ void splitk_reduce_kernel(int64_t m, int64_t n, int splits, const double *__restrict__ P, int64_t stride,
                                     double alpha, double beta, double *__restrict__ C, int64_t ldc, int lower)
{
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % m, j = idx / m;
        if (lower && i < j) continue;
        double s = 0.0;
        for (int z = 0; z < splits; ++z) s += P[z * stride + i + j * m];
        double *cp = &C[i + j * ldc];
        double v = alpha * s;
        if (beta != 0.0) v += beta * (*cp);
        *cp = v;
    }
}

// Split-K sum for small outputs with many partials: SPL adjacent lanes of a
// wavefront share one output entry, each adding the partials z = part,
// part + SPL, ..., then the SPL sums are combined by lane shuffles (in a
// fixed order: the result does not depend on the launch).
template <int SPL>
__global__ __launch_bounds__(256) void splitk_reduce_wide_kernel(int64_t m, int64_t n, int splits,
                                                                 const double *__restrict__ P, int64_t stride,
                                                                 double alpha, double beta, double *__restrict__ C,
                                                                 int64_t ldc, int lower)
{
    const int64_t total = m * n;
    const int part = threadIdx.x % SPL;
    for (int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / SPL; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x / SPL) {
        const int64_t i = idx % m, j = idx / m;
        double s = 0.0;
        for (int z = part; z < splits; z += SPL) s += P[z * stride + i + j * m];
#pragma unroll
        for (int off = SPL / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (part == 0 && !(lower && i < j)) {
            double *cp = &C[i + j * ldc];
            double v = alpha * s;
            if (beta != 0.0) v += beta * (*cp);
            *cp = v;
        }
    }
}

template <int BM, int BN, int WM, int WN, int OPA, int OPB, int LOWER>
void launch_cfg(hipStream_t s, dim3 grid, int64_t m, int64_t n, int64_t k, int64_t kchunk, double alpha,
                const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                int64_t split_stride)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    // lower-triangular outputs of square tiles: a one-dimensional grid of the
    // T (T + 1) / 2 tiles on or below the diagonal (no workgroups that exit)
    int swz = LOWER ? 0 : g_gemm_swizzle;
    if (LOWER && BM == BN && grid.z == 1 && m == n) {
        const unsigned T = grid.x;
        grid = dim3(T * (T + 1) / 2, 1, 1);
        swz = 1 + GEMM_LOWER_BAND;
    }
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WM, WN, OPA, OPB, LOWER>), grid, dim3(NT), 0, s, m, n, k, kchunk,
                       alpha, A, lda, B, ldb, beta, C, ldc, split_stride, swz);
}

// direct-load kernel for 128 x BN tiles (op N or T, m >= 128, n >= BN, whole K slices)
template <int OPA, int OPB, int LOWER, int BN>
void launch_dl(hipStream_t s, dim3 grid, int64_t m, int64_t n, int64_t k, int64_t kchunk, double alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
               int64_t split_stride)
{
    int swz = LOWER ? 0 : g_gemm_swizzle;
    if (LOWER && grid.z == 1 && m == n) {
        const unsigned T = grid.x;
        grid = dim3(T * (T + 1) / 2, 1, 1);
        swz = 1 + GEMM_LOWER_BAND;
    }
    hipLaunchKernelGGL((gemm_f64_dl_kernel<OPA, OPB, LOWER, BN>), grid, dim3(512), 0, s, m, n, k, kchunk, alpha, A, lda, B,
                       ldb, beta, C, ldc, split_stride, swz);
}

template <int BM, int BN, int WM, int WN>
void launch_ops(hipStream_t s, int opa, int opb, int lower, dim3 grid, int64_t m, int64_t n, int64_t k,
                int64_t kchunk, double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                double beta, double *C, int64_t ldc, int64_t split_stride)
{
#define EVD_GEMM_CASE(OA, OB, LW)                                                                          \
    if (opa == OA && opb == OB && lower == LW) {                                                          \
        launch_cfg<BM, BN, WM, WN, OA, OB, LW>(s, grid, m, n, k, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, \
                                               split_stride);                                             \
        return;                                                                                           \
    }
    EVD_GEMM_CASE(OP_N, OP_N, 0)
    EVD_GEMM_CASE(OP_N, OP_T, 0)
    EVD_GEMM_CASE(OP_T, OP_N, 0)
    EVD_GEMM_CASE(OP_T, OP_T, 0)
    EVD_GEMM_CASE(OP_S, OP_N, 0)
    EVD_GEMM_CASE(OP_S, OP_T, 0)
    EVD_GEMM_CASE(OP_N, OP_N, 1)
    EVD_GEMM_CASE(OP_N, OP_T, 1)
    EVD_GEMM_CASE(OP_T, OP_N, 1)
    EVD_GEMM_CASE(OP_T, OP_T, 1)
    EVD_GEMM_CASE(OP_N, OP_T, 2)
#undef EVD_GEMM_CASE
}

struct GemmPlan {
    int bm, bn, splits;
    int64_t kchunk;
};

GemmPlan plan_gemm(int64_t m, int64_t n, int64_t k, size_t ws_elems)
{
    GemmPlan p;
    p.bm = (m > 64) ? 128 : 64;
    p.bn = (n > 64) ? 128 : 64;
    int64_t tiles = evd_ceil_div(m, p.bm) * evd_ceil_div(n, p.bn);
    if (tiles < 512 && p.bm == 128 && p.bn == 128) {
        // prefer more, smaller tiles when the grid is small
        if (m >= n) p.bn = 64; else p.bm = 64;
        tiles = evd_ceil_div(m, p.bm) * evd_ceil_div(n, p.bn);
    }
    p.splits = 1;
    p.kchunk = k;
    // Split K when the output grid fills under about one and a half rounds of
    // the resident workgroups (two per CU for every tile shape) and K is long.
    // Outputs of under one round (the SBR products m x b x m, W^T X, ...)
    // take at least 8 splits and at least one full round of workgroups: the
    // K-chunk of the narrow operand then stays in L2, and on m x 64 x m
    // 8-16 splits beat the 2-5 that merely fill the CUs by up to 12 %.
    const int64_t slots = 2 * (int64_t)g_gemm_cus;
    if (tiles < (3 * slots) / 2 && k >= 1024) {
        int64_t sp = (tiles < slots) ? evd_ceil_div(slots, tiles) : evd_ceil_div((3 * slots) / 2, tiles);
        if (tiles < slots && sp < 8) sp = 8;
        // (outputs of a few tiles, W^T X or [Z Y]^T W in SBR, take up to 256
        // splits: one workgroup per CU; their partial sums are few)
        const int64_t smax = (tiles <= 4) ? 256 : 64;
        if (sp > smax) sp = smax;
        if (sp > k / 128) sp = k / 128;
        if (sp >= 2 && (size_t)(sp * m * n) <= ws_elems) {
            p.kchunk = evd_ceil_div(evd_ceil_div(k, sp), BK) * BK;
            p.splits = (int)evd_ceil_div(k, p.kchunk);
        }
    }
    return p;
}

}  // namespace

evd_status_t gemm_f64_grouped(hipStream_t s, const GemmProblem *probs, int nprob, int64_t max_m, int64_t max_n)
{
    if (nprob <= 0 || max_m <= 0 || max_n <= 0) return EVD_OK;
    // the problem index is the grid's z dimension (at most 65535 per launch)
    constexpr int ZMAX = 65535;
    for (int p0 = 0; p0 < nprob; p0 += ZMAX) {
        const unsigned np = (unsigned)((nprob - p0) < ZMAX ? (nprob - p0) : ZMAX);
        if (max_m > 64 && max_n > 64 && max_m * max_n >= (int64_t)512 * 128 * 128) {
            dim3 grid((unsigned)evd_ceil_div(max_m, 128), (unsigned)evd_ceil_div(max_n, 128), np);
            if (g_gemm_dl) hipLaunchKernelGGL(gemm_f64_grouped_dl_kernel, grid, dim3(512), 0, s, probs + p0);
            hipLaunchKernelGGL((gemm_f64_grouped_kernel<128, 128, 64, 32>), grid, dim3(512), 0, s, probs + p0, g_gemm_dl);
        } else {
            dim3 grid((unsigned)evd_ceil_div(max_m, 64), (unsigned)evd_ceil_div(max_n, 64), np);
            hipLaunchKernelGGL((gemm_f64_grouped_kernel<64, 64, 32, 32>), grid, dim3(256), 0, s, probs + p0, 0);
        }
    }
    return evd_check_last();
}

void gemm_set_cu_count(int cus)
{
    if (cus > 0) g_gemm_cus = cus;
}

void gemm_set_staged(int on) { g_gemm_dl = on ? 0 : 1; }

size_t gemm_splitk_ws_elems(int64_t m, int64_t n, int64_t k)
{
    GemmPlan p = plan_gemm(m, n, k, (size_t)-1);
    return p.splits > 1 ? (size_t)p.splits * (size_t)m * (size_t)n : 0;
}

evd_status_t gemm_f64(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k, double alpha,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                      int64_t ldc, double *ws, size_t ws_elems)
{
    if (m <= 0 || n <= 0) return EVD_OK;
    if (k <= 0 || alpha == 0.0) {
        // C = beta C on the referenced part
        if (beta == 1.0) return EVD_OK;
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)evd_ceil_div(m * n, 256 * 4) < 65535
                                                          ? (unsigned)evd_ceil_div(m * n, 256 * 4) : 65535u),
                           dim3(256), 0, s, m, n, 0, (const double *)nullptr, (int64_t)0, 0.0, beta, C, ldc,
                           lower_c);
        return evd_check_last();
    }
    if (!evd_gemm_ld_ok(lda) || !evd_gemm_ld_ok(ldb)) return EVD_ERR_INVALID_ARG;  // slice loader offsets
    // lower_c: 0 full C, 1 lower triangle only, 2 lower triangle computed and
    // also written transposed into the upper triangle (square C, op N/T, no
    // K splitting)
    const int lower = (lower_c == 2) ? 2 : (lower_c ? 1 : 0);
    if (lower == 2 && (m != n || opa != OP_N || opb != OP_T)) return EVD_ERR_INVALID_ARG;
    GemmPlan p = plan_gemm(m, n, k, (ws && lower != 2) ? ws_elems : 0);
    dim3 grid((unsigned)evd_ceil_div(m, p.bm), (unsigned)evd_ceil_div(n, p.bn), (unsigned)p.splits);
    double *Cout = C;
    int64_t ldo = ldc, sstride = 0;
    double a = alpha, bta = beta;
    if (p.splits > 1) {
        Cout = ws;
        ldo = m;
        sstride = m * n;
        a = 1.0;
        bta = 0.0;
    }
    // (split K: every chunk but the last is whole slices; unsplit: any K)
    const bool kok = p.splits == 1 || p.kchunk % BK == 0;
    const bool dl = g_gemm_dl && p.bm == 128 && p.bn == 128 && m >= 128 && n >= 128 && opa != OP_S && kok;
    if (dl) {
#define EVD_DL_CASE(OA, OB, LW)                                                                                \
    if (opa == OA && opb == OB && lower == LW)                                                                 \
        launch_dl<OA, OB, LW, 128>(s, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo, sstride);
        EVD_DL_CASE(OP_N, OP_N, 0)
        EVD_DL_CASE(OP_N, OP_T, 0)
        EVD_DL_CASE(OP_T, OP_N, 0)
        EVD_DL_CASE(OP_T, OP_T, 0)
        EVD_DL_CASE(OP_N, OP_N, 1)
        EVD_DL_CASE(OP_N, OP_T, 1)
        EVD_DL_CASE(OP_T, OP_N, 1)
        EVD_DL_CASE(OP_T, OP_T, 1)
        EVD_DL_CASE(OP_N, OP_T, 2)
#undef EVD_DL_CASE
    } else if (g_gemm_dl && p.bm == 128 && p.bn == 64 && m >= 128 && n >= 64 && opb == OP_N && lower == 0 &&
               opa != OP_S && kok) {
        if (opa == OP_N) launch_dl<OP_N, OP_N, 0, 64>(s, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo, sstride);
        else launch_dl<OP_T, OP_N, 0, 64>(s, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo, sstride);
    } else if (p.bm == 128 && p.bn == 128)
        launch_ops<128, 128, 64, 32>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                     sstride);
    else if (p.bm == 128 && p.bn == 64)
        launch_ops<128, 64, 32, 32>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                    sstride);
    else if (p.bm == 64 && p.bn == 128)
        launch_ops<64, 128, 32, 32>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                    sstride);
    else
        launch_ops<64, 64, 32, 32>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                   sstride);
    EVD_CHECK(evd_check_last());
    if (p.splits > 1) {
        if (m * n <= 65536 && p.splits >= 16) {
            // few entries, many partials: 16 lanes per entry
            const int64_t blocks = evd_ceil_div(m * n * 16, 256);
            hipLaunchKernelGGL(splitk_reduce_wide_kernel<16>, dim3((unsigned)blocks), dim3(256), 0, s, m, n,
                               p.splits, ws, sstride, alpha, beta, C, ldc, lower);
        } else {
            int64_t blocks = evd_ceil_div(m * n, 256);
            if (blocks > 65535) blocks = 65535;
            hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, n, p.splits, ws,
                               sstride, alpha, beta, C, ldc, lower);
        }
        EVD_CHECK(evd_check_last());
    }
    return EVD_OK;
}
