// FP32 GEMM through split-BF16x3 on gfx950 matrix cores (mixed-precision path).
//
// Every FP32 operand x is split as x_hi = bf16(x), x_lo = bf16(x - x_hi) and
// C = alpha (A_hi B_hi + A_hi B_lo + A_lo B_hi) + beta C with FP32
// accumulation (v_mfma_f32_16x16x32_bf16).  The split keeps about 17
// significant bits of each product (the dropped term A_lo B_lo is below
// 2^-16 relative), well short of FP32's 24: the mixed path relies on FP64
// refinement afterwards for full accuracy.
//
// Tiling mirrors the FP64 kernel: BM x BN workgroup tile, (BM/WM) x (BN/WN)
// wavefronts, K staged through LDS in slices of 32 (one MFMA K-step) with two
// buffers.  LDS holds the hi and lo parts k-contiguous per row so each lane
// reads its 8-element fragment with one 16-byte load.
#include "common.h"

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int BK3 = 32;
constexpr int KP = BK3 + 8;  // padded row length (bf16 elements) in LDS

__device__ __forceinline__ void split_bf16(float x, __bf16 *hi, __bf16 *lo)
{
    const __bf16 h = (__bf16)x;          // round to nearest even
    *hi = h;
    *lo = (__bf16)(x - (float)h);
}

template <int BM, int BN, int WM, int WN, int OPA, int OPB, int LOWER>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void gemm_f32x3_kernel(
    int64_t m, int64_t n, int64_t k, int64_t kchunk, float alpha, const float *__restrict__ A, int64_t lda,
    const float *__restrict__ B, int64_t ldb, float beta, float *__restrict__ C, int64_t ldc, int64_t split_stride)
{
    constexpr int NW = (BM / WM) * (BN / WN);
    constexpr int NT = NW * 64;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int EA = BM * BK3 / NT;
    constexpr int EB = BN * BK3 / NT;
    static_assert(EA * NT == BM * BK3 && EB * NT == BN * BK3, "tile/thread mismatch");

    __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][KP];
    __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM][KP];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN][KP];
    __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BN][KP];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % (BM / WM), wn = wave / (BM / WM);
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    if (LOWER && n0 > m0 + BM - 1) return;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;
    C += (int64_t)blockIdx.z * split_stride;

    using SAm = TileSlice<float, BM, BK3, NT>;  // contiguous along M
    using SAk = TileSlice<float, BK3, BM, NT>;  // contiguous along K
    using SBk = TileSlice<float, BK3, BN, NT>;
    using SBn = TileSlice<float, BN, BK3, NT>;
    const int ilda = (int)lda, ildb = (int)ldb;
    float ra[EA], rb[EB];
    int amap = 0;
    auto load_a = [&](int64_t kt) {
        const int64_t mrem = m - m0, krem = kend - kt;
        const bool full = mrem >= BM && krem >= BK3;
        if (OPA == OP_N) {
            amap = 0;
            SAm::load(ra, A + m0 + kt * lda, ilda, tid, full, mrem, krem);
        } else if (OPA == OP_T) {
            amap = 1;
            SAk::load(ra, A + kt + m0 * lda, ilda, tid, full, krem, mrem);
        } else {
            if (m0 >= kt + BK3 - 1) {
                amap = 0;
                SAm::load(ra, A + m0 + kt * lda, ilda, tid, full, mrem, krem);
            } else if (m0 + BM - 1 <= kt) {
                amap = 1;
                SAk::load(ra, A + kt + m0 * lda, ilda, tid, full, krem, mrem);
            } else {
                amap = 0;
#pragma unroll
                for (int r = 0; r < EA; ++r) {
                    const int64_t gi = m0 + SAm::c(tid, r), gk = kt + SAm::s(tid, r);
                    float v = 0.0f;
                    if (gi < m && gk < kend) v = (gi >= gk) ? A[gi + gk * lda] : A[gk + gi * lda];
                    ra[r] = v;
                }
            }
        }
    };
    auto store_a = [&](int buf) {
#pragma unroll
        for (int r = 0; r < EA; ++r) {
            const int i = (amap == 0) ? SAm::c(tid, r) : SAk::s(tid, r);
            const int kk = (amap == 0) ? SAm::s(tid, r) : SAk::c(tid, r);
            split_bf16(ra[r], &Ah[buf][i][kk], &Al[buf][i][kk]);
        }
    };
    auto load_b = [&](int64_t kt) {
        const int64_t nrem = n - n0, krem = kend - kt;
        const bool full = nrem >= BN && krem >= BK3;
        if (OPB == OP_N) SBk::load(rb, B + kt + n0 * ldb, ildb, tid, full, krem, nrem);
        else SBn::load(rb, B + n0 + kt * ldb, ildb, tid, full, nrem, krem);
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int r = 0; r < EB; ++r) {
            const int j = (OPB == OP_N) ? SBk::s(tid, r) : SBn::c(tid, r);
            const int kk = (OPB == OP_N) ? SBk::c(tid, r) : SBn::s(tid, r);
            split_bf16(rb[r], &Bh[buf][j][kk], &Bl[buf][j][kk]);
        }
    };

    float4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (float4_t){0.0f, 0.0f, 0.0f, 0.0f};

    const int64_t nkt = (kend > kbeg) ? (kend - kbeg + BK3 - 1) / BK3 : 0;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    if (nkt > 0) {
        load_a(kbeg);
        load_b(kbeg);
        store_a(0);
        store_b(0);
        __syncthreads();
        for (int64_t t = 0; t < nkt; ++t) {
            const int cur = (int)(t & 1);
            if (t + 1 < nkt) {
                load_a(kbeg + (t + 1) * BK3);
                load_b(kbeg + (t + 1) * BK3);
            }
            bf16x8_t ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                ah[i] = *(const bf16x8_t *)&Ah[cur][wm * WM + i * 16 + lr][lk];
                al[i] = *(const bf16x8_t *)&Al[cur][wm * WM + i * 16 + lr][lk];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                bh[j] = *(const bf16x8_t *)&Bh[cur][wn * WN + j * 16 + lr][lk];
                bl[j] = *(const bf16x8_t *)&Bl[cur][wn * WN + j * 16 + lr][lk];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah[i], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al[i], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah[i], acc[i][j], 0, 0, 0);
                }
            if (t + 1 < nkt) {
                store_a(cur ^ 1);
                store_b(cur ^ 1);
            }
            __syncthreads();
        }
    }
    // epilogue: D(row, col) of the MFMA is C(i = col, j = row)
    const int lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int64_t gi = m0 + wm * WM + i * 16 + lr;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gj = n0 + wn * WN + j * 16 + EVD_F32_MFMA_ROW(lq, r);
                if (gi < m && gj < n && (!LOWER || gi >= gj)) {
                    float v = alpha * acc[i][j][r];
                    float *cp = &C[gi + gj * ldc];
                    if (beta != 0.0f) v += beta * (*cp);
                    *cp = v;
                    if (LOWER == 2 && gi > gj) C[gj + gi * ldc] = v;  // mirror into the upper triangle
                }
            }
        }
    }
}

__global__ void splitk_reduce_f32_kernel(int64_t m, int64_t n, int splits, const float *__restrict__ P,
                                         int64_t stride, float alpha, float beta, float *__restrict__ C, int64_t ldc,
                                         int lower)
{
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % m, j = idx / m;
        if (lower && i < j) continue;
        float s = 0.0f;
        for (int z = 0; z < splits; ++z) s += P[z * stride + i + j * m];
        float *cp = &C[i + j * ldc];
        float v = alpha * s;
        if (beta != 0.0f) v += beta * (*cp);
        *cp = v;
    }
}

template <int BM, int BN, int WM, int WN>
void launch_ops3(hipStream_t s, int opa, int opb, int lower, dim3 grid, int64_t m, int64_t n, int64_t k,
                 int64_t kchunk, float alpha, const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                 float *C, int64_t ldc, int64_t sstride)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
#define EVD_G3_CASE(OA, OB, LW)                                                                                    \
    if (opa == OA && opb == OB && lower == LW) {                                                                  \
        hipLaunchKernelGGL((gemm_f32x3_kernel<BM, BN, WM, WN, OA, OB, LW>), grid, dim3(NT), 0, s, m, n, k, kchunk, \
                           alpha, A, lda, B, ldb, beta, C, ldc, sstride);                                         \
        return;                                                                                                   \
    }
    EVD_G3_CASE(OP_N, OP_N, 0)
    EVD_G3_CASE(OP_N, OP_T, 0)
    EVD_G3_CASE(OP_T, OP_N, 0)
    EVD_G3_CASE(OP_T, OP_T, 0)
    EVD_G3_CASE(OP_S, OP_N, 0)
    EVD_G3_CASE(OP_N, OP_T, 1)
    EVD_G3_CASE(OP_N, OP_N, 1)
    EVD_G3_CASE(OP_N, OP_T, 2)
#undef EVD_G3_CASE
}

struct Plan3 {
    int bm, bn, splits;
    int64_t kchunk;
};

Plan3 plan3(int64_t m, int64_t n, int64_t k, size_t ws_elems)
{
    Plan3 p;
    p.bm = (m > 64) ? 128 : 64;
    p.bn = (n > 64) ? 128 : 64;
    int64_t tiles = evd_ceil_div(m, p.bm) * evd_ceil_div(n, p.bn);
    if (tiles < 512 && p.bm == 128 && p.bn == 128) {
        if (m >= n) p.bn = 64; else p.bm = 64;
        tiles = evd_ceil_div(m, p.bm) * evd_ceil_div(n, p.bn);
    }
    p.splits = 1;
    p.kchunk = k;
    if (tiles < 256 && k >= 2048) {
        int64_t want = evd_ceil_div(512, tiles);
        int64_t maxs = k / 512;
        int64_t sp = want < maxs ? want : maxs;
        if (sp > 64) sp = 64;
        if (sp >= 2 && (size_t)(sp * m * n) <= ws_elems) {
            p.kchunk = evd_ceil_div(evd_ceil_div(k, sp), BK3) * BK3;
            p.splits = (int)evd_ceil_div(k, p.kchunk);
        }
    }
    return p;
}

}  // namespace

size_t gemm_f32x3_ws_elems(int64_t m, int64_t n, int64_t k)
{
    Plan3 p = plan3(m, n, k, (size_t)-1);
    return p.splits > 1 ? (size_t)p.splits * (size_t)m * (size_t)n : 0;
}

evd_status_t gemm_f32x3(hipStream_t s, int opa, int opb, int lower_c, int64_t m, int64_t n, int64_t k, float alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                        float *ws, size_t ws_elems)
{
    if (m <= 0 || n <= 0) return EVD_OK;
    if (opa == OP_S && opb == OP_T) return EVD_ERR_INVALID_ARG;
    if (k <= 0 || alpha == 0.0f) {
        if (beta == 1.0f) return EVD_OK;
        hipLaunchKernelGGL(splitk_reduce_f32_kernel, dim3(1024), dim3(256), 0, s, m, n, 0, (const float *)nullptr,
                           (int64_t)0, 0.0f, beta, C, ldc, lower_c);
        return evd_check_last();
    }
    if (!evd_gemm_ld_ok(lda) || !evd_gemm_ld_ok(ldb)) return EVD_ERR_INVALID_ARG;  // slice loader offsets
    // lower_c 2: lower triangle computed and mirrored (see gemm_f64)
    const int lower = (lower_c == 2) ? 2 : (lower_c ? 1 : 0);
    if (lower == 2 && (m != n || opa != OP_N || opb != OP_T)) return EVD_ERR_INVALID_ARG;
    Plan3 p = plan3(m, n, k, (ws && lower != 2) ? ws_elems : 0);
    dim3 grid((unsigned)evd_ceil_div(m, p.bm), (unsigned)evd_ceil_div(n, p.bn), (unsigned)p.splits);
    float *Cout = C;
    int64_t ldo = ldc, sstride = 0;
    float a = alpha, bta = beta;
    if (p.splits > 1) {
        Cout = ws;
        ldo = m;
        sstride = m * n;
        a = 1.0f;
        bta = 0.0f;
    }
    if (p.bm == 128 && p.bn == 128)
        launch_ops3<128, 128, 64, 64>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                      sstride);
    else if (p.bm == 128 && p.bn == 64)
        launch_ops3<128, 64, 64, 32>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                     sstride);
    else if (p.bm == 64 && p.bn == 128)
        launch_ops3<64, 128, 32, 64>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                     sstride);
    else
        launch_ops3<64, 64, 32, 32>(s, opa, opb, lower, grid, m, n, k, p.kchunk, a, A, lda, B, ldb, bta, Cout, ldo,
                                    sstride);
    EVD_CHECK(evd_check_last());
    if (p.splits > 1) {
        int64_t blocks = evd_ceil_div(m * n, 256);
        if (blocks > 65535) blocks = 65535;
        hipLaunchKernelGGL(splitk_reduce_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, n, p.splits, ws,
                           sstride, alpha, beta, C, ldc, lower);
        EVD_CHECK(evd_check_last());
    }
    return EVD_OK;
}

extern "C" {

evd_status_t evd_sgemm_x3(evd_ctx_t ctx, char opa, char opb, int lower_c, int64_t m, int64_t n, int64_t k,
                          float alpha, const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                          int64_t ldc, void *work, size_t work_bytes)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    auto code = [](char c, bool allow_s) {
        if (c == 'N' || c == 'n') return (int)OP_N;
        if (c == 'T' || c == 't') return (int)OP_T;
        if (allow_s && (c == 'S' || c == 's')) return (int)OP_S;
        return -1;
    };
    const int oa = code(opa, true), ob = code(opb, false);
    int bad = 0;
    if (oa < 0) bad = 2;
    else if (ob < 0 || (oa == OP_S && ob != OP_N)) bad = 3;
    else if (lower_c && (m != n || oa == OP_S)) bad = 4;
    else if (m < 0) bad = 5;
    else if (n < 0) bad = 6;
    else if (k < 0 || (oa == OP_S && k != m)) bad = 7;
    else if (m > 0 && k > 0 && !A) bad = 9;
    else if (lda < ((oa == OP_T) ? (k > 1 ? k : 1) : (m > 1 ? m : 1))) bad = 10;
    else if (n > 0 && k > 0 && !B) bad = 11;
    else if (ldb < ((ob == OP_N) ? (k > 1 ? k : 1) : (n > 1 ? n : 1))) bad = 12;
    else if (m > 0 && n > 0 && !C) bad = 14;
    else if (ldc < (m > 1 ? m : 1)) bad = 15;
    ctx->last_invalid_arg = bad;
    if (bad) return EVD_ERR_INVALID_ARG;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    return gemm_f32x3(ctx->stream, oa, ob, lower_c ? 1 : 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, (float *)work,
                      work ? work_bytes / sizeof(float) : 0);
}

evd_status_t evd_sgemm_x3_work_size(evd_ctx_t ctx, int64_t m, int64_t n, int64_t k, size_t *bytes)
{
    if (!ctx || !bytes || m < 0 || n < 0 || k < 0) return EVD_ERR_INVALID_ARG;
    *bytes = gemm_f32x3_ws_elems(m, n, k) * sizeof(float);
    return EVD_OK;
}

}  // extern "C"
