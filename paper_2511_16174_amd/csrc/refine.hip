// FP64 eigenpair refinement of Ogita and Aishima (JJIAM 2018, "RefSyEv"),
// used by the mixed-precision path (not in the paper): from an approximate
// eigenvector matrix X of the symmetric A,
//   R = I - X^T X,  S = X^T A X,  lam_i = s_ii / (1 - r_ii),
//   delta = 2 (||S - diag(lam)|| + ||A|| ||R||),
//   E_ij = (s_ij + lam_j r_ij) / (lam_j - lam_i)   if |lam_i - lam_j| > delta
//          r_ij / 2                                 otherwise,
//   X <- X + X E.
// The norms are Frobenius norms (upper bounds of the 2-norms), ||A|| is
// bounded by max |lam_i| (1 + ||R||).  Eigenvalues closer than delta form a
// cluster whose invariant subspace the update refines but whose basis it
// does not; every cluster of 2..OA_KMAX members is therefore resolved by a
// Rayleigh-Ritz step in the same sweep: with N = I + R_CC/2 (first-order
// (X_C^T X_C)^(-1/2)), N S_CC N = V diag(mu) V^T is diagonalised by cyclic
// Jacobi in FP64 and W_C = N V.  With the block-diagonal W (identity outside
// the clusters) the sweep continues in the basis Y = X W:
// S' = W^T S W, R' = I - W^T (I - R) W, lam_C = mu, E' from S', R' as above,
// and X <- X W (I + E') = X + X (W (I + E') - I).
// All large products are FP64 MFMA GEMMs.
#include <vector>

#include "common.h"

namespace {

__global__ void oa_eye_kernel(int64_t n, double *M, int64_t ld)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        M[i + j * ld] = (i == j) ? 1.0 : 0.0;
    }
}

__global__ void oa_copy_kernel(int64_t n, const double *src, int64_t lds, double *dst, int64_t ldd)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        dst[i + j * ldd] = src[i + j * lds];
    }
}

// lam_i = s_ii / (1 - r_ii)
__global__ void oa_lambda_kernel(int64_t n, const double *S, const double *R, double *lam)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        lam[i] = S[i + i * n] / (1.0 - R[i + i * n]);
}

// partial sums per block: [0] ||S - diag(lam)||_F^2, [1] ||R||_F^2, [2] max |lam|
__global__ __launch_bounds__(256) void oa_norms_kernel(int64_t n, const double *S, const double *R, const double *lam,
                                                       double *part)
{
    __shared__ double r0[4], r1[4], r2[4];
    double a = 0.0, b = 0.0, c = 0.0;
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const double s = S[idx] - ((i == j) ? lam[i] : 0.0);
        a += s * s;
        b += R[idx] * R[idx];
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c = fmax(c, fabs(lam[i]));
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_max(c);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { r0[w] = a; r1[w] = b; r2[w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = r0[0] + r0[1] + r0[2] + r0[3];
        part[blockIdx.x * 3 + 1] = r1[0] + r1[1] + r1[2] + r1[3];
        part[blockIdx.x * 3 + 2] = fmax(fmax(r2[0], r2[1]), fmax(r2[2], r2[3]));
    }
}

// delta from the per-block partials (one thread; fixed order -> deterministic)
__global__ void oa_delta_kernel(int nblk, int64_t n, const double *part, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int q = 0; q < nblk; ++q) {
        a += part[q * 3 + 0];
        b += part[q * 3 + 1];
        c = fmax(c, part[q * 3 + 2]);
    }
    const double rn = sqrt(b);
    // at least sqrt(n eps) max|lam|: below that gap the Newton-type update
    // divides the rounding noise of S by the gap and loses orthogonality
    const double floor_ = sqrt((double)n * 2.220446049250313e-16) * c;
    out[0] = fmax(2.0 * (sqrt(a) + c * (1.0 + rn) * rn), floor_);  // delta
    out[1] = sqrt(a);
    out[2] = rn;
    out[3] = c;
}

constexpr int OA_KMAX = 64;  // largest cluster resolved by Rayleigh-Ritz

// Clusters along the column order (eigenvalue estimates arrive in ascending
// order up to errors far below delta): consecutive |lam_i - lam_{i-1}| <=
// delta.  Clusters of 2..OA_KMAX members are listed (begin, size, offset of
// their k x k blocks); cid[i] is the list index of column i's cluster or -1;
// larger clusters go to a second list (begin, size) resolved on the host side.
// meta: [0] listed small clusters, [1] largest cluster size, [2] large clusters.
__global__ void oa_cluster_kernel(int64_t n, const double *lam, const double *dl, int *cid, int *cl, int *meta,
                                  int *big)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double delta = dl[0];
    int ncl = 0, kmax = 1, nbig = 0;
    int64_t off = 0;
    int64_t b0 = 0;
    for (int64_t i = 1; i <= n; ++i) {
        if (i == n || fabs(lam[i] - lam[i - 1]) > delta) {
            const int k = (int)(i - b0);
            if (k > kmax) kmax = k;
            const bool rr = k >= 2 && k <= OA_KMAX;
            for (int64_t q = b0; q < i; ++q) cid[q] = rr ? ncl : -1;
            if (rr) {
                cl[3 * ncl + 0] = (int)b0;
                cl[3 * ncl + 1] = k;
                cl[3 * ncl + 2] = (int)off;
                off += (int64_t)k * k;
                ++ncl;
            } else if (k > OA_KMAX) {
                big[2 * nbig + 0] = (int)b0;
                big[2 * nbig + 1] = k;
                ++nbig;
            }
            b0 = i;
        }
    }
    meta[0] = ncl;
    meta[1] = kmax;
    meta[2] = nbig;
}

// Rayleigh-Ritz on one cluster per workgroup: N = I + R_CC/2, M = N S_CC N,
// cyclic Jacobi M = V diag(mu) V^T; writes W = N V (column-major k x k) and mu.
__global__ __launch_bounds__(256) void oa_rr_kernel(int64_t n, const double *S, const double *R, const int *cl,
                                                    const int *meta, double *Wg, double *lam)
{
    constexpr int LD = OA_KMAX + 1;
    __shared__ double A0[OA_KMAX * LD];
    __shared__ double A1[OA_KMAX * LD];
    __shared__ double A2[OA_KMAX * LD];
    __shared__ double rot[2];
    __shared__ double red[4];
    const int ncl = meta[0];
    for (int q = blockIdx.x; q < ncl; q += gridDim.x) {
    const int64_t b0 = cl[3 * q];
    const int k = cl[3 * q + 1];
    const int64_t off = cl[3 * q + 2];
    const int tid = threadIdx.x;
    __syncthreads();
    for (int e = tid; e < k * k; e += 256) {
        const int a = e % k, c = e / k;
        A0[a * LD + c] = S[(b0 + a) + (b0 + c) * n];
        A1[a * LD + c] = ((a == c) ? 1.0 : 0.0) + 0.5 * R[(b0 + a) + (b0 + c) * n];
    }
    __syncthreads();
    // A2 = S N, then A0 = N A2 = N S N
    for (int e = tid; e < k * k; e += 256) {
        const int a = e % k, c = e / k;
        double t = 0.0;
        for (int p = 0; p < k; ++p) t += A0[a * LD + p] * A1[p * LD + c];
        A2[a * LD + c] = t;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += 256) {
        const int a = e % k, c = e / k;
        double t = 0.0;
        for (int p = 0; p < k; ++p) t += A1[a * LD + p] * A2[p * LD + c];
        A0[a * LD + c] = t;
    }
    __syncthreads();
    // symmetrise (rounding) and V = I in A2
    for (int e = tid; e < k * k; e += 256) {
        const int a = e % k, c = e / k;
        if (a > c) {
            const double m = 0.5 * (A0[a * LD + c] + A0[c * LD + a]);
            A0[a * LD + c] = m;
            A0[c * LD + a] = m;
        }
        A2[a * LD + c] = (a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // cyclic Jacobi (Rutishauser's rotation, rotated pair set to zero), until
    // off(M) <= 1e-16 ||M||_F
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off2 = 0.0, tot = 0.0;
        for (int e = tid; e < k * k; e += 256) {
            const int a = e % k, c = e / k;
            const double m = A0[a * LD + c];
            tot += m * m;
            if (a != c) off2 += m * m;
        }
        off2 = block_sum(off2, red);
        tot = block_sum(tot, red);
        if (off2 <= 1e-32 * tot) break;
        for (int p = 0; p < k - 1; ++p) {
            for (int r = p + 1; r < k; ++r) {
                if (tid == 0) {
                    const double apq = A0[p * LD + r];
                    double c = 1.0, sn = 0.0;
                    if (apq != 0.0) {
                        const double th = (A0[r * LD + r] - A0[p * LD + p]) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                    rot[0] = c;
                    rot[1] = sn;
                }
                __syncthreads();
                const double c = rot[0], sn = rot[1];
                if (sn != 0.0) {
                    // rows p, r of M
                    for (int j = tid; j < k; j += 256) {
                        const double x = A0[p * LD + j], y = A0[r * LD + j];
                        A0[p * LD + j] = c * x - sn * y;
                        A0[r * LD + j] = sn * x + c * y;
                    }
                    __syncthreads();
                    // columns p, r of M and of V
                    for (int j = tid; j < k; j += 256) {
                        const double x = A0[j * LD + p], y = A0[j * LD + r];
                        A0[j * LD + p] = c * x - sn * y;
                        A0[j * LD + r] = sn * x + c * y;
                        const double u = A2[j * LD + p], w = A2[j * LD + r];
                        A2[j * LD + p] = c * u - sn * w;
                        A2[j * LD + r] = sn * u + c * w;
                    }
                    __syncthreads();
                    if (tid == 0) {
                        A0[p * LD + r] = 0.0;
                        A0[r * LD + p] = 0.0;
                    }
                }
                __syncthreads();
            }
        }
    }
    // Ritz values ascending (ties by index): column c of N V goes to position
    // rank(c), so the cluster's columns stay in eigenvalue order for the
    // next sweep's consecutive-gap clustering
    __shared__ int rank_[OA_KMAX];
    for (int c = tid; c < k; c += 256) {
        const double key = A0[c * LD + c];
        int r = 0;
        for (int q = 0; q < k; ++q) {
            const double v = A0[q * LD + q];
            r += (v < key || (v == key && q < c)) ? 1 : 0;
        }
        rank_[c] = r;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += 256) {
        const int a = e % k, c = e / k;
        double t = 0.0;
        for (int p = 0; p < k; ++p) t += A1[a * LD + p] * A2[p * LD + c];
        Wg[off + a + rank_[c] * k] = t;
    }
    for (int a = tid; a < k; a += 256) lam[b0 + rank_[a]] = A0[a * LD + a];
    }
}

// M(i, C) <- M(i, C) W_C for every row i and resolved cluster C (one thread
// per row; the cluster's k entries of the row stay in registers).
__global__ __launch_bounds__(256) void oa_colrot_kernel(int64_t n, double *M, const int *cl, const int *meta,
                                                        const double *Wg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ncl = meta[0];
    for (int q = blockIdx.y; q < ncl; q += gridDim.y) {
        const int64_t b0 = cl[3 * q];
        const int k = cl[3 * q + 1];
        const double *W = Wg + cl[3 * q + 2];
        double *Mr = M + i + b0 * n;
        double e[OA_KMAX];
#pragma unroll
        for (int c = 0; c < OA_KMAX; ++c) e[c] = (c < k) ? Mr[c * n] : 0.0;
        for (int c = 0; c < k; ++c) {
            double t = 0.0;
#pragma unroll
            for (int p = 0; p < OA_KMAX; ++p)
                if (p < k) t += e[p] * W[p + c * k];
            Mr[c * n] = t;
        }
    }
}

// M(C, j) <- op(W_C) M(C, j) for every column j (op = transpose if trans).
__global__ __launch_bounds__(256) void oa_rowrot_kernel(int64_t n, double *M, const int *cl, const int *meta,
                                                        const double *Wg, int trans)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int ncl = meta[0];
    for (int q = blockIdx.y; q < ncl; q += gridDim.y) {
        const int64_t b0 = cl[3 * q];
        const int k = cl[3 * q + 1];
        const double *W = Wg + cl[3 * q + 2];
        double *Mc = M + b0 + j * n;
        double e[OA_KMAX];
#pragma unroll
        for (int c = 0; c < OA_KMAX; ++c) e[c] = (c < k) ? Mc[c] : 0.0;
        for (int a = 0; a < k; ++a) {
            double t = 0.0;
#pragma unroll
            for (int p = 0; p < OA_KMAX; ++p)
                if (p < k) t += (trans ? W[p + a * k] : W[a + p * k]) * e[p];
            Mc[a] = t;
        }
    }
}

// Diagonal blocks after the rotation Y_C = X_C W_C:
//   R'_CC = I - W^T (I - R_CC) W  (the passes left W^T R_CC W: add I - W^T W);
//   mode 1 (update): E_CC += W - I.
__global__ __launch_bounds__(256) void oa_diagfix_kernel(double *M, int64_t n, const int *cl, const int *meta,
                                                         const double *Wg, int mode)
{
    const int ncl = meta[0];
    for (int q = blockIdx.x; q < ncl; q += gridDim.x) {
        const int64_t b0 = cl[3 * q];
        const int k = cl[3 * q + 1];
        const double *W = Wg + cl[3 * q + 2];
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
            const int a = e % k, c = e / k;
            double v;
            if (mode == 0) {
                double t = 0.0;
                for (int p = 0; p < k; ++p) t += W[p + a * k] * W[p + c * k];
                v = ((a == c) ? 1.0 : 0.0) - t;
            } else {
                v = W[a + c * k] - ((a == c) ? 1.0 : 0.0);
            }
            M[(b0 + a) + (b0 + c) * n] += v;
        }
    }
}

// N = I + R_CC / 2 for a large cluster (k x k, leading dimension k)
__global__ void oa_make_n_kernel(int64_t k, const double *Rc, int64_t ldr, double *N)
{
    const int64_t total = k * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = idx % k, c = idx / k;
        N[idx] = ((a == c) ? 1.0 : 0.0) + 0.5 * Rc[a + c * ldr];
    }
}

__global__ void oa_copy2d_kernel(int64_t m, int64_t ncol, const double *src, int64_t lds, double *dst, int64_t ldd)
{
    const int64_t total = m * ncol;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % m, j = idx / m;
        dst[i + j * ldd] = src[i + j * lds];
    }
}

// M_CC += sign * (I or W): mode 0 adds I, mode 1 adds W - I
__global__ void oa_add_block_kernel(int64_t k, double *Mc, int64_t ldm, const double *W, int mode)
{
    const int64_t total = k * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = idx % k, c = idx / k;
        const double id = (a == c) ? 1.0 : 0.0;
        Mc[a + c * ldm] += (mode == 0) ? id : W[idx] - id;
    }
}

// E_ij as in RefSyEv from the symmetric parts of S and R (the computed
// products are symmetric only up to rounding; the asymmetric part divided by
// a small eigenvalue gap would break the orthogonality E_ij + E_ji = r_ij).
__global__ void oa_e_kernel(int64_t n, const double *S, const double *R, const double *lam, const double *dl,
                            double *E)
{
    const double delta = dl[0];
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const int64_t tdx = j + i * n;
        const double r = 0.5 * (R[idx] + R[tdx]);
        const double sv = 0.5 * (S[idx] + S[tdx]);
        const double d = lam[j] - lam[i];
        E[idx] = (i != j && fabs(d) > delta) ? (sv + lam[j] * r) / d : 0.5 * r;
    }
}

// residual partials: ||A X - X diag(lam)||_F^2 (AX given) and ||A||_F^2 (lower stored)
__global__ __launch_bounds__(256) void oa_resid_kernel(int64_t n, const double *AX, const double *X, const double *lam,
                                                       const double *A, int64_t lda, double *part)
{
    __shared__ double r0[4], r1[4];
    double a = 0.0, b = 0.0;
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        const double r = AX[idx] - X[idx] * lam[j];
        a += r * r;
        if (i >= j) {
            const double v = A[i + j * lda];
            b += (i == j) ? v * v : 2.0 * v * v;
        }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { r0[w] = a; r1[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2 + 0] = r0[0] + r0[1] + r0[2] + r0[3];
        part[blockIdx.x * 2 + 1] = r1[0] + r1[1] + r1[2] + r1[3];
    }
}

__global__ void oa_resid_final_kernel(int nblk, int64_t n, const double *part, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int q = 0; q < nblk; ++q) { a += part[q * 2]; b += part[q * 2 + 1]; }
    out[0] = (b > 0.0) ? sqrt(a) / ((double)n * sqrt(b)) : sqrt(a);
}

// Rayleigh quotients lam_j = (x_j . (A x_j)) / (x_j . x_j), one wavefront per column
__global__ __launch_bounds__(64) void oa_rayleigh_kernel(int64_t n, const double *AX, const double *X, int64_t ldx,
                                                         double *lam)
{
    const int64_t j = blockIdx.x;
    if (j >= n) return;
    double num = 0.0, den = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 64) {
        const double x = X[i + j * ldx];
        num += x * AX[i + j * n];
        den += x * x;
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if (threadIdx.x == 0) lam[j] = num / den;
}

// M(j, i) <- M(i, j) for i > j: the products whose lower triangle alone is
// computed (R = I - X^T X and S = X^T (A X), symmetric) in full storage
__global__ void oa_mirror_kernel(int64_t n, double *M)
{
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        if (i > j) M[j + i * n] = M[idx];
    }
}

// ||R||_F^2 partials (R = I - X^T X in full storage)
__global__ __launch_bounds__(256) void oa_rnorm_kernel(int64_t n, const double *R, double *part)
{
    __shared__ double r0[4];
    double a = 0.0;
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x)
        a += R[idx] * R[idx];
    a = wave_sum(a);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) r0[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = r0[0] + r0[1] + r0[2] + r0[3];
}

__global__ void oa_orth_final_kernel(int nblk, int64_t n, const double *part, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0;
    for (int q = 0; q < nblk; ++q) a += part[q];
    out[0] = sqrt(a) / (double)n;
}

// last sweep's figures into the caller's statistics: [2] sweeps, [3] delta,
// [4] clusters resolved, [5] largest cluster, [6] ||S - diag(lam)||_F, [7] ||R||_F
__global__ void oa_meta_stats_kernel(const int *meta, const double *dl, int sweeps, double *stats)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        stats[2] = (double)sweeps;
        stats[3] = sweeps > 0 ? dl[0] : 0.0;
        stats[4] = sweeps > 0 ? (double)meta[0] : 0.0;
        stats[5] = sweeps > 0 ? (double)meta[1] : 0.0;
        stats[6] = sweeps > 0 ? dl[1] : 0.0;
        stats[7] = sweeps > 0 ? dl[2] : 0.0;
    }
}

constexpr int OA_BLOCKS = 1024;

}  // namespace

size_t dsyevd_work_bytes_any_b(int64_t n);

namespace {

// Large clusters (more than OA_KMAX members) are resolved with the FP64
// two-stage solver on their k x k block; their rotations share one store of
// n^2 doubles (the clusters are disjoint, so every cluster fits: a cluster
// left unresolved would get Newton updates between members whose gaps only
// just exceed delta, and lose orthogonality).
int64_t big_capacity(int64_t n) { return n > OA_KMAX ? n : 0; }

struct RefWork {
    double *R, *AX, *S, *Xn, *part, *Wg, *dl;
    int *cid, *cl, *meta, *big;
    double *bN, *bM, *bW, *bmu;
    void *bws;
    size_t bws_bytes;
    int64_t kcap;
};

size_t ref_layout(int64_t n, char *base, RefWork *w)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += evd_align256(bytes > 0 ? bytes : 1);
        return (void *)p;
    };
    RefWork t;
    t.R = (double *)take(nn * nn * 8);
    t.AX = (double *)take(nn * nn * 8);
    t.S = (double *)take(nn * nn * 8);
    t.Xn = (double *)take(nn * nn * 8);
    t.part = (double *)take((size_t)OA_BLOCKS * 3 * 8);
    t.Wg = (double *)take(nn * OA_KMAX * 8);
    t.dl = (double *)take(64);
    t.cid = (int *)take(nn * 4);
    t.cl = (int *)take(nn * 3 * 4);
    t.meta = (int *)take(64);
    t.big = (int *)take(nn * 2 * 4);
    t.kcap = big_capacity(n);
    const size_t kc = (size_t)t.kcap;
    t.bN = (double *)take(kc * kc * 8);
    t.bM = (double *)take(kc * kc * 8);
    t.bW = (double *)take(kc * kc * 8);
    t.bmu = (double *)take(kc * 8);
    t.bws_bytes = kc > 0 ? dsyevd_work_bytes_any_b((int64_t)kc) : 0;
    t.bws = take(t.bws_bytes);
    if (w) *w = t;
    return off;
}

struct BigC {
    int64_t b0, k;
    double *W;
};

// Rayleigh-Ritz of the large clusters (host loop; reads the cluster list back):
// N = I + R_CC/2, N S_CC N = V diag(mu) V^T by evd_dsyevd, W = N V; then
// S' and R' in the rotated basis for those clusters.
evd_status_t big_clusters_begin(evd_ctx_t ctx, int64_t n, double *S, double *R, double *lam, RefWork &w,
                                std::vector<BigC> &done)
{
    hipStream_t s = ctx->stream;
    done.clear();
    if (w.kcap <= 0) return EVD_OK;
    int hm[4] = {0, 0, 0, 0};
    EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(hm, w.meta, sizeof(hm), hipMemcpyDeviceToHost, s)));
    EVD_CHECK(evd_hip(ctx, hipStreamSynchronize(s)));
    const int nbig = hm[2];
    if (nbig <= 0) return EVD_OK;
    std::vector<int> bl(2 * (size_t)nbig);
    EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(bl.data(), w.big, bl.size() * sizeof(int), hipMemcpyDeviceToHost, s)));
    EVD_CHECK(evd_hip(ctx, hipStreamSynchronize(s)));
    const dim3 g(256), t(256);
    size_t used = 0;
    const size_t capacity = (size_t)w.kcap * (size_t)w.kcap;
    const int64_t saved_timing = ctx->timing;
    for (int q = 0; q < nbig; ++q) {
        const int64_t b0 = bl[2 * q], k = bl[2 * q + 1];
        if (k > w.kcap || used + (size_t)(k * k) > capacity) continue;
        double *Wk = w.bW + used;
        hipLaunchKernelGGL(oa_make_n_kernel, g, t, 0, s, k, (const double *)(R + b0 + b0 * n), n, w.bN);
        // T = S_CC N (in the W slot), M = N T
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, k, k, k, 1.0, S + b0 + b0 * n, n, w.bN, k, 0.0, Wk, k, nullptr, 0));
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, k, k, k, 1.0, w.bN, k, Wk, k, 0.0, w.bM, k, nullptr, 0));
        ctx->timing = 0;
        const evd_status_t st = evd_dsyevd(ctx, 'V', 'L', k, w.bM, k, w.bmu, w.bws, w.bws_bytes, w.meta + 4);
        ctx->timing = saved_timing;
        EVD_CHECK(st);
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, k, k, k, 1.0, w.bN, k, w.bM, k, 0.0, Wk, k, nullptr, 0));
        hipLaunchKernelGGL(oa_copy2d_kernel, dim3(64), t, 0, s, k, (int64_t)1, (const double *)w.bmu, k, lam + b0, k);
        done.push_back({b0, k, Wk});
        used += (size_t)(k * k);
    }
    // S' = W^T S W and R' = W^T R W on the resolved clusters' rows and columns
    for (const BigC &c : done) {
        for (int which = 0; which < 2; ++which) {
            double *M = which ? R : S;
            EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, n, c.k, c.k, 1.0, M + c.b0 * n, n, c.W, c.k, 0.0, w.Xn, n, nullptr, 0));
            hipLaunchKernelGGL(oa_copy2d_kernel, g, t, 0, s, n, c.k, (const double *)w.Xn, n, M + c.b0 * n, n);
            EVD_CHECK(gemm_f64(s, OP_T, OP_N, 0, c.k, n, c.k, 1.0, c.W, c.k, M + c.b0, n, 0.0, w.Xn, c.k, nullptr, 0));
            hipLaunchKernelGGL(oa_copy2d_kernel, g, t, 0, s, c.k, n, (const double *)w.Xn, c.k, M + c.b0, n);
        }
        // R'_CC = I - W^T (I - R_CC) W = (W^T R_CC W) + I - W^T W
        EVD_CHECK(gemm_f64(s, OP_T, OP_N, 0, c.k, c.k, c.k, -1.0, c.W, c.k, c.W, c.k, 1.0, R + c.b0 + c.b0 * n, n,
                           nullptr, 0));
        hipLaunchKernelGGL(oa_add_block_kernel, g, t, 0, s, c.k, R + c.b0 + c.b0 * n, n, (const double *)c.W, 0);
    }
    return evd_hip(ctx, hipGetLastError());
}

// F = W (I + E') - I on the large clusters' rows: E(C, :) <- W E(C, :), E_CC += W - I
evd_status_t big_clusters_end(evd_ctx_t ctx, int64_t n, double *E, RefWork &w, const std::vector<BigC> &done)
{
    hipStream_t s = ctx->stream;
    const dim3 g(256), t(256);
    for (const BigC &c : done) {
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, c.k, n, c.k, 1.0, c.W, c.k, E + c.b0, n, 0.0, w.Xn, c.k, nullptr, 0));
        hipLaunchKernelGGL(oa_copy2d_kernel, g, t, 0, s, c.k, n, (const double *)w.Xn, c.k, E + c.b0, n);
        hipLaunchKernelGGL(oa_add_block_kernel, g, t, 0, s, c.k, E + c.b0 + c.b0 * n, n, (const double *)c.W, 1);
    }
    return evd_hip(ctx, hipGetLastError());
}

}  // namespace

size_t refine_work_bytes(int64_t n) { return ref_layout(n, nullptr, nullptr); }

// RefSyEv sweeps on X (n x n, ldx), A FP64 symmetric in full storage (both
// triangles; the residual norms read the lower one), on the context's
// stream, at most max_sweeps of them.  Before each sweep (and after the
// last) the current X is checked: R = I - X^T X and A X are formed (they are
// the sweep's first products anyway), lam = the Rayleigh quotients of X's
// columns, stats[0] = ||A X - X diag(lam)||_F / (n ||A||_F) and stats[1] =
// ||X^T X - I||_F / n.  With target > 0 the check is read on the host (one
// synchronisation per sweep) and the sweeps stop once both are <= target;
// with target <= 0 exactly max_sweeps sweeps run without a host round trip
// (resolving clusters of more than 64 members reads the cluster list back,
// once per sweep).  stats (device, 8 doubles): [0] residual and [1]
// orthogonality of the returned X, [2] sweeps run, then of the last sweep
// [3] delta, [4] clusters resolved by Rayleigh-Ritz, [5] the largest cluster
// size, [6] ||S - diag(lam)||_F, [7] ||R||_F.  lam (n) receives the Rayleigh
// quotients of the returned X.  Returns the sweep count in *done.
evd_status_t refine_run(evd_ctx_t ctx, int64_t n, const double *A, int64_t lda, double *X, int64_t ldx, double *lam,
                        int max_sweeps, double target, void *work, double *stats, int *done)
{
    hipStream_t s = ctx->stream;
    RefWork w;
    ref_layout(n, (char *)work, &w);
    double *R = w.R, *AX = w.AX, *S = w.S, *Xn = w.Xn, *part = w.part;
    const dim3 g(OA_BLOCKS), t(256);
    std::vector<BigC> big;
    int sw = 0;
    for (;; ++sw) {
        // R = I - X^T X (lower triangle computed, mirrored), A X
        hipLaunchKernelGGL(oa_eye_kernel, g, t, 0, s, n, R, n);
        EVD_CHECK(gemm_f64(s, OP_T, OP_N, 1, n, n, n, -1.0, X, ldx, X, ldx, 1.0, R, n, nullptr, 0));
        hipLaunchKernelGGL(oa_mirror_kernel, g, t, 0, s, n, R);
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, n, n, n, 1.0, A, lda, X, ldx, 0.0, AX, n, nullptr, 0));
        // check of the current X
        hipLaunchKernelGGL(oa_rayleigh_kernel, dim3((unsigned)n), dim3(64), 0, s, n, (const double *)AX,
                           (const double *)X, ldx, lam);
        hipLaunchKernelGGL(oa_resid_kernel, g, t, 0, s, n, (const double *)AX, (const double *)X,
                           (const double *)lam, A, lda, part);
        hipLaunchKernelGGL(oa_resid_final_kernel, dim3(1), dim3(64), 0, s, OA_BLOCKS, n, (const double *)part,
                           stats);
        hipLaunchKernelGGL(oa_rnorm_kernel, g, t, 0, s, n, (const double *)R, part);
        hipLaunchKernelGGL(oa_orth_final_kernel, dim3(1), dim3(64), 0, s, OA_BLOCKS, n, (const double *)part,
                           stats + 1);
        if (sw >= max_sweeps) break;
        if (target > 0.0) {
            double h[2] = {0.0, 0.0};
            EVD_CHECK(evd_hip(ctx, hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, s)));
            EVD_CHECK(evd_hip(ctx, hipStreamSynchronize(s)));
            if (h[0] <= target && h[1] <= target) break;
        }
        // S = X^T (A X) (lower triangle computed, mirrored)
        EVD_CHECK(gemm_f64(s, OP_T, OP_N, 1, n, n, n, 1.0, X, ldx, AX, n, 0.0, S, n, nullptr, 0));
        hipLaunchKernelGGL(oa_mirror_kernel, g, t, 0, s, n, S);
        hipLaunchKernelGGL(oa_lambda_kernel, dim3(64), t, 0, s, n, (const double *)S, (const double *)R, lam);
        hipLaunchKernelGGL(oa_norms_kernel, g, t, 0, s, n, (const double *)S, (const double *)R, (const double *)lam,
                           part);
        hipLaunchKernelGGL(oa_delta_kernel, dim3(1), dim3(64), 0, s, OA_BLOCKS, n, (const double *)part, w.dl);
        hipLaunchKernelGGL(oa_cluster_kernel, dim3(1), dim3(64), 0, s, n, (const double *)lam, (const double *)w.dl,
                           w.cid, w.cl, w.meta, w.big);
        // Rayleigh-Ritz on the clusters, then S' = Wbd^T S Wbd, R' = I - Wbd^T (I - R) Wbd
        const unsigned maxcl = (unsigned)(n / 2 < 1024 ? (n / 2 > 0 ? n / 2 : 1) : 1024);
        const dim3 gr((unsigned)evd_ceil_div(n, 256), maxcl < 64 ? maxcl : 64);
        hipLaunchKernelGGL(oa_rr_kernel, dim3(maxcl), t, 0, s, n, (const double *)S, (const double *)R,
                           (const int *)w.cl, (const int *)w.meta, w.Wg, lam);
        for (int which = 0; which < 2; ++which) {
            double *M = which ? R : S;
            hipLaunchKernelGGL(oa_colrot_kernel, gr, t, 0, s, n, M, (const int *)w.cl, (const int *)w.meta,
                               (const double *)w.Wg);
            hipLaunchKernelGGL(oa_rowrot_kernel, gr, t, 0, s, n, M, (const int *)w.cl, (const int *)w.meta,
                               (const double *)w.Wg, 1);
        }
        hipLaunchKernelGGL(oa_diagfix_kernel, dim3(maxcl), t, 0, s, R, n, (const int *)w.cl, (const int *)w.meta,
                           (const double *)w.Wg, 0);
        EVD_CHECK(big_clusters_begin(ctx, n, S, R, lam, w, big));
        // E' in the rotated basis, then F = Wbd (I + E') - I
        double *E = AX;  // A X is no longer needed
        hipLaunchKernelGGL(oa_e_kernel, g, t, 0, s, n, (const double *)S, (const double *)R, (const double *)lam,
                           (const double *)w.dl, E);
        hipLaunchKernelGGL(oa_rowrot_kernel, gr, t, 0, s, n, E, (const int *)w.cl, (const int *)w.meta,
                           (const double *)w.Wg, 0);
        hipLaunchKernelGGL(oa_diagfix_kernel, dim3(maxcl), t, 0, s, E, n, (const int *)w.cl, (const int *)w.meta,
                           (const double *)w.Wg, 1);
        EVD_CHECK(big_clusters_end(ctx, n, E, w, big));
        hipLaunchKernelGGL(oa_copy_kernel, g, t, 0, s, n, (const double *)X, ldx, Xn, n);
        EVD_CHECK(gemm_f64(s, OP_N, OP_N, 0, n, n, n, 1.0, X, ldx, E, n, 1.0, Xn, n, nullptr, 0));
        hipLaunchKernelGGL(oa_copy_kernel, g, t, 0, s, n, (const double *)Xn, n, X, ldx);
    }
    hipLaunchKernelGGL(oa_meta_stats_kernel, dim3(1), dim3(64), 0, s, (const int *)w.meta, (const double *)w.dl, sw,
                       stats);
    if (done) *done = sw;
    return evd_hip(ctx, hipGetLastError());
}
