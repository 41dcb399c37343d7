// Stage 3: symmetric tridiagonal eigensolver (paper Section 2.1.1: divide and
// conquer after Cuppen, Gu-Eisenstat and Tisseur-Dongarra; the reordered
// stages of Section 3.3 make it independent of the back transformation).
//
// T = tridiag(e, d, e) is torn at every boundary of a binary partition whose
// leaves have size 1:  T = diag(T_1, T_2) + |rho| v v^T,  v = e_k + sign(rho)
// e_{k+1},  so every diagonal entry is first reduced by the couplings on both
// sides and the leaves are solved (eigenvalue d'_j, eigenvector e_j).  The
// merges run bottom-up, one launch per kernel per tree level for all nodes of
// that level:
//   prep     z = [last row of Q_1; sign(rho) first row of Q_2] / sqrt 2,
//            sigma = 2 |rho|; merge the two sorted eigenvalue lists
//            (merge path); deflate small sigma |z_i| <= tol and close pairs
//            (a Givens rotation that zeroes z_p moves D by |t c s| <= tol),
//            tol = 8 eps max(max|D|, sigma); group the surviving columns by
//            which child they draw from (left / mixed / right).
//   qp       permuted, rotated copy of the children's eigenvectors.
//   secular  one root per lane: f(lam) = 1 + sigma sum z_i^2/(D_i - lam) = 0
//            in (D_j, D_j+1) (or beyond the last pole), kept as
//            (nearest pole, offset tau); bracketing plus a two-pole rational
//            model (Bunch-Nielsen-Sorensen), bisection fallback.
//   zhat     Gu-Eisenstat: z_i recomputed from the computed roots (Loewner).
//   vec      u_j = zhat ./ (D - lam_j), normalised (one wavefront per column).
//   gemm     Q = [Q_1 0; 0 Q_2] P G U as two grouped products that skip the
//            zero blocks (rows of the left child only meet left/mixed columns).
//   final    ascending order of (roots, deflated values), columns scattered.
// Eigenvalues only ('N'): Sturm-count bisection, one eigenvalue per lane.
#include "common.h"

namespace {

constexpr double DC_EPS = 2.220446049250313e-16;  // 2^-52

__device__ __forceinline__ void node_range(int64_t n, int t, int64_t i, int64_t *lo, int64_t *mid, int64_t *hi)
{
    *lo = (i * n) >> t;
    *hi = ((i + 1) * n) >> t;
    *mid = ((2 * i + 1) * n) >> (t + 1);
}

struct DcArrays {
    double *Dw;      // n: working eigenvalues (node blocks)
    double *Dsort;   // n: merged D (node-local sorted index u)
    double *zsort;   // n
    int *srcCol;     // n: sorted u -> original column within node
    int *status;     // n: 0 deflated, 1 left, 2 right, 3 mixed
    double *Dfin;    // n: D after deflation rotations (sorted u)
    double *zfin;    // n
    int *destCol;    // n: sorted u -> column of Qp
    double *Dk;      // n: non-deflated D (sorted, index j)
    double *zk;      // n
    int *gpos;       // n: non-deflated j -> row of U / column of Qp
    double *lam;     // n: roots
    int *org;        // n: pole index of root j
    double *tauj;    // n: offset of root j from its pole
    double *zhat;    // n
    double *Ddef;    // n: deflated values (index r)
    int *rotP;       // n
    int *rotI;       // n
    double *rotC;    // n
    double *rotS;    // n
    int *outSrc;     // n: output position -> source column (j < K: product column, else Qp column)
    int *info;       // node info, 8 ints per node: K, K1, K2, K3, nrot, ndef, active, -
    GemmProblem *probs;
    double *Qp;      // n x n
    double *U;       // n x n
    double *Tmp;     // n x n
    int *flag;       // 1 int: non-convergence
};

__global__ void dc_init_kernel(int64_t n, const double *d, const double *e, double *Dw, double *Z, int64_t ldz)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double left = (j > 0) ? fabs(e[j - 1]) : 0.0;
        const double right = (j + 1 < n) ? fabs(e[j]) : 0.0;
        Dw[j] = d[j] - left - right;
    }
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        Z[i + j * ldz] = (i == j) ? 1.0 : 0.0;
    }
}

constexpr int PREP_T = 256;
constexpr int PREP_CH = 1024;

__global__ __launch_bounds__(PREP_T) void dc_prep_kernel(int64_t n, int t, const double *e, const double *Z,
                                                         int64_t ldz, DcArrays a)
{
    __shared__ double sD[PREP_CH];
    __shared__ double sZ[PREP_CH];
    __shared__ int sSt[PREP_CH];
    __shared__ double red[PREP_T / 64];
    __shared__ int cnt[5][PREP_T + 1];

    const int64_t i = blockIdx.x;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int64_t s = hi - lo, n1 = mid - lo, n2 = hi - mid;
    int *info = a.info + i * 8;
    const int tid = threadIdx.x;
    if (n1 == 0 || n2 == 0) {
        if (tid == 0) {
            info[6] = 0;
            a.probs[2 * i] = GemmProblem{nullptr, nullptr, nullptr, 1, 1, 1, 0, 0, 0};
            a.probs[2 * i + 1] = GemmProblem{nullptr, nullptr, nullptr, 1, 1, 1, 0, 0, 0};
        }
        return;
    }
    const double rho = e[mid - 1];
    const double sigma = 2.0 * fabs(rho);
    const double sgn = (rho >= 0.0) ? 1.0 : -1.0;
    const double rs2 = 0.70710678118654752440;
    const double *DL = a.Dw + lo, *DR = a.Dw + mid;

    // ---- merge path: thread tid produces outputs [u0, u1)
    {
        const int64_t per = (s + PREP_T - 1) / PREP_T;
        const int64_t u0 = tid * per < s ? tid * per : s;
        const int64_t u1 = u0 + per < s ? u0 + per : s;
        int64_t l = u0 > n2 ? u0 - n2 : 0, h = u0 < n1 ? u0 : n1;
        while (l < h) {
            const int64_t md = (l + h) >> 1;
            if (DL[md] <= DR[u0 - md - 1]) l = md + 1;
            else h = md;
        }
        int64_t pa = l, pb = u0 - l;
        for (int64_t u = u0; u < u1; ++u) {
            const bool takeA = pa < n1 && (pb >= n2 || DL[pa] <= DR[pb]);
            if (takeA) {
                a.Dsort[lo + u] = DL[pa];
                a.zsort[lo + u] = Z[(mid - 1) + (lo + pa) * ldz] * rs2;
                a.srcCol[lo + u] = (int)pa;
                ++pa;
            } else {
                a.Dsort[lo + u] = DR[pb];
                a.zsort[lo + u] = sgn * Z[mid + (mid + pb) * ldz] * rs2;
                a.srcCol[lo + u] = (int)(n1 + pb);
                ++pb;
            }
        }
    }
    __syncthreads();
    // ---- tolerance
    double dm = 0.0;
    for (int64_t u = tid; u < s; u += PREP_T) dm = fmax(dm, fabs(a.Dsort[lo + u]));
    dm = wave_max(dm);
    if ((tid & 63) == 0) red[tid >> 6] = dm;
    __syncthreads();
    dm = red[0];
    for (int w = 1; w < PREP_T / 64; ++w) dm = fmax(dm, red[w]);
    const double tol = 8.0 * DC_EPS * fmax(dm, sigma);

    // ---- deflation scan (sequential chain; data staged through LDS)
    int pend = -1, pendSt = 0, nrot = 0;
    double pD = 0.0, pZ = 0.0;
    for (int64_t c0 = 0; c0 < s; c0 += PREP_CH) {
        const int len = (int)((s - c0) < PREP_CH ? (s - c0) : PREP_CH);
        __syncthreads();
        for (int q = tid; q < len; q += PREP_T) {
            sD[q] = a.Dsort[lo + c0 + q];
            sZ[q] = a.zsort[lo + c0 + q];
            sSt[q] = (a.srcCol[lo + c0 + q] < n1) ? 1 : 2;
        }
        __syncthreads();
        if (tid == 0) {
            for (int q = 0; q < len; ++q) {
                const int u = (int)(c0 + q);
                const double Du = sD[q], zu = sZ[q];
                if (sigma * fabs(zu) <= tol) {
                    a.status[lo + u] = 0;
                    a.Dfin[lo + u] = Du;
                    a.zfin[lo + u] = 0.0;
                    continue;
                }
                if (pend < 0) { pend = u; pD = Du; pZ = zu; pendSt = sSt[q]; continue; }
                const double tt = Du - pD;
                const double r = hypot(pZ, zu);
                const double cc = zu / r, sn = pZ / r;
                if (fabs(tt * cc * sn) <= tol) {
                    // rotate in the plane (pend, u): z_pend -> 0, pend deflates
                    const double dp = pD * cc * cc + Du * sn * sn;
                    const double du = pD * sn * sn + Du * cc * cc;
                    a.rotP[lo + nrot] = pend;
                    a.rotI[lo + nrot] = u;
                    a.rotC[lo + nrot] = cc;
                    a.rotS[lo + nrot] = sn;
                    ++nrot;
                    a.status[lo + pend] = 0;
                    a.Dfin[lo + pend] = dp;
                    a.zfin[lo + pend] = 0.0;
                    pend = u;
                    pD = du;
                    pZ = r;
                    pendSt = pendSt | sSt[q];
                } else {
                    a.status[lo + pend] = pendSt;
                    a.Dfin[lo + pend] = pD;
                    a.zfin[lo + pend] = pZ;
                    pend = u;
                    pD = Du;
                    pZ = zu;
                    pendSt = sSt[q];
                }
            }
        }
    }
    if (tid == 0 && pend >= 0) {
        a.status[lo + pend] = pendSt;
        a.Dfin[lo + pend] = pD;
        a.zfin[lo + pend] = pZ;
    }
    __syncthreads();
    __threadfence_block();

    // ---- positions: counts per category over contiguous segments
    const int64_t per = (s + PREP_T - 1) / PREP_T;
    const int64_t u0 = tid * per < s ? tid * per : s;
    const int64_t u1 = u0 + per < s ? u0 + per : s;
    int c[5] = {0, 0, 0, 0, 0};  // deflated, left, right, mixed, all non-deflated
    for (int64_t u = u0; u < u1; ++u) {
        const int st = a.status[lo + u];
        c[st]++;
        if (st) c[4]++;
    }
    for (int k = 0; k < 5; ++k) cnt[k][tid] = c[k];
    __syncthreads();
    if (tid < 5) {
        int acc = 0;
        for (int q = 0; q < PREP_T; ++q) { const int v = cnt[tid][q]; cnt[tid][q] = acc; acc += v; }
        cnt[tid][PREP_T] = acc;
    }
    __syncthreads();
    const int K1 = cnt[1][PREP_T], K3r = cnt[2][PREP_T], K2m = cnt[3][PREP_T];
    const int K = cnt[4][PREP_T];
    int pos[5];
    for (int k = 0; k < 5; ++k) pos[k] = cnt[k][tid];
    for (int64_t u = u0; u < u1; ++u) {
        const int st = a.status[lo + u];
        int dc;
        if (st == 0) {
            dc = K + pos[0];
            a.Ddef[lo + pos[0]] = a.Dfin[lo + u];
            pos[0]++;
        } else {
            if (st == 1) dc = pos[1]++;
            else if (st == 3) dc = K1 + pos[3]++;
            else dc = K1 + K2m + pos[2]++;
            const int j = pos[4]++;
            a.Dk[lo + j] = a.Dfin[lo + u];
            a.zk[lo + j] = a.zfin[lo + u];
            a.gpos[lo + j] = dc;
        }
        a.destCol[lo + u] = dc;
    }
    if (tid == 0) {
        info[0] = K;
        info[1] = K1;
        info[2] = K2m;
        info[3] = K3r;
        info[4] = nrot;
        info[5] = (int)(s - K);
        info[6] = 1;
        const int64_t ld = n;
        double *Qb = a.Qp + lo + lo * ld;
        double *Ub = a.U + lo + lo * ld;
        double *Tb = a.Tmp + lo + lo * ld;
        // rows of the left child meet columns [0, K1+K2) only; right child [K1, K)
        a.probs[2 * i] = GemmProblem{Qb, Ub, Tb, ld, ld, ld, n1, K, K1 + K2m};
        a.probs[2 * i + 1] = GemmProblem{Qb + n1 + (int64_t)K1 * ld, Ub + K1, Tb + n1, ld, ld, ld, n2, K, K2m + K3r};
    }
}

// Columns of a node block per workgroup of the column copies (grid z): the
// copies of a large node are spread over the whole chip instead of one
// thread per row walking every column.
constexpr int DC_CC = 256;

// Qp[:, destCol[u]] = Z[:, srcCol[u]] for the node block: thread per row,
// workgroup z for columns [z DC_CC, (z + 1) DC_CC), eight loads in flight.
__global__ __launch_bounds__(256) void dc_qp_kernel(int64_t n, int t, const double *Z, int64_t ldz, DcArrays a)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int64_t s = hi - lo;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t u0 = (int64_t)blockIdx.z * DC_CC;
    if (r >= s || u0 >= s) return;
    const int64_t u1 = (u0 + DC_CC < s) ? u0 + DC_CC : s;
    const int64_t ld = n;
    const double *Zr = Z + lo + r + lo * ldz;
    double *Qr = a.Qp + lo + r + lo * ld;
    const int *src = a.srcCol + lo, *dst = a.destCol + lo;
    int64_t u = u0;
    for (; u + 8 <= u1; u += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = Zr[(int64_t)src[u + q] * ldz];
#pragma unroll
        for (int q = 0; q < 8; ++q) Qr[(int64_t)dst[u + q] * ld] = v[q];
    }
    for (; u < u1; ++u) Qr[(int64_t)dst[u] * ld] = Zr[(int64_t)src[u] * ldz];
}

// The deflation rotations on Qp, in order; one thread per row (after the
// column copies of dc_qp_kernel).
__global__ __launch_bounds__(256) void dc_rot_kernel(int64_t n, int t, DcArrays a)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int64_t s = hi - lo;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= s) return;
    const int64_t ld = n;
    double *Qr = a.Qp + lo + r + lo * ld;
    const int nrot = info[4];
    for (int k = 0; k < nrot; ++k) {
        const int64_t ca = a.destCol[lo + a.rotP[lo + k]], cb = a.destCol[lo + a.rotI[lo + k]];
        const double c = a.rotC[lo + k], sn = a.rotS[lo + k];
        const double x = Qr[ca * ld], y = Qr[cb * ld];
        Qr[ca * ld] = c * x - sn * y;
        Qr[cb * ld] = sn * x + c * y;
    }
}

// Sum over the L consecutive lanes of a lane group (L a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int L)
{
    for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double group_prod(double v, int L)
{
    for (int off = L >> 1; off > 0; off >>= 1) v *= __shfl_xor(v, off, 64);
    return v;
}

// Secular equation 1 + sigma sum_q z_q^2 / (D_q - lambda) = 0, one root per
// group of L lanes (each lane sums every L-th pole; the group's lanes hold
// identical reduced sums, so they take identical decisions).  The root is
// kept as (origin pole, offset tau) and refined by a bracketed two-pole
// rational model.
__global__ __launch_bounds__(64) void dc_secular_kernel(int64_t n, int t, const double *e, DcArrays a, int L,
                                                       int maxit)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int K = info[0];
    const int sub = threadIdx.x & (L - 1);
    const int64_t j = (int64_t)blockIdx.x * (64 / L) + threadIdx.x / L;
    if (j >= K) return;  // whole groups leave together
    const double sigma = 2.0 * fabs(e[mid - 1]);
    const double *D = a.Dk + lo, *z = a.zk + lo;

    int o;
    double tlo, thi;
    if (j < K - 1) {
        const double gap = D[j + 1] - D[j];
        const double half = 0.5 * gap;
        double f = 0.0;
        for (int q = sub; q < K; q += L) f += sigma * z[q] * z[q] / ((D[q] - D[j]) - half);
        f = 1.0 + group_sum(f, L);
        if (f > 0.0) { o = (int)j; tlo = 0.0; thi = half; }
        else { o = (int)j + 1; tlo = -half; thi = 0.0; }
    } else {
        double zz = 0.0;
        for (int q = sub; q < K; q += L) zz += z[q] * z[q];
        zz = group_sum(zz, L);
        o = K - 1;
        tlo = 0.0;
        thi = sigma * zz;
    }
    const double Do = D[o];
    double tau = 0.5 * (tlo + thi);
    double last = 1e300;
    bool done = false;
    for (int it = 0; it < maxit; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int q = sub; q < K; q += L) {
            const double inv = 1.0 / ((D[q] - Do) - tau);
            const double tq = z[q] * z[q] * inv;
            if (q <= j) {
                psi += tq;
                dpsi += tq * inv;
            } else {
                phi += tq;
                dphi += tq * inv;
            }
        }
        psi = sigma * group_sum(psi, L);
        dpsi = sigma * group_sum(dpsi, L);
        phi = sigma * group_sum(phi, L);
        dphi = sigma * group_sum(dphi, L);
        const double f = 1.0 + psi + phi;
        if (f > 0.0) thi = tau;
        else tlo = tau;
        if (f == 0.0 || thi - tlo <= 2.0 * DC_EPS * fmax(fabs(tlo), fabs(thi))) { done = true; break; }
        if (fabs(f) <= DC_EPS * (1.0 + fabs(psi) + fabs(phi)) && it > 0 && fabs(last) <= 4.0 * DC_EPS * fabs(tau)) {
            done = true;
            break;
        }
        // two-pole rational model around the current point
        const double dj = (D[j] - Do) - tau;
        double eta = 0.0;
        bool ok = false;
        if (j < K - 1) {
            const double dj1 = (D[j + 1] - Do) - tau;
            const double Bc = dpsi * dj * dj, Ac = psi - dpsi * dj;
            const double Ec = dphi * dj1 * dj1, Cc = phi - dphi * dj1;
            const double cq = 1.0 + Ac + Cc;
            const double aq = cq * (dj + dj1) + Bc + Ec;
            const double bq = cq * dj * dj1 + Bc * dj1 + Ec * dj;
            const double disc = fmax(aq * aq - 4.0 * cq * bq, 0.0);
            const double sq = sqrt(disc);
            const double qq = 0.5 * (aq + (aq >= 0.0 ? sq : -sq));
            if (cq != 0.0) {
                const double e1 = qq / cq;
                if (tau + e1 > tlo && tau + e1 < thi) { eta = e1; ok = true; }
            }
            if (!ok && qq != 0.0) {
                const double e2 = bq / qq;
                if (tau + e2 > tlo && tau + e2 < thi) { eta = e2; ok = true; }
            }
        } else {
            const double Bc = dpsi * dj * dj, Ac = psi - dpsi * dj;
            if (1.0 + Ac != 0.0) {
                const double e1 = dj + Bc / (1.0 + Ac);
                if (tau + e1 > tlo && tau + e1 < thi) { eta = e1; ok = true; }
            }
        }
        const double nt = ok ? tau + eta : 0.5 * (tlo + thi);
        last = nt - tau;
        tau = nt;
    }
    if (sub != 0) return;
    if (!done) atomicMax(a.flag, 1);
    if (tau == 0.0) tau = (o == (int)j) ? 1e-300 : -1e-300;  // never exactly on the pole
    a.org[lo + j] = o;
    a.tauj[lo + j] = tau;
    a.lam[lo + j] = Do + tau;
}

// Gu-Eisenstat: zhat_i^2 = (lam_K - D_i)/sigma prod_{j<i} (lam_j - D_i)/(D_j - D_i)
//                          prod_{i<=j<K-1} (lam_j - D_i)/(D_j+1 - D_i)
// Every factor of the two products lies in (0, 1) by interlacing, so partial
// products over any subset stay between the full product and 1: the group of
// L lanes multiplies strided subsets and combines them.
__global__ __launch_bounds__(64) void dc_zhat_kernel(int64_t n, int t, const double *e, DcArrays a, int L)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int K = info[0];
    const int sub = threadIdx.x & (L - 1);
    const int64_t q = (int64_t)blockIdx.x * (64 / L) + threadIdx.x / L;
    if (q >= K) return;
    const double sigma = 2.0 * fabs(e[mid - 1]);
    const double *D = a.Dk + lo;
    const int *org = a.org + lo;
    const double *tj = a.tauj + lo;
    const double Dq = D[q];
    double prod = 1.0;
    for (int j = sub; j < K - 1; j += L) {
        const double den = (j < q) ? (D[j] - Dq) : (D[j + 1] - Dq);
        prod *= ((D[org[j]] - Dq) + tj[j]) / den;
    }
    prod = group_prod(prod, L) * (((D[org[K - 1]] - Dq) + tj[K - 1]) / sigma);
    if (sub == 0) a.zhat[lo + q] = copysign(sqrt(fmax(prod, 0.0)), a.zk[lo + q]);
}

// Column j of U: zhat ./ (D - lam_j), normalised; rows placed at gpos.
__global__ __launch_bounds__(64) void dc_vec_kernel(int64_t n, int t, DcArrays a)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int K = info[0];
    const int64_t j = blockIdx.x;
    if (j >= K) return;
    const int lane = threadIdx.x;
    const double *D = a.Dk + lo, *zh = a.zhat + lo;
    const double Do = D[a.org[lo + j]], tj = a.tauj[lo + j];
    double ss = 0.0;
    for (int q = lane; q < K; q += 64) {
        const double u = zh[q] / ((D[q] - Do) - tj);
        ss += u * u;
    }
    ss = wave_sum(ss);
    const double inv = 1.0 / sqrt(ss);
    const int64_t ld = n;
    double *Uc = a.U + lo + (lo + j) * ld;
    for (int q = lane; q < K; q += 64) {
        const double u = zh[q] / ((D[q] - Do) - tj);
        Uc[a.gpos[lo + q]] = u * inv;
    }
}

// Final order: position of every root / deflated value among the node's s values.
__global__ __launch_bounds__(256) void dc_rank_kernel(int64_t n, int t, DcArrays a)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int64_t s = hi - lo;
    const int K = info[0], nd = info[5];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s) return;
    const double *lam = a.lam + lo, *Dd = a.Ddef + lo;
    double key;
    int64_t pos;
    if (q < K) {
        key = lam[q];
        // roots are ascending; count deflated values strictly below (ties: roots first)
        int64_t c = 0;
        for (int r = 0; r < nd; ++r) c += (Dd[r] < key) ? 1 : 0;
        pos = q + c;
    } else {
        const int r0 = (int)(q - K);
        key = Dd[r0];
        // roots <= key (binary search), deflated values before it in (value, index) order
        int64_t l = 0, h = K;
        while (l < h) {
            const int64_t md = (l + h) >> 1;
            if (lam[md] <= key) l = md + 1;
            else h = md;
        }
        int64_t c = l;
        for (int r = 0; r < nd; ++r) {
            const double v = Dd[r];
            c += (v < key || (v == key && r < r0)) ? 1 : 0;
        }
        pos = c;
    }
    a.Dw[lo + pos] = key;
    a.outSrc[lo + pos] = (int)q;
}

// Z block column p <- product column (src < K) or deflated Qp column (src >= K);
// thread per row, workgroup z for columns [z DC_CC, (z + 1) DC_CC).
__global__ __launch_bounds__(256) void dc_scatter_kernel(int64_t n, int t, double *Z, int64_t ldz, DcArrays a)
{
    const int64_t i = blockIdx.y;
    int64_t lo, mid, hi;
    node_range(n, t, i, &lo, &mid, &hi);
    const int *info = a.info + i * 8;
    if (!info[6]) return;
    const int64_t s = hi - lo;
    const int K = info[0];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.z * DC_CC;
    if (r >= s || p0 >= s) return;
    const int64_t p1 = (p0 + DC_CC < s) ? p0 + DC_CC : s;
    const int64_t ld = n;
    const double *Tr = a.Tmp + lo + r + lo * ld;
    const double *Qr = a.Qp + lo + r + lo * ld;
    double *Zr = Z + lo + r + lo * ldz;
    const int *osrc = a.outSrc + lo;
    auto col = [&](int64_t p) {
        const int src = osrc[p];
        return (src < K) ? Tr[(int64_t)src * ld] : Qr[(int64_t)src * ld];
    };
    int64_t p = p0;
    for (; p + 8 <= p1; p += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = col(p + q);
#pragma unroll
        for (int q = 0; q < 8; ++q) Zr[(p + q) * ldz] = v[q];
    }
    for (; p < p1; ++p) Zr[p * ldz] = col(p);
}

// ---------------------------------------------------------------- eigenvalues only
__device__ __forceinline__ int64_t sturm_count(int64_t n, const double *d, const double *e, double x, double pivmin)
{
    int64_t cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int64_t k = 1; k < n; ++k) {
        q = (d[k] - x) - e[k - 1] * e[k - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// k-th smallest eigenvalue by bisection on the Sturm count; bounds from
// dc_gersh_kernel (g[0] <= lambda <= g[1], g[2] = max e_i^2).  Stops when
// the bracket is below 2 eps max(|lo|, |hi|) + eps ||T||.
__global__ void dc_bisect_kernel(int64_t n, const double *d, const double *e, double *W, const double *g)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double tnorm = fmax(fabs(g[0]), fabs(g[1]));
    const double pivmin = 2.2250738585072014e-308 * fmax(g[2], 1.0);
    const double pad = 2.0 * DC_EPS * tnorm * (double)n + 2.0 * pivmin;
    const double atol = DC_EPS * tnorm;
    double lo = g[0] - pad, hi = g[1] + pad;
    for (int it = 0; it < 200; ++it) {
        const double md = 0.5 * (lo + hi);
        if (md <= lo || md >= hi) break;
        if (hi - lo <= 2.0 * DC_EPS * fmax(fabs(lo), fabs(hi)) + atol) break;
        if (sturm_count(n, d, e, md, pivmin) > k) hi = md;
        else lo = md;
    }
    W[k] = 0.5 * (lo + hi);
}

__global__ void dc_gersh_kernel(int64_t n, const double *d, const double *e, double *out)
{
    // single workgroup: out[0] = min(d_i - r_i), out[1] = max(d_i + r_i), out[2] = max |e_i|^2
    __shared__ double s0[256], s1[256], s2[256];
    double lo = 1e300, hi = -1e300, em = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double r = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
        if (i + 1 < n) em = fmax(em, e[i] * e[i]);
    }
    s0[threadIdx.x] = lo;
    s1[threadIdx.x] = hi;
    s2[threadIdx.x] = em;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)blockDim.x; ++q) {
            lo = fmin(lo, s0[q]);
            hi = fmax(hi, s1[q]);
            em = fmax(em, s2[q]);
        }
        out[0] = lo;
        out[1] = hi;
        out[2] = em;
    }
}

__global__ void dc_copy_kernel(int64_t n, const double *src, double *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void dc_info_kernel(const int *flag, int32_t *info)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) info[0] = flag[0] ? EVD_ERR_NOT_CONVERGED : 0;
}

__global__ void dc_zero_int(int *p, int64_t cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

size_t dc_layout(int64_t n, char *base, DcArrays *out)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += evd_align256(bytes);
        return p;
    };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int levels = (n > 1) ? (int)ceil(log2((double)n)) : 0;
    const size_t maxnodes = (size_t)1 << (levels > 0 ? levels - 1 : 0);
    DcArrays a;
    a.Dw = (double *)take(nn * 8);
    a.Dsort = (double *)take(nn * 8);
    a.zsort = (double *)take(nn * 8);
    a.srcCol = (int *)take(nn * 4);
    a.status = (int *)take(nn * 4);
    a.Dfin = (double *)take(nn * 8);
    a.zfin = (double *)take(nn * 8);
    a.destCol = (int *)take(nn * 4);
    a.Dk = (double *)take(nn * 8);
    a.zk = (double *)take(nn * 8);
    a.gpos = (int *)take(nn * 4);
    a.lam = (double *)take(nn * 8);
    a.org = (int *)take(nn * 4);
    a.tauj = (double *)take(nn * 8);
    a.zhat = (double *)take(nn * 8);
    a.Ddef = (double *)take(nn * 8);
    a.rotP = (int *)take(nn * 4);
    a.rotI = (int *)take(nn * 4);
    a.rotC = (double *)take(nn * 8);
    a.rotS = (double *)take(nn * 8);
    a.outSrc = (int *)take(nn * 4);
    a.info = (int *)take(maxnodes * 8 * 4);
    a.probs = (GemmProblem *)take(maxnodes * 2 * sizeof(GemmProblem));
    a.flag = (int *)take(256);
    a.Qp = (double *)take(nn * nn * 8);
    a.U = (double *)take(nn * nn * 8);
    a.Tmp = (double *)take(nn * nn * 8);
    if (out) *out = a;
    return off;
}

size_t dc_values_layout(int64_t n) { (void)n; return 256; }

}  // namespace

size_t dc_work_bytes(char compz, int64_t n)
{
    if (compz == 'N' || compz == 'n') return dc_values_layout(n);
    return dc_layout(n, nullptr, nullptr);
}

evd_status_t dc_run(evd_ctx_t ctx, char compz, int64_t n, const double *d, const double *e, double *W, double *Z,
                    int64_t ldz, void *work, int32_t *info)
{
    hipStream_t s = ctx->stream;
    auto grid1 = [](int64_t cnt) { return dim3((unsigned)(evd_ceil_div(cnt, 256) < 4096 ? evd_ceil_div(cnt, 256) : 4096)); };
    if (compz == 'N' || compz == 'n') {
        double *g = (double *)work;
        hipLaunchKernelGGL(dc_gersh_kernel, dim3(1), dim3(256), 0, s, n, d, e, g);
        hipLaunchKernelGGL(dc_bisect_kernel, dim3((unsigned)evd_ceil_div(n, 64)), dim3(64), 0, s, n, d, e, W,
                           (const double *)g);
        if (info) hipLaunchKernelGGL(dc_zero_int, dim3(1), dim3(64), 0, s, (int *)info, (int64_t)1);
        return evd_check_last();
    }
    DcArrays a;
    dc_layout(n, (char *)work, &a);
    // iterations per secular root; "dc_max_iter" lowers it to force the
    // non-convergence status (failure-path tests)
    const int maxit = (ctx->dc_max_iter > 0 && ctx->dc_max_iter < 200) ? (int)ctx->dc_max_iter : 200;
    hipLaunchKernelGGL(dc_zero_int, dim3(1), dim3(64), 0, s, a.flag, (int64_t)1);
    hipLaunchKernelGGL(dc_init_kernel, grid1(n * n), dim3(256), 0, s, n, d, e, a.Dw, Z, ldz);
    const int levels = (n > 1) ? (int)ceil(log2((double)n)) : 0;
    for (int t = levels - 1; t >= 0; --t) {
        const int64_t M = (int64_t)1 << t;
        const int64_t smax = evd_ceil_div(n, M);
        hipLaunchKernelGGL(dc_prep_kernel, dim3((unsigned)M), dim3(PREP_T), 0, s, n, t, e, (const double *)Z, ldz, a);
        const unsigned cz = (unsigned)evd_ceil_div(smax, DC_CC);
        hipLaunchKernelGGL(dc_qp_kernel, dim3((unsigned)evd_ceil_div(smax, 256), (unsigned)M, cz), dim3(256), 0, s, n,
                           t, (const double *)Z, ldz, a);
        hipLaunchKernelGGL(dc_rot_kernel, dim3((unsigned)evd_ceil_div(smax, 256), (unsigned)M), dim3(256), 0, s, n, t,
                           a);
        // lanes per root: enough roots in flight, at least ~32 poles per lane
        int L = 1;
        while (L < 64 && (int64_t)L * 64 <= smax) L *= 2;
        const unsigned gx = (unsigned)evd_ceil_div(smax, 64 / L);
        hipLaunchKernelGGL(dc_secular_kernel, dim3(gx, (unsigned)M), dim3(64), 0, s, n, t, e, a, L, maxit);
        hipLaunchKernelGGL(dc_zhat_kernel, dim3(gx, (unsigned)M), dim3(64), 0, s, n, t, e, a, L);
        hipLaunchKernelGGL(dc_vec_kernel, dim3((unsigned)smax, (unsigned)M), dim3(64), 0, s, n, t, a);
        EVD_CHECK(gemm_f64_grouped(s, a.probs, (int)(2 * M), smax, smax));
        hipLaunchKernelGGL(dc_rank_kernel, dim3((unsigned)evd_ceil_div(smax, 256), (unsigned)M), dim3(256), 0, s, n,
                           t, a);
        hipLaunchKernelGGL(dc_scatter_kernel, dim3((unsigned)evd_ceil_div(smax, 256), (unsigned)M, cz), dim3(256), 0,
                           s, n, t, Z, ldz, a);
        EVD_CHECK(evd_check_last());
    }
    hipLaunchKernelGGL(dc_copy_kernel, grid1(n), dim3(256), 0, s, n, (const double *)a.Dw, W);
    if (info) hipLaunchKernelGGL(dc_info_kernel, dim3(1), dim3(64), 0, s, (const int *)a.flag, info);
    return evd_check_last();
}

extern "C" {

evd_status_t evd_dstedc_work_size(evd_ctx_t ctx, char compz, int64_t n, size_t *bytes)
{
    if (!ctx || !bytes) return EVD_ERR_INVALID_ARG;
    if (!(compz == 'N' || compz == 'n' || compz == 'I' || compz == 'i')) { ctx->last_invalid_arg = 2; return EVD_ERR_INVALID_ARG; }
    if (n < 0) { ctx->last_invalid_arg = 3; return EVD_ERR_INVALID_ARG; }
    *bytes = dc_work_bytes(compz, n);
    return EVD_OK;
}

evd_status_t evd_dstedc(evd_ctx_t ctx, char compz, int64_t n, const double *d, const double *e, double *W, double *Z,
                        int64_t ldz, void *work, size_t work_bytes, int32_t *info)
{
    if (!ctx) return EVD_ERR_INVALID_ARG;
    const bool vec = (compz == 'I' || compz == 'i');
    int bad = 0;
    if (!(vec || compz == 'N' || compz == 'n')) bad = 2;
    else if (n < 0) bad = 3;
    else if (n > 0 && !d) bad = 4;
    else if (n > 1 && !e) bad = 5;
    else if (n > 0 && !W) bad = 6;
    else if (vec && n > 0 && !Z) bad = 7;
    else if (vec && ldz < (n > 1 ? n : 1)) bad = 8;
    else if (n > 0 && !work) bad = 9;
    else if (work_bytes < dc_work_bytes(compz, n)) bad = 10;
    ctx->last_invalid_arg = bad;
    if (bad) return bad == 10 ? EVD_ERR_WORKSPACE : EVD_ERR_INVALID_ARG;
    if (n == 0) return EVD_OK;
    if (ctx->device < 0) return EVD_ERR_HIP;
    EVD_CHECK(evd_hip(ctx, hipSetDevice(ctx->device)));
    return dc_run(ctx, vec ? 'I' : 'N', n, d, e, W, Z, ldz, work, info);
}

}  // extern "C"
