// Tridiagonal divide and conquer on the host CPU: the paper's placement of
// the D&C stage (Algorithm 1 runs it in a CPU thread while the GPUs carry
// out the back transformation, Section 3.3), kept as an alternative to the
// GPU D&C of dc.hip.  The arithmetic is the same method:
//   * Cuppen tear at the middle coupling, T = diag(T1, T2) + |rho| v v^T,
//     v = e_last(T1) + sign(rho) e_first(T2), recursively down to size 1;
//   * merge: z = [last row of Q1; sign(rho) first row of Q2] / sqrt 2,
//     sigma = 2 |rho|; poles sorted; deflation of sigma |z_i| <= tol and of
//     close poles by a Givens rotation (off-diagonal |c s (D_i - D_p)| <= tol),
//     tol = 8 eps max(max|D|, sigma);
//   * secular equation f(lam) = 1 + sigma sum z_i^2 / (D_i - lam) = 0 per
//     root, the root kept as (nearest pole, offset tau), bracketed, with a
//     two-pole rational model (Bunch, Nielsen and Sorensen 1978) and
//     bisection as the fallback;
//   * z recomputed from the roots (Gu and Eisenstat 1995, Loewner), vectors
//     u_j = zhat ./ (D - lam_j) normalised, Q = diag(Q1, Q2) P G U as two
//     products that skip the zero blocks (rows of T1 meet only columns that
//     come from Q1 or were rotated with one, likewise for T2).
// Work is spread over std::thread workers: the two halves of the upper tree
// levels run side by side, and every merge splits its root solves, vectors
// and products over the threads it owns.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "common.h"

namespace {

constexpr double HEPS = 2.220446049250313e-16;  // 2^-52

template <typename F>
void par_for(int64_t count, int threads, F &&fn)
{
    if (count <= 0) return;
    if (threads <= 1 || count == 1) {
        fn((int64_t)0, count);
        return;
    }
    const int t = (int)std::min<int64_t>(threads, count);
    std::vector<std::thread> pool;
    pool.reserve(t);
    for (int w = 0; w < t; ++w) {
        const int64_t a = count * w / t, b = count * (w + 1) / t;
        pool.emplace_back([&fn, a, b] { fn(a, b); });
    }
    for (auto &th : pool) th.join();
}

// C (m x n) = A (m x k) B (k x n), column-major; blocks of 256 rows x 4
// columns of C accumulate over K-blocks of 256 (the four C columns stay in L1).
__attribute__((target("avx2,fma"))) void gemm_block_avx2(int64_t m, int64_t n, int64_t k, const double *A,
                                                         int64_t lda, const double *B, int64_t ldb, double *C,
                                                         int64_t ldc)
{
    constexpr int64_t MB = 256, KB = 256;
    for (int64_t i0 = 0; i0 < m; i0 += MB) {
        const int64_t mb = std::min(MB, m - i0);
        for (int64_t j = 0; j < n; j += 4) {
            const int64_t nc = std::min<int64_t>(4, n - j);
            double *c[4];
            for (int q = 0; q < 4; ++q) c[q] = C + i0 + (j + (q < nc ? q : 0)) * ldc;
            for (int q = 0; q < nc; ++q)
                for (int64_t i = 0; i < mb; ++i) c[q][i] = 0.0;
            for (int64_t p0 = 0; p0 < k; p0 += KB) {
                const int64_t pe = std::min(k, p0 + KB);
                if (nc == 4) {
                    double *__restrict c0 = c[0], *__restrict c1 = c[1], *__restrict c2 = c[2], *__restrict c3 = c[3];
                    for (int64_t p = p0; p < pe; ++p) {
                        const double *__restrict a = A + i0 + p * lda;
                        const double b0 = B[p + j * ldb], b1 = B[p + (j + 1) * ldb], b2 = B[p + (j + 2) * ldb],
                                     b3 = B[p + (j + 3) * ldb];
                        for (int64_t i = 0; i < mb; ++i) {
                            const double av = a[i];
                            c0[i] += av * b0;
                            c1[i] += av * b1;
                            c2[i] += av * b2;
                            c3[i] += av * b3;
                        }
                    }
                } else {
                    for (int q = 0; q < nc; ++q) {
                        double *__restrict cq = c[q];
                        for (int64_t p = p0; p < pe; ++p) {
                            const double *__restrict a = A + i0 + p * lda;
                            const double bq = B[p + (j + q) * ldb];
                            for (int64_t i = 0; i < mb; ++i) cq[i] += a[i] * bq;
                        }
                    }
                }
            }
        }
    }
}

void gemm_block_plain(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                      double *C, int64_t ldc)
{
    for (int64_t j = 0; j < n; ++j) {
        double *cj = C + j * ldc;
        for (int64_t i = 0; i < m; ++i) cj[i] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double b = B[p + j * ldb];
            const double *a = A + p * lda;
            for (int64_t i = 0; i < m; ++i) cj[i] += a[i] * b;
        }
    }
}

bool have_avx2()
{
    static const bool ok = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    return ok;
}

// C = A B over column blocks of C, in parallel
void gemm(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
          int64_t ldc, int threads)
{
    if (m <= 0 || n <= 0) return;
    if (k <= 0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) C[i + j * ldc] = 0.0;
        return;
    }
    const int64_t nb = (n + 63) / 64;
    const int t = (int)std::min<int64_t>(threads, std::max<int64_t>(1, (m * n * k) / (1 << 21)));
    par_for(nb, t, [&](int64_t b0, int64_t b1) {
        const int64_t j0 = b0 * 64, j1 = std::min(n, b1 * 64);
        if (have_avx2()) gemm_block_avx2(m, j1 - j0, k, A, lda, B + j0 * ldb, ldb, C + j0 * ldc, ldc);
        else gemm_block_plain(m, j1 - j0, k, A, lda, B + j0 * ldb, ldb, C + j0 * ldc, ldc);
    });
}

struct Root {
    int org;      // pole index the root is measured from
    double tau;   // root = D[org] + tau
};

// Root j of f(lam) = 1 + sigma sum w_k / (D_k - lam), D ascending (K poles),
// w_k = z_k^2 > 0: lam_j in (D_j, D_j+1), the last one in (D_K-1, D_K-1 + sigma sum w).
// Returns false if it did not converge in maxit iterations.
bool secular_root(int K, const double *D, const double *w, double sigma, double wsum, int j, int maxit, Root *out)
{
    const bool last = (j == K - 1);
    int o;
    double lo, hi;  // bracket of tau around pole o
    if (last) {
        o = j;
        lo = 0.0;
        hi = sigma * wsum;
    } else {
        const double gap = D[j + 1] - D[j], mid = 0.5 * gap;
        double f = 1.0;
        for (int k = 0; k < K; ++k) f += sigma * w[k] / ((D[k] - D[j]) - mid);
        if (f >= 0.0) {
            o = j;
            lo = 0.0;
            hi = mid;
        } else {
            o = j + 1;
            lo = -mid;
            hi = 0.0;
        }
    }
    const double dj = D[j] - D[o];                     // left pole of the interval, shifted
    const double dj1 = last ? 0.0 : D[j + 1] - D[o];   // right pole, shifted (unused for the last root)
    double tau = 0.5 * (lo + hi);
    for (int it = 0; it < maxit; ++it) {
        // f and the derivatives of its left (k <= j) and right (k > j) parts at tau
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int k = 0; k <= j; ++k) {
            const double r = 1.0 / ((D[k] - D[o]) - tau);
            const double t = sigma * w[k] * r;
            psi += t;
            dpsi += t * r;
        }
        for (int k = j + 1; k < K; ++k) {
            const double r = 1.0 / ((D[k] - D[o]) - tau);
            const double t = sigma * w[k] * r;
            phi += t;
            dphi += t * r;
        }
        const double f = 1.0 + psi + phi;
        if (f > 0.0) hi = tau;
        else lo = tau;
        const double err = 8.0 * HEPS * (1.0 + std::fabs(psi) + std::fabs(phi));
        if (std::fabs(f) <= err || (hi - lo) <= 4.0 * HEPS * std::max(std::fabs(lo), std::fabs(hi))) {
            *out = {o, tau};
            return true;
        }
        // two-pole model: psi ~ a + b / (dj - t), phi ~ c + e / (dj1 - t)
        double tn;
        const double xl = dj - tau;
        const double b = dpsi * xl * xl, a = psi - b / xl;
        if (last) {
            const double A = 1.0 + a + phi;   // phi = 0 for the last root
            tn = (A != 0.0) ? dj + b / A : 0.5 * (lo + hi);
        } else {
            const double xr = dj1 - tau;
            const double e = dphi * xr * xr, c = phi - e / xr;
            const double A = 1.0 + a + c;
            // A (dj - t)(dj1 - t) + b (dj1 - t) + e (dj - t) = 0, in u = t - tau
            // with p = dj - tau, q = dj1 - tau:  A (p - u)(q - u) + b (q - u) + e (p - u) = 0
            const double p = xl, q = xr;
            const double qa = A, qb = -(A * (p + q) + b + e), qc = A * p * q + b * q + e * p;
            double u;
            if (std::fabs(qa) < 1e-300) {
                u = (qb != 0.0) ? -qc / qb : 0.0;
            } else {
                const double disc = qb * qb - 4.0 * qa * qc;
                const double sq = std::sqrt(std::max(disc, 0.0));
                const double r1 = (qb >= 0.0) ? (-qb - sq) / (2.0 * qa) : (-qb + sq) / (2.0 * qa);
                const double r2 = (r1 != 0.0) ? qc / (qa * r1) : 0.0;
                // the root between the two poles (p < u < q)
                u = (r1 > p && r1 < q) ? r1 : r2;
            }
            tn = tau + u;
        }
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == tau) {
            *out = {o, tau};
            return true;
        }
        tau = tn;
    }
    *out = {o, tau};
    return false;
}

struct Ctx {
    int maxit;
    std::atomic<int> failed{0};
};

// Solve the size-n tridiagonal whose (torn) diagonal is Dw[0:n) and couplings
// e[0:n-1), eigenvalues ascending into lam[0:n), eigenvectors into Z (ldz).
void dc_rec(int64_t n, double *Dw, const double *e, double *lam, double *Z, int64_t ldz, int threads, Ctx &cx)
{
    if (n == 1) {
        lam[0] = Dw[0];
        Z[0] = 1.0;
        return;
    }
    const int64_t n1 = n / 2, n2 = n - n1;
    const double rho = e[n1 - 1];
    const double beta = std::fabs(rho), sg = (rho >= 0.0) ? 1.0 : -1.0;
    Dw[n1 - 1] -= beta;
    Dw[n1] -= beta;
    // children: Q1 in Z[0:n1, 0:n1], Q2 in Z[n1:n, n1:n]; the off-diagonal blocks zero
    for (int64_t j = 0; j < n1; ++j)
        for (int64_t i = n1; i < n; ++i) Z[i + j * ldz] = 0.0;
    for (int64_t j = n1; j < n; ++j)
        for (int64_t i = 0; i < n1; ++i) Z[i + j * ldz] = 0.0;
    if (threads > 1 && n >= 512) {
        const int t1 = threads / 2, t2 = threads - t1;
        std::thread th([&] { dc_rec(n1, Dw, e, lam, Z, ldz, t1, cx); });
        dc_rec(n2, Dw + n1, e + n1, lam + n1, Z + n1 + n1 * ldz, ldz, t2, cx);
        th.join();
    } else {
        dc_rec(n1, Dw, e, lam, Z, ldz, 1, cx);
        dc_rec(n2, Dw + n1, e + n1, lam + n1, Z + n1 + n1 * ldz, ldz, 1, cx);
    }

    // ---- merge
    const double sigma = 2.0 * beta;
    std::vector<double> z(n);
    for (int64_t j = 0; j < n1; ++j) z[j] = Z[(n1 - 1) + j * ldz] / std::sqrt(2.0);
    for (int64_t j = n1; j < n; ++j) z[j] = sg * Z[n1 + j * ldz] / std::sqrt(2.0);
    // poles ascending (merge of the two ascending lists)
    std::vector<int64_t> perm(n);
    {
        int64_t a = 0, b = n1, u = 0;
        while (a < n1 || b < n) perm[u++] = (b >= n || (a < n1 && lam[a] <= lam[b])) ? a++ : b++;
    }
    std::vector<double> D(n), zz(n);
    std::vector<int> side(n);  // 1 = column from Q1 only, 2 = from Q2 only, 3 = mixed (after a rotation)
    std::vector<int64_t> col(n);  // column of the children's Q behind sorted index u
    double dmax = 0.0;
    for (int64_t u = 0; u < n; ++u) {
        D[u] = lam[perm[u]];
        zz[u] = z[perm[u]];
        col[u] = perm[u];
        side[u] = perm[u] < n1 ? 1 : 2;
        dmax = std::max(dmax, std::fabs(D[u]));
    }
    const double tol = 8.0 * HEPS * std::max(dmax, sigma);
    // Q columns in sorted order (rotations act on this copy)
    std::vector<double> Qs((size_t)n * n);
    for (int64_t u = 0; u < n; ++u) std::memcpy(&Qs[(size_t)u * n], Z + col[u] * ldz, sizeof(double) * n);
    std::vector<char> defl(n, 0);
    int64_t prev = -1;
    for (int64_t u = 0; u < n; ++u) {
        if (sigma * std::fabs(zz[u]) <= tol) {
            defl[u] = 1;
            continue;
        }
        if (prev >= 0) {
            const double r = std::hypot(zz[prev], zz[u]);
            const double c = zz[u] / r, s = zz[prev] / r;
            if (std::fabs(c * s * (D[u] - D[prev])) <= tol) {
                // rotate (prev, u): prev deflates with c^2 D_p + s^2 D_u, u keeps z = r
                const double dp = c * c * D[prev] + s * s * D[u], du = s * s * D[prev] + c * c * D[u];
                double *qp = &Qs[(size_t)prev * n], *qu = &Qs[(size_t)u * n];
                for (int64_t i = 0; i < n; ++i) {
                    const double x = qp[i], y = qu[i];
                    qp[i] = c * x - s * y;
                    qu[i] = s * x + c * y;
                }
                D[prev] = dp;
                D[u] = du;
                zz[prev] = 0.0;
                zz[u] = r;
                defl[prev] = 1;
                if (side[prev] != side[u]) side[u] = side[prev] = 3;
            }
        }
        prev = u;
    }
    // non-deflated poles (ascending after the rotations? rotations only mix
    // values closer than tol, so the order holds up to tol; sort to be exact)
    std::vector<int64_t> nd;
    for (int64_t u = 0; u < n; ++u)
        if (!defl[u]) nd.push_back(u);
    std::stable_sort(nd.begin(), nd.end(), [&](int64_t x, int64_t y) { return D[x] < D[y]; });
    const int K = (int)nd.size();
    std::vector<double> Dk(K), wk(K), zk(K);
    double wsum = 0.0;
    for (int k = 0; k < K; ++k) {
        Dk[k] = D[nd[k]];
        zk[k] = zz[nd[k]];
        wk[k] = zk[k] * zk[k];
        wsum += wk[k];
    }
    std::vector<Root> roots(K);
    par_for(K, threads, [&](int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j)
            if (!secular_root(K, Dk.data(), wk.data(), sigma, wsum, (int)j, cx.maxit, &roots[j])) cx.failed = 1;
    });
    // Gu-Eisenstat zhat and the vectors of D + sigma zhat zhat^T
    std::vector<double> zh(K);
    par_for(K, threads, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            auto diff = [&](int j) { return (Dk[roots[j].org] - Dk[i]) + roots[j].tau; };  // lam_j - D_i
            double prod = diff(K - 1) / sigma;
            for (int j = 0; j < i; ++j) prod *= diff(j) / (Dk[j] - Dk[i]);
            for (int j = (int)i; j < K - 1; ++j) prod *= diff(j) / (Dk[j + 1] - Dk[i]);
            zh[i] = std::copysign(std::sqrt(std::fabs(prod)), zk[i]);
        }
    });
    // U (K x K, column j = normalised zhat ./ (D - lam_j)), rows grouped
    // [Q1-only | mixed | Q2-only] for the two products
    std::vector<int> ord(K);
    {
        int t = 0;
        for (int g : {1, 3, 2})
            for (int k = 0; k < K; ++k)
                if (side[nd[k]] == g) ord[t++] = k;
    }
    int k1 = 0, k3 = 0;
    for (int k = 0; k < K; ++k) {
        if (side[nd[k]] == 1) ++k1;
        else if (side[nd[k]] == 3) ++k3;
    }
    std::vector<double> U((size_t)K * K);
    par_for(K, threads, [&](int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j) {
            double *uj = &U[(size_t)j * K];
            double nrm = 0.0;
            for (int r = 0; r < K; ++r) {
                const int i = ord[r];
                const double v = zh[i] / ((Dk[i] - Dk[roots[j].org]) - roots[j].tau);
                uj[r] = v;
                nrm += v * v;
            }
            const double sc = 1.0 / std::sqrt(nrm);
            for (int r = 0; r < K; ++r) uj[r] *= sc;
        }
    });
    // Q columns of the non-deflated poles in the same grouped order
    std::vector<double> Qn((size_t)n * K);
    for (int r = 0; r < K; ++r) std::memcpy(&Qn[(size_t)r * n], &Qs[(size_t)nd[ord[r]] * n], sizeof(double) * n);
    // products: rows of T1 meet groups 1 and 3, rows of T2 groups 3 and 2
    std::vector<double> P((size_t)n * K);
    gemm(n1, K, k1 + k3, Qn.data(), n, U.data(), K, P.data(), n, threads);
    gemm(n2, K, K - k1, Qn.data() + n1 + (size_t)k1 * n, n, U.data() + k1, K, P.data() + n1, n, threads);
    // output: all n eigenvalues ascending (roots and deflated values)
    std::vector<double> val(n);
    std::vector<int64_t> src(n);  // < K: column of P, else n... index into Qs (deflated column u) + K
    int64_t t = 0;
    for (int j = 0; j < K; ++j) {
        val[t] = Dk[roots[j].org] + roots[j].tau;
        src[t++] = j;
    }
    for (int64_t u = 0; u < n; ++u)
        if (defl[u]) {
            val[t] = D[u];
            src[t++] = K + u;
        }
    std::vector<int64_t> fin(n);
    for (int64_t i = 0; i < n; ++i) fin[i] = i;
    std::stable_sort(fin.begin(), fin.end(), [&](int64_t x, int64_t y) { return val[x] < val[y]; });
    par_for(n, threads, [&](int64_t a, int64_t b) {
        for (int64_t q = a; q < b; ++q) {
            const int64_t s = src[fin[q]];
            const double *from = (s < K) ? &P[(size_t)s * n] : &Qs[(size_t)(s - K) * n];
            std::memcpy(Z + q * ldz, from, sizeof(double) * n);
        }
    });
    for (int64_t q = 0; q < n; ++q) lam[q] = val[fin[q]];
}

// eigenvalues only: Sturm-count bisection, eigenvalues split over the threads
void bisect_all(int64_t n, const double *d, const double *e, double *W, int threads)
{
    double lo = 1e300, hi = -1e300, em = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
        if (i + 1 < n) em = std::max(em, e[i] * e[i]);
    }
    const double tnorm = std::max(std::fabs(lo), std::fabs(hi));
    const double pivmin = 2.2250738585072014e-308 * std::max(em, 1.0);
    const double pad = 2.0 * HEPS * tnorm * (double)n + 2.0 * pivmin;
    lo -= pad;
    hi += pad;
    par_for(n, threads, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            double l = lo, h = hi;
            for (int it = 0; it < 200; ++it) {
                const double md = 0.5 * (l + h);
                if (md <= l || md >= h) break;
                if (h - l <= 2.0 * HEPS * std::max(std::fabs(l), std::fabs(h)) + HEPS * tnorm) break;
                int64_t cnt = 0;
                double q = d[0] - md;
                if (std::fabs(q) < pivmin) q = -pivmin;
                if (q < 0.0) ++cnt;
                for (int64_t i = 1; i < n; ++i) {
                    q = (d[i] - md) - e[i - 1] * e[i - 1] / q;
                    if (std::fabs(q) < pivmin) q = -pivmin;
                    if (q < 0.0) ++cnt;
                }
                if (cnt > k) h = md;
                else l = md;
            }
            W[k] = 0.5 * (l + h);
        }
    });
}

int host_threads(int requested)
{
    if (requested > 0) return requested;
    if (const char *s = std::getenv("OMP_NUM_THREADS")) {
        const int v = std::atoi(s);
        if (v > 0) return v;
    }
    const unsigned hc = std::thread::hardware_concurrency();
    return hc > 0 ? (int)hc : 1;
}

}  // namespace

// Host D&C (also used by evd_dsyevd with "dc_host" = 1): returns 0, or
// EVD_ERR_NOT_CONVERGED if a secular equation did not converge.
int host_dc_run(char compz, int64_t n, const double *d, const double *e, double *W, double *Z, int64_t ldz,
                int threads, int maxit)
{
    threads = host_threads(threads);
    if (n <= 0) return 0;
    if (compz == 'N' || compz == 'n') {
        bisect_all(n, d, e, W, threads);
        return 0;
    }
    std::vector<double> Dw(d, d + n);
    Ctx cx;
    cx.maxit = maxit > 0 ? maxit : 200;
    dc_rec(n, Dw.data(), e, W, Z, ldz, threads, cx);
    return cx.failed ? (int)EVD_ERR_NOT_CONVERGED : 0;
}

extern "C" {

evd_status_t evd_dstedc_host(char compz, int64_t n, const double *d, const double *e, double *W, double *Z,
                             int64_t ldz, int32_t threads, int32_t *info)
{
    const bool vec = (compz == 'I' || compz == 'i');
    if (!(vec || compz == 'N' || compz == 'n')) return EVD_ERR_INVALID_ARG;
    if (n < 0) return EVD_ERR_INVALID_ARG;
    if (n > 0 && (!d || !W || (n > 1 && !e))) return EVD_ERR_INVALID_ARG;
    if (vec && n > 0 && (!Z || ldz < n)) return EVD_ERR_INVALID_ARG;
    if (threads < 0) return EVD_ERR_INVALID_ARG;
    const int st = host_dc_run(compz, n, d, e, W, Z, ldz, threads, 0);
    if (info) *info = st;
    return EVD_OK;
}

}  // extern "C"
