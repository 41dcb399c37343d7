/*
 * oracle.c -- plain, slow, FP64 CPU reference for the dense symmetric
 * eigenvalue decomposition A = Q * Lambda * Q^T (paper, Section 1 and the
 * ENSURE clause of Algorithm 1: eigenvalues Lambda and orthogonal Q).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and must never be used as a
 * fallback for it.
 *
 * The method of the paper (two-stage reduction: band reduction + bulge
 * chasing, divide and conquer, back transformation) reaches, up to rounding,
 * the plain eigendecomposition of A, which is unique for the eigenvalues and
 * unique up to signs / rotations inside degenerate eigenspaces for Q.  This
 * file therefore computes that plain definition with the classical one-stage
 * route, which the paper names as the alternative family (Section 1: one-stage
 * Householder tridiagonalization; iterative solver; back transformation):
 *
 *   O-2  one-stage Householder tridiagonalization  S -> T = H^T S H
 *   O-3  backward accumulation of H = H_0 H_1 ... H_{n-3}
 *   O-4  implicit QL iteration with Wilkinson shift on T (Givens rotations)
 *   O-5  ascending sort of the eigenvalues, columns permuted alike
 *   O-6  cyclic-by-row Jacobi, an independent brute force for small n
 *   O-7  Sturm count nu(T, sigma) = #{ eigenvalues of T < sigma }
 *
 * Storage: column-major, element (i, j) of an n x n matrix with leading
 * dimension ld lives at M[i + j*ld].  All arithmetic is IEEE double.
 * Loops parallelised with OpenMP do not change the arithmetic of any single
 * entry (each thread owns whole rows or whole columns), so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * O-2: one-stage Householder tridiagonalization (Golub & Van Loan, 4th ed.,
 * Algorithm 8.3.1).  S is the full symmetric n x n matrix (both triangles
 * valid) and is overwritten: on exit S[k+2:n, k] holds the tail of the
 * Householder vector v_k (v_k[0] = 1 implicit, acting on rows k+1..n-1),
 * d holds the diagonal, e the sub-diagonal and tau the reflector scalars,
 * with H_k = I - tau_k v_k v_k^T and T = H_{n-3}...H_0 S H_0...H_{n-3}.
 *
 * For column k, x = S[k+1:n, k]:
 *   if ||x[1:]|| == 0:  tau = 0 (H = I), e_k = x_0
 *   else beta = -sign(x_0) ||x||, v = (x - beta e_1)/(x_0 - beta), v_0 = 1,
 *        tau = (beta - x_0)/beta, e_k = beta
 *   p = tau * S2 v,  w = p - (tau/2)(p^T v) v,  S2 <- S2 - v w^T - w v^T
 * where S2 = S[k+1:n, k+1:n].  Cost ~ 4n^3/3 flops (plus the full-storage
 * update, which this plain version does not halve).
 * ------------------------------------------------------------------------ */
int oracle_tridiag(int64_t n, double *S, int64_t lds, double *d, double *e, double *tau)
{
    if (n <= 0) return 0;
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    if (!p || !v) { free(p); free(v); return -1; }

    for (int64_t k = 0; k + 2 < n; ++k) {
        const int64_t m = n - k - 1;            /* length of x */
        double *x = &S[IDX(k + 1, k, lds)];
        double x0 = x[0];
        double sig = 0.0;
        for (int64_t i = 1; i < m; ++i) sig += x[i] * x[i];
        d[k] = S[IDX(k, k, lds)];
        if (sig == 0.0) {
            tau[k] = 0.0;
            e[k] = x0;
            for (int64_t i = 1; i < m; ++i) x[i] = 0.0;
            continue;
        }
        double nrm = sqrt(x0 * x0 + sig);
        double beta = (x0 >= 0.0) ? -nrm : nrm;
        double t = (beta - x0) / beta;
        double scale = 1.0 / (x0 - beta);
        v[0] = 1.0;
        for (int64_t i = 1; i < m; ++i) v[i] = x[i] * scale;
        tau[k] = t;
        e[k] = beta;

        /* p = tau * S2 * v  (S2 full symmetric, rows/cols k+1..n-1) */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int64_t j = 0; j < m; ++j) acc += S[IDX(k + 1 + i, k + 1 + j, lds)] * v[j];
            p[i] = t * acc;
        }
        double pv = 0.0;
        for (int64_t i = 0; i < m; ++i) pv += p[i] * v[i];
        const double half = 0.5 * t * pv;
        /* w = p - (tau/2)(p^T v) v, kept in p */
        for (int64_t i = 0; i < m; ++i) p[i] -= half * v[i];
        /* S2 <- S2 - v w^T - w v^T (both triangles) */
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            double vj = v[j], wj = p[j];
            double *col = &S[IDX(k + 1, k + 1 + j, lds)];
            for (int64_t i = 0; i < m; ++i) col[i] -= v[i] * wj + p[i] * vj;
        }
        /* the column below the sub-diagonal now holds the reflector tail */
        x[0] = beta;
        for (int64_t i = 1; i < m; ++i) x[i] = v[i];
        /* keep the symmetric copy of the annihilated row consistent */
        S[IDX(k, k + 1, lds)] = beta;
        for (int64_t i = 1; i < m; ++i) S[IDX(k, k + 1 + i, lds)] = 0.0;
    }
    if (n >= 2) {
        d[n - 2] = S[IDX(n - 2, n - 2, lds)];
        e[n - 2] = S[IDX(n - 1, n - 2, lds)];
        if (n >= 3) tau[n - 2] = 0.0;
    }
    d[n - 1] = S[IDX(n - 1, n - 1, lds)];
    free(p);
    free(v);
    return 0;
}

/* ------------------------------------------------------------------------
 * O-3: backward accumulation (Golub & Van Loan, Section 5.1.6) of
 * H = H_0 H_1 ... H_{n-3} from the reflectors stored by oracle_tridiag:
 *   Q = I;  for k = n-3 down to 0:  Q[k+1:, k+1:] <- (I - tau_k v_k v_k^T) Q[k+1:, k+1:]
 * ------------------------------------------------------------------------ */
int oracle_form_q(int64_t n, const double *S, int64_t lds, const double *tau, double *Q, int64_t ldq)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) Q[IDX(i, j, ldq)] = (i == j) ? 1.0 : 0.0;
    for (int64_t k = n - 3; k >= 0; --k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        const int64_t m = n - k - 1;
        const double *vt = &S[IDX(k + 1, k, lds)]; /* vt[0] is e_k, v[0] = 1 implied */
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            double *col = &Q[IDX(k + 1, k + 1 + j, ldq)];
            double s = col[0];
            for (int64_t i = 1; i < m; ++i) s += vt[i] * col[i];
            s *= t;
            col[0] -= s;
            for (int64_t i = 1; i < m; ++i) col[i] -= s * vt[i];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * O-4: implicit QL iteration with Wilkinson shift on the symmetric
 * tridiagonal T = tridiag(e, d, e) (Golub & Van Loan, Section 8.3, QL
 * orientation: convergence at the top of each unreduced block).
 *
 * T is held as an explicit symmetric band of half-bandwidth 2 (the extra
 * diagonal carries the bulge), and every rotation is applied two-sided to
 * that band with the plain formulas below, so each step can be checked
 * against the textbook by eye:
 *   plane (k, k+1), G = [[c, s], [-s, c]] in rows/cols k, k+1,  T <- G^T T G
 *   Q <- Q G   (columns k, k+1)
 * Deflation: |T(m+1, m)| <= eps (|T(m, m)| + |T(m+1, m+1)|).
 * Shift: the eigenvalue of the leading 2 x 2 block [[d_l, e_l], [e_l, d_l+1]]
 * that is closer to d_l.
 * Returns 0 on success, or l+1 if eigenvalue l did not converge in 30 steps.
 * If Q is NULL no vectors are accumulated.
 * ------------------------------------------------------------------------ */
typedef struct { double *b0, *b1, *b2; int64_t n; } band2_t;

static double b2_get(const band2_t *B, int64_t i, int64_t j)
{
    if (i < j) { int64_t t = i; i = j; j = t; }
    int64_t dd = i - j;
    if (dd == 0) return B->b0[j];
    if (dd == 1) return B->b1[j];
    if (dd == 2) return B->b2[j];
    return 0.0;
}

static void b2_set(band2_t *B, int64_t i, int64_t j, double val)
{
    if (i < j) { int64_t t = i; i = j; j = t; }
    int64_t dd = i - j;
    if (dd == 0) B->b0[j] = val;
    else if (dd == 1) B->b1[j] = val;
    else if (dd == 2) B->b2[j] = val;
    /* entries further out are structurally zero during a QL sweep */
}

/* T <- G^T T G for the plane (k, k+1); only entries within distance 2 of the
 * diagonal can be touched, so the row loop runs over k-2 .. k+3. */
static void b2_rotate(band2_t *B, int64_t k, double c, double s, int64_t lo, int64_t hi)
{
    const double a = b2_get(B, k, k), bb = b2_get(B, k + 1, k), dd = b2_get(B, k + 1, k + 1);
    for (int64_t j = k - 2; j <= k + 3; ++j) {
        if (j < lo || j > hi || j == k || j == k + 1) continue;
        const double x = b2_get(B, k, j), y = b2_get(B, k + 1, j);
        b2_set(B, k, j, c * x - s * y);
        b2_set(B, k + 1, j, s * x + c * y);
    }
    b2_set(B, k, k, c * c * a - 2.0 * c * s * bb + s * s * dd);
    b2_set(B, k + 1, k + 1, s * s * a + 2.0 * c * s * bb + c * c * dd);
    b2_set(B, k + 1, k, c * s * (a - dd) + (c * c - s * s) * bb);
}

int oracle_ql(int64_t n, double *d, double *e, double *Q, int64_t ldq)
{
    if (n <= 1) return 0;
    const double eps = 2.220446049250313e-16; /* 2^-52 */
    band2_t B;
    B.n = n;
    B.b0 = d;
    B.b1 = (double *)calloc((size_t)n, sizeof(double));
    B.b2 = (double *)calloc((size_t)n, sizeof(double));
    double *cs = (double *)calloc((size_t)n, sizeof(double));
    double *sn = (double *)calloc((size_t)n, sizeof(double));
    if (!B.b1 || !B.b2 || !cs || !sn) { free(B.b1); free(B.b2); free(cs); free(sn); return -1; }
    for (int64_t i = 0; i + 1 < n; ++i) B.b1[i] = e[i];
    int info = 0;

    for (int64_t l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int64_t m = l;
            while (m + 1 < n) {
                double off = fabs(B.b1[m]);
                if (off <= eps * (fabs(B.b0[m]) + fabs(B.b0[m + 1]))) { B.b1[m] = 0.0; break; }
                ++m;
            }
            if (m == l) break;                 /* d_l has converged */
            if (iter++ == 30) { info = (int)l + 1; goto done; }

            /* Wilkinson shift from the leading 2 x 2 of the block [l, m] */
            const double a = B.b0[l], bv = B.b1[l], c2 = B.b0[l + 1];
            const double delta = 0.5 * (c2 - a);
            const double sg = (delta >= 0.0) ? 1.0 : -1.0;
            const double mu = a - bv * bv / (delta + sg * hypot(delta, bv));

            /* first rotation, plane (m-1, m): annihilate the (m-1) entry of
             * the last column of (T - mu I) against its (m) entry */
            double xk = B.b1[m - 1];
            double xk1 = B.b0[m] - mu;
            for (int64_t k = m - 1; k >= l; --k) {
                double r = hypot(xk, xk1);
                double c, s;
                if (r == 0.0) { c = 1.0; s = 0.0; }
                else { c = xk1 / r; s = xk / r; }
                b2_rotate(&B, k, c, s, l, m);
                if (k + 2 <= m) B.b2[k] = 0.0;  /* the bulge at (k+2, k) is annihilated */
                cs[k] = c;
                sn[k] = s;
                if (k > l) {
                    /* next rotation, plane (k-1, k): annihilate the bulge at
                     * (k-1, k+1) against the entry (k, k+1) */
                    xk = B.b2[k - 1];
                    xk1 = B.b1[k];
                }
            }
            if (Q) {
                /* Q <- Q G_{m-1} G_{m-2} ... G_l, rows independent */
                const int64_t rb = 64;
                #pragma omp parallel for schedule(static)
                for (int64_t i0 = 0; i0 < n; i0 += rb) {
                    const int64_t i1 = (i0 + rb < n) ? i0 + rb : n;
                    for (int64_t k = m - 1; k >= l; --k) {
                        const double c = cs[k], s = sn[k];
                        double *qa = &Q[IDX(0, k, ldq)], *qb = &Q[IDX(0, k + 1, ldq)];
                        for (int64_t i = i0; i < i1; ++i) {
                            const double x = qa[i], y = qb[i];
                            qa[i] = c * x - s * y;
                            qb[i] = s * x + c * y;
                        }
                    }
                }
            }
        }
    }
done:
    for (int64_t i = 0; i + 1 < n; ++i) e[i] = B.b1[i];
    free(B.b1);
    free(B.b2);
    free(cs);
    free(sn);
    return info;
}

/* ------------------------------------------------------------------------
 * O-5: sort eigenvalues ascending and permute the columns of Q (if any).
 * Plain insertion sort over an index array (stable).
 * ------------------------------------------------------------------------ */
int oracle_sort(int64_t n, double *w, double *Q, int64_t ldq)
{
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *wt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!idx || !wt) { free(idx); free(wt); return -1; }
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    for (int64_t i = 1; i < n; ++i) {
        int64_t key = idx[i];
        int64_t j = i - 1;
        while (j >= 0 && w[idx[j]] > w[key]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = key;
    }
    for (int64_t i = 0; i < n; ++i) wt[i] = w[idx[i]];
    memcpy(w, wt, sizeof(double) * (size_t)n);
    if (Q) {
        double *Qt = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        if (!Qt) { free(idx); free(wt); return -1; }
        for (int64_t j = 0; j < n; ++j)
            memcpy(&Qt[IDX(0, j, n)], &Q[IDX(0, idx[j], ldq)], sizeof(double) * (size_t)n);
        for (int64_t j = 0; j < n; ++j)
            memcpy(&Q[IDX(0, j, ldq)], &Qt[IDX(0, j, n)], sizeof(double) * (size_t)n);
        free(Qt);
    }
    free(idx);
    free(wt);
    return 0;
}

/* ------------------------------------------------------------------------
 * Full oracle: A (n x n, the triangle 'L' or 'U' is read) -> w ascending and,
 * if Q != NULL, orthonormal eigenvectors with A Q = Q diag(w).
 * A is not modified.  Returns 0, a negative value on allocation failure, or
 * the QL non-convergence index.
 * ------------------------------------------------------------------------ */
int oracle_syev(char uplo, int64_t n, const double *A, int64_t lda, double *w, double *Q, int64_t ldq)
{
    if (n <= 0) return 0;
    double *S = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *tau = (double *)calloc((size_t)n, sizeof(double));
    if (!S || !e || !tau) { free(S); free(e); free(tau); return -1; }
    /* O-1: symmetrize from the referenced triangle */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            int64_t r = i, c = j;
            if (uplo == 'L' || uplo == 'l') { if (r < c) { r = j; c = i; } }
            else { if (r > c) { r = j; c = i; } }
            S[IDX(i, j, n)] = A[IDX(r, c, lda)];
        }
    oracle_tridiag(n, S, n, w, e, tau);
    if (Q) oracle_form_q(n, S, n, tau, Q, ldq);
    int info = oracle_ql(n, w, e, Q, ldq);
    if (info == 0) oracle_sort(n, w, Q, ldq);
    free(S);
    free(e);
    free(tau);
    return info;
}

/* Tridiagonal driver: eigenvalues (and vectors of T if Q != NULL) of
 * tridiag(e, d, e).  d, e are not modified. */
int oracle_stev(int64_t n, const double *d, const double *e, double *w, double *Q, int64_t ldq)
{
    if (n <= 0) return 0;
    double *et = (double *)calloc((size_t)n, sizeof(double));
    if (!et) return -1;
    memcpy(w, d, sizeof(double) * (size_t)n);
    if (n > 1) memcpy(et, e, sizeof(double) * (size_t)(n - 1));
    if (Q)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) Q[IDX(i, j, ldq)] = (i == j) ? 1.0 : 0.0;
    int info = oracle_ql(n, w, et, Q, ldq);
    if (info == 0) oracle_sort(n, w, Q, ldq);
    free(et);
    return info;
}

/* ------------------------------------------------------------------------
 * O-6: cyclic-by-row Jacobi (Golub & Van Loan, Algorithms 8.5.2/8.5.3) on the
 * full symmetric n x n matrix A (overwritten), accumulating V.  For each pair
 * (p, q) with a_pq != 0:
 *   theta = (a_qq - a_pp) / (2 a_pq),  t = sign(theta)/(|theta| + sqrt(1+theta^2)),
 *   c = 1/sqrt(1+t^2), s = t c,   J = [[c, s], [-s, c]] in rows/cols p, q,
 *   A <- J^T A J,  V <- V J.
 * Sweeps until off(A) <= 1e-3 * eps * ||A||_F, at most max_sweeps.
 * Returns the number of sweeps used, or -1 if it did not converge.
 * ------------------------------------------------------------------------ */
int oracle_jacobi(int64_t n, double *A, int64_t lda, double *w, double *V, int64_t ldv, int max_sweeps)
{
    const double eps = 2.220446049250313e-16;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) V[IDX(i, j, ldv)] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) fro += A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
    fro = sqrt(fro);
    int sweep = 0;
    for (;;) {
        double off = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                if (i != j) off += A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
        off = sqrt(off);
        if (off <= 1e-3 * eps * fro) break;
        if (sweep == max_sweeps) return -1;
        ++sweep;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                const double apq = A[IDX(p, q, lda)];
                if (apq == 0.0) continue;
                const double app = A[IDX(p, p, lda)], aqq = A[IDX(q, q, lda)];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = ((theta >= 0.0) ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* columns p, q:  A <- A J */
                for (int64_t k = 0; k < n; ++k) {
                    const double akp = A[IDX(k, p, lda)], akq = A[IDX(k, q, lda)];
                    A[IDX(k, p, lda)] = c * akp - s * akq;
                    A[IDX(k, q, lda)] = s * akp + c * akq;
                }
                /* rows p, q:  A <- J^T A */
                for (int64_t k = 0; k < n; ++k) {
                    const double apk = A[IDX(p, k, lda)], aqk = A[IDX(q, k, lda)];
                    A[IDX(p, k, lda)] = c * apk - s * aqk;
                    A[IDX(q, k, lda)] = s * apk + c * aqk;
                }
                A[IDX(p, q, lda)] = 0.0;
                A[IDX(q, p, lda)] = 0.0;
                for (int64_t k = 0; k < n; ++k) {
                    const double vkp = V[IDX(k, p, ldv)], vkq = V[IDX(k, q, ldv)];
                    V[IDX(k, p, ldv)] = c * vkp - s * vkq;
                    V[IDX(k, q, ldv)] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) w[i] = A[IDX(i, i, lda)];
    oracle_sort(n, w, V, ldv);
    return sweep;
}

/* ------------------------------------------------------------------------
 * O-7: Sturm count.  nu(T, sigma) = number of eigenvalues of
 * T = tridiag(e, d, e) strictly below sigma, from the signs of the pivots of
 * the LDL^T factorization of T - sigma I:
 *   q_0 = d_0 - sigma,  q_i = (d_i - sigma) - e_{i-1}^2 / q_{i-1}
 * An exact zero pivot is replaced by a tiny negative number (Kahan 1966).
 * ------------------------------------------------------------------------ */
int64_t oracle_sturm(int64_t n, const double *d, const double *e, double sigma)
{
    const double tiny = -1e-300;
    int64_t cnt = 0;
    double q = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0) q = d[0] - sigma;
        else q = (d[i] - sigma) - (e[i - 1] * e[i - 1]) / q;
        if (q == 0.0) q = tiny;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}
