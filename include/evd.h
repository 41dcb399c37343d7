/*
 * evd.h -- C ABI of the MI355X (gfx950) two-stage dense symmetric eigensolver.
 *
 * Problem (paper, Section 1; Algorithm 1, REQUIRE/ENSURE): for a dense
 * symmetric A in R^{n x n} compute A = Q diag(W) Q^T with W the eigenvalues
 * (ascending) and, if requested, Q the orthogonal eigenvector matrix.
 *
 * Method (paper, Sections 2.1 and 3.3): successive band reduction (SBR) of A
 * to a band matrix B of half-bandwidth b with blocked Householder panels and
 * the two-sided ZY update of Eq. 1; bulge chasing (BC) of B to a tridiagonal
 * T; divide and conquer (D&C) on T; back transformation, by default in the
 * conventional order Q = Q_s (H_1 ... H_m Q_d) (BC-back on the D&C vectors,
 * then SBR-back from the left), or in the reordered order of Section 3.3
 * (SBR-back and BC-back applied to the identity, then one extra GEMM
 * Q = Q_sb * Q_d; "order" = 0).
 *
 * Conventions for every entry point:
 *  - Matrices are column-major; element (i, j) of M with leading dimension
 *    ld is M[i + j*ld].  Sizes and leading dimensions are 64-bit.
 *  - Pointers are DEVICE pointers (memory of the context's device) unless
 *    marked [host].  The caller owns all buffers; the library allocates no
 *    device memory inside compute calls (scratch comes from `work`).
 *  - Calls are asynchronous on the context's stream (evd_set_stream); results
 *    are valid after the stream is synchronised.  Numerical status goes to the
 *    device integer `info` where present.
 *  - Argument errors are detected on the host before any launch: the call
 *    returns EVD_ERR_INVALID_ARG and evd_last_invalid_arg() gives the 1-based
 *    position of the offending argument (LAPACK's -info convention).
 *  - No call throws across the ABI.  One context per host thread.
 */
#ifndef EVD_H
#define EVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct evd_ctx_s *evd_ctx_t;

typedef enum {
    EVD_OK = 0,
    EVD_ERR_INVALID_ARG = 1,   /* see evd_last_invalid_arg()                  */
    EVD_ERR_WORKSPACE = 2,     /* work buffer smaller than the queried size   */
    EVD_ERR_HIP = 3,           /* a HIP runtime call failed                   */
    EVD_ERR_NONFINITE = 4,     /* non-finite input (reported in device info)  */
    EVD_ERR_NOT_CONVERGED = 5, /* non-convergence (reported in device info)   */
    EVD_ERR_NOT_IMPLEMENTED = 6,
    EVD_ERR_TIMEOUT = 7        /* a wait between workgroups gave up (device info) */
} evd_status_t;

/* ------------------------------------------------------------------ context */

/* Create a context bound to HIP device `device`.  [host] *ctx receives the
 * handle.  The context owns only events and tunables.  device = -1 creates a
 * validation-only context: every entry point checks its arguments as usual
 * and then returns EVD_ERR_HIP without touching any device (for testing the
 * argument checks on machines without a GPU). */
evd_status_t evd_create(evd_ctx_t *ctx, int device);
evd_status_t evd_destroy(evd_ctx_t ctx);

/* Borrow a HIP stream (hipStream_t passed as void*; NULL = default stream). */
evd_status_t evd_set_stream(evd_ctx_t ctx, void *stream);

/* Tunables ([host] key strings):
 *   "b"            band half-width of SBR/BC, 0 = automatic (power of two, 4..64)
 *   "bc_waves"     number of persistent bulge-chasing wavefronts, 0 = automatic
 *   "order"        1 (default) = conventional stage order Q = Q_s (H_1 ... H_m Q_d),
 *                  2n^3 + 2n^3 back-transformation flops; 0 = the reordered
 *                  stages of Section 3.3 (Q_s H_1 ... H_m formed on the
 *                  identity, then Q = Q_sb Q_d: 4n^3/3 flops more, but
 *                  independent of D&C until the last product)
 *   "timing"       1 = record per-stage times (host-synchronising; for benchmarks)
 *   "panel_wgs"    0 (default) = each panel-QR workgroup holds as many rows
 *                  as its registers take (512 at b = 64), the fewest
 *                  workgroups; k > 0 = the rows spread over about k workgroups
 *   "panel_generic" 1: b = 64 panels in the generic thread layout (eight
 *                  lanes of a wavefront per column); 0 (default): each
 *                  wavefront holds eight whole columns over 64 rows per lane
 *                  step (the sums are formed in another order)
 *   "bcback_valu"  1 = apply the bulge-chasing reflectors one by one on the
 *                  vector ALUs; 0 (default) = in compact-WY groups of sweeps on
 *                  the matrix cores (b = 16, 32, 64)
 *   "bcback_group" sweeps per group of the blocked BC-back: 0 = automatic
 *                  (64 for b = 64, else 32), 32 = always 32
 *   "bcback_sub"   sweeps per block reflector inside a 64-sweep BC-back group,
 *                  applied one after another: 16, 32 (0 = default, 32) or 64
 *                  (one block reflector per group)
 *   "bcback_rows"  rows of Q per workgroup of the 64-sweep BC-back: 64 or 128
 *                  for all rows; 0 = automatic (128 for whole rounds of one
 *                  workgroup per compute unit, a remainder of at most one
 *                  round of 64-row workgroups as such, else 128)
 *   "bcback_rt"    16-row tiles per wavefront of the 128-row workgroups of
 *                  the 64-sweep BC-back with block reflectors: 1 (eight
 *                  wavefronts; 0 = default) or 2 (four wavefronts, each LDS
 *                  operand feeding two row tiles)
 *   "bcback_lds2"  1: 64-row workgroups of the 64-sweep BC-back double-buffer
 *                  their groups in LDS, one workgroup per compute unit;
 *                  0 (default): one buffer (61 KB), two workgroups per CU
 *   "gemm_staged"  1: every FP64 product stages its K slices through registers;
 *                  0 (default): 128 x 128 tiles with K slices of 16 that are
 *                  all whole load them straight into LDS (same results, bit
 *                  for bit).  Applies to every context of the process.
 *   "orgsb_nb"     panels of b columns aggregated into one block reflector in
 *                  SBR-back, in columns (0 = 512)
 *   "sbr_nb"       SBR outer (double-blocking) block in columns, 0 = 320;
 *                  a value <= b gives single blocking (one update per panel)
 *   "last_hip_error" first HIP error code a call met (read; set 0 to clear)
 *   "capture_error"  HIP error that made the last batched graph capture fall
 *                  back to a direct run (read only)
 *   "batch_streams", "batch_graph", "batch_plain", "last_graph_used"  see evd_dsyevd_batched
 *   "dc_max_iter"  iterations allowed per secular-equation root in D&C
 *                  (0 = 200); a small value forces the EVD_ERR_NOT_CONVERGED
 *                  status in `info` (for tests of the failure path)
 *   "bc_overlap"   1 = bulge chasing runs beside SBR (Section 2.1.1, Alg. 1):
 *                  launched on an auxiliary stream before the first panel,
 *                  each of its steps waits until SBR has published the band
 *                  columns it touches (panel by panel); 0 (default) = after
 *                  SBR.  Results are bitwise the same either way.
 *   "spin_limit_ms" longest wait (ms) of a workgroup for another workgroup's
 *                  progress (bulge-chasing sweeps, SBR's published band, the
 *                  panel-QR records) before the call gives up with
 *                  EVD_ERR_TIMEOUT in `info` and NaN outputs (0 = 30000)
 *   "dc_host"      1 = with vectors, D&C runs on the host CPU in a thread
 *                  (evd_dstedc_host) while the GPU forms Q_s H_1 ... H_m, as
 *                  in the paper's Algorithm 1; then Q = (Q_s H_1 ... H_m) Q_d
 *                  on the GPU.  The call then synchronises with its stream.
 *                  "dc_host_threads": its host threads (0 = automatic).
 *   "debug_gate"   1 = bulge chasing waits for band columns that are never
 *                  published (forces EVD_ERR_TIMEOUT; for tests of that path)
 * Unknown keys return EVD_ERR_INVALID_ARG. */
evd_status_t evd_set_param(evd_ctx_t ctx, const char *key, int64_t value);
evd_status_t evd_get_param(evd_ctx_t ctx, const char *key, int64_t *value /*[host]*/);

/* 1-based index of the argument that made the last call fail, 0 if none. */
int evd_last_invalid_arg(evd_ctx_t ctx);
const char *evd_status_string(evd_status_t s);

/* Per-stage wall times (ms) of the last evd_dsyevd call when "timing" = 1:
 * [0] SBR, [1] BC, [2] D&C / eigenvalue solve, [3] SBR-back, [4] BC-back,
 * [5] final GEMM, [6] total, [7] reserved.  [host] ms[8]. */
evd_status_t evd_get_stage_times(evd_ctx_t ctx, float *ms);

/* ------------------------------------------------------------------ GEMM */

/* C = alpha * op(A) * op(B) + beta * C on FP64 matrix cores (MFMA).
 * The products of Eq. 1 (Section 2.1.1), of SBR-back and of the final
 * eigenvector GEMM Q = Q_sb * Q_d (Section 3.3) are all of this form.
 *   opa: 'N' op(A) = A (m x k), 'T' op(A) = A^T (A is k x m),
 *        'S' op(A) = the symmetric m x m matrix whose lower triangle is stored
 *            in A (k must equal m; the strict upper triangle is not read).
 *   opb: 'N' op(B) = B (k x n), 'T' op(B) = B^T (B is n x k).
 *   lower_c: nonzero -> only entries C(i, j) with i >= j are written (SYR2K-style);
 *            2 -> each of them is also stored at C(j, i) (square C, opa 'N',
 *            opb 'T'; the symmetric rank-k update that keeps both triangles).
 * `work` (may be NULL) is scratch for split-K partial sums; when it is NULL or
 * smaller than evd_dgemm_work_size() the product runs without K splitting. */
evd_status_t evd_dgemm(evd_ctx_t ctx, char opa, char opb, int lower_c, int64_t m, int64_t n, int64_t k,
                       double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                       double beta, double *C, int64_t ldc, void *work, size_t work_bytes);
evd_status_t evd_dgemm_work_size(evd_ctx_t ctx, int64_t m, int64_t n, int64_t k, size_t *bytes /*[host]*/);

/* FP32 GEMM through split-BF16x3 on matrix cores (mixed-precision path; not
 * in the paper): each FP32 operand is split into bf16 hi + lo parts and
 * C = alpha (A_hi B_hi + A_hi B_lo + A_lo B_hi) + beta C with FP32
 * accumulation; about 17 significant bits per product (relative error of a
 * dot product ~ 3 * 2^-17 + FP32 accumulation).  Same op conventions as
 * evd_dgemm ('S' only with opb 'N'; lower_c not with 'S'). */
evd_status_t evd_sgemm_x3(evd_ctx_t ctx, char opa, char opb, int lower_c, int64_t m, int64_t n, int64_t k,
                          float alpha, const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                          float *C, int64_t ldc, void *work, size_t work_bytes);
evd_status_t evd_sgemm_x3_work_size(evd_ctx_t ctx, int64_t m, int64_t n, int64_t k, size_t *bytes /*[host]*/);

/* ------------------------------------------------------------------ full EVD */

/* dsyevd-style driver (LAPACK convention; paper Section 1).
 *   jobz 'N': eigenvalues only -> W (ascending); A is destroyed.
 *   jobz 'V': eigenvalues -> W and orthonormal eigenvectors -> A (column i
 *             pairs with W[i]).
 *   uplo 'L' or 'U': the triangle of A that is read.
 *   A: n x n, max(1, n) <= lda <= EVD_MAX_N.  W: n doubles.
 *   info: one device int32 holding an evd_status_t: 0 on success,
 *     EVD_ERR_NONFINITE if the referenced triangle of A holds a NaN or an
 *       infinity (W, and A for jobz 'V', are then set to NaN),
 *     EVD_ERR_NOT_CONVERGED if a secular equation of D&C did not converge,
 *     EVD_ERR_TIMEOUT if a wait between workgroups gave up ("spin_limit_ms";
 *       W, and A for jobz 'V', are then set to NaN).
 *   The input scan and the status stay on the stream (no host round trip):
 *   the host return value reports only argument and runtime errors.
 *   work: at least evd_dsyevd_work_size() bytes, 256-byte aligned. */
#define EVD_MAX_N ((int64_t)1 << 21) /* largest n and lda: the tile loaders' 32-bit byte offsets */
evd_status_t evd_dsyevd_work_size(evd_ctx_t ctx, char jobz, char uplo, int64_t n, int64_t lda,
                                  size_t *bytes /*[host]*/);
evd_status_t evd_dsyevd(evd_ctx_t ctx, char jobz, char uplo, int64_t n, double *A, int64_t lda,
                        double *W, void *work, size_t work_bytes, int32_t *info);

/* evd_dsyevd without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, outputs, `info` and host status
 * as evd_dsyevd; the scratch is a static device array of
 * EVD_NOALLOC_SCRATCH_BYTES per GPU, held by the library on every GPU it
 * runs on until the process ends, whose address is looked up by evd_create.
 * The call itself allocates nothing (no device allocation, no stream or event
 * creation).  Returns EVD_ERR_WORKSPACE (evd_last_invalid_arg = 4) when
 * evd_dsyevd_work_size(jobz, uplo, n, lda) exceeds that size: at the default
 * band width n <= 1151 fits with vectors, n <= 5262 for eigenvalues only.
 * All calls on one GPU share its array: calls that overlap on one GPU (two
 * streams, two host threads, two contexts) race and must be serialised by the
 * caller; consecutive calls on one stream are safe. */
#define EVD_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
evd_status_t evd_dsyevd_noalloc(evd_ctx_t ctx, char jobz, char uplo, int64_t n, double *A, int64_t lda,
                                double *W, int32_t *info);

/* Mixed-precision EVD with FP64 refinement (an extension beside the paper's
 * FP64 path; not in the paper).  The pipeline of evd_dsyevd runs in FP32
 * (panel QR, bulge chasing and BC-back on FP32 vector units; every product
 * through split-BF16x3 matrix cores, see evd_sgemm_x3), the tridiagonal
 * eigenproblem in FP64, then FP64 Ogita-Aishima refinement sweeps
 * (R = I - X^T X, S = X^T A X, lam_i = s_ii/(1 - r_ii),
 * E_ij = (s_ij + lam_j r_ij)/(lam_j - lam_i) if |lam_i - lam_j| > delta else
 * r_ij/2, X <- X + X E; eigenvalues closer than delta are resolved by a
 * Rayleigh-Ritz step inside the sweep) improve the eigenpairs.  Outputs as
 * evd_dsyevd (jobz must be 'V'; W ascending, eigenvectors in A; W holds the
 * Rayleigh quotients of the returned vectors).
 *   max_sweeps: 0..8 refinement sweeps at most.
 *   target_residual > 0: the sweeps stop as soon as the scaled residual
 *     ||A X - X diag(W)||_F / (n ||A||_F) and the orthogonality
 *     ||X^T X - I||_F / n are both <= target_residual (the call then
 *     synchronises with its stream once per sweep); if they are not reached
 *     after max_sweeps, info = EVD_ERR_NOT_CONVERGED (the pairs are still
 *     returned).  target_residual <= 0: exactly max_sweeps sweeps, no status.
 *   achieved (optional, device, 8 doubles): [0] the achieved scaled residual,
 *     [1] the orthogonality above, [2] sweeps run, and of the last sweep
 *     [3] delta, [4] clusters resolved by Rayleigh-Ritz, [5] the largest
 *     cluster size, [6] ||S - diag(lam)||_F, [7] ||R||_F.  Not written for
 *     n < 3 (solved by the FP64 driver).
 * Stage times ("timing" = 1): [0] SBR, [1] BC, [2] D&C, [3] SBR-back,
 * [4] BC-back, [5] final product, [6] refinement, [7] total. */
evd_status_t evd_dsyevd_mixed_work_size(evd_ctx_t ctx, char jobz, char uplo, int64_t n, int64_t lda,
                                        size_t *bytes /*[host]*/);
evd_status_t evd_dsyevd_mixed(evd_ctx_t ctx, char jobz, char uplo, int64_t n, double *A, int64_t lda,
                              double *W, int32_t max_sweeps, double target_residual, void *work,
                              size_t work_bytes, int32_t *info, double *achieved);

/* Autotuner for the band half-width b (the paper fixes b = 32 for its
 * platform, Section 4.1; the best b depends on the GPU and on n) and the
 * blocking of the kernels around it.  Times evd_dsyevd on A (n x n, lower
 * triangle, not modified) for the configurations (b, SBR outer block
 * "sbr_nb", BC-back block width "bcback_sub") in
 *   (16, 256), (16, 512), (32, 256), (32, 512),
 *   (64, 256, 32), (64, 320, 32), (64, 512, 32), (64, 320, 64)
 * (two calls each, the second timed with events on the stream; this call
 * synchronises) and records the fastest for n's size bucket floor(log2 n) in
 * the context, where evd_dsyevd, evd_dsyevd_mixed, the batched driver and
 * the work-size queries use them while the parameters are 0.
 * [host] best_b, best_ms may be NULL; the other choices are read back as the
 * parameters "last_tuned_nb" and "last_tuned_sub". */
evd_status_t evd_autotune_work_size(evd_ctx_t ctx, char jobz, int64_t n, size_t *bytes /*[host]*/);
evd_status_t evd_autotune(evd_ctx_t ctx, char jobz, int64_t n, const double *A, int64_t lda, void *work,
                          size_t work_bytes, int64_t *best_b, float *best_ms);

/* Batched EVD of many uneven-size matrices (an extension beside the paper's
 * method; tight-binding models are one of its applications, Section 1).
 * Matrix i (n[i] x n[i], leading dimension lda[i]) is solved exactly as by
 * evd_dsyevd: eigenvalues into W[i], eigenvectors into A[i] (jobz 'V').
 * n, lda: [host] arrays of `batch` sizes.  A, W: [host] arrays of `batch`
 * DEVICE pointers.  info: device int32[batch] (per-matrix status).
 * t_start_end (optional): device uint64[2*batch], wall_clock64 (100 MHz) ticks
 * at the start and end of every matrix.
 * Matrices are ordered by decreasing n^3 and spread over "batch_streams"
 * (default 8) streams, launched directly (default) or, with "batch_graph" =
 * 1, captured once into a hipGraph that is replayed while sizes and pointers
 * are unchanged ("last_graph_used" reports whether the graph ran; on ROCm 7
 * the replay runs the streams' branches one after another, 2.2x slower than
 * the direct launches on the tight-binding batch).  Persistent kernels are
 * capped at (compute units / streams) workgroups each and, with
 * "batch_plain" = 1 (default), launched plainly so that the streams run side
 * by side (0 = cooperative launches, which the runtime serialises).
 * work: evd_dsyevd_batched_work_size() bytes. */
evd_status_t evd_dsyevd_batched_work_size(evd_ctx_t ctx, char jobz, int32_t batch, const int64_t *n /*[host]*/,
                                          const int64_t *lda /*[host]*/, size_t *bytes /*[host]*/);
evd_status_t evd_dsyevd_batched(evd_ctx_t ctx, char jobz, char uplo, int32_t batch, const int64_t *n /*[host]*/,
                                double *const *A /*[host] array of device pointers*/,
                                const int64_t *lda /*[host]*/, double *const *W /*[host] array of device pointers*/,
                                void *work, size_t work_bytes, int32_t *info, uint64_t *t_start_end);

/* ------------------------------------------------------------------ stages */

/* Stage 1, SBR (Section 2.1.1, Fig. 1, Eq. 1): reduce the symmetric A (lower
 * triangle read; 'U' is first mirrored into it) to a band matrix B of
 * half-bandwidth b by panels of b columns: panel k is QR-factored,
 * P_k = (I - Y_k T_k Y_k^T) R_k, and the trailing matrix A_2 receives
 * Z = A_2 W - 1/2 Y (W^T A_2 W), A_2 <- A_2 - Y Z^T - Z Y^T with W = Y T.
 * Outputs:
 *   AB (ldab >= 2b+1, n columns): B in lower band storage, AB[d + j*ldab] =
 *      B(j+d, j) for 0 <= d <= b; rows b+1..2b are zeroed (room for bulges).
 *   A: columns kb..kb+b-1, rows (k+1)b..n-1 hold the explicit Y_k
 *      (unit lower trapezoidal: ones on its diagonal, zeros above); the rest
 *      of A (both triangles) is used as scratch.
 * The trailing updates are double-blocked (Section 4.1): deferred over outer
 * blocks of "sbr_nb" columns, with the trailing matrix kept in full storage
 * (each block's update writes both triangles) so that A_2 W is a plain
 * product.
 *   T: the b x b upper triangular T_k of panel k at T + k*b*b (column-major,
 *      leading dimension b); evd_sbr_num_panels(n, b) panels.
 * Requires 1 <= b <= 64, b | 64 (b in {1,2,4,8,16,32,64}). */
int64_t evd_sbr_num_panels(int64_t n, int64_t b);
evd_status_t evd_dsy2sb_work_size(evd_ctx_t ctx, int64_t n, int64_t b, size_t *bytes /*[host]*/);
evd_status_t evd_dsy2sb(evd_ctx_t ctx, char uplo, int64_t n, int64_t b, double *A, int64_t lda,
                        double *AB, int64_t ldab, double *T, void *work, size_t work_bytes);

/* Stage 2, BC (Section 2.1.1; Section 4.2 for its sweep/step structure):
 * reduce the band matrix in AB to tridiagonal T = tridiag(e, d, e) by
 * Householder bulge chasing.  Sweep c (0 <= c < n-2) annihilates column c
 * below its sub-diagonal with a reflector on rows c+1..c+b and chases the
 * bulge down in steps s = 1, 2, ...; step s acts on rows r = c+1+s*b ..
 * r+b-1.  Reflector (c, s) is H = I - tau v v^T with v[0] = 1, stored at
 *   V  [ (s*n + c) * b + i ],  i = 0..b-1 (zero-padded), and
 *   TAU[  s*n + c ]             (0 for reflectors that do not exist),
 * for s < evd_bc_num_steps(n, b).  T = H_m ... H_1 B H_1 ... H_m in
 * generation order.  AB is overwritten.  V/TAU may be NULL when jobz = 'N'.
 * work: evd_dsb2st_work_size() bytes (one progress counter per sweep). */
int64_t evd_bc_num_steps(int64_t n, int64_t b);
evd_status_t evd_dsb2st_work_size(evd_ctx_t ctx, int64_t n, size_t *bytes /*[host]*/);
evd_status_t evd_dsb2st(evd_ctx_t ctx, char jobz, int64_t n, int64_t b, double *AB, int64_t ldab,
                        double *d, double *e, double *V, double *TAU, void *work, size_t work_bytes);

/* Stage 3, tridiagonal eigensolver on T = tridiag(e, d, e) (Section 2.1.1;
 * divide and conquer of Cuppen / Gu-Eisenstat, Tisseur-Dongarra):
 *   compz 'I': W (ascending) and eigenvectors of T in Z (n x n, ldz >= n).
 *   compz 'N': eigenvalues only (Sturm bisection); Z is not referenced.
 * d, e are not modified.  info: device int32, 0 on success,
 * EVD_ERR_NOT_CONVERGED if a secular equation did not converge (compz 'I'). */
evd_status_t evd_dstedc_work_size(evd_ctx_t ctx, char compz, int64_t n, size_t *bytes /*[host]*/);
evd_status_t evd_dstedc(evd_ctx_t ctx, char compz, int64_t n, const double *d, const double *e,
                        double *W, double *Z, int64_t ldz, void *work, size_t work_bytes, int32_t *info);

/* The same stage on the host CPU, as the paper places it (Algorithm 1 runs
 * D&C in a CPU thread beside the GPUs' back transformation, Section 3.3):
 * divide and conquer with the same tear, deflation, secular solver,
 * Gu-Eisenstat zhat and zero-block-skipping products, spread over `threads`
 * std::thread workers (0 = OMP_NUM_THREADS, else all hardware threads).
 * All pointers are [host]: d (n), e (n-1), W (n), Z (ldz x n, compz 'I').
 * *info [host, optional] = 0 or EVD_ERR_NOT_CONVERGED.  No context, no
 * device.  evd_dsyevd uses it when "dc_host" = 1. */
evd_status_t evd_dstedc_host(char compz, int64_t n, const double *d, const double *e, double *W, double *Z,
                             int64_t ldz, int32_t threads, int32_t *info);

/* Stage 4a, SBR-back (Section 2.1.2; Algorithm 1 genW/genQ): form
 * Q_s = (I - Y_0 T_0 Y_0^T)(I - Y_1 T_1 Y_1^T) ... in Q (n x n, ldq >= n),
 * from the Y_k stored in A and the T_k in T by evd_dsy2sb. */
evd_status_t evd_dorgsb_work_size(evd_ctx_t ctx, int64_t n, int64_t b, size_t *bytes /*[host]*/);
evd_status_t evd_dorgsb(evd_ctx_t ctx, int64_t n, int64_t b, const double *A, int64_t lda, const double *T,
                        double *Q, int64_t ldq, void *work, size_t work_bytes);

/* Stage 4b, BC-back (Sections 2.1.2 and 4.3): with the bulge-chasing
 * reflectors H_1 ... H_m of evd_dsb2st (V, TAU as it wrote them),
 *   trans 'N': Q <- Q H_1 H_2 ... H_m   (Q_d = H_1 ... H_m applied from the right)
 *   trans 'T': Q <- Q H_m ... H_2 H_1   (= Q Q_d^T: the rows of Q_d^T Z)
 * Q is m_rows x n, column-major, ldq >= m_rows; rows are independent.
 * work: device scratch of evd_dbcback_work_size() bytes, 8-byte aligned, for
 * the T factors of the blocked matrix-core path (reflector groups of 32
 * sweeps, compact WY; used for b = 16, 32, 64 while "bcback_valu" is 0).  A
 * size of 0 means the reflector-by-reflector kernel runs and work may be NULL.
 * Returns EVD_ERR_WORKSPACE if work_bytes is below the queried size. */
evd_status_t evd_dbcback_work_size(evd_ctx_t ctx, int64_t n, int64_t b, size_t *bytes /*[host]*/);
evd_status_t evd_dbcback(evd_ctx_t ctx, char trans, int64_t m_rows, int64_t n, int64_t b, const double *V,
                         const double *TAU, double *Q, int64_t ldq, void *work, size_t work_bytes);

#ifdef __cplusplus
}
#endif

#endif /* EVD_H */
