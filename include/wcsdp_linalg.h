/*
 * wcsdp_linalg.h -- hand-written FP64 dense linear algebra on MI355X (gfx950).
 *
 * These are the building blocks the interior-point method uses to form the
 * Nesterov-Todd scaling point (Introduction, eq. newt), its eigen-split
 * (Section 3, eq. EQSigdef) and the Schur complement of the indefinite
 * preconditioner (Section 6).  They are exported so they can be tested on
 * their own.
 *
 * Conventions: column-major FP64, leading dimensions in elements, every
 * matrix pointer is a device pointer, `stream` is a hipStream_t or NULL.
 * Work is enqueued on `stream`; functions that return a count or a status
 * computed on the GPU synchronise it.  Return value 0 = success, -1 = invalid
 * argument, -3 = HIP error, -5 = numerical failure (see each function).
 * Temporary device memory is allocated and freed internally.
 */
#ifndef WCSDP_LINALG_H
#define WCSDP_LINALG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * C = alpha op(A) op(B) + beta C with op(X) = X (trans 'N') or X^T ('T');
 * op(A) is m x k, op(B) is k x n, C is m x n.  FP64 MFMA (16x16x4) tiles;
 * with op(B) = B and n <= 16 a row-parallel thin kernel instead.  Products
 * with few output tiles and a long K (and thin ones with a long K) are split
 * over K into partial products summed in a fixed order (a temporary
 * workspace; the stream is then synchronised before returning).  When
 * beta == 0, C is not read.
 */
int32_t wc_dgemm(void* stream, char transa, char transb, int32_t m, int32_t n, int32_t k, double alpha,
                 const double* A, int32_t lda, const double* B, int32_t ldb, double beta, double* C, int32_t ldc);

/*
 * C = A B (n x n; A n x k, B k x n, column-major, no transposes) where the
 * caller knows the product to be symmetric -- the second product E (Y E) of
 * the augmented operator's E Y E (Section 5), with E and Y symmetric.  Every
 * entry with row >= col is written; entries above the diagonal may or may not
 * be.  For n >= 3969 only the 128 x 128 tiles on or below the diagonal of the
 * first 128 floor(n / 128) rows are computed (spread evenly over the XCDs),
 * plus the rows below them; smaller n take the full product.  A temporary
 * workspace; the stream is synchronised before returning.  Returns 0, or -1
 * with the reason in sdp_last_error() for bad sizes.
 */
int32_t wc_dgemm_sym_lower(void* stream, int32_t n, int32_t k, const double* A, int32_t lda, const double* B,
                           int32_t ldb, double* C, int32_t ldc);

/*
 * y = alpha A x + beta y for a symmetric d x d matrix A held in full
 * (column-major, lda even, A 16-byte aligned): only one triangle is read,
 * half the bytes of a general product -- the preconditioner applies C^{-1}
 * (Section 6) this way.  x and y have d entries; when beta == 0, y is not
 * read.  A temporary workspace; the stream is synchronised before returning.
 */
int32_t wc_dsymv(void* stream, int32_t d, double alpha, const double* A, int32_t lda, const double* x, double beta,
                 double* y);

/*
 * wc_dsymv for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product and kernels, with the tile partial sums kept in a file-scope
 * device array of the library (one per GPU, about 32 MiB, held until the
 * process ends) instead of a workspace allocated per call.  Allocates and
 * frees nothing and does not synchronise the stream.  d must not exceed
 * WC_DSYMV_NOALLOC_MAX_D (-1 otherwise, nothing enqueued); the other
 * arguments and the result are as for wc_dsymv.  All calls on one GPU share
 * that array: calls that overlap on one GPU (different streams or host
 * threads without ordering between them) race and give wrong results.
 */
#define WC_DSYMV_NOALLOC_MAX_D 16384
int32_t wc_dsymv_noalloc(void* stream, int32_t d, double alpha, const double* A, int32_t lda, const double* x,
                         double beta, double* y);

/*
 * In-place Cholesky factorisation A = L L^T of the n x n symmetric positive
 * definite A (lower triangle read and overwritten with L; the strict upper
 * triangle is set to zero).  Returns 0, or -5 when a pivot is not positive;
 * *info_host (may be NULL) receives 0 or the 1-based index of that pivot.
 */
int32_t wc_dpotrf(void* stream, int32_t n, double* A, int32_t lda, int32_t* info_host);

/*
 * Linv = L^{-1} for the n x n lower-triangular L (strict upper triangle of L
 * ignored).  Linv's strict upper triangle is set to zero.  Linv must not
 * alias L.
 */
int32_t wc_dtrtri(void* stream, int32_t n, const double* L, int32_t ldl, double* Linv, int32_t ldi);

/*
 * One-sided (Hestenes) block Jacobi on the n x n matrix A: rotates the
 * columns of A in place until they are mutually orthogonal to within
 * tol * ||a_i|| ||a_j|| (tol <= 0 selects n * 2^-53), so that on return
 * A_in V = A_out.  Then sigma[k] (device, n) = ||A_out(:, k)|| in decreasing
 * order, V (device, n x n, may be NULL) holds the matching right singular
 * vectors with the sign convention "entry of largest magnitude positive"
 * (the columns of A_out are permuted and signed to match).  The number of
 * sweeps is returned through *sweeps_host (may be NULL).  Returns -5 if
 * max_sweeps were not enough.
 */
int32_t wc_djacobi_svd(void* stream, int32_t n, double* A, int32_t lda, double* V, int32_t ldv, double* sigma,
                       double tol, int32_t max_sweeps, int32_t* sweeps_host);

/*
 * Smallest Ritz value of the symmetric n x n matrix T (device, column-major,
 * leading dimension ldt >= n, 1 <= n <= 4096) after at most kmax (<= 64)
 * Lanczos steps with full reorthogonalisation.  It is an upper bound on
 * lambda_min(T), equal to it once converged, and it is the estimate the
 * interior-point step length max{alpha : X + alpha dX PSD} is taken from.
 * The value is written to *out_host; T is not modified.
 */
int32_t wc_dlanczos_min_eig(void* stream, int32_t n, const double* T, int32_t ldt, int32_t kmax, double* out_host);

/*
 * Low-precision GEMM of the mixed-precision inner operator: C = A B for
 * column-major A (m x k) and B (k x n) given in FP32 (prec_in = 1) or as BF16
 * bit patterns (prec_in = 2, uint16 per element), multiplied on the matrix
 * cores with FP32 accumulation.  out_kind 0 writes C as FP32, 1 as BF16
 * (round to nearest even), 2 adds the result to an FP64 C (C += A B), 3
 * writes C as FP64.
 */
int32_t wc_gemm_lp(void* stream, int32_t prec_in, int32_t out_kind, int32_t m, int32_t n, int32_t k, const void* A,
                   int32_t lda, const void* B, int32_t ldb, void* C, int32_t ldc);

/*
 * C = A B for a symmetric m x m matrix A and an m x n matrix B, both stored in
 * precision prec_in (1 FP32, 2 BF16 bit patterns; column-major) and
 * accumulated in FP32, written as out_kind says (as in wc_gemm_lp).  A is
 * read by rows, which is what makes both operands k-contiguous; only a
 * symmetric A may be passed.  With lda and ldb multiples of 4 (FP32) or 8
 * (BF16), 16-byte aligned A and B and at least 64 output tiles of 128 x 128,
 * a 128 x 128-tile kernel runs; otherwise the general kernel of wc_gemm_lp.
 */
int32_t wc_gemm_lp_sym(void* stream, int32_t prec_in, int32_t out_kind, int32_t m, int32_t n, const void* A,
                       int32_t lda, const void* B, int32_t ldb, void* C, int32_t ldc);

/*
 * B = A rounded to FP32 (prec = 1, round to nearest) or to BF16 (prec = 2,
 * round to FP32 then to nearest even), column-major rows x cols.
 */
int32_t wc_to_lowp(void* stream, int32_t prec, int32_t rows, int32_t cols, const double* A, int32_t lda, void* B,
                   int32_t ldb);

#ifdef __cplusplus
}
#endif

#endif /* WCSDP_LINALG_H */
