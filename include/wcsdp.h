/*
 * wcsdp.h -- C ABI of the MI355X well-conditioned low-rank SDP solver.
 *
 * Solves the standard-form primal/dual pair (Introduction, eq. sdp-pd)
 *     min <C, X>  s.t.  A(X) = b, X PSD;      max <b, y>  s.t.  A^T(y) + S = C, S PSD
 * with a primal-dual interior-point method whose Newton systems (Section 3,
 * eq. Newt-eps) are solved through the well-conditioned augmented system of
 * eq. augsys by indefinite-preconditioned PCG (Corollary pcg, Section 6) and
 * recovered with eq. recover.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are n x n, column-major, FP64.  Symmetric inputs must be
 *    symmetric to within 1e-12 of their Frobenius norm.
 *  - "device pointer" means memory the caller allocated on the GPU that
 *    the context was set up on (hipMalloc, or a torch CUDA tensor); the
 *    caller keeps ownership.  "host pointer" means ordinary CPU memory.
 *  - Every GPU operation is issued on the stream given to sdp_setup (NULL =
 *    the default stream) and is stream-ordered with the caller's work.  Entry
 *    points that return scalars or statistics synchronise that stream.
 *  - No C++ exception crosses this boundary.  On error the return value is
 *    negative, sdp_last_error() describes it, and outputs are unspecified
 *    unless stated otherwise.
 *  - Augmented-system vectors have length sdp_aug_dim() = m + d with
 *    d = n r - r (r - 1) / 2 (Proposition correct).  The first m entries are
 *    u; the remaining d entries are v = [svec(B); vec(N)] with B an r x r
 *    symmetric block (svec: column-major lower triangle, off-diagonal entries
 *    times sqrt(2), Notations) and N an (n - r) x r block stored
 *    column-major, both expressed in the eigenbasis [Q Qp] of the scaling
 *    point W (eq. EQSigdef).  Eigenvalues are ordered decreasingly and every
 *    eigenvector is signed so that its entry of largest magnitude is
 *    positive (lowest index on ties).
 */
#ifndef WCSDP_H
#define WCSDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdp_ctx sdp_ctx;
typedef int32_t sdp_status;

enum {
    SDP_OK = 0,
    SDP_EINVAL = -1,    /* invalid argument: shapes, indices, NaN/Inf, asymmetry */
    SDP_ENOMEM = -2,    /* device allocation failed */
    SDP_EDEVICE = -3,   /* a HIP call failed */
    SDP_ENOTCONV = -4,  /* inner Krylov solve reached inner_maxit */
    SDP_ENUMERIC = -5,  /* a factorisation met a non-positive pivot */
    SDP_ESTALL = -6,    /* the interior-point method hit max_ipm_iter or stalled */
    SDP_ECENTER = -7    /* sdp_adjoint could not bring the iterate onto the central path */
};

/* Largest distance to the central path at which sdp_adjoint reports SDP_OK. */
#define SDP_ADJOINT_CENTER_TOL 1e-6

enum { SDP_A_DENSE = 0, SDP_A_ENTRY = 1, SDP_A_SPARSE = 2 };
enum { SDP_SOLVER_PCG = 0, SDP_SOLVER_MINRES = 1 };
enum { SDP_PREC_F64 = 0, SDP_PREC_F32 = 1, SDP_PREC_BF16 = 2 };
enum { SDP_REFINE_SWEEPS = 0, SDP_REFINE_REPLACE = 1 };

/*
 * Problem data (Introduction, eq. sdp-pd).
 *  a_kind == SDP_A_DENSE: A holds m rows of n*n values, row i = vec(A_i); each
 *      A_i must be symmetric.
 *  a_kind == SDP_A_ENTRY: jk holds m pairs (j, k), 0-based, j <= k < n, all
 *      distinct; A_i = (e_j e_k^T + e_k e_j^T)/2, so <A_i, X> = X_jk.
 *  a_kind == SDP_A_SPARSE: A and jk are unused; the entries come in an
 *      sdp_sparse_rows given to sdp_setup_ex.
 *  b has m entries; C is n x n symmetric.
 *  on_device != 0 means A / jk / b / C are device pointers, else host
 *  pointers.  Validation of values (NaN, symmetry, index range, duplicates)
 *  is done for host inputs only; device inputs are checked for shape only.
 *  sdp_setup copies everything it needs: the caller may free the inputs
 *  afterwards.
 */
typedef struct sdp_problem {
    int32_t n;
    int32_t m;
    int32_t a_kind;
    const double* A;
    const int32_t* jk;
    const double* b;
    const double* C;
    int32_t on_device;
} sdp_problem;

/*
 * Sparse constraint matrices (a_kind == SDP_A_SPARSE): constraint i owns the
 * entries ptr[i] .. ptr[i+1]-1 of (row, col, val), 0-based, row <= col < n,
 * with A_i[row][col] = A_i[col][row] = val (repeated positions add).
 * ptr has m + 1 entries, ptr[0] = 0, nondecreasing.  on_device as in
 * sdp_lp_block.  Suited to constraints with few nonzeros each, such as the
 * distance rows a a^T of eq. snl-sdp.
 */
typedef struct sdp_sparse_rows {
    const int32_t* ptr;
    const int32_t* row;
    const int32_t* col;
    const double* val;
    int32_t on_device;
} sdp_sparse_rows;

/*
 * A nonnegative-orthant (LP) block beside the PSD variable: the problem
 * becomes  min <C, X> + c^T x  s.t.  A(X) + B x = b,  X PSD,  x >= 0  (the
 * cone of eq. rmc-sdp and eq. snl-sdp in the experiments section), with the
 * dual slack s = c - B^T y >= 0.
 *  l           LP coordinates (>= 1)
 *  col_ptr     l + 1 offsets into row / val, col_ptr[0] = 0, nondecreasing:
 *              column j of B holds the entries col_ptr[j] .. col_ptr[j+1]-1
 *  row, val    0-based constraint index (< m) and value of each entry; a
 *              row may repeat within a column (the values add)
 *  c           the cost, l entries
 *  on_device   nonzero: the four arrays are device pointers (checked for shape
 *              only), else host pointers (also checked for range and finite
 *              values).  sdp_setup_lp copies what it needs.
 */
typedef struct sdp_lp_block {
    int32_t l;
    const int32_t* col_ptr;
    const int32_t* row;
    const double* val;
    const double* c;
    int32_t on_device;
} sdp_lp_block;

/*
 * Solver options.  sdp_default_options fills the defaults given in brackets.
 *  rank_max     rhat of the rank rule r = argmax_{i <= rhat} lambda_i/lambda_{i+1}
 *               (Experiments section) [10, clipped to n - 1]
 *  rank_fixed   > 0 forces r [0]
 *  beta         > 0 fixes the preconditioner's beta (Corollary pcg); <= 0 uses
 *               (median eigenvalue of E)^2 * mean ||A_i||_F^2, with an LP block
 *               raised to max_i (B diag(e2) B^T)_ii when that is larger (e2 the
 *               LP coordinates' script-E entries: 1 on T) [0]
 *  solver       SDP_SOLVER_PCG (Corollary pcg) or SDP_SOLVER_MINRES (Corollary minres) [PCG]
 *  inner_tol    PCG stops when ||r_u|| <= inner_tol * ||r_u(0)|| [1e-10]
 *  inner_maxit  [2000]
 *  inner_prec   precision of the inner operator [SDP_PREC_F64].  SDP_PREC_F32:
 *               the A E A^T block of the augmented operator with E Y E on the
 *               FP32 matrix cores and, for dense A, the two constraint passes
 *               over an FP32 copy of the packed rows (FP64 accumulation);
 *               SDP_PREC_BF16: the same with the GEMM operands in BF16 (FP32
 *               accumulation; the constraint data stays FP32).  The
 *               off-diagonal and bottom blocks stay FP64.  The Newton step is
 *               brought to inner_tol by FP64 iterative refinement; the scaling
 *               point, its eigen-decomposition, the preconditioner, residuals
 *               and step lengths stay FP64.
 *  max_refine   most FP64 refinement sweeps around a low-precision inner
 *               solve; SDP_REFINE_SWEEPS also stops once two sweeps in a row
 *               fail to halve the FP64 residual [20]
 *  refine_mode  how the FP64 refinement corrects the low-precision inner
 *               solve [SDP_REFINE_SWEEPS]: SDP_REFINE_SWEEPS restarts a
 *               low-precision PCG run on each FP64 residual (classic
 *               iterative refinement); SDP_REFINE_REPLACE runs one PCG with
 *               the low-precision operator and replaces its recursive
 *               residual by the FP64 residual g - K x whenever it has dropped
 *               by refine_tol since the last replacement, keeping the search
 *               direction (the Krylov space survives the correction)
 *  refine_tol   SWEEPS: relative residual reduction asked of each low-precision
 *               PCG run (0: 1e-6 for FP32, 1e-2 for BF16); later sweeps ask
 *               only for the reduction still missing to inner_tol when that is
 *               larger.  REPLACE: reduction between two replacements (0: 1e-2
 *               for FP32, 1e-1 for BF16) [0]
 *  gap_tol, feas_tol   stopping tolerances of the interior-point method [1e-8]
 *  max_ipm_iter [100]
 *  step_frac    fraction of the step to the boundary [0.98]
 *  verbose      0 silent, 1 one line per interior-point iteration and one per
 *               scaling setup with its phase timings (the stream is synchronised
 *               between phases), 2 also one line per Krylov iteration (stderr) [0]
 *  sparse_sandwich  entry-sampling constraints only, n <= 16384: nonzero
 *               forms the A E A^T block of the FP64 operator (with a
 *               low-precision inner_prec: of the FP64 products that the
 *               refinement takes its residuals with)
 *               (Section 5) at the sampled pairs only, as Z = A^T(u) E (a
 *               sparse-dense product) followed by one length-n dot product
 *               per constraint, instead of the two dense n x n x n products
 *               of E Y E.  Same operator up to rounding; it pays when m is far
 *               below n^2 [0]
 *  lp_top_max   LP block only: most LP coordinates that join the low-rank
 *               part T of the split (those with w_j = sqrt(x_j/s_j) above
 *               2 tau; past the cap only the largest stay, a tied group as a
 *               whole or not at all).  The augmented system and the
 *               preconditioner's Schur complement grow by |T| [2048]
 */
typedef struct sdp_options {
    int32_t rank_max;
    int32_t rank_fixed;
    double beta;
    int32_t solver;
    double inner_tol;
    int32_t inner_maxit;
    int32_t inner_prec;
    int32_t max_refine;
    double gap_tol;
    double feas_tol;
    int32_t max_ipm_iter;
    double step_frac;
    int32_t verbose;
    double refine_tol;
    int32_t sparse_sandwich;
    int32_t refine_mode;
    int32_t lp_top_max;
} sdp_options;

typedef struct sdp_inner_stats {
    int32_t iterations;     /* Krylov iterations (summed over refinement sweeps) */
    int32_t refinements;    /* FP64 refinement sweeps, or FP64 residual replacements (0 in FP64 mode) */
    int32_t converged;      /* 1 if the tolerance was met */
    int32_t r;              /* rank parameter of the split */
    double tau;             /* lambda_{r+1}(W) / 2 */
    double beta;            /* preconditioner beta */
    double rel_res;         /* final ||r_u|| / ||r_u(0)|| */
} sdp_inner_stats;

typedef struct sdp_step_stats {
    double mu, pobj, dobj, relgap, pinf, dinf;   /* at the start of the step */
    double alpha_p, alpha_d, sigma;
    int32_t r;
    int32_t pcg_pred, pcg_corr;
    int32_t converged;      /* 1 if the point already met the tolerances (no step taken) */
    double t_scaling_ms, t_inner_ms, t_total_ms;
} sdp_step_stats;

typedef struct sdp_result {
    int32_t status;
    int32_t iterations;
    int64_t pcg_iterations;
    int64_t newton_matvecs;  /* FP64 applications of the augmented operator */
    double pobj, dobj, relgap, pinf, dinf, mu;
    double time_ms;
    int64_t lp_matvecs;      /* applications of its low-precision form (mixed mode) */
} sdp_result;

/* Fill *opt with the defaults listed above. */
void sdp_default_options(sdp_options* opt);

/*
 * Create a context for one problem.  Validates and uploads the data, builds
 * the device layout of A (dense: packed lower-triangle rows; entry: index
 * pairs) and sets the starting point X = xi I, S = eta I, y = 0.
 * hip_stream: a hipStream_t, or NULL.  *out receives the context; on error
 * *out is NULL and the message is available from sdp_last_error(NULL).
 */
sdp_status sdp_setup(const sdp_problem* prob, const sdp_options* opt, void* hip_stream, sdp_ctx** out);

/*
 * sdp_setup for a problem with an LP block (see sdp_lp_block; lp may be NULL,
 * which is sdp_setup).  The starting point adds x = xi 1, s = eta 1 with the
 * magnitudes of X0 and S0.  On such a context the augmented system gains one
 * v-coordinate per LP coordinate in T after the SDP ones (sdp_aug_dim counts
 * them); sdp_newton_apply, sdp_precond_apply, sdp_ipm_step, sdp_solve and
 * sdp_get_point work as documented, with the LP block included; use
 * sdp_set_point_lp, sdp_get_point_lp and sdp_inner_solve_lp for the parts that
 * carry x, s or c~.  sdp_set_point, sdp_inner_solve, sdp_adjoint and
 * sdp_solve_batched return SDP_EINVAL on it.
 */
sdp_status sdp_setup_lp(const sdp_problem* prob, const sdp_lp_block* lp, const sdp_options* opt, void* hip_stream,
                        sdp_ctx** out);

/*
 * sdp_setup_lp for any constraint kind: sparse carries the constraint entries
 * when prob->a_kind == SDP_A_SPARSE (NULL otherwise); lp may be NULL.  The
 * sparse kind forms script-A script-Q explicitly from the entries (as for
 * dense rows) and runs with inner_prec SDP_PREC_F64; sdp_adjoint and
 * sdp_solve_batched do not take it (SDP_EINVAL).
 */
sdp_status sdp_setup_ex(const sdp_problem* prob, const sdp_sparse_rows* sparse, const sdp_lp_block* lp,
                        const sdp_options* opt, void* hip_stream, sdp_ctx** out);

/* Release every device buffer the context owns.  NULL is allowed. */
void sdp_destroy(sdp_ctx* ctx);

/* Message of the last error on ctx (or of the last failed sdp_setup when ctx is NULL). */
const char* sdp_last_error(const sdp_ctx* ctx);

/* m + d at the current scaling (d depends on the rank parameter r). */
int64_t sdp_aug_dim(sdp_ctx* ctx);

/*
 * One application of the augmented operator of eq. augsys,
 *   [u'; v'] = [A E A^T, A Q; Q^T A^T, -tau^2 Sigma] [u; v],
 * evaluated with the Section 5 products at the scaling point of the current
 * iterate (computed on first use after sdp_setup / sdp_set_point /
 * sdp_ipm_step).  uv_in, uv_out: device pointers of sdp_aug_dim() doubles,
 * not aliased.
 */
sdp_status sdp_newton_apply(sdp_ctx* ctx, const double* uv_in, double* uv_out);

/*
 * The same product in a chosen precision: SDP_PREC_F64 is sdp_newton_apply;
 * otherwise prec must equal the inner_prec the context was set up with, and
 * the product is the low-precision form used inside the refinement sweeps
 * (see sdp_options.inner_prec).  Returns SDP_EINVAL for any other prec.
 */
sdp_status sdp_newton_apply_prec(sdp_ctx* ctx, int32_t prec, const double* uv_in, double* uv_out);

/*
 * The preconditioner of Section 6 applied to a vector of the augmented space:
 * uv_out = P^{-1} uv_in with P = [beta I, AQ; (AQ)^T, -tau^2 Sigma], by block
 * elimination through the Schur complement C = tau^2 Sigma + (AQ)^T (AQ) / beta
 * followed by one step of iterative refinement -- the operation every PCG
 * iteration of sdp_inner_solve performs.  FP64.  Same layout and pointer
 * rules as sdp_newton_apply (device pointers of length m + d, not aliased);
 * the scaling point is prepared first if needed.
 */
sdp_status sdp_precond_apply(sdp_ctx* ctx, const double* uv_in, double* uv_out);

/*
 * Solve eq. Newt-eps at the current scaling point: given b_tilde (m) and the
 * symmetric C_tilde (n x n), return dX (n x n) and dy (m) with
 *   dX = W (A^T(dy) - C_tilde) W,   A(dX) = b_tilde
 * through eq. augsys (indefinite PCG, Corollary pcg) and eq. recover.
 * All four arrays are device pointers.  stats may be NULL.  Returns
 * SDP_ENOTCONV (with the last iterate's recovery written) when inner_maxit
 * is reached.
 */
sdp_status sdp_inner_solve(sdp_ctx* ctx, const double* b_tilde, const double* C_tilde, double* dX, double* dy,
                           sdp_inner_stats* stats);

/*
 * sdp_inner_solve on a context with an LP block: eq. Newt-eps extended by
 * B dx with dx = w^2 (B^T dy - c~) (w = sqrt(x/s) elementwise) and
 * A(dX) + B dx = b_tilde.  c_tilde_lp and dx_lp are device pointers of l
 * entries; the other arguments as for sdp_inner_solve.
 */
sdp_status sdp_inner_solve_lp(sdp_ctx* ctx, const double* b_tilde, const double* C_tilde, const double* c_tilde_lp,
                              double* dX, double* dy, double* dx_lp, sdp_inner_stats* stats);

/*
 * The LP split at the current scaling point (prepared first if needed):
 * *t = |T|; top_idx (device, at least lp_top_max int32 entries, or NULL)
 * receives T in increasing order; w (device, l doubles, or NULL) receives
 * w = sqrt(x/s).  SDP_EINVAL without an LP block.
 */
sdp_status sdp_get_lp_split(sdp_ctx* ctx, int32_t* t, int32_t* top_idx, double* w);

/*
 * One Mehrotra predictor-corrector iteration with the Nesterov-Todd
 * direction, both Newton systems solved by sdp_inner_solve.  stats may be NULL.
 */
sdp_status sdp_ipm_step(sdp_ctx* ctx, sdp_step_stats* stats);

/*
 * Iterate sdp_ipm_step until the relative gap and the primal and dual
 * infeasibilities are all <= the tolerances.  Returns SDP_ESTALL after
 * max_ipm_iter iterations.  res may be NULL.
 */
sdp_status sdp_solve(sdp_ctx* ctx, sdp_result* res);

typedef struct sdp_adjoint_stats {
    int32_t centring_steps;   /* Newton centring steps that led to the point used */
    int32_t inner_iterations; /* Krylov iterations, centring and gradient solves together */
    int32_t converged;        /* 1 if the gradient solve met inner_tol */
    double centrality;        /* max(||X S / mu - I||_F, pinf, dinf) at that point */
    double mu;                /* the mu of the central-path point aimed at */
} sdp_adjoint_stats;

/*
 * Gradient of a loss L(X) of the solution with respect to the data b and C
 * (the paper does not treat derivatives; this follows from eq. Newt-eps).
 * The Newton KKT operator [dX; dy] -> [-W^{-1} dX W^{-1} + A^T(dy); A(dX)] is
 * self-adjoint and, on the central path, is exactly the linearisation of the
 * path point in the data; so (dL/dC, dL/db) is the Newton direction with
 * C~ = dL/dX, b~ = 0.  The current iterate (normally the output of sdp_solve)
 * is first moved onto the central path at its own mu by pure centring Newton
 * steps, to a distance of 1e-8 or until they stall (at most 12; the closest
 * point is kept and becomes the context's iterate), and the gradient is that
 * of the central-path point, which tends to the solution map's derivative as
 * mu -> 0 when that derivative exists (nondegenerate, strictly complementary
 * problems).  Without a strictly feasible point there is no central path:
 * centring stalls, and when the closest point reached is farther than
 * SDP_ADJOINT_CENTER_TOL from it the call returns SDP_ECENTER (the outputs
 * then hold the Newton-system solution at that point, which is not a
 * derivative of the solution; stats->centrality gives the distance).
 * dL_dX (n x n symmetric, read), dL_db (m, written), dL_dC (n x n symmetric,
 * written): device pointers.  stats may be NULL.  The inner solves use the
 * context's inner precision.  Returns SDP_ENOTCONV if the gradient solve
 * reached inner_maxit (checked before SDP_ECENTER).
 */
sdp_status sdp_adjoint(sdp_ctx* ctx, const double* dL_dX, double* dL_db, double* dL_dC, sdp_adjoint_stats* stats);

/*
 * Pass configuration of the batched solver, chosen per size bucket by
 * sdp_autotune_batched: packed constraint rows each wave streams at once in
 * the A(M) pass (1 to 4), constraints per group when script-A script-Q is
 * formed (1 to 16), and the edge of the output tile each wave computes in the
 * workgroup's MFMA products (16 or 32; 0 selects 32): 16 keeps more of the
 * workgroup's waves busy on small products.
 */
typedef struct sdp_batch_tune {
    int32_t rows_per_wave;
    int32_t aq_group;
    int32_t gemm_tile;
} sdp_batch_tune;

/*
 * Solve `count` independent problems in one persistent launch: each
 * workgroup takes instances from a queue (largest first) and runs the whole
 * interior-point method of sdp_solve (PCG) for one instance at a time.
 * opt->inner_prec SDP_PREC_F64 (default) or SDP_PREC_F32: with FP32 the inner
 * operator reads an FP32 copy of the packed rows in both constraint passes
 * and forms E Y E on the FP32 matrix cores (off-diagonal blocks through the
 * FP64 script-A script-Q), and FP64 refinement sweeps (max_refine, refine_tol
 * with 0 meaning 1e-6) bring each Newton step to inner_tol; results count the
 * FP64 and low-precision operator products.
 * Dense constraint data only (a_kind SDP_A_DENSE), host inputs (on_device 0),
 * n_i <= 128 recommended (every workgroup keeps O(n^2 + m d + d^2) doubles of
 * scratch).  results: count entries (time_ms is the whole launch).  X_out,
 * y_out: NULL or host arrays of `count` device pointers (NULL entries
 * allowed) receiving X_i (n_i x n_i) and y_i (m_i).  tune: NULL (defaults) or
 * `count` configurations.  Uses opt's rank_max, inner_tol, inner_maxit,
 * gap_tol, feas_tol, max_ipm_iter and step_frac; status per instance in
 * results[i].status.
 */
sdp_status sdp_solve_batched(const sdp_problem* probs, int32_t count, const sdp_options* opt, void* hip_stream,
                             sdp_result* results, double* const* X_out, double* const* y_out,
                             const sdp_batch_tune* tune);

/*
 * Autotuner of the batched solver: for each size bucket (n < 48, n < 96,
 * larger) times every candidate configuration on up to 8 of the bucket's
 * instances for two interior-point iterations and writes the fastest to
 * tune_out[i] for every instance; bucket_ms (3 entries, may be NULL) receives
 * the winning times.
 */
sdp_status sdp_autotune_batched(const sdp_problem* probs, int32_t count, const sdp_options* opt, void* hip_stream,
                                sdp_batch_tune* tune_out, double* bucket_ms);

/* Copy the current iterate into device buffers (any may be NULL). */
sdp_status sdp_get_point(sdp_ctx* ctx, double* X, double* y, double* S);

/*
 * Replace the current iterate with device buffers X (n x n), y (m),
 * S (n x n); X and S must be positive definite (checked when the scaling is
 * next computed, SDP_ENUMERIC otherwise).  Resets the iteration counter.
 */
sdp_status sdp_set_point(sdp_ctx* ctx, const double* X, const double* y, const double* S);

/* sdp_get_point with the LP block: x and s (device, l entries each; any may be NULL). */
sdp_status sdp_get_point_lp(sdp_ctx* ctx, double* X, double* y, double* S, double* x, double* s);

/*
 * sdp_set_point with the LP block: x and s (device, l entries each) must be
 * positive (checked when the scaling is next computed, SDP_ENUMERIC otherwise).
 */
sdp_status sdp_set_point_lp(sdp_ctx* ctx, const double* X, const double* y, const double* S, const double* x,
                            const double* s);

/*
 * The eigen-split of the scaling point (eq. EQSigdef) at the current
 * iterate: lam (n, host, decreasing eigenvalues of W), V (n x n, device,
 * eigenvectors with the sign convention above), and the scalars r, tau,
 * beta (host).  Any pointer may be NULL.
 */
sdp_status sdp_get_scaling(sdp_ctx* ctx, double* lam, double* V, int32_t* r, double* tau, double* beta);

/*
 * Kernel classes whose launches can be timed with HIP events.  The two dense
 * constraint passes are timed from the kernel's own start and end timestamps
 * (events handed to the launch); GEMM and NEWTON are bracketed by events
 * recorded on the stream, which adds a few microseconds of dispatch per launch.
 */
enum {
    SDP_K_A_APPLY = 0,   /* A(M): packed dense rows times the weighted packed M */
    SDP_K_AT_APPLY = 1,  /* A^T(u): slab partial column sums of the packed rows */
    SDP_K_GEMM = 2,      /* every FP64 GEMM launch */
    SDP_K_NEWTON = 3,    /* a whole sdp_newton_apply */
    SDP_K_SANDWICH = 4,  /* each n x n x n GEMM of E Y E inside the operator, FP64 or low precision
                            (2 n^3 flops per launch; bytes = its operands and result) */
    SDP_K_SAMPLED_YE = 5,   /* sparse_sandwich: Z = A^T(u) E from the sliced pattern (bytes = E read
                               and Z written once, 10 per pattern slot) */
    SDP_K_SAMPLED_DOTS = 6, /* sparse_sandwich: E[:, j] . Z[:, k] per constraint (algorithmic HBM
                               bytes = E and Z read once each, 16 per constraint for the pair
                               index and the result; the per-constraint re-reads of Z's
                               columns are cache traffic and not counted) */
    SDP_K_SANDWICH_LOWER = 7, /* FP64 operator at large n: the second product of E Y E as its lower
                                 triangle (plus the ragged strip of rows below the last full
                                 128-row block), E Y E being symmetric; n^2 (n + 1) flops and
                                 the entries it writes as bytes.  The first product stays in
                                 SDP_K_SANDWICH */
    SDP_K_COUNT = 8
};

/*
 * Event timing of the kernel classes above: bit k of class_mask enables class
 * k (0 disables all).  Resets the accumulated figures.
 */
sdp_status sdp_profile_enable(sdp_ctx* ctx, int32_t class_mask);

/*
 * Accumulated time (ms), launch count and algorithmic bytes moved for one
 * kernel class since profiling was enabled.  Synchronises the stream.
 */
sdp_status sdp_profile_get(sdp_ctx* ctx, int32_t kernel_class, double* total_ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* WCSDP_H */
