/*
 * amgpoly.h -- C ABI of the MI355X (gfx950) polynomial-smoothed AMG library.
 *
 * Method: D'Ambra, Durastante, Filippone, Massei, Thomas, "Optimal polynomial
 * smoothers for parallel AMG" (arXiv 2407.09848).  The library solves SPD
 * systems A x = b (eq. sys1) with a conjugate-gradient method preconditioned
 * by one multiplicative V-cycle (eq. amg) whose smoother on every level is a
 * polynomial in M^{-1}A, M the l1-Jacobi diagonal (eq. l1smooth):
 *
 *   AMG_L1JAC     plain l1-Jacobi sweeps, p(x) = (1-x)^k
 *   AMG_CHEB4     4th-kind Chebyshev recurrence (eq. polsmoother)
 *   AMG_OPTCHEB4  the same with the optimal weights beta_{j,k} (eq. polsmootheropt)
 *   AMG_OPTCHEB1  1st-kind Chebyshev on [a*_k, 1] (eq. polsmootheropt1kind, Algorithm 1)
 *
 * The spectral scale rho(M^{-1}A) of those recurrences is taken as 1, which
 * the l1-Jacobi M guarantees (Algorithm 1, comments).  The coarse levels are
 * Galerkin products A_{l+1} = P^T A_l P with P piecewise constant on fixed
 * 2x2x2 boxes of the structured grid (Section 2, first display); the
 * coarsest level is solved directly (dense Cholesky, factor formed at setup).
 * Setup options give the ingredients of the paper's own runs (Section 4):
 * boxes of another edge, algebraic aggregates (compatible weighted matching or
 * the classical smoothed aggregation, VBM), the smoothed prolongator and a
 * coarsest solve by a fixed number of l1-Jacobi sweeps.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device (HBM) pointers; pointers named h_* are
 *     host pointers.  Vectors are contiguous, length n_level, float64 unless
 *     stated.  The caller owns every buffer it passes; the library never
 *     frees or retains them past the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Kernels are enqueued on it; calls return once the work is enqueued
 *     unless stated otherwise (setup and pcg_solve synchronise the stream).
 *   - Return value: AMG_OK (0) on success, AMG_NOT_CONVERGED (1) when an
 *     iteration limit was hit (outputs are valid), a negative AMG_E* code on
 *     error (outputs undefined).  amg_strerror() names every code.
 *   - A handle is not thread safe: calls on one handle must not overlap
 *     (they share the handle's workspace).
 */
#ifndef AMGPOLY_H
#define AMGPOLY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define AMG_OK             0
#define AMG_NOT_CONVERGED  1
#define AMG_EINVAL        -1  /* bad argument: null pointer, size, kind, degree, level */
#define AMG_ENOTSPD       -2  /* non-positive diagonal / l1 row sum, or Cholesky pivot <= 0 */
#define AMG_ENOMEM        -3  /* device allocation failed */
#define AMG_EHIP          -4  /* a HIP runtime call failed */
#define AMG_EBREAKDOWN    -5  /* CG breakdown: (p, A p) <= 0 */
#define AMG_ENAN          -6  /* non-finite value in the input or the iteration */
#define AMG_ECAPACITY     -7  /* a product row exceeds the Galerkin kernels' column capacity */

/* ---- smoother kinds ---- */
#define AMG_L1JAC     0
#define AMG_CHEB4     1
#define AMG_OPTCHEB4  2
#define AMG_OPTCHEB1  3

/* ---- hierarchy precision ---- */
#define AMG_FP64  0  /* all levels, smoothers and transfers in float64 */
#define AMG_FP32  1  /* smoothers, transfers and level matrices in float32 with float32
                        accumulation; the coarsest solve, the outer CG residual, its dot
                        products and direction updates stay float64 */

/* ---- aggregation ---- */
#define AMG_AGG_BOX       0  /* fixed boxes of the structured grid (agg_edge) */
#define AMG_AGG_MATCHING  1  /* compatible weighted matching (Section 4), one problem only */
#define AMG_AGG_VBM       2  /* classical smoothed aggregation (Section 4, VBM), one problem only */

/* Highest supported polynomial degree (tabulated constants exist for 1..AMG_MAX_DEGREE). */
#define AMG_MAX_DEGREE 12

typedef struct amg_handle amg_handle;

typedef struct amg_opts {
  int32_t nx, ny, nz;   /* per-problem interior grid extents; row = i + nx*j + nx*ny*k */
  int32_t nbatch;       /* >= 1 problems stacked along z (block-diagonal A); 0 means 1 */
  int32_t max_coarse;   /* coarsen while rows per problem > max_coarse; 0 means 4096 */
  int32_t precision;    /* AMG_FP64 or AMG_FP32 */
  /* The preconditioner ingredients of Section 4 (all zero: 2x2x2 boxes, plain
   * aggregation, dense Cholesky coarsest solve). */
  int32_t agg_edge;      /* box aggregate edge in 2..4; 0 means 2 */
  int32_t smoothed;      /* 1: smoothed prolongator P = (I - omega D^{-1} A) P_hat, D = diag(A),
                            omega = 4 / (3 ||D^{-1} A||_inf) per stacked problem (Section 4) */
  int32_t coarse_sweeps; /* > 0: the coarsest level is solved by this many l1-Jacobi sweeps from
                            zero (at most 1000) instead of the dense Cholesky factorisation */
  int32_t aggregation;   /* AMG_AGG_BOX (0), AMG_AGG_VBM (below) or AMG_AGG_MATCHING: aggregates from match_steps
                            approximate maximum-weight matchings of the graph of A_l, edge weight
                            1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2) for the smooth vector w
                            (ones on level 0, then the coarse one), matched greedily in decreasing
                            weight; a pair forms an aggregate, the tentative prolongator column
                            holds w restricted to it, normalised.  Requires nbatch = 1 and a
                            structurally symmetric A; the grid extents are not used then */
  int32_t match_steps;   /* matching steps per level, 1..3 (aggregates of up to 2^steps rows); 0 means 3 */
  double vbm_theta;      /* AMG_AGG_VBM: strength threshold on level 0, halved on each coarser level
                            (finite, >= 0; 0 makes every nonzero coupling strong).  The edge {i, j}
                            is strong when a_ij != 0 and q_ij >= rint(2^30 theta_l^2), where
                            q_ij = rint(2^30 a_ij^2 / |a_ii a_jj|) with a_ij from the smaller row
                            (the grid keeps couplings that are equal in exact arithmetic equal).
                            Roots: the greedy maximal set of vertices pairwise at
                            least three strong edges apart, in decreasing SplitMix64 order of the
                            index; a root's aggregate is it and its strong neighbours; every other
                            vertex joins the aggregate of its aggregated neighbour of largest q_ij
                            (ties: smaller index); aggregates are numbered by root, the tentative
                            prolongator is piecewise constant (entries 1.0).  Requires nbatch = 1
                            and a structurally symmetric A; the grid extents are not used then */
  int32_t drop_fine_csr; /* 1: keep no CSR form of level 0 (12 bytes per stored entry, read
                            after setup only by amg_level_export and amg_level_features, which
                            then return AMG_EINVAL for it): setup reads the caller's arrays in
                            place (never writing them) instead of copying them.  0 keeps a copy */
} amg_opts;

/* ---------------------------------------------------------------------------
 * Setup (Section 2: Galerkin hierarchy; eq. l1smooth: M_i = a_ii + sum_{j!=i} |a_ij|).
 *
 * A is n x n CSR on the device: d_row_ptr[n+1] (int32, d_row_ptr[0] = 0),
 * d_col[nnz] (int32, strictly increasing within a row), d_val[nnz] float64.
 * n must equal nx*ny*nz*nbatch and A must be symmetric with a positive
 * diagonal (symmetry is the caller's promise; it is not checked).  The
 * library copies what it needs: A may be freed after return.  Builds every
 * level's l1 diagonal, the aggregates, the Galerkin operators, the
 * sliced-ELL copies used by the kernels and the coarsest factor, and
 * allocates all workspace.  Synchronises `stream`.  Coarsening stops at the
 * first level with at most max_coarse rows per problem, or where the
 * aggregation no longer reduces the level.
 * With agg_edge != 2, smoothed != 0 or a graph aggregation the transfers use
 * explicit P and P^T (sliced ELL), built with general sparse products; entries
 * of the smoothed P and of the Galerkin operators whose magnitude is at most
 * 2^-46 times the largest of their row are dropped (exact cancellations up to
 * rounding).
 * Errors: AMG_EINVAL (null, n mismatch, nnz < n, a row_ptr that is not monotone from
 * 0 to nnz, a column index out of range or not increasing in its row, an option out
 * of range, nbatch > 1 with a graph aggregation), AMG_ENOTSPD, AMG_ECAPACITY (a product
 * row with more than 3072 distinct columns), AMG_ENOMEM, AMG_EHIP.  On error *out is NULL.
 * ------------------------------------------------------------------------- */
int amg_setup(int64_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
              const double* d_val, const amg_opts* h_opts, void* stream, amg_handle** out);

/* Release everything the handle owns.  NULL is a no-op.  Returns AMG_OK. */
int amg_destroy(amg_handle* h);

/* Number of levels (fine level 0 .. coarsest L), and the size of level l. */
int amg_num_levels(const amg_handle* h, int* h_nlevels);
int amg_level_info(const amg_handle* h, int level, int64_t* h_n, int64_t* h_nnz);

/* Storage of level l's operator in the kernels' sliced-ELL format (host outputs, any may be
 * NULL): *h_padded stored entries including padding, *h_lanes lanes per row (1, 4, 16 or
 * 64), *h_aligned 1 when its slices are offset-aligned (columns formed as row + a per-slice
 * offset, no column indices read), else 0. */
int amg_level_layout(const amg_handle* h, int level, int64_t* h_padded, int* h_lanes, int* h_aligned);

/* How the restriction from level l to level l + 1 is computed (host outputs, any may be NULL;
 * AMG_EINVAL on the coarsest level): *h_form = AMG_TRANSFER_RESIDUAL (2x2x2 boxes: the fine
 * residual b - A x, then the sum over each aggregate's rows), AMG_TRANSFER_PRODUCT (2x2x2 boxes:
 * b_c = P^T b - R x with the restriction product R = P^T A, the Galerkin construction's first
 * factor of Section 2, stored in offset-aligned slices with offsets taken against each
 * aggregate's first row; no fine residual is formed) or AMG_TRANSFER_EXPLICIT (smoothed or
 * other prolongators: P^T as a sparse matrix).  *h_stored: stored entries of R or P^T
 * including padding, 0 for the residual form. */
#define AMG_TRANSFER_RESIDUAL 0
#define AMG_TRANSFER_PRODUCT 1
#define AMG_TRANSFER_EXPLICIT 2
int amg_level_transfer(const amg_handle* h, int level, int* h_form, int64_t* h_stored);

/* Copy level l's Galerkin operator (CSR, sorted columns) and its l1 inverse
 * diagonal 1/M_i into caller buffers: d_row_ptr[n+1], d_col[nnz], d_val[nnz],
 * d_minv[n] (float64).  Any pointer may be NULL to skip it.  Asynchronous.
 * AMG_EINVAL for a level out of range, or for CSR outputs of level 0 when the handle was
 * set up with drop_fine_csr = 1 (d_minv alone is still served). */
int amg_level_export(const amg_handle* h, int level, int32_t* d_row_ptr, int32_t* d_col,
                     double* d_val, double* d_minv, void* stream);

/* Copy the aggregate index of every row of level l (0 <= l < number of levels - 1) into
 * d_agg[n_l] (int32): the coarse row of level l+1 that the row's tentative prolongator
 * column belongs to (box, VBM or, for compatible matching, the composite of the matching
 * steps).  Asynchronous.  AMG_EINVAL for the coarsest level or a null pointer. */
int amg_level_aggregates(const amg_handle* h, int level, int32_t* d_agg, void* stream);

/* ---------------------------------------------------------------------------
 * Polynomial coefficients (Section 2.1, eq. polsmootheropt; Section 2.3, eq. optimalparameter).
 * The tables are computed offline and compiled in (the paper tabulates them too).
 * ------------------------------------------------------------------------- */
/* Default optimal 4th-kind weights beta_{1..k,k} into h_beta[k]. */
int amg_default_beta(int degree, double* h_beta);
/* Default left end a*_k of the optimal 1st-kind interval. */
int amg_default_astar(int degree, double* h_a);
/* Override the beta_{1..k} used by AMG_OPTCHEB4 at `degree` on one level
 * (level = -1: all levels).  h_beta has `degree` finite entries; copied.
 * p(0) = 1 holds for any beta (the weights only move the polynomial within Pi_k). */
int amg_set_beta(amg_handle* h, int degree, int level, const double* h_beta);
/* Restore the default table on every level. */
int amg_reset_beta(amg_handle* h);

/* ---------------------------------------------------------------------------
 * Kernel-level operations on one level (the steps the V-cycle is built from).
 * All asynchronous on `stream`; d_* vectors have the level's length unless stated.
 * ------------------------------------------------------------------------- */
/* y = A_l x (SpMV; the matrix-vector product every recurrence step is built on). */
int amg_spmv(amg_handle* h, int level, const double* d_x, double* d_y, void* stream);

/* Apply the degree-k smoother of `kind` on level l once (Sections 2.1-2.2,
 * Algorithm 1): x <- x + p_k-correction, i.e. on exit x - A^{-1}b = p_k(M^{-1}A)(x_in - A^{-1}b).
 * x_is_zero != 0 declares x_in = 0 (x is then write-only and r^(0) = b needs
 * no SpMV).  d_b is read only.  1 <= degree <= AMG_MAX_DEGREE. */
int smoother_apply(amg_handle* h, int level, int kind, int degree, const double* d_b,
                   double* d_x, int x_is_zero, void* stream);

/* smoother_apply in the FP32 hierarchy (amg_opts.precision = AMG_FP32): the same recurrence on
 * the level's float32 matrix and l1 diagonal with float32 accumulation (the smoother the FP32
 * V-cycle applies), on float32 vectors d_b, d_x.  smoother_apply on such a handle runs the
 * float64 copy of the level.  AMG_EINVAL also for a float64 handle. */
int smoother_apply_f32(amg_handle* h, int level, int kind, int degree, const float* d_b, float* d_x,
                       int x_is_zero, void* stream);

/* b_c = P_l^T (b - A_l x): the restriction of the residual to level l+1 (Section 2, eq. amg),
 * computed as P_l^T b - (P_l^T A_l) x on box levels with a restriction product
 * (amg_level_transfer), else from the residual.  d_b, d_x have n_l entries, d_bc has n_{l+1}.
 * Asynchronous; AMG_EINVAL for a null pointer or the coarsest level. */
int amg_restrict_residual(amg_handle* h, int level, const double* d_b, const double* d_x,
                          double* d_bc, void* stream);

/* x += P_l x_c: prolongation of the level-(l+1) correction and addition. */
int amg_prolong_add(amg_handle* h, int level, const double* d_xc, double* d_x, void* stream);

/* x = A_L^{-1} b on the coarsest level (direct solve with the setup's Cholesky factor). */
int amg_coarse_solve(amg_handle* h, const double* d_b, double* d_x, void* stream);

/* ---------------------------------------------------------------------------
 * V-cycle (eq. amg): z = B r with pre- and post-smoothing by the same degree-k
 * polynomial of `kind` on every level (Section 2: p^l = p_k for all l), so B
 * is symmetric.  d_r and d_z have n_0 entries; d_r is not modified; d_z is
 * overwritten.  In AMG_FP32 handles the cycle runs in float32 between a
 * rounding of r on entry and a widening of z on exit.
 * ------------------------------------------------------------------------- */
int vcycle_apply(amg_handle* h, int kind, int degree, const double* d_r, double* d_z, void* stream);

/* ---------------------------------------------------------------------------
 * Preconditioned CG (Section 4 uses a CG variant with one global reduction).
 * x0 is taken from d_x (x_is_zero != 0 declares it zero).  Stops at the first
 * iteration k with ||r_k||_2 <= rtol ||b||_2, r_k the recursively updated
 * residual, or after maxit iterations.  flexible != 0 uses the Polak-Ribiere
 * beta (robust to a preconditioner that is not exactly fixed, e.g. the FP32
 * V-cycle).  Outputs (host): *h_iters, *h_relres = ||r_k||/||b||, and when
 * h_hist is not NULL the relative residual history h_hist[0..iters] (length
 * >= maxit+1).  Synchronises `stream`.  ||b|| = 0 returns x = 0, iters = 0.
 * Returns AMG_OK, AMG_NOT_CONVERGED, AMG_EBREAKDOWN, AMG_ENAN or an argument error.
 * On AMG_EBREAKDOWN ((p, A p) <= 0: A, or the preconditioner, is not positive
 * definite) the step along p is not taken: x and *h_relres are those of the
 * last iterate before the breakdown, *h_iters counts the failed iteration.
 * ------------------------------------------------------------------------- */
int pcg_solve(amg_handle* h, int kind, int degree, const double* d_b, double* d_x, int x_is_zero,
              double rtol, int maxit, int flexible, int* h_iters, double* h_relres,
              double* h_hist, void* stream);

/* ---------------------------------------------------------------------------
 * Preconditioned CG with the level-0 smoother alone as the preconditioner:
 * z = p_k(M^{-1}A) M^{-1} r, the degree-k `kind` polynomial of l1-Jacobi run
 * from z = 0 (the polynomial preconditioning of the remark after
 * Fig. boundcomparison, Fig. better-than-optimal).  No coarse correction is
 * applied, so the hierarchy below level 0 is unused (a single-level handle,
 * n <= max_coarse, is the natural setup).  The smoother always runs in
 * float64, also in AMG_FP32 handles.  Arguments, outputs, synchronisation and
 * return codes are those of pcg_solve.
 * ------------------------------------------------------------------------- */
int pcg_solve_smoother(amg_handle* h, int kind, int degree, const double* d_b, double* d_x,
                       int x_is_zero, double rtol, int maxit, int flexible, int* h_iters,
                       double* h_relres, double* h_hist, void* stream);

/* ---------------------------------------------------------------------------
 * Differentiable V-cycle and the learned optimal-4th-kind weights.
 *
 * Weight table layout (device, float64): d_beta[(p * nlevels + l) * degree + j - 1]
 * is beta_j of the degree-`degree` optimal 4th-kind smoother (eq. polsmootheropt)
 * used for stacked problem p on level l (pre- and post-smoothing alike).
 * These calls always use the optimal 4th kind.  Vectors are float64 at the
 * boundary; the cycle runs in the handle's precision.
 * ------------------------------------------------------------------------- */
/* Bytes of checkpoint storage one differentiable V-cycle needs (caller allocates it). */
int amg_ckpt_bytes(const amg_handle* h, int64_t* h_bytes);

/* z = B(beta) r (the V-cycle of eq. amg with per-problem, per-level weights), saving
 * each level's smoother inputs (the level right-hand side and the post-smoothing
 * residual) into d_ckpt.  d_r is read only. */
int vcycle_fwd_ckpt(amg_handle* h, int degree, const double* d_beta, const double* d_r, double* d_z,
                    void* d_ckpt, void* stream);

/* Adjoint of vcycle_fwd_ckpt: given d_gz = dL/dz, writes d_gr = dL/dr (= B(beta) d_gz, the
 * V-cycle being symmetric) and ADDS dL/dbeta into d_gbeta (layout of d_beta).  Each
 * smoother's correction is a symmetric operator in M^{-1}A, so its adjoint is the same
 * recurrence run on the incoming adjoint; dL/dbeta_j is the dot product of that run's
 * j-th direction with the checkpointed recurrence input.  The SpMV is reused (A = A^T). */
int vcycle_bwd(amg_handle* h, int degree, const double* d_beta, const void* d_ckpt, const double* d_gz,
               double* d_gr, double* d_gbeta, void* stream);

/* Residual-reduction loss of two V-cycle iterations from x = 0 on d_b:
 *   r_0 = b, r_1 = r_0 - A B r_0, r_2 = r_1 - A B r_1,
 *   loss = mean over stacked problems p of ||r_2,p|| / ||r_0,p||,
 * its gradient d_gbeta = d loss / d beta (overwritten), and h_loss[0] = loss,
 * h_loss[1 + p] = ratio of problem p (host, nbatch + 1 entries).  Synchronises. */
int amg_train_loss_grad(amg_handle* h, int degree, const double* d_beta, const double* d_b, double* h_loss,
                        double* d_gbeta, void* stream);

/* Eight features per (stacked problem p, smoothing level l < nlevels-1), row (p * (nlevels-1) + l)
 * of d_feat (float32): degree/6, l/(nlevels-1), 1 - lambda_max(M^{-1}A_l) estimated by 20
 * power iterations from the ones vector (the margin below the l1-Jacobi bound rho <= 1),
 * (nnz_l/n_l)/27, log2(rows per problem)/24, h_sigma[p], n_{l+1}/n_l, and the mean over
 * rows of sum_{j!=i}|a_ij| / a_ii.  Synchronises.  AMG_EINVAL for a single-level handle or
 * one set up with drop_fine_csr = 1. */
int amg_level_features(amg_handle* h, int degree, const double* h_sigma, float* d_feat, void* stream);

/* MLP 8 -> 64 -> 64 -> 6 (tanh hidden units, output scaled by 0.1), float32.
 * Parameters d_params[mlp_num_params()] = W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6].
 * mlp_fwd: d_y[batch][6] from d_x[batch][8]; d_cache[batch][128] keeps the hidden activations.
 * mlp_bwd: d_gparams = d(sum of d_gy . y)/d params (overwritten); d_work[2 * batch * 64].
 * mlp_adam: one bias-corrected Adam step (step >= 1) on d_params.  1 <= batch <= 256. */
int mlp_num_params(void);
int mlp_fwd(const float* d_params, const float* d_x, int batch, float* d_y, float* d_cache, void* stream);
int mlp_bwd(const float* d_params, const float* d_x, int batch, const float* d_cache, const float* d_gy,
            float* d_gparams, float* d_work, void* stream);
int mlp_adam(float* d_params, const float* d_g, float* d_m, float* d_v, int n, int step, float lr, float b1,
             float b2, float eps, void* stream);

/* mlp_bwd for callers that cannot allocate device memory (code under HIP graph capture, serving
 * or training loops that forbid allocation): the same gradients, bitwise, with no workspace
 * argument.  Its scratch (2 * batch * 64 floats) is a static array inside the library, one per
 * GPU (128 KB, held until the process ends); the call allocates and frees nothing.  Limit:
 * 1 <= batch <= 256 (AMG_ECAPACITY above, AMG_EINVAL for batch < 1 or a null pointer).  Calls
 * on one GPU share its array, so calls that overlap in time on one GPU (other streams, other
 * host threads) race and must be ordered by the caller.  Asynchronous on `stream`. */
int mlp_bwd_noalloc(const float* d_params, const float* d_x, int batch, const float* d_cache, const float* d_gy,
                    float* d_gparams, void* stream);

/* d_valid[q] = 1 when the weighted 4th-kind polynomial of row q of d_beta (count rows of
 * `degree` weights) stays inside Pi_k (eq. polspace): |p(x)| < 1 at x = m/ngrid, m = 1..ngrid
 * (p(0) = 1 holds for any weights); else 0.  Used to fall back to the tabulated weights. */
int amg_beta_valid(const double* d_beta, int count, int degree, int ngrid, int* d_valid, void* stream);

/* Learned weights on the device (eq. polsmootheropt with corrected beta, kept inside Pi_k of
 * eq. polspace).  d_y[(p * (nlevels - 1) + l) * 6 + j] is the network output (mlp_fwd) for
 * stacked problem p and smoothing level l; only its first `degree` columns are used
 * (1 <= degree <= 6).  Writes the weight table d_beta (layout of vcycle_fwd_ckpt, all
 * nbatch * nlevels rows):
 *   beta[p][l][j] = beta_opt_{j,k} + (double)y[p, l][j]   on the smoothing levels l < nlevels - 1,
 *   beta[p][nlevels-1][j] = beta_opt_{j,k}                on the coarsest level (not smoothed),
 * beta_opt the compiled-in optimal table.  A smoothing row whose polynomial leaves Pi_k
 * (|p(x)| >= 1 at some x = m/ngrid, m = 1..ngrid, as amg_beta_valid) falls back to beta_opt;
 * d_valid[p * (nlevels - 1) + l] = 1 for a kept row, 0 for a fallback.  d_y = NULL writes the
 * plain table (every row valid).  Asynchronous.  AMG_EINVAL: null handle or outputs, degree
 * outside 1..6, ngrid < 1, a handle with a single level. */
int amg_learned_beta(const amg_handle* h, int degree, const float* d_y, int ngrid, double* d_beta, int* d_valid,
                     void* stream);

/* Gradient hand-over from the weights to the network output: d_gy[q][j] (float32, q = p *
 * (nlevels - 1) + l, 6 columns) = dL/dbeta[p][l][j] (d_gbeta, layout of d_beta) for j < degree
 * on the rows amg_learned_beta kept (d_valid[q] = 1), and 0 elsewhere (fallback rows and the
 * unused columns), since a fallback row does not depend on y.  Asynchronous.  AMG_EINVAL as
 * amg_learned_beta. */
int amg_learned_beta_grad(const amg_handle* h, int degree, const double* d_gbeta, const int* d_valid, float* d_gy,
                          void* stream);

/* ---------------------------------------------------------------------------
 * Bandwidth ceiling of the device memory: kernels with known byte counts that
 * the smoother kernels are measured against (16-byte nontemporal accesses,
 * AMG_HBM_PARTIALS blocks of 256 threads, grid-stride).  d_x, d_y 16-byte aligned.
 * ------------------------------------------------------------------------- */
#define AMG_HBM_PARTIALS 16384
/* Reads d_x[n] once (8 n bytes): d_partial[AMG_HBM_PARTIALS] receives block sums whose total
 * is sum_i x_i (rounding order fixed by the grid).  Asynchronous.  d_x must be 16-byte aligned;
 * it may be NULL when n = 0 (the block sums are then zeros).  AMG_EINVAL otherwise. */
int amg_hbm_read(const double* d_x, int64_t n, double* d_partial, void* stream);
/* d_y[i] = d_x[i], i < n (8 n bytes read, 8 n written); the ranges must not overlap and both
 * must be 16-byte aligned (AMG_EINVAL otherwise).  n = 0 does nothing.  Asynchronous. */
int amg_hbm_copy(const double* d_x, double* d_y, int64_t n, void* stream);

/* Human-readable name of a return code (static storage). */
const char* amg_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* AMGPOLY_H */
