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
#define AMG_ECAPACITY     -7  /* a coarse row exceeds the Galerkin kernel's column capacity */

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

/* Highest supported polynomial degree (tabulated constants exist for 1..AMG_MAX_DEGREE). */
#define AMG_MAX_DEGREE 12

typedef struct amg_handle amg_handle;

typedef struct amg_opts {
  int32_t nx, ny, nz;   /* per-problem interior grid extents; row = i + nx*j + nx*ny*k */
  int32_t nbatch;       /* >= 1 problems stacked along z (block-diagonal A); 0 means 1 */
  int32_t max_coarse;   /* coarsen while rows per problem > max_coarse; 0 means 4096 */
  int32_t precision;    /* AMG_FP64 or AMG_FP32 */
} amg_opts;

/* ---------------------------------------------------------------------------
 * Setup (Section 2: Galerkin hierarchy; eq. l1smooth: M_i = a_ii + sum_{j!=i} |a_ij|).
 *
 * A is n x n CSR on the device: d_row_ptr[n+1] (int32, d_row_ptr[0] = 0),
 * d_col[nnz] (int32, strictly increasing within a row), d_val[nnz] float64.
 * n must equal nx*ny*nz*nbatch and A must be symmetric with a positive
 * diagonal (symmetry is the caller's promise; it is not checked).  The
 * library copies what it needs: A may be freed after return.  Builds every
 * level's l1 diagonal, the box aggregates, the Galerkin operators, the
 * sliced-ELL copies used by the kernels and the coarsest factor, and
 * allocates all workspace.  Synchronises `stream`.
 * Errors: AMG_EINVAL (null, n mismatch, nnz < n, a row_ptr that is not monotone from
 * 0 to nnz, a column index out of range or not increasing in its row), AMG_ENOTSPD, AMG_ECAPACITY,
 * AMG_ENOMEM, AMG_EHIP.  On error *out is NULL.
 * ------------------------------------------------------------------------- */
int amg_setup(int64_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
              const double* d_val, const amg_opts* h_opts, void* stream, amg_handle** out);

/* Release everything the handle owns.  NULL is a no-op.  Returns AMG_OK. */
int amg_destroy(amg_handle* h);

/* Number of levels (fine level 0 .. coarsest L), and the size of level l. */
int amg_num_levels(const amg_handle* h, int* h_nlevels);
int amg_level_info(const amg_handle* h, int level, int64_t* h_n, int64_t* h_nnz);

/* Copy level l's Galerkin operator (CSR, sorted columns) and its l1 inverse
 * diagonal 1/M_i into caller buffers: d_row_ptr[n+1], d_col[nnz], d_val[nnz],
 * d_minv[n] (float64).  Any pointer may be NULL to skip it.  Asynchronous. */
int amg_level_export(const amg_handle* h, int level, int32_t* d_row_ptr, int32_t* d_col,
                     double* d_val, double* d_minv, void* stream);

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

/* b_c = P_l^T (b - A_l x): fused residual and restriction to level l+1 (Section 2, eq. amg).
 * d_b, d_x have n_l entries, d_bc has n_{l+1}. */
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
 * ------------------------------------------------------------------------- */
int pcg_solve(amg_handle* h, int kind, int degree, const double* d_b, double* d_x, int x_is_zero,
              double rtol, int maxit, int flexible, int* h_iters, double* h_relres,
              double* h_hist, void* stream);

/* Human-readable name of a return code (static storage). */
const char* amg_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* AMGPOLY_H */
