/*
 * proxsdp.h -- C interface of a GPU (MI355X, gfx950) implementation of the
 * primal-dual hybrid gradient method for general semidefinite programs with
 * approximate (truncated, adaptive-rank) projection onto the PSD cone.
 *
 * Method: Souto, Garcia, Veiga, "Exploiting Low-Rank Structure in
 * Semidefinite Programming by Approximate Operator Splitting"
 * (arXiv 1810.05231):
 *   problem          Section 1.3, general SDP form:
 *                      minimize tr(C X)  s.t.  A(X) = b, G(X) <= h, X PSD
 *   dual             Section 1.3 (dual problem; inequality duals <= 0)
 *   iteration        Section 2.2 fixed-point iteration, Algorithm 1 (PD-SDP)
 *   residuals        Section 2.2 (primal, dual, combined residual)
 *   aproj            Section 3.1, truncated eigen-projection (eq_trunc_eig)
 *   rank control     Section 3.2, Algorithm 2 (LR-PD-SDP)
 *
 * Conventions shared by every call:
 *  - All functions return an int: PROXSDP_OK (0) or a negative error code.
 *    proxsdp_last_error() returns a thread-local message for the last error.
 *  - Symmetric matrices are passed by their upper triangle (i <= j) as
 *    0-based COO triplets.  An off-diagonal triplet v at (i, j) stands for v
 *    at (i, j) and at (j, i), so it contributes 2 v X_ij to tr(A X).
 *    Duplicated triplets are summed.  A triplet with i > j, an index out of
 *    range or a non-finite value is rejected with PROXSDP_ERR_INVALID.
 *  - Constraint rows 0..m-1 are equalities A(X) = b, rows m..m+p-1 are
 *    inequalities G(X) <= h.  A row is the sum of its triplets and of its
 *    rank-one terms sigma * u u^T.
 *  - The dual vector y has the sign of the Section 1.3 dual problem:
 *    inequality duals are <= 0 and the dual constraint reads
 *    C - sum_i y_i M_i PSD.  (Algorithm 1's y is the negative of this y.)
 *  - Host arrays passed to a call are read during the call and copied; the
 *    caller may free them on return.
 *  - Device memory is the caller's: every call that needs device memory
 *    takes a workspace pointer and size.  The library never frees the
 *    caller's memory and allocates no device memory itself, with one
 *    exception: the exact projection for n > 64 (proxsdp_project_psd, r = 0)
 *    creates one rocBLAS handle per process on first use, which holds a small
 *    allocation of its own (its work buffers come from the workspace).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Work
 *    is enqueued on it; calls that return host results synchronise it.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef PROXSDP_H
#define PROXSDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ codes */
#define PROXSDP_OK 0
#define PROXSDP_ERR_INVALID (-1)       /* bad argument or problem data        */
#define PROXSDP_ERR_WORKSPACE (-2)     /* workspace NULL, misaligned or small */
#define PROXSDP_ERR_HIP (-3)           /* a HIP runtime call failed           */
#define PROXSDP_ERR_UNSUPPORTED (-4)   /* valid input outside supported sizes */

/* solver status (proxsdp_info.status) */
#define PROXSDP_STATUS_RUNNING 0       /* step() returned before a stop      */
#define PROXSDP_STATUS_CONVERGED 1     /* residual and rank tests passed     */
#define PROXSDP_STATUS_MAX_ITERS 2
#define PROXSDP_STATUS_TIME_LIMIT 3
#define PROXSDP_STATUS_NUMERICAL 4     /* NaN/Inf in the iterate             */
/* The residual test passed but convergence could not be decided: either
 * Algorithm 2's rank test stayed undecided at the rank cap (after the
 * confirmation rounds of the partial eigensolve the tested Ritz value lies
 * below the rank-test threshold while its upper estimate, Ritz value plus
 * the norm of its Ritz residual, lies above it, and the r <- 2r step that an
 * undecided test calls for cannot be taken), or the exact-step check could
 * not converge its eigensolve within 1000 rounds three times.  The iterate is returned
 * as it is; it is not certified optimal. */
#define PROXSDP_STATUS_EIG_NOT_CONVERGED 5
/* The residual test passed, the rank test failed and r is at its cap
 * (r_max < n, or the automatic cap of the partial path), so Algorithm 2's
 * r <- 2r cannot be taken.  The iterate is Algorithm 2's intermediate
 * feasible solution X_[r] (Section 3.2), not an optimum of the SDP. */
#define PROXSDP_STATUS_RANK_LIMIT 6

/* Quantity in Algorithm 2's rank test (n - r) max(lambda, 0) <= eps_lambda */
#define PROXSDP_RANK_TEST_LAMBDA_R 0        /* lambda_r, as Algorithm 2 states it  */
#define PROXSDP_RANK_TEST_LAMBDA_R_PLUS_1 1 /* lambda_{r+1}, the first excluded
                                               eigenvalue, which the Section 3.1
                                               error bound of aproj is about      */

/* storage / arithmetic of the dense n x n iterate and its block products */
#define PROXSDP_FP64 0
#define PROXSDP_FP32 1
#define PROXSDP_BF16 2
/* No dense iterate at all: every pass of the partial eigensolve applies
 * W = X - alpha (C - M*(y)) exactly in FP64 through its structure,
 * W B = V (Lambda (V^T B)) + D B + sum_q gamma_q u_q (u_q^T B), with X =
 * V diag(Lambda) V^T the factors of the current iterate, D = -alpha C +
 * alpha M*(y) on the sparsity pattern of C and the constraint rows, and the
 * rank-one constraint terms.  O(n (r + k) k + nnz k) per pass instead of the
 * n^2 of a dense pass, and no n x n buffer; the iterates are those of
 * PROXSDP_FP64 up to rounding order.  For sparse / low-rank data (a C or
 * constraint rows with O(n^2) triplets cost as much as a dense pass). */
#define PROXSDP_IMPLICIT 3

/* --------------------------------------------------------- problem */
/* General SDP form, Section 1.3.  All pointers are host pointers. */
typedef struct {
  int32_t n;            /* X is n x n symmetric, n >= 1                       */
  int32_t m;            /* number of equality rows (A(X) = b)                 */
  int32_t p;            /* number of inequality rows (G(X) <= h)              */
  int64_t nnz_c;        /* C as upper-triangle triplets                        */
  const int32_t *c_i, *c_j;
  const double *c_v;
  int64_t nnz_a;        /* constraint triplets; a_row in [0, m + p)           */
  const int32_t *a_row, *a_i, *a_j;
  const double *a_v;
  int32_t n_r1;         /* rank-one terms sigma_t u_t u_t^T added to row r1_row[t] */
  const int32_t *r1_row;
  const double *r1_sigma;
  const double *r1_u;   /* n_r1 x n, row-major                                 */
  const double *b;      /* m values                                            */
  const double *h;      /* p values                                            */
} proxsdp_problem;

/* ----------------------------------------------------------- options */
typedef struct {
  double tol;           /* stop when max(rho_p, rho_d) <= tol (default 1e-4); rho as
                           in proxsdp_info                                      */
  double eps_lambda;    /* rank test (n - r) max(lambda_r, 0) <= eps_lambda of
                           Algorithm 2; < 0 means eps_lambda = tol (default -1) */
  double alpha;         /* step size; 0 = 0.95 / ||M||_2 of the row-scaled operator
                           (Section 2.2 requires 0 < alpha < 1/||M||_2)         */
  int32_t window;       /* l of Algorithm 2's windowed residual test (default 50);
                           must be a multiple of check_every                     */
  int32_t check_every;  /* iterations between host-side control checks (10)     */
  int32_t r0;           /* initial target rank (default 1, Algorithm 2)          */
  int32_t r_max;        /* largest target rank (0 = automatic: n on the exact path,
                           otherwise 64 with the lambda_r test and 48 with the
                           lambda_{r+1} test, which needs one more Ritz value
                           than r inside the 64-wide subspace)                   */
  int32_t full_eig;     /* 1 = PD-SDP (Algorithm 1, exact projection; n <= 64)   */
  int32_t precision;    /* storage of the dense iterate W: PROXSDP_FP64 (default,
                           plain form), PROXSDP_FP32 or PROXSDP_BF16 (precision
                           form: Chebyshev filter passes over the low-precision W
                           on FP32 / BF16 MFMA; every Rayleigh-Ritz pass applies W
                           exactly in FP64 from the factors of X, the sparse part
                           and the rank-one terms; factors, Rayleigh-Ritz,
                           residuals and the dual step stay FP64), or
                           PROXSDP_IMPLICIT (no dense W, every pass through the
                           factors in FP64).  The exact small-n path (n <= 64 or
                           full_eig) always uses a dense FP64 W.                 */
  int32_t max_iters;    /* default 200000                                        */
  double time_limit_s;  /* default 1200 (the paper's cap); <= 0 = none           */
  int32_t row_scaling;  /* 1 (default): rows scaled to unit Frobenius norm        */
  int32_t block;        /* subspace width k (0 = automatic, multiple of 16, <= 64);
                           a fixed width also caps r at k (k - 1 with the
                           lambda_{r+1} rank test)                               */
  double eig_tol;       /* relative Ritz residual target of the partial
                           eigensolve, floor of the adaptive schedule (1e-10)    */
  int32_t max_passes;   /* max dense passes per iteration (default 8)             */
  int32_t seed;         /* seed of the initial random subspace (default 1)        */
  int32_t eig_strict;   /* 1: every iteration repeats eigensolver rounds until the
                           kept Ritz pairs meet eig_tol (synchronises per round;
                           for verification), 0 (default): adaptive schedule    */
  double eig_rel;       /* adaptive schedule: the absolute Ritz residual of the
                           kept pairs is held below max(eig_tol * max|theta|,
                           eig_rel * alpha * eps_p), a fraction of the current
                           primal step (default 0.2)                              */
  int32_t graphs;       /* 1: rounds of check_every iterations are captured once
                           per configuration (rank, width, passes, ...) into HIP
                           graphs and replayed (fewer launches; serving); needs
                           a stream other than the null stream.  0 (default):
                           every kernel is launched directly                    */
  int32_t rank_test;    /* PROXSDP_RANK_TEST_LAMBDA_R (default, Algorithm 2) or
                           PROXSDP_RANK_TEST_LAMBDA_R_PLUS_1.  On the partial
                           path a passing test is confirmed on a converged
                           subspace and must hold for the upper estimate
                           theta + ||W u - theta u|| of the tested Ritz pair   */
} proxsdp_options;

/* ------------------------------------------------------------- info */
typedef struct {
  int32_t status;       /* PROXSDP_STATUS_*                                       */
  int32_t iters;        /* PDHG iterations done since create                      */
  int32_t r;            /* current target rank                                    */
  int32_t k;            /* current subspace width                                  */
  int32_t rank_updates; /* number of r <- 2r updates so far                       */
  int32_t passes;       /* total dense passes over the n x n iterate               */
  double lambda_r;      /* r-th largest eigenvalue of the last projected matrix   */
  double lambda_r1;     /* (r+1)-th (first excluded) Ritz value, or NaN            */
  double eps_p, eps_d;  /* Section 2.2 residuals of the last iteration (scaled rows) */
  double rho_p, rho_d;  /* eps_p / (1 + ||C||_F), eps_d / (1 + ||[b; h]||_2)       */
  double obj;           /* tr(C X) at the last check                               */
  double dual_obj;      /* b^T y_eq + h^T y_ineq at the last check                 */
  double alpha;         /* step size in use                                        */
  double norm_M;        /* ||M||_2 of the (scaled) operator                        */
  double ritz_res;      /* largest relative Ritz residual of the kept pairs        */
  double time_s;        /* wall time inside step/solve since create                */
  double gap;           /* |obj - dual_obj| / (1 + |obj| + |dual_obj|) at the last check */
  double rank_value;    /* value of the last rank test decided on a confirmed
                           subspace: upper estimate of lambda_r (or lambda_{r+1}),
                           NaN if none was taken                                  */
  int32_t saved;        /* number of intermediate solutions X_[r] kept so far      */
  int32_t verify_steps; /* exact-step convergence checks taken: once the residual
                           and rank tests pass on the partial path with the
                           adaptive eigensolve accuracy, one more iteration runs
                           with eigensolver rounds until the error bound of its
                           projection, sqrt(sum over the kept pairs of
                           min(||W v - theta v||, theta)^2), is below
                           0.1 alpha tol min(1 + ||C||_F, (1 + ||[b; h]||) / 0.95),
                           a tenth of what the stopping rule allows either
                           residual (at most 1000 rounds; after three
                           checks that cannot get there the solve stops with
                           EIG_NOT_CONVERGED), and the solve stops only if that
                           exact step's residuals meet tol.  Otherwise the iteration
                           continues: with the exact residual q times the
                           reported one, the next check waits for reported
                           residuals below tol / (1.02 q), and eig_rel is
                           scaled by 0.1 / (q - 1) (floor 1e-3) if q > 1.1      */
} proxsdp_info;

typedef struct proxsdp_handle proxsdp_handle;

/* Fills *opt with the defaults listed above. */
int proxsdp_default_options(proxsdp_options *opt);

/* Device workspace (bytes) that proxsdp_create needs for this problem and these
 * options.  Validates the problem (same checks as create); host-only, makes
 * no HIP call. */
int proxsdp_workspace_size(const proxsdp_problem *prob, const proxsdp_options *opt,
                           size_t *bytes);

/* Builds a solver: validates and preprocesses the data (duplicate summing,
 * row scaling, sparsity pattern, ||M||_2 and alpha), uploads it into
 * d_workspace (device memory of at least proxsdp_workspace_size bytes,
 * 256-byte aligned) and sets X0 = 0, y0 = 0.  The workspace must stay valid
 * and untouched until proxsdp_destroy.  Enqueues on `stream` and
 * synchronises it before returning.  Besides the caller's device workspace
 * the handle owns a pinned host buffer of check_every + 1 iteration records
 * (the control checks' copy target), freed by proxsdp_destroy. */
int proxsdp_create(const proxsdp_problem *prob, const proxsdp_options *opt, void *d_workspace,
                   size_t ws_bytes, void *stream, proxsdp_handle **out);

/* Runs up to n_iters PDHG iterations (Algorithm 2's inner loop, with its rank
 * control every check_every iterations) and stops early on a terminal
 * status.  If info != NULL the stream is synchronised and *info filled. */
int proxsdp_step(proxsdp_handle *h, int32_t n_iters, proxsdp_info *info);

/* Iterates until a terminal status (converged, iteration or time limit,
 * numerical failure); fills *info (may be NULL).  Synchronises. */
int proxsdp_solve(proxsdp_handle *h, proxsdp_info *info);

/* Serving form: advances every running handle in hs[0 .. count) by up to
 * n_iters PDHG iterations.  Handles progress independently: each one's next
 * round (up to its next control check) is launched on its own stream as soon
 * as its previous round has finished and been checked, so solves of different
 * sizes overlap on the device and none waits for a slower one.  With flags &
 * PROXSDP_STEP_UNTIL_ANY_STOPS the call returns once any handle stops
 * (converged, limits), after the rounds in flight have finished; handles that
 * did not finish their n_iters continue in the next call.  Handles on the same
 * stream are valid but run one after the other, and so do streams that HIP
 * maps onto the same hardware queue (GPU_MAX_HW_QUEUES, 4 unless set before
 * HIP initialises; measured best at one queue per stream, 16 streams).  infos (host array of count
 * entries, nullable) receives each handle's state.  Synchronises every stream
 * before returning.  Errors: PROXSDP_ERR_INVALID for a NULL entry or
 * n_iters < 0. */
#define PROXSDP_STEP_UNTIL_ANY_STOPS 1
int proxsdp_step_many(proxsdp_handle **hs, int32_t count, int32_t n_iters, int32_t flags,
                      proxsdp_info *infos);

/* Current iterate: X (n x n, row-major, formed from the rank-r factors) and
 * the dual y (m + p values, unscaled, Section 1.3 sign).  Either pointer may
 * be NULL.  on_device = 0: host pointers; 1: device pointers.  Synchronises. */
int proxsdp_get_solution(proxsdp_handle *h, double *X, double *y, int32_t on_device);

/* Current factors X = V diag(lambda) V^T: V is n x r row-major (lds = r),
 * lambda has r values (>= 0).  Host pointers; either may be NULL.  *r_out gets r. */
int proxsdp_get_factors(proxsdp_handle *h, double *V, double *lambda, int32_t *r_out);

/* Resumable state in one call: the factors of X (as proxsdp_get_factors) and
 * the dual y (m + p values, unscaled, as proxsdp_get_solution).  Host
 * pointers; any may be NULL (call once with NULLs to learn r).  Synchronises.
 * Algorithm 2 keeps its intermediate (X, y) in memory; this is the way to
 * take it out for a later warm start. */
int proxsdp_get_state(proxsdp_handle *h, double *V, double *lambda, double *y, int32_t *r_out);

/* Intermediate feasible solutions X_[r] of Algorithm 2 (Section 3.2): every
 * time the residual test passes and the rank test fails, before r doubles (or
 * before the solve stops with PROXSDP_STATUS_RANK_LIMIT /
 * EIG_NOT_CONVERGED), the handle keeps a host copy of that iterate: its
 * factors X_[r] = V diag(lambda) V^T (V n x r row-major, lambda r values) and
 * its dual y_[r] (m + p values, unscaled, Section 1.3 sign).  `idx` counts
 * from 0 in the order they were kept; *iter_out gets the iteration after which
 * the copy was made and *r_out its rank.  Any output pointer may be NULL (a
 * call with NULL arrays returns r).  proxsdp_saved_count gives how many exist.
 * reset / set_state drop them.  Errors: PROXSDP_ERR_INVALID for a bad idx. */
int proxsdp_saved_count(proxsdp_handle *h, int32_t *count);
int proxsdp_get_saved(proxsdp_handle *h, int32_t idx, double *V, double *lambda, double *y,
                      int32_t *r_out, int32_t *iter_out);

/* Random-hyperplane rounding (Goemans-Williamson, the rounding of the max-cut
 * relaxation that the paper's Section 1.1 cites) of the current iterate
 * X = V diag(lambda) V^T: for each trial t,
 *   x_t = sign(V diag(sqrt(lambda)) g_t) in {-1, +1}^n   (+1 where the sum is >= 0)
 * and its value <C, x_t x_t^T> (for the max-cut relaxation C = -L/4 this is
 * minus the weight of the cut, and x_t x_t^T satisfies diag = 1).
 *   trials  1 .. 64
 *   g       host, trials x r row-major Gaussian vectors drawn by the caller
 *           (r = the rank proxsdp_get_factors reports; NULL allowed if r = 0)
 *   values  host, trials values <C, x_t x_t^T> (or NULL)
 *   x_best  host, n entries of the trial with the smallest value (or NULL)
 *   best    host, index of that trial (or NULL); ties go to the first
 * Synchronises.  Errors: PROXSDP_ERR_INVALID (trials out of range, g NULL or
 * non-finite). */
int proxsdp_round_hyperplane(proxsdp_handle *h, int32_t trials, const double *g, double *values,
                             int8_t *x_best, int32_t *best);

/* Warm start: restarts the iteration (counters, rank control and history
 * cleared, as proxsdp_reset) from X0 = V diag(lambda) V^T and y0 instead of
 * X0 = 0, y0 = 0 (Algorithm 1 from a given point).  V: n x r row-major host
 * array (columns need not be orthonormal), lambda: r values, finite and
 * >= 0 (X0 must be PSD), y: m + p values in the problem's own (unscaled)
 * units and Section 1.3 sign, inequality duals <= 0, or NULL for y0 = 0.
 * 0 <= r <= min(64, r cap) (n on the exact path).  The working rank becomes
 * max(r0, r) (within the cap); the first Ritz basis starts from V's columns.
 * Copies the arrays; synchronises `stream` of the handle.  Errors:
 * PROXSDP_ERR_INVALID (bad r, NULL arrays for r > 0, negative or non-finite
 * lambda, non-finite V or y, a positive inequality dual), PROXSDP_ERR_HIP. */
int proxsdp_set_state(proxsdp_handle *h, int32_t r, const double *V, const double *lambda,
                      const double *y);

/* Restarts the iteration from X0 = 0, y0 = 0 (Algorithm 2 with r = r0) on the
 * problem data already on the device; no host transfer of problem data.
 * Synchronises the stream. */
int proxsdp_reset(proxsdp_handle *h);

/* Kernel timing for benchmarks: enable = 1 records HIP events on the handle's
 * stream around every dense pass W B and every dense write of W (up to 8192
 * launches each); proxsdp_profile_read synchronises, returns the summed
 * milliseconds and launch counts since enabling, and stops recording.
 * Any pointer may be NULL. */
int proxsdp_profile_enable(proxsdp_handle *h, int32_t enable);
int proxsdp_profile_read(proxsdp_handle *h, double *pass_ms, int32_t *pass_count,
                         double *write_ms, int32_t *write_count);

/* Kernel timing totals since proxsdp_profile_enable (synchronises, disables
 * profiling): out[0] summed dense-pass time (ms), out[1] timed passes,
 * out[2] their algorithmic flops (2 npad^2 k per pass, k its subspace width),
 * out[3] their algorithmic bytes (s npad^2 per pass, one read of W stored
 * with s bytes per element: 8 FP64, 4 FP32, 2 BF16), out[4] summed
 * dense-write time (ms), out[5] timed writes, out[6] their MFMA flops (2 r
 * per cell of the upper tile pairs), out[7] their bytes (s n^2 written).  Copies min(count, 8) values to the host array `out`. */
int proxsdp_profile_totals(proxsdp_handle *h, double *out, int32_t count);

/* Rank path of Algorithm 2 since create/reset: for each change of the target
 * rank, the iteration after which it happened, the new rank and the reason
 * (1 = residual converged but the rank test failed, 2 = the windowed residual
 * test found no decrease, 3 = residual converged and the rank test could not
 * be decided on a confirmed subspace).  Writes up to `cap` entries; *count gets the total.
 * Host pointers; any may be NULL. */
int proxsdp_rank_path(proxsdp_handle *h, int32_t *iters, int32_t *ranks, int32_t *reasons,
                      int32_t cap, int32_t *count);

/* Diagnostics: copies min(count, 64) internal device scalars to host `out`
 * (0 step size, 1 lower spectral bound used by the filter, 2 largest relative
 * Ritz residual of the kept pairs, 3 lambda_r, 4 lambda_{r+1}, 5 max |theta|,
 * 6 eps_p, 7 eps_d, 8 objective, 9 dual objective, 10 ||X+ - X||_F^2,
 * 13 non-finite code (0 none, 1 Rayleigh-Ritz, 2 full eigensolve, 3 dual
 * step, 4 residuals), 14 dropped basis columns, 15 filter centre, 16 filter
 * half-width, 17 Jacobi sweeps, 18 Newton refinement steps of the last
 * Rayleigh-Ritz step or -1 if it took the Cholesky path, 19 number of
 * Rayleigh-Ritz steps on the Cholesky path and 20 of all Rayleigh-Ritz steps
 * since the last create/reset, 21 iteration counter, 22 / 23 / 24 Cholesky-path
 * steps that left the Newton refinement because the Gram matrix stayed
 * non-orthonormal / couplings among the kept pairs stayed above 1e-4 max|theta|
 * / the bound on the unresolved tail exceeded the r-th value, 25 .. 28 seconds
 * the Rayleigh-Ritz steps spent in their Newton refinement / Cholesky path /
 * diagonalisation / coefficient output, from the device clock, 29 positive
 * kept Ritz values, 30 the top Ritz value in the filter's variable, 31 Newton
 * refinement steps of all Rayleigh-Ritz calls, 32 calls whose refinement
 * reached its step limit, 33 Jacobi sweeps after accepted refinements) followed
 * by the Ritz values of the last
 * Rayleigh-Ritz step in out[64 ..] if count > 64.  Synchronises. */
int proxsdp_debug_scalars(proxsdp_handle *h, double *out, int32_t count);

/* Releases host-side state.  Does not touch the caller's workspace. */
void proxsdp_destroy(proxsdp_handle *h);

/* --------------------------------------------------- projection only */
/* Device workspace (bytes) for proxsdp_project_psd with these sizes. */
int proxsdp_project_workspace_size(int32_t n, int32_t r, int32_t precision, size_t *bytes);

/* aproj(S, r) of Section 3.1 (eq_trunc_eig): sum over the r algebraically
 * largest eigenvalues lambda_i of the symmetric S of max(0, lambda_i) u_i u_i^T;
 * r = 0 or r >= n gives the exact projection of Section 2.3.2 (one-workgroup
 * Jacobi for n <= 64, rocSOLVER dsyevd and a rocBLAS product above); for
 * 0 < r < n and n > 64 the target rank must be <= 48 (partial eigensolve).
 *   S       device, n x n row-major with leading dimension lds >= n, FP64
 *           (precision = PROXSDP_FP64); only read.  Must be symmetric.
 *   P       device, n x n output with leading dimension ldp, or NULL.
 *   evals   host, r values: the r largest eigenvalues, decreasing (or NULL).
 *   evecs   host, n x r row-major eigenvectors (or NULL).
 *   rank_out host: number of positive eigenvalues kept (or NULL).
 *   tol     relative residual target ||S v - lambda v|| <= tol ||S||_2 of the kept
 *           pairs (<= 0: 1e-12).
 * Synchronises `stream`.  Returns PROXSDP_ERR_UNSUPPORTED if the iteration does
 * not reach tol within its pass budget. */
int proxsdp_project_psd(const void *S, int32_t n, int64_t lds, int32_t r, int32_t precision,
                        double tol, void *P, int64_t ldp, double *evals, double *evecs,
                        int32_t *rank_out, void *d_workspace, size_t ws_bytes, void *stream);

/* proxsdp_project_psd for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and arguments, without the workspace.
 * Its device memory is a static 32 MiB array that the library holds on every
 * GPU it runs on until the process ends (enough for n = 2000 at r <= 48, or
 * n up to about 2800 at r = 16); it calls no hipMalloc / hipFree and no
 * allocating library routine.  Every call on one GPU shares that GPU's array
 * and overwrites it, so calls that overlap on one GPU (other threads, other
 * streams) race; serialise them.  The exact projection for n > 64 (r = 0 or
 * r >= n) needs rocSOLVER and is refused with PROXSDP_ERR_UNSUPPORTED; a size
 * whose scratch (proxsdp_project_workspace_size) exceeds 32 MiB is refused
 * with PROXSDP_ERR_WORKSPACE.  Synchronises `stream`. */
int proxsdp_project_psd_noalloc(const void *S, int32_t n, int64_t lds, int32_t r, int32_t precision,
                                double tol, void *P, int64_t ldp, double *evals, double *evecs,
                                int32_t *rank_out, void *stream);

/* Thread-local description of the last error (empty string if none). */
const char *proxsdp_last_error(void);

/* Library version string. */
const char *proxsdp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PROXSDP_H */
