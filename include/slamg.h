/* slamg.h -- C ABI of the MI355X self-learning algebraic multigrid solver for a few extremal
 * singular triplets of a sparse matrix, and for extremal eigenpairs of an SPD matrix.
 *
 * The method is H. De Sterck, "A Self-learning Algebraic Multigrid Method for Extremal Singular
 * Triplets and Eigenpairs" (arXiv:1102.0919):
 *   problem statement ......... §1, eq. (1.2): A v_j = sigma_j u_j, A^t u_j = sigma_j v_j,
 *                               n_b dominant (largest sigma) or minimal (smallest sigma) triplets;
 *                               the SPD eigenpair special case (§1, §5.2);
 *   setup (multiplicative) .... §3 (bootstrap V-cycles, relaxation §3.4-3.5, coarsest solve §3.6,
 *                               coarsening and LS interpolation §3.7-3.8);
 *   solve (additive + Ritz) ... §4 (additive V-cycles §4.1-4.2, Ritz projection §4.3);
 *   minimal targets ........... §5.3 (Kaczmarz relaxation, inverse-RQ LS weights).
 *
 * Conventions
 *   - Every function returns slamg_status; no C++ exception crosses this interface.
 *   - All floating-point inputs and outputs are IEEE double.
 *   - Ownership: the caller owns A and every output array; the library copies A to the device
 *     during slamg_solve / slamg_submit, so the caller may free it when the call returns.  The
 *     context owns all device memory (hierarchy, vectors, workspaces) until slamg_destroy.
 *   - Results: sigma sorted descending (dominant) or ascending (minimal); columns of U and V have
 *     unit 2-norm; the entry of largest magnitude of v_j (of x_j for eigenproblems; lowest index on
 *     ties) is positive.  m < n is handled by solving with A^t and swapping U and V.  Empty rows
 *     and columns of A are removed before solving and get zero entries in U and V.
 *   - A context is used by one host thread at a time; distinct contexts may run concurrently.
 */
#ifndef SLAMG_H
#define SLAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLAMG_OK = 0,
  SLAMG_NOT_CONVERGED = 1,  /* results filled, tolerance not reached within max_add iterations */
  SLAMG_E_INVALID = -1,     /* bad CSR, n_b < 1 or > min(m, n), tol <= 0, SPD with m != n, ...  */
  SLAMG_E_OOM = -2,         /* a device allocation failed                                       */
  SLAMG_E_BUDGET = -3,      /* the device footprint would exceed the context's HBM budget      */
  SLAMG_E_DEVICE = -4,      /* a HIP runtime call failed                                        */
  SLAMG_E_NUMERIC = -5,     /* NaN/Inf, factorisation breakdown, coarsest level too large        */
  SLAMG_E_BUSY = -6         /* request not finished yet (slamg_fetch)                           */
} slamg_status;

typedef enum { SLAMG_DOMINANT = 0, SLAMG_MINIMAL = 1 } slamg_target;
typedef enum { SLAMG_SVD = 0, SLAMG_SPD_EIG = 1 } slamg_kind;
typedef enum {
  SLAMG_FP64 = 0,           /* every step in FP64                                               */
  SLAMG_MIXED_FP32 = 1,     /* FP32 V-cycles on the error equation inside an FP64 refinement     */
  SLAMG_MIXED_BF16 = 2      /* as MIXED_FP32 with the V-cycle's operator values stored in BF16
                               (rounded to nearest even); vectors and sums stay FP32           */
} slamg_precision;

/* Sparse matrix in CSR: row_ptr (m+1, int64), col_idx (nnz, int32, sorted within a row, no
 * duplicates), val (nnz, double).  on_device = 0: host pointers.  on_device = 1: device pointers
 * on the context's device (read on the context stream). */
typedef struct {
  int64_t m, n, nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
  int32_t on_device;
} slamg_csr;

/* Method parameters.  slamg_params_init fills the defaults listed here. */
typedef struct {
  double theta;             /* strength threshold of §3.7 (0.06)                                */
  int32_t strength_rule;    /* 0 row-sum rule of §3.7, 1 max-based rule, 2 top-s rule (0)       */
  int32_t top_s;            /* s of the top-s rule, 1..16 (4)                                   */
  double df_filter;         /* top-s rule: rows with more than df_filter*n nonzeros are ignored
                               when measuring strength on the finest level (0 = off)            */
  int32_t n_t;              /* number of test vectors (8)                                       */
  int32_t mu_t, mu_b;       /* test / boot relaxations per level (4, 4)                         */
  double omega_J;           /* weighted-Jacobi weight of §3.4 (0.7)                             */
  int32_t n_mult;           /* multiplicative cycles (10)                                       */
  int32_t max_add;          /* maximum additive iterations (200)                                */
  int32_t coarse_max;       /* coarsest-level size: n (eigen) or m+n (SVD) at most this (64)     */
  int32_t max_levels;       /* (25)                                                            */
  double stall_ratio;       /* stop coarsening when the coarse level keeps more (0.9)           */
  double tol;               /* relative residual tolerance (1e-8)                               */
  uint64_t seed;            /* SplitMix64 seed of the initial test vectors (1102)               */
  int32_t precision;        /* slamg_precision (SLAMG_FP64)                                     */
  int32_t ritz_in_mult;     /* Ritz step at the end of each multiplicative cycle (1)            */
  int32_t coarse_pinv;      /* additive coarsest solve: 0 pseudo-inverse from the SVD of
                               X - sigma Y without its smallest component (§4.2); 1 the same
                               with the pencil eigenbasis of (X, Y) computed once (0)           */
  int32_t profile_mask;     /* bit c set: time every launch of kernel class c with HIP events on
                               the context stream and report it (0 = off).  Classes:
                               0 fused row kernel on the finest level (Jacobi-type relaxation),
                               1 Kaczmarz sweeps on the finest level, 2 MFMA Gram products,
                               3 Galerkin SpGEMM, 4 coarsest dense solves, 5 block SpMM on the
                               finest level, 6 operator reductions (dot products of a block with
                               an operator product) on the finest level, 7 fused row kernel
                               computing residuals on the finest level */
  int32_t verbose;          /* k > 0: one progress line on stderr after each multiplicative cycle
                               and every k additive iterations (0)                              */
  int32_t graphs;           /* 1: capture one additive iteration (V-cycle, Ritz step, residual
                               reductions) in a HIP graph and replay it; 0: launch every kernel
                               on the stream.  Both give bitwise the same results (1)           */
  int32_t square_coarsening;  /* SVD of a square A (§5.1): strength, C/F split and interpolatory
                               sets of both sides from A itself, so P and Q share one pattern and
                               every level is square; the LS weights of P and Q are fitted
                               separately.  Needs a square matrix without empty rows or
                               columns (SLAMG_E_INVALID otherwise); ignored for SPD (0)         */
  int32_t n_guard;          /* guard pairs: the method runs on a block of n_b + n_guard pairs
                               (coarsest selection, boot vectors, V-cycles and the Ritz step of
                               §4.3 on the whole block); the stopping test and the outputs take
                               the n_b extremal pairs.  n_b + n_guard <= 16 (0)                 */
  int32_t mu_tJ, mu_bJ;     /* inner weighted-Jacobi steps per outer test / boot relaxation of
                               dominant targets (§3.4, §3.5) (1, 1)                             */
  int32_t kaczmarz_order;   /* row order of the Kaczmarz sweeps of minimal targets (§5.3): 0
                               multicolour (rows of one colour share no column, colours
                               ascending, rows ascending), 1 lexicographic (row by row) (0)     */
  int32_t coarse_dense_max; /* completed C-sets: where coarsening would stop at a level of more
                               than this many unknowns, each side with fewer than n_b + n_guard
                               + n_t C-points gets its most influential F-points as further
                               C-points (Algorithm 1's initial measure, lowest index on ties)
                               and coarsening continues.  1 .. 1024, the largest coarsest level
                               the dense coarsest solves take (1024)                            */
  int32_t redo_p;           /* redetermined interpolation in the additive phase (§6.3): a pair
                               counts as converged once its sigma changes by at most redo_tol
                               relative between two iterations; whenever that set grows while a
                               pair of the block is not converged, one downward sweep of the
                               multiplicative phase refits P, Q and the coarse operators, the LS
                               weights of the test vectors and of the converged pairs multiplied
                               by 1e-3; the iterates are kept (0)                               */
  double redo_tol;          /* relative change of sigma that counts as converged (1e-14)         */
  int32_t cycle_gamma;      /* additive cycle (§3.3): 1 V-cycle, 2 W-cycle (every level but the
                               last one above the coarsest visits its coarser level twice, the
                               second visit from the first one's correction) (1)                */
  int32_t ritz_coarse;      /* Ritz step on coarse levels (§4.3): in the upward sweep of a
                               multiplicative cycle, after each coarse level's boot relaxation, the
                               boot triplets become the Ritz triplets of their span in the B and C
                               metrics (0)                                                       */
  int32_t solve_phase;      /* 0 the multigrid-Ritz additive phase of §4; 1 LOBPCG on the learned
                               hierarchy (§7 names it as a replacement): the preconditioned
                               direction of a pair is the change the additive cycle makes to it,
                               and the Ritz step of §4.3 runs on the span of the pairs, those
                               directions and the previous search directions (3 n_b columns; the
                               previous directions are left out in an iteration where they are
                               numerically dependent on the others).  Minimal SVD targets take
                               the left basis from A times the right one.  Iterations run
                               without graph replay (0)                                         */
  int32_t fmg;              /* additive cycle (§3.3 names FMG): 1 an FMG cycle: the finest block's
                               residual restricted through every level, the coarsest level solved,
                               then from the coarsest upwards every coarse level starts from the
                               prolonged correction of the level below it and runs one cycle
                               (cycle_gamma) against its restricted residual; the finest block
                               adds the prolonged correction and runs one cycle.  0 the cycle of
                               cycle_gamma alone (0)                                            */
} slamg_params;

/* Report of one solve.  Arrays are filled up to the counts given. */
typedef struct {
  int32_t levels, mult_cycles, add_iters, converged;
  int64_t rows[32], cols[32], nnz[32];      /* per level: A_l is rows x cols with nnz entries  */
  int32_t colours[32];                       /* Kaczmarz colours of the rows of A_l            */
  int32_t capped[32];                        /* interpolatory sets capped on level l           */
  double anorm;                              /* ||A||_2 estimate used by the residuals         */
  double resid[16];                          /* final relative residual per triplet            */
  double rho_history[256];                   /* max relative residual after the mult phase (0)
                                                and after each additive iteration              */
  double mult_sigma[32][16];                 /* sigma_b after each multiplicative cycle        */
  double t_setup_ms, t_solve_ms;             /* multiplicative phase / additive phase           */
  double err_bound[16];                      /* residual-based error bound per sigma_j         */
  double prof_ms[8];                         /* per profiled class: summed device time (ms)     */
  int64_t prof_launches[8];                  /*   number of launches                            */
  double prof_bytes[8];                      /*   summed algorithmic bytes of those launches    */
  int32_t graph_iters;                       /* additive iterations run as graph replays        */
  int32_t redo_count;                        /* redetermined interpolations (redo_p)            */
  int64_t device_bytes;                      /* peak device memory the solve held (all levels)  */
  double t_queue_ms, t_latency_ms;           /* requests: submit -> start, submit -> result      */
  int32_t p_dropped;                         /* LOBPCG iterations that left out the previous
                                                search directions (solve_phase 1)              */
  int32_t reserved_r;
} slamg_report;

typedef struct slamg_ctx slamg_ctx;

/* Default parameters for a problem kind and target. */
slamg_status slamg_params_init(slamg_params* p, slamg_kind kind, slamg_target target);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run on, or NULL for a
 * stream owned by the context.  hbm_budget_bytes: device-memory cap of this context (0 = none). */
slamg_status slamg_create(slamg_ctx** ctx, int device, void* hip_stream, size_t hbm_budget_bytes);
void slamg_destroy(slamg_ctx* ctx);

/* Solve for n_b triplets (kind SVD) or eigenpairs (kind SPD_EIG, m == n) of A: the problem of §1,
 * eq. (1.2), for the dominant or minimal end of the spectrum (§5.2, §5.3), by the multiplicative
 * set-up cycles of §3 (hierarchy, interpolation and test vectors learnt together) followed by the
 * additive multigrid-Ritz iterations of §4 (or, solve_phase = 1, LOBPCG preconditioned by the
 * learnt hierarchy, §7) until every pair's residual max(||A v - sigma u||, ||A^t u - sigma v||) /
 * ||A|| (eigenpairs: ||A x - lambda x|| / ||A||; ||A|| the estimate reported as anorm) is at
 * most tol.
 * init_tests: NULL (seeded SplitMix64 uniform[-1,1) test vectors) or a column-major
 *   (m'+n') x n_t (SVD) / n' x n_t (eigen) array for the prepared matrix (m' >= n' after the
 *   optional transposition, empty rows and columns removed).
 * sigma: n_b; U: m x n_b column-major or NULL; V: n x n_b column-major or NULL (ignored for SPD);
 * rep: NULL or a report.  Returns SLAMG_OK, SLAMG_NOT_CONVERGED (outputs hold the last iterate)
 * or an error. */
slamg_status slamg_solve(slamg_ctx* ctx, const slamg_csr* A, slamg_kind kind, slamg_target target,
                         int32_t n_b, const slamg_params* p, const double* init_tests, double* sigma,
                         double* U, double* V, slamg_report* rep);

/* Prepared matrices.  slamg_matrix_create validates A, prepares it (transposition when m < n,
 * removal of empty rows and columns) and keeps it resident in device memory, so that repeated
 * solves start with A already in HBM.  The handle belongs to ctx and must be destroyed before it.
 * slamg_solve_matrix solves like slamg_solve.  outputs_on_device = 0: U, V are host arrays (or
 * NULL); outputs_on_device = 1: U (m x n_b) and V (n x n_b) are column-major device arrays on the
 * context's device (or NULL), written on the context stream; sigma is always a host array. */
typedef struct slamg_matrix slamg_matrix;
slamg_status slamg_matrix_create(slamg_ctx* ctx, const slamg_csr* A, slamg_kind kind, slamg_matrix** M);
void slamg_matrix_destroy(slamg_matrix* M);
slamg_status slamg_solve_matrix(slamg_ctx* ctx, const slamg_matrix* M, slamg_target target, int32_t n_b,
                                const slamg_params* p, const double* init_tests, double* sigma, double* U,
                                double* V, int32_t outputs_on_device, slamg_report* rep);

/* Request interface (the problem of §1 as a stream of requests).  submit copies A, checks the
 * request's device-memory estimate against the context's HBM budget (SLAMG_E_BUDGET if it can
 * never fit) and returns an id at once.  Without the serving loop, the request is solved on the
 * context stream when slamg_poll, slamg_wait or slamg_fetch asks for it (first come, first
 * served).  poll sets *done; wait blocks until the request is done; fetch returns SLAMG_E_BUSY
 * while unfinished, else the request's status, outputs (as slamg_solve) and report (with its
 * queueing time and latency), and frees it. */
slamg_status slamg_submit(slamg_ctx* ctx, const slamg_csr* A, slamg_kind kind, slamg_target target,
                          int32_t n_b, const slamg_params* p, uint64_t* request_id);
slamg_status slamg_poll(slamg_ctx* ctx, uint64_t request_id, int32_t* done);
slamg_status slamg_wait(slamg_ctx* ctx, uint64_t request_id);
slamg_status slamg_fetch(slamg_ctx* ctx, uint64_t request_id, double* sigma, double* U, double* V,
                         slamg_report* rep);

/* Serving loop: `slots` (1..64) worker threads, each with its own HIP stream on the context's
 * device, solve submitted requests as they arrive.  A request starts when a slot is free and its
 * device-memory estimate fits the context's HBM budget beside the running requests (first fit
 * among the 64 oldest pending ones); its solve then overlaps on the device with the others and
 * may use at most its estimate.  Results are the same as those of slamg_solve on the request
 * alone.  stop finishes the pending requests, then joins the workers (slamg_destroy calls it).
 * The context's API calls stay single-threaded; only the workers run concurrently. */
slamg_status slamg_serve_start(slamg_ctx* ctx, int32_t slots);
slamg_status slamg_serve_stop(slamg_ctx* ctx);

const char* slamg_status_string(slamg_status s);
const char* slamg_last_error(const slamg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SLAMG_H */
