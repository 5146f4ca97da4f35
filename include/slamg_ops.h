/* slamg_ops.h -- step-level C entry points of the slamg library.
 *
 * Each entry point runs ONE step of the method's multilevel cycles with the same HIP kernels (or
 * host graph code) that slamg_solve uses, on caller-owned buffers, so that every step can be
 * compared with an independent reference.  The passage of the paper (H. De Sterck,
 * arXiv:1102.0919) that defines each step is cited at the declaration.
 *
 * Conventions
 *   - "d_" pointers are device pointers on the current HIP device, "h_" pointers host pointers.
 *   - Sparse matrices are CSR with int32 row pointers / column indices and double values; a NULL
 *     B or C operator means the identity.  Dense blocks are row-major (row i holds w entries).
 *   - w (block width) is 1..16.  stream: a hipStream_t or NULL for the null stream.
 *   - Device entry points are synchronous (they wait for their kernels), allocate and free their
 *     own temporaries with hipMalloc/hipFree, and return SLAMG_E_DEVICE on a HIP error and
 *     SLAMG_E_INVALID on bad sizes.  Outputs are written only on success.
 *   - Host graph entry points touch no device and are deterministic.
 */
#ifndef SLAMG_OPS_H
#define SLAMG_OPS_H

#include <stdint.h>

#include "slamg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Block sparse product Y = A X + beta Y (A: m rows).  Every operator application of §3.4-§4.3. */
slamg_status slamg_op_spmm(int32_t m, int32_t w, const int32_t* d_rp, const int32_t* d_ci, const double* d_v,
                           const double* d_x, double* d_y, double beta, void* stream);
/* The same product in FP32 (mixed-precision V-cycles). */
slamg_status slamg_op_spmm_f32(int32_t m, int32_t w, const int32_t* d_rp, const int32_t* d_ci, const float* d_v,
                               const float* d_x, float* d_y, double beta, void* stream);
/* The FP32 product reading BF16 operator values (SLAMG_MIXED_BF16 V-cycles): d_v holds nnz BF16 bit
 * patterns (the high 16 bits of an FP32 word); x, y and the sums are FP32. */
slamg_status slamg_op_spmm_bf16(int32_t m, int32_t w, const int32_t* d_rp, const int32_t* d_ci, const uint16_t* d_v,
                                const float* d_x, float* d_y, double beta, void* stream);
/* BF16 copy of n FP64 values as the SLAMG_MIXED_BF16 mode stores them: each value rounded to FP32,
 * then to BF16, both to nearest with ties to even; a NaN stays a (quiet) NaN.  d_out: n uint16. */
slamg_status slamg_op_cast_bf16(int64_t n, const double* d_in, uint16_t* d_out, void* stream);

/* Test-vector relaxation, dominant targets (§3.4): one power step with one weighted-Jacobi inner
 * step of weight omega, normalised in the C / B norm.  SVD: A (m x n) and its transpose At, B
 * (m x m), C (n x n) (NULL: identity), U (m x w), V (n x w) updated in place.  Eigenproblem
 * (spd = 1): A (n x n), d_bv = values of B on A's pattern (NULL: identity), X in d_u. */
slamg_status slamg_op_relax_test(int32_t spd, int32_t m, int32_t n, int32_t w, const int32_t* d_arp,
                                 const int32_t* d_aci, const double* d_av, const int32_t* d_atrp,
                                 const int32_t* d_atci, const double* d_atv, const int32_t* d_brp,
                                 const int32_t* d_bci, const double* d_bv, const int32_t* d_crp,
                                 const int32_t* d_cci, const double* d_cv, double omega, double* d_u, double* d_v,
                                 void* stream);

/* Boot-vector relaxation, dominant targets (§3.5, eqs. of the block Gauss-Seidel step): u from
 * A v = sigma B u + kappa, then v from A^t u = sigma C v + tau, each by one weighted-Jacobi step.
 * d_sig: w values; d_kap (m x w) / d_tau (n x w) may be NULL (zero).  Same operand layout as
 * slamg_op_relax_test. */
slamg_status slamg_op_relax_boot(int32_t spd, int32_t m, int32_t n, int32_t w, const int32_t* d_arp,
                                 const int32_t* d_aci, const double* d_av, const int32_t* d_atrp,
                                 const int32_t* d_atci, const double* d_atv, const int32_t* d_brp,
                                 const int32_t* d_bci, const double* d_bv, const int32_t* d_crp,
                                 const int32_t* d_cci, const double* d_cv, const double* d_sig,
                                 const double* d_kap, const double* d_tau, double omega, double* d_u, double* d_v,
                                 void* stream);

/* One Kaczmarz sweep (minimal targets, §5.3) on M x = rhs, rows taken colour by colour in the order
 * h_rows[h_cptr[c] .. h_cptr[c+1]) (rows of one colour must not share a column).  With d_lam
 * (w shifts) the operator of column j is M - lam_j B, B given by d_bv on M's pattern (NULL: B = I,
 * M square).  d_rhs (nrows x w) may be NULL.  x (ncols x w) is updated in place. */
slamg_status slamg_op_kaczmarz(int32_t nrows, int32_t ncols, int32_t w, const int32_t* d_rp, const int32_t* d_ci,
                               const double* d_v, const double* d_bv, const double* d_lam, const int32_t* h_rows,
                               const int32_t* h_cptr, int32_t ncolours, const double* d_rhs, double* d_x,
                               void* stream);

/* Additive residual (§4.1, eq. (4.1)): out = kap - (K z - sigma_j M y) over the rows of K; M NULL
 * means identity.  Restriction and prolongation (eqs. (4.2)-(4.3)) are slamg_op_spmm with P^t / P. */
slamg_status slamg_op_residual(int32_t nrows, int32_t w, const int32_t* d_krp, const int32_t* d_kci,
                               const double* d_kv, const double* d_z, const int32_t* d_mrp, const int32_t* d_mci,
                               const double* d_mv, const double* d_y, const double* d_kap, const double* d_sig,
                               double* d_out, void* stream);

/* Column reductions out_j = sum_i a_ij (K z)_ij (K NULL: z itself) or, with a NULL,
 * sum_i ((K z)_ij - sig_j y_ij)^2.  h_out: w values (host). */
slamg_status slamg_op_dots(int32_t nrows, int32_t w, const double* d_a, const int32_t* d_krp, const int32_t* d_kci,
                           const double* d_kv, const double* d_z, const double* d_y, const double* d_sig,
                           double* h_out, void* stream);

/* Tall-skinny Gram product G = X^t Y on the FP64 matrix cores (rows x w blocks; h_g: w x w). */
slamg_status slamg_op_gram(int32_t rows, int32_t w, const double* d_x, const double* d_y, double* h_g,
                           void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): slamg_op_gram with the result G = X^t Y (w x w,
 * row-major) written to the device array d_g, and the reduction's per-workgroup partial sums kept
 * in a fixed device array of slamg_op_gram_noalloc_scratch_bytes() bytes (4 MiB; one per GPU,
 * held until the process ends) instead of memory it allocates.  It allocates and frees nothing,
 * does not synchronise (the kernels are queued on `stream`; read d_g after the stream's work), and
 * needs no zeroed scratch (every launch writes the slots it reads).  Every call on one GPU uses
 * that GPU's one scratch array: calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller.  rows >= 0, w in 1..16 (SLAMG_E_INVALID otherwise;
 * SLAMG_E_BUDGET if the reduction would need more scratch than the array holds), SLAMG_E_DEVICE
 * on a HIP error at launch. */
slamg_status slamg_op_gram_noalloc(int32_t rows, int32_t w, const double* d_x, const double* d_y, double* d_g,
                                   void* stream);
size_t slamg_op_gram_noalloc_scratch_bytes(void);

/* Ritz projection on the finest level (§4.3): Cholesky-QR2 orthonormalisation of U (and V), the
 * projected w x w problem and the rotation of the bases.  spd = 1: X in d_u, eigenproblem.
 * minimal selects ascending order.  h_sig: w values (host). */
slamg_status slamg_op_ritz(int32_t spd, int32_t minimal, int32_t m, int32_t n, int32_t w, const int32_t* d_arp,
                           const int32_t* d_aci, const double* d_av, double* d_u, double* d_v, double* h_sig,
                           void* stream);

/* Least-squares interpolation weights (§3.8, eq. (LS)): for every F-point (h_is_c[i] == 0) the
 * weighted normal equations on its interpolatory set h_fine_cols[h_ptr[i] .. h_ptr[i+1]) (fine ids
 * of C-points).  Fitted vectors: U1 (npts x w1) then U2 (npts x w2, may be NULL with w2 = 0);
 * values at F-points: B1, B2 (same shapes; NULL = U1, U2); weights d_wts (w1 + w2).
 * h_pval receives the P values in pattern order (C rows = 1). */
slamg_status slamg_op_ls_fit(int32_t npts, const int32_t* h_ptr, const int32_t* h_fine_cols, const int8_t* h_is_c,
                             int32_t w1, const double* d_u1, const double* d_b1, int32_t w2, const double* d_u2,
                             const double* d_b2, const double* d_wts, double* h_pval, void* stream);

/* Numeric sparse product on a given pattern (Galerkin operators, eq. (3.4), and the strength
 * operators A A^t, A^t A of §3.7): entry e of C (row d_rowc[e], column d_colc[e]) = row i of L
 * dotted with row j of R^t.  d_out: nnz values. */
slamg_status slamg_op_spgemm(int32_t nnz, const int32_t* d_rowc, const int32_t* d_colc, const int32_t* d_lrp,
                             const int32_t* d_lci, const double* d_lv, const int32_t* d_rtrp, const int32_t* d_rtci,
                             const double* d_rtv, double* d_out, void* stream);

/* Top-s rule of §3.7 on a strength operator: for every row i of the m-row CSR matrix (device
 * row pointers d_rp, columns d_col, values d_val) the s (1..16) off-diagonal entries with the
 * largest |n_ij| > 0, ties to the lower j, written to d_out_col / d_out_val (m x s, row-major) in
 * ascending j, -1 (and 0.0) after the last.  SLAMG_E_INVALID for s outside 1..16 or m < 0. */
slamg_status slamg_op_topsel(int32_t m, const int32_t* d_rp, const int32_t* d_col, const double* d_val, int32_t s,
                             int32_t* d_out_col, double* d_out_val, void* stream);

/* Coarsest generalized SVD (§3.6, Theorem 3.1): n_b extremal triplets of dense A (mL x nL) w.r.t.
 * SPD B (mL x mL) and C (nL x nL), or (spd = 1) eigenpairs of the pencil (A, B).  Host dense
 * row-major inputs; h_u (mL x nb), h_v (nL x nb) row-major, h_sig (nb). */
slamg_status slamg_op_coarse_gsvd(int32_t spd, int32_t minimal, int32_t mL, int32_t nL, int32_t nb,
                                  const double* h_a, const double* h_b, const double* h_c, double* h_sig,
                                  double* h_u, double* h_v);

/* SVD of the k x k projected matrix of the LOBPCG step (§7, the Rayleigh-Ritz step on span[X, W, P]
 * of an SVD target with orthonormal bases): the nb singular triplets M z_j = sigma_j y_j with the
 * largest (minimal = 0) or smallest (minimal = 1) sigma, in that order, by one-sided Jacobi on M.
 * h_m: dense row-major k x k (host); h_sig (nb), h_y (k x nb), h_z (k x nb) row-major (host,
 * caller-owned).  Singular values at or below 1e-13 sigma_max get y completed to an orthonormal
 * set.  SLAMG_E_INVALID unless 1 <= nb <= k <= 32 and every pointer is non-null. */
slamg_status slamg_op_proj_svd(int32_t minimal, int32_t k, int32_t nb, const double* h_m, double* h_sig,
                               double* h_y, double* h_z);

/* Additive coarsest solve (§4.2): per column j, variant 0 applies the pseudo-inverse of
 * X - sig_j Y from its SVD without the smallest singular component; variant 1 the pencil variant;
 * variants 2, 3 and 4 are variant 0 computed the way consecutive additive iterations compute it,
 * starting from the eigenvectors of X - sig'_j Y at sig'_j = sig_j (1 + delta): delta = 1e-6
 * (variant 2: Newton-type steps when N <= 64, else Jacobi sweeps), 1e-12 (variant 3: the
 * first-order update) or 1e-3 (variant 4: Jacobi sweeps); variant 5 is variant 2 with the basis
 * re-orthonormalised first (one Newton-Schulz step, as every 32nd additive iteration does).  Returns
 * SLAMG_E_INVALID for another variant or N outside [1, 1024].
 * Host dense inputs X, Y (N x N), h_rhs / h_out (N x nb) row-major. */
slamg_status slamg_op_coarse_solve(int32_t variant, int32_t N, int32_t nb, const double* h_x, const double* h_y,
                                   const double* h_sig, const double* h_rhs, double* h_out);

/* Host graph steps of the first multiplicative cycle (§3.7). */
/* Strength sets S_i (rule 0 row-sum, 1 max-based, 2 top-s); h_sp (n+1), h_si (capacity nnz). */
slamg_status slamg_graph_strength(int32_t n, const int32_t* h_rp, const int32_t* h_ci, const double* h_v,
                                  double theta, int32_t rule, int32_t top_s, int32_t* h_sp, int32_t* h_si);
/* Algorithm 1 (one-pass Ruge-Stueben coarsening): h_is_c (n) receives 1 for C-points. */
slamg_status slamg_graph_rs(int32_t n, const int32_t* h_sp, const int32_t* h_si, int8_t* h_is_c);
/* Interpolatory sets capped to `cap` strongest: h_ptr (n+1), h_cols (capacity nnz(S) + n). */
slamg_status slamg_graph_interp(int32_t n, const int32_t* h_sp, const int32_t* h_si, const int32_t* h_rp,
                                const int32_t* h_ci, const double* h_v, const int8_t* h_is_c, int32_t cap,
                                int32_t* h_ptr, int32_t* h_cols, int32_t* h_capped);
/* Greedy first-fit colouring of the rows of an m x n pattern (rows sharing a column conflict). */
slamg_status slamg_graph_colour(int32_t m, int32_t n, const int32_t* h_rp, const int32_t* h_ci, int32_t* h_colour);

#ifdef __cplusplus
}
#endif
#endif /* SLAMG_OPS_H */
