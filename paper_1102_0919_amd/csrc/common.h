// Internal declarations shared by the HIP kernels, the host-side graph code and the solver.
// Nothing here crosses the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace slamg {

// ------------------------------------------------------------------------------------------------
// Device CSR (int32 row pointers and column indices; all supported problems have nnz < 2^31).
// Values are kept in FP64 and, in the mixed-precision mode, also in FP32.
// ------------------------------------------------------------------------------------------------
struct DCsr {
  int m = 0, n = 0;
  int nnz = 0;
  int* rp = nullptr;      // m + 1
  int* ci = nullptr;      // nnz, sorted within a row
  double* v = nullptr;    // nnz
  float* vf = nullptr;    // nnz, FP32 copy (mixed precision only)
};

// Host CSR pattern (+ optional values)
struct HCsr {
  int m = 0, n = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  int nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Launch configuration helpers ------------------------------------------------------------------
struct ErrorState {
  std::string msg;
  int code = 0;
};

// status codes (mirrors slamg.h)
enum {
  ST_OK = 0,
  ST_NOT_CONVERGED = 1,
  ST_E_INVALID = -1,
  ST_E_OOM = -2,
  ST_E_BUDGET = -3,
  ST_E_DEVICE = -4,
  ST_E_NUMERIC = -5,
  ST_E_BUSY = -6
};

// ------------------------------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All take a stream; none synchronises.
// Blocks are row-major rows x w, w <= 16 unless stated.
// ------------------------------------------------------------------------------------------------
enum MMode { M_NONE = 0, M_IDENT = 1, M_CSR = 2, M_SHARED = 3 };
enum CMode {
  C_JAC_TEST = 0,   // out = x + D*( w*(Kz) - w*(My) )
  C_JAC_BOOT = 1,   // out = x + D*( (w/s)*(Kz) - w*(My) - (w/s)*kap )
  C_RESID = 2,      // out = -(Kz) + s*(My) + kap
  C_SMOOTH = 3,     // out = x + D*( -w*(Kz) )
  C_COPYK = 4       // out = Kz (+ x if given)
};

template <typename T>
struct RowOpArgs {
  int nrows = 0, w = 0;
  const int* Krp = nullptr; const int* Kci = nullptr; const T* Kv = nullptr; const T* z = nullptr;
  int mmode = M_NONE;
  const int* Mrp = nullptr; const int* Mci = nullptr; const T* Mv = nullptr; const T* y = nullptr;
  const T* x = nullptr;      // nullable
  const T* D = nullptr;      // nullable per-row scale
  const T* kap = nullptr;    // nullable
  const double* sig = nullptr;
  int cmode = C_JAC_TEST;
  double omega = 0.7;
  T* out = nullptr;
  int nnzK = -1;             // nonzeros of K (chooses the row split); -1: unknown
  double avgM = 0.0;         // mean row length of M (M_CSR; also chooses the row split)
  int vbf = 0;               // Kv, Mv hold BF16 bit patterns (T = float only)
  // rows with very many nonzeros in K or M: flag per row (1 = long) and the list of those rows;
  // each long row gets a workgroup of its own (none: all rows by lane groups)
  const unsigned char* lflag = nullptr;
  const int* lrows = nullptr;
  int nlong = 0;
};

template <typename T> void launch_rowop(const RowOpArgs<T>& a, hipStream_t s);
// two independent row operations (same w, same value form vbf) in one launch
template <typename T> void launch_rowop2(const RowOpArgs<T>& a, const RowOpArgs<T>& b, hipStream_t s);

// vbf: v holds BF16 bit patterns (T = float only)
template <typename T>
void launch_spmm(int m, int w, const int* rp, const int* ci, const T* v, const T* x, T* y,
                 double beta, hipStream_t s, int nnz = -1, int vbf = 0);

// y = K x (+ beta y) for one operand set of a paired SpMM
template <typename T>
struct SpmmArgs {
  int m = 0, nnz = -1;
  const int* rp = nullptr; const int* ci = nullptr; const T* v = nullptr;
  const T* x = nullptr; T* y = nullptr; double beta = 0.0;
  int vbf = 0;               // v holds BF16 bit patterns (T = float only)
};
// two independent products with w columns (same value form vbf) in one launch
template <typename T> void launch_spmm2(const SpmmArgs<T>& a, const SpmmArgs<T>& b, int w, hipStream_t s);

template <typename T>
struct KaczArgs {
  int nrows = 0;             // rows in this colour
  const int* rows = nullptr; // row ids of this colour
  int w = 0;
  const int* rp = nullptr; const int* ci = nullptr; const T* av = nullptr;
  const T* bv = nullptr;     // shared-pattern B values (eigenproblem boot relaxation) or null
  const double* lam = nullptr;
  const T* rn_aa = nullptr; const T* rn_ab = nullptr; const T* rn_bb = nullptr;
  int rmode = M_NONE;        // right-hand side operator on y: none / identity / CSR
  const int* Mrp = nullptr; const int* Mci = nullptr; const T* Mv = nullptr; const T* y = nullptr;
  const double* rsig = nullptr;
  const T* kap = nullptr;
  T* x = nullptr;
  long nnz_total = -1, nnz_rows = 0;   // row-length statistics of the operator (row split)
  double avgM = 0.0;                    // mean row length of the right-hand side operator (M_CSR)
  int vbf = 0;                          // av, bv, Mv hold BF16 bit patterns (T = float only)
};
template <typename T> void launch_kacz(const KaczArgs<T>& a, hipStream_t s);
// nhalf (1 or 2) half-sweeps per sweep, nsweeps sweeps, all in one workgroup; halves[h].rows is the
// colour-ordered row list and cptr[h] its device colour pointer (ncol[h] colours).
template <typename T>
void launch_kacz_wg(const KaczArgs<T>* halves, const int* const* cptr, const int* ncol, int nhalf, int nsweeps,
                    hipStream_t s);
// Whole sweeps with one workgroup per block column, the updated vectors' column held in LDS
// (nx[h]: length of half-sweep h's updated vector; with two half-sweeps each one's y is the other
// one's x).  Returns false, having launched nothing, when the vectors do not fit one workgroup's LDS.
template <typename T>
bool launch_kacz_lds(const KaczArgs<T>* halves, const int* const* cptr, const int* ncol, const int* nx, int nhalf,
                     int nsweeps, hipStream_t s);

// Column reductions: partial sums over a fixed grid, then a fixed-order finalisation.
// value_ic = (K ? (K z)_ic : z_ic) - (y ? s_c y_ic : 0);  acc_c += a ? a_ic * value_ic : value_ic^2
template <typename T>
struct DotArgs {
  int nrows = 0, w = 0;
  const T* a = nullptr;
  const int* Krp = nullptr; const int* Kci = nullptr; const T* Kv = nullptr;
  const T* z = nullptr;
  const T* y = nullptr; const double* sig = nullptr;
  int nnzK = -1;
};
// Column reductions and the Gram product: partials per workgroup, then a fixed-order finalisation
// launch (bitwise reproducible).
template <typename T> void launch_dots(const DotArgs<T>& a, double* partial, double* out, hipStream_t s);
int dots_grid(int nrows, int w);
// largest reduction grids: a partial buffer of DOTS_MAX_GRID * 16 (dots) or GRAM_MAX_GRID * 256 (Gram)
// doubles serves every launch
constexpr int DOTS_MAX_GRID = 8192;
constexpr int GRAM_MAX_GRID = 2048;
constexpr size_t PARTIAL_DOUBLES = (size_t)GRAM_MAX_GRID * 256;

void launch_gram(int rows, int w, const double* X, const double* Y, double* partial, double* G, hipStream_t s);
// two independent reductions / Gram products in one launch (each with its own partials and output)
template <typename T>
void launch_dots2(const DotArgs<T>& a, double* pa, double* oa, const DotArgs<T>& b, double* pb, double* ob,
                  hipStream_t s);
void launch_gram2(int w, int rows_a, const double* Xa, const double* Ya, double* pa, double* Ga, int rows_b,
                  const double* Xb, const double* Yb, double* pb, double* Gb, hipStream_t s);
int gram_grid(int rows);

template <typename T>
void launch_rotate(int rows, int win, int wout, const T* X, const double* S, T* out, hipStream_t s);
// out_a = X_a S_a and out_b = X_b S_b (w x w) in one launch
template <typename T>
void launch_rotate2(int w, int rows_a, const T* Xa, const double* Sa, T* outa, int rows_b, const T* Xb,
                    const double* Sb, T* outb, hipStream_t s);
template <typename T>
void launch_gather_rows(int nout, int w, const int* idx, const T* X, T* out, hipStream_t s);
template <typename T>
void launch_scale_cols(int rows, int w, T* X, const double* d, int mode, hipStream_t s);
void launch_rq_update(int w, const double* num, const double* nu, const double* nv, double* sig,
                      double* flip, hipStream_t s);
void launch_fill(double* p, size_t n, double val, hipStream_t s);
void launch_axpby(size_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t s);
// out = Y + alpha X S (rows x w blocks, S w x w row-major, w <= 16); out may be Y, not X
void launch_rotate_acc(int rows, int w, const double* X, const double* S, double alpha, const double* Y, double* out,
                       hipStream_t s);
// the leading wr x wc part of a w x w block G into the ld-wide row-major M at (r0, c0); sym also at
// (c0, r0) transposed
void launch_place_block(int w, int wr, int wc, const double* G, double* M, int ld, int r0, int c0, int sym,
                        hipStream_t s);
// dst (rows x w) = the columns idx[0..n) of src (rows x w), then zero columns (w <= 16)
void launch_gather_cols(int rows, int w, const int* idx, int n, const double* src, double* dst, hipStream_t s);
void launch_eye(int k, double* M, hipStream_t s);
// rowC[k] = i for the entries k of row i of an m-row CSR pattern
void launch_row_index(int m, const int* rp, int* rowC, hipStream_t s);
// rowC[k] = the row of entry e0 + k (k < cnt) of a CSR pattern whose rows [r0, r1) hold those entries
void launch_row_index_range(int r0, int r1, const int* rp, long e0, long cnt, int* rowC, hipStream_t s);
// top-s rule (§3.7) per row of a strength operator chunk: rows [r0, r1), entries rp[i] - e0 ..
// rp[i + 1] - e0 of col / val; out (rows x s): the selected (j, n_ij) ascending in j, -1 after
void launch_topsel(int r0, int r1, const int* rp, long e0, const int* col, const double* val, int s, int* out_col,
                   double* out_val, hipStream_t st);
void launch_fillf(float* p, size_t n, float val, hipStream_t s);
void launch_copy_cast_df(const double* in, float* out, size_t n, hipStream_t s);
// FP64 -> BF16 bit patterns (out: n 16-bit words), rounded to FP32 and then to the nearest BF16
void launch_cast_bf16(const double* in, void* out, size_t n, hipStream_t s);
void launch_copy_cast_fd(const float* in, double* out, size_t n, hipStream_t s);
void launch_axpy_fd(const float* in, double* out, size_t n, hipStream_t s);   // out += in
void launch_splitmix_block(long ru, long rv, int w, unsigned long long seed, double* U, double* V, hipStream_t s);
void launch_sign_argmax(int rows, int ncols, int w, const double* X, double* sgn, hipStream_t s);
void launch_scatter_out(int rows, int ncols, int w, const double* X, const int* keep, const double* sgn, double* out,
                        long ld, hipStream_t s);
void launch_recip(int n, const double* in, double* out, hipStream_t s);
void launch_perm_gather(int n, const int* perm, const double* in, double* out, hipStream_t s);
void launch_spgemm_dot(int nnz, const int* rowC, const int* colC, const int* rpL, const int* ciL,
                       const double* vL, const int* rpR, const int* ciR, const double* vR, double* out,
                       hipStream_t s);
void launch_diag_inv(int m, const int* rp, const int* ci, const double* v, double* dinv, hipStream_t s);
void launch_row_sq(int m, const int* rp, const double* v, const double* bv, double* aa, double* ab,
                   double* bb, const int* ci, hipStream_t s);
void launch_csr_to_dense(int m, const int* rp, const int* ci, const double* v, double* D, int ld,
                         int roff, int coff, bool transpose, hipStream_t s);
void launch_ls_fit(int nF, const int* Fpts, const int* prp, const int* fine_cols, int w1,
                   const double* U1, int w2, const double* U2, const double* B1, const double* B2,
                   const double* wts, double* pval, int qmax, hipStream_t s);
// LS weights of the fitted pairs (R19), each multiplied by scale[c] when scale is given
void launch_rq_weights(int nf, const double* num, const double* nu, const double* nv, int minimal,
                       double floor_abs, const double* scale, double* w, hipStream_t s);

// dense.hip (single-workgroup dense FP64 procedures)
void launch_chol_inv_upper(int w, const double* G, double* T, int* status, hipStream_t s);
// the same; *pivot_min = the smallest of the first wpiv pivots of the unshifted factorisation of
// the column-scaled matrix, -1 when it failed within them
void launch_chol_inv_upper_pivot(int w, int wpiv, const double* G, double* T, int* status, double* pivot_min,
                                 hipStream_t s);
// two factorisations (G0 -> T0, G1 -> T1) in one launch
void launch_chol_inv_upper2(int w, const double* G0, double* T0, const double* G1, double* T1, int* status,
                            hipStream_t s);
// SVD of a k x k projected matrix (k <= 32), the nb triplets in target order: Y, Z (k x nb), sig
void launch_proj_svd(int k, int nb, int minimal, const double* M, double* Y, double* Z, double* sig, hipStream_t s);
void launch_small_ritz(int w, int spd, int minimal, const double* M, double* Y, double* Z, double* sig,
                       double* work, int* status, hipStream_t s);
void launch_coarse_gsvd(int spd, int minimal, int mL, int nL, int nb, double* A, double* B, double* C,
                        double* work, double* sig, double* U, double* V, int* status, hipStream_t s);
// basis: nb N^2 eigenvector store; warm = 1 reuses it from the previous call (same X, Y, nearby sigma)
void launch_pinv_solve(int N, int nb, const double* X, const double* Y, const double* sig,
                       const double* rhs, double* out, double* work, double* basis, int warm, int* status,
                       hipStream_t s);
void launch_pencil_setup(int N, double* X, double* Y, double* mu, double* Z, double* work,
                         int* status, hipStream_t s);
void launch_pencil_solve(int N, int nb, const double* mu, const double* Z, const double* sig,
                         const double* rhs, double* out, hipStream_t s);
void launch_dense_sym_eig(int n, double* A, double* V, double* lam, int* status, hipStream_t s);

}  // namespace slamg
