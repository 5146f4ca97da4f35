// Step-level C entry points (include/slamg_ops.h): one step of the cycles on caller buffers,
// with the kernels the solver uses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/slamg_ops.h"
#include "graph.h"
#include "solver.h"

using namespace slamg;

namespace {

struct Tmp {
  std::vector<void*> p;
  ~Tmp() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  T* get(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw SolverError{ST_E_OOM, "hipMalloc"};
    p.push_back(q);
    return (T*)q;
  }
};

#define OPCHK(x)                                                                        \
  do {                                                                                  \
    if ((x) != hipSuccess) throw SolverError{ST_E_DEVICE, #x};                          \
  } while (0)

template <class F>
slamg_status guarded(hipStream_t s, F&& f) {
  try {
    f();
    OPCHK(hipGetLastError());
    OPCHK(hipStreamSynchronize(s));
    return SLAMG_OK;
  } catch (const SolverError& e) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    return (slamg_status)e.code;
  } catch (...) {
    return SLAMG_E_OOM;
  }
}

template <class T>
void up(T* d, const T* h, size_t n, hipStream_t s) {
  if (n) OPCHK(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
void down(T* h, const T* d, size_t n, hipStream_t s) {
  if (n) OPCHK(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  OPCHK(hipStreamSynchronize(s));
}

bool bad_w(int w) { return w < 1 || w > 16; }

// Nonzero count of a device CSR operator (its last row pointer); chooses the kernels' row split.
int dev_nnz(const int* rp, int m, hipStream_t s) {
  if (!rp || m <= 0) return -1;
  int v = 0;
  down(&v, rp + m, 1, s);
  return v;
}

// one Jacobi-type half step: out = x + D (a K z - w M y ...) then optional normalisation; copy to x
void jac_half(hipStream_t s, Tmp& t, int rows, int w, const int* krp, const int* kci, const double* kv,
              const double* z, int mmode, const int* mrp, const int* mci, const double* mv, double* x,
              const double* kap, const double* sig, int cmode, double omega, bool normalise) {
  double* dinv = nullptr;
  if (mmode != M_IDENT) {
    dinv = t.get<double>(rows);
    if (mmode == M_SHARED) launch_diag_inv(rows, krp, kci, mv, dinv, s);
    else launch_diag_inv(rows, mrp, mci, mv, dinv, s);
  }
  double* out = t.get<double>((size_t)rows * w);
  RowOpArgs<double> a;
  a.nrows = rows; a.w = w; a.Krp = krp; a.Kci = kci; a.Kv = kv; a.z = z;
  a.mmode = mmode; a.Mrp = mrp; a.Mci = mci; a.Mv = mv; a.y = x; a.x = x; a.D = dinv; a.kap = kap; a.sig = sig;
  a.cmode = cmode; a.omega = omega; a.out = out;
  a.nnzK = dev_nnz(krp, rows, s);
  if (mmode == M_CSR && rows > 0) a.avgM = (double)dev_nnz(mrp, rows, s) / rows;
  launch_rowop(a, s);
  if (normalise) {
    double* part = t.get<double>((size_t)DOTS_MAX_GRID * 16);
    double* nrm = t.get<double>(16);
    DotArgs<double> d;
    d.nrows = rows; d.w = w; d.a = out; d.z = out;
    if (mmode == M_SHARED) { d.Krp = krp; d.Kci = kci; d.Kv = mv; d.nnzK = a.nnzK; }
    if (mmode == M_CSR) { d.Krp = mrp; d.Kci = mci; d.Kv = mv; d.nnzK = dev_nnz(mrp, rows, s); }
    launch_dots(d, part, nrm, s);
    launch_scale_cols<double>(rows, w, out, nrm, 0, s);
  }
  OPCHK(hipMemcpyAsync(x, out, sizeof(double) * rows * w, hipMemcpyDeviceToDevice, s));
}

}  // namespace

extern "C" slamg_status slamg_op_spmm(int32_t m, int32_t w, const int32_t* d_rp, const int32_t* d_ci,
                                      const double* d_v, const double* d_x, double* d_y, double beta, void* stream) {
  if (m < 0 || bad_w(w)) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] { launch_spmm<double>(m, w, d_rp, d_ci, d_v, d_x, d_y, beta, s, dev_nnz(d_rp, m, s)); });
}

extern "C" slamg_status slamg_op_spmm_f32(int32_t m, int32_t w, const int32_t* d_rp, const int32_t* d_ci,
                                          const float* d_v, const float* d_x, float* d_y, double beta, void* stream) {
  if (m < 0 || bad_w(w)) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] { launch_spmm<float>(m, w, d_rp, d_ci, d_v, d_x, d_y, beta, s, dev_nnz(d_rp, m, s)); });
}

extern "C" slamg_status slamg_op_spmm_bf16(int32_t m, int32_t w, const int32_t* d_rp, const int32_t* d_ci,
                                           const uint16_t* d_v, const float* d_x, float* d_y, double beta,
                                           void* stream) {
  if (m < 0 || bad_w(w)) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    launch_spmm<float>(m, w, d_rp, d_ci, reinterpret_cast<const float*>(d_v), d_x, d_y, beta, s, dev_nnz(d_rp, m, s), 1);
  });
}

extern "C" slamg_status slamg_op_cast_bf16(int64_t n, const double* d_in, uint16_t* d_out, void* stream) {
  if (n < 0 || (n > 0 && (!d_in || !d_out))) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] { launch_cast_bf16(d_in, d_out, (size_t)n, s); });
}

extern "C" slamg_status slamg_op_relax_test(int32_t spd, int32_t m, int32_t n, int32_t w, const int32_t* d_arp,
                                            const int32_t* d_aci, const double* d_av, const int32_t* d_atrp,
                                            const int32_t* d_atci, const double* d_atv, const int32_t* d_brp,
                                            const int32_t* d_bci, const double* d_bv, const int32_t* d_crp,
                                            const int32_t* d_cci, const double* d_cv, double omega, double* d_u,
                                            double* d_v, void* stream) {
  if (m < 1 || n < 1 || bad_w(w) || (spd && m != n)) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    if (spd) {
      jac_half(s, t, m, w, d_arp, d_aci, d_av, d_u, d_bv ? M_SHARED : M_IDENT, nullptr, nullptr, d_bv, d_u,
               nullptr, nullptr, C_JAC_TEST, omega, true);
    } else {
      jac_half(s, t, n, w, d_atrp, d_atci, d_atv, d_u, d_cv ? M_CSR : M_IDENT, d_crp, d_cci, d_cv, d_v, nullptr,
               nullptr, C_JAC_TEST, omega, true);
      jac_half(s, t, m, w, d_arp, d_aci, d_av, d_v, d_bv ? M_CSR : M_IDENT, d_brp, d_bci, d_bv, d_u, nullptr,
               nullptr, C_JAC_TEST, omega, true);
    }
  });
}

extern "C" slamg_status slamg_op_relax_boot(int32_t spd, int32_t m, int32_t n, int32_t w, const int32_t* d_arp,
                                            const int32_t* d_aci, const double* d_av, const int32_t* d_atrp,
                                            const int32_t* d_atci, const double* d_atv, const int32_t* d_brp,
                                            const int32_t* d_bci, const double* d_bv, const int32_t* d_crp,
                                            const int32_t* d_cci, const double* d_cv, const double* d_sig,
                                            const double* d_kap, const double* d_tau, double omega, double* d_u,
                                            double* d_v, void* stream) {
  if (m < 1 || n < 1 || bad_w(w) || (spd && m != n) || !d_sig) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    if (spd) {
      jac_half(s, t, m, w, d_arp, d_aci, d_av, d_u, d_bv ? M_SHARED : M_IDENT, nullptr, nullptr, d_bv, d_u, d_kap,
               d_sig, C_JAC_BOOT, omega, false);
    } else {
      jac_half(s, t, m, w, d_arp, d_aci, d_av, d_v, d_bv ? M_CSR : M_IDENT, d_brp, d_bci, d_bv, d_u, d_kap, d_sig,
               C_JAC_BOOT, omega, false);
      jac_half(s, t, n, w, d_atrp, d_atci, d_atv, d_u, d_cv ? M_CSR : M_IDENT, d_crp, d_cci, d_cv, d_v, d_tau,
               d_sig, C_JAC_BOOT, omega, false);
    }
  });
}

extern "C" slamg_status slamg_op_kaczmarz(int32_t nrows, int32_t ncols, int32_t w, const int32_t* d_rp,
                                          const int32_t* d_ci, const double* d_v, const double* d_bv,
                                          const double* d_lam, const int32_t* h_rows, const int32_t* h_cptr,
                                          int32_t ncolours, const double* d_rhs, double* d_x, void* stream) {
  if (nrows < 0 || ncols < 1 || bad_w(w) || ncolours < 0 || !h_cptr) return SLAMG_E_INVALID;
  if (d_lam && !d_bv && nrows != ncols) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    double* aa = t.get<double>(nrows);
    double* ab = t.get<double>(nrows);
    double* bb = t.get<double>(nrows);
    launch_row_sq(nrows, d_rp, d_v, d_bv, aa, ab, bb, d_ci, s);
    const int total = h_cptr[ncolours];
    const long nnz = dev_nnz(d_rp, nrows, s);
    int* rows = t.get<int>(total);
    up(rows, h_rows, total, s);
    for (int c = 0; c < ncolours; ++c) {
      KaczArgs<double> k;
      k.nrows = h_cptr[c + 1] - h_cptr[c]; k.rows = rows + h_cptr[c]; k.w = w;
      k.rp = d_rp; k.ci = d_ci; k.av = d_v; k.bv = d_bv; k.lam = d_lam;
      k.rn_aa = aa; k.rn_ab = ab; k.rn_bb = bb; k.kap = d_rhs; k.x = d_x;
      k.nnz_total = nnz; k.nnz_rows = nrows;
      launch_kacz(k, s);
    }
  });
}

extern "C" slamg_status slamg_op_residual(int32_t nrows, int32_t w, const int32_t* d_krp, const int32_t* d_kci,
                                          const double* d_kv, const double* d_z, const int32_t* d_mrp,
                                          const int32_t* d_mci, const double* d_mv, const double* d_y,
                                          const double* d_kap, const double* d_sig, double* d_out, void* stream) {
  if (nrows < 0 || bad_w(w) || !d_sig) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    RowOpArgs<double> a;
    a.nrows = nrows; a.w = w; a.Krp = d_krp; a.Kci = d_kci; a.Kv = d_kv; a.z = d_z;
    a.mmode = d_mv ? M_CSR : M_IDENT; a.Mrp = d_mrp; a.Mci = d_mci; a.Mv = d_mv; a.y = d_y;
    a.kap = d_kap; a.sig = d_sig; a.cmode = C_RESID; a.out = d_out;
    a.nnzK = dev_nnz(d_krp, nrows, s);
    if (d_mv && nrows > 0) a.avgM = (double)dev_nnz(d_mrp, nrows, s) / nrows;
    launch_rowop(a, s);
  });
}

extern "C" slamg_status slamg_op_dots(int32_t nrows, int32_t w, const double* d_a, const int32_t* d_krp,
                                      const int32_t* d_kci, const double* d_kv, const double* d_z, const double* d_y,
                                      const double* d_sig, double* h_out, void* stream) {
  if (nrows < 0 || bad_w(w) || !h_out) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    double* part = t.get<double>((size_t)DOTS_MAX_GRID * 16);
    double* out = t.get<double>(16);
    DotArgs<double> d;
    d.nrows = nrows; d.w = w; d.a = d_a; d.Krp = d_krp; d.Kci = d_kci; d.Kv = d_kv; d.z = d_z; d.y = d_y;
    d.sig = d_sig;
    if (d_kv) d.nnzK = dev_nnz(d_krp, nrows, s);
    launch_dots(d, part, out, s);
    down(h_out, out, w, s);
  });
}

extern "C" slamg_status slamg_op_gram(int32_t rows, int32_t w, const double* d_x, const double* d_y, double* h_g,
                                      void* stream) {
  if (rows < 0 || bad_w(w) || !h_g) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    double* part = t.get<double>((size_t)gram_grid(rows) * 256);
    double* G = t.get<double>(256);
    launch_gram(rows, w, d_x, d_y, part, G, s);
    down(h_g, G, (size_t)w * w, s);
  });
}

extern "C" slamg_status slamg_op_ritz(int32_t spd, int32_t minimal, int32_t m, int32_t n, int32_t w,
                                      const int32_t* d_arp, const int32_t* d_aci, const double* d_av, double* d_u,
                                      double* d_v, double* h_sig, void* stream) {
  if (m < 1 || n < 1 || bad_w(w) || (spd && m != n) || !h_sig) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    double* part = t.get<double>((size_t)std::max(gram_grid(std::max(m, n)), 1) * 256);
    double* G = t.get<double>(256);
    double* T1 = t.get<double>(256);
    double* T2 = t.get<double>(256);
    double* work = t.get<double>(4 * 32 * 32);
    double* sig = t.get<double>(16);
    int* status = t.get<int>(1);
    OPCHK(hipMemsetAsync(status, 0, sizeof(int), s));
    auto cholqr2 = [&](double* X, int rows, double* tmp, double* out) {
      launch_gram(rows, w, X, X, part, G, s);
      launch_chol_inv_upper(w, G, T1, status, s);
      launch_rotate<double>(rows, w, w, X, T1, tmp, s);
      launch_gram(rows, w, tmp, tmp, part, G, s);
      launch_chol_inv_upper(w, G, T1, status, s);
      launch_rotate<double>(rows, w, w, tmp, T1, out, s);
    };
    double* tU = t.get<double>((size_t)m * w);
    double* Uh = t.get<double>((size_t)m * w);
    double* W = t.get<double>((size_t)m * w);
    if (spd) {
      cholqr2(d_u, m, tU, Uh);
      launch_spmm<double>(m, w, d_arp, d_aci, d_av, Uh, W, 0.0, s);
      launch_gram(m, w, Uh, W, part, G, s);
      launch_small_ritz(w, 1, minimal, G, T1, T2, sig, work, status, s);
      launch_rotate<double>(m, w, w, Uh, T1, d_u, s);
    } else {
      // the U- and V-side Cholesky-QR2 in paired launches, as the solver runs them
      double* tV = t.get<double>((size_t)n * w);
      double* Vh = t.get<double>((size_t)n * w);
      double* part2 = t.get<double>((size_t)std::max(gram_grid(std::max(m, n)), 1) * 256);
      double* G2 = t.get<double>(256);
      double* T3 = t.get<double>(256);
      launch_gram2(w, m, d_u, d_u, part, G, n, d_v, d_v, part2, G2, s);
      launch_chol_inv_upper2(w, G, T1, G2, T3, status, s);
      launch_rotate2<double>(w, m, d_u, T1, tU, n, d_v, T3, tV, s);
      launch_gram2(w, m, tU, tU, part, G, n, tV, tV, part2, G2, s);
      launch_chol_inv_upper2(w, G, T1, G2, T3, status, s);
      launch_rotate2<double>(w, m, tU, T1, Uh, n, tV, T3, Vh, s);
      launch_spmm<double>(m, w, d_arp, d_aci, d_av, Vh, W, 0.0, s);
      launch_gram(m, w, Uh, W, part, G, s);
      launch_small_ritz(w, 0, minimal, G, T1, T2, sig, work, status, s);
      launch_rotate2<double>(w, m, Uh, T1, d_u, n, Vh, T2, d_v, s);
    }
    int st = 0;
    down(&st, status, 1, s);
    if (st) throw SolverError{ST_E_NUMERIC, "Cholesky-QR breakdown"};
    down(h_sig, sig, w, s);
  });
}

extern "C" slamg_status slamg_op_ls_fit(int32_t npts, const int32_t* h_ptr, const int32_t* h_fine_cols,
                                        const int8_t* h_is_c, int32_t w1, const double* d_u1, const double* d_b1,
                                        int32_t w2, const double* d_u2, const double* d_b2, const double* d_wts,
                                        double* h_pval, void* stream) {
  if (npts < 1 || w1 < 1 || w2 < 0 || w1 + w2 > 32 || !h_ptr || !h_fine_cols || !h_is_c) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    Tmp t;
    const int nnz = h_ptr[npts];
    std::vector<int> F;
    int qmax = 0;
    std::vector<double> pv(nnz, 0.0);
    for (int i = 0; i < npts; ++i) {
      if (h_is_c[i]) { pv[h_ptr[i]] = 1.0; continue; }
      F.push_back(i);
      qmax = std::max(qmax, h_ptr[i + 1] - h_ptr[i]);
    }
    if (qmax > 16) throw SolverError{ST_E_INVALID, "interpolatory set larger than 16"};
    int* dF = t.get<int>(F.size());
    int* dptr = t.get<int>(npts + 1);
    int* dfc = t.get<int>(nnz);
    double* dp = t.get<double>(nnz);
    up(dF, F.data(), F.size(), s);
    up(dptr, h_ptr, npts + 1, s);
    up(dfc, h_fine_cols, nnz, s);
    up(dp, pv.data(), nnz, s);
    launch_ls_fit((int)F.size(), dF, dptr, dfc, w1, d_u1, w2, d_u2, d_b1 ? d_b1 : d_u1, d_b2 ? d_b2 : d_u2, d_wts,
                  dp, qmax, s);
    down(h_pval, dp, nnz, s);
  });
}

extern "C" slamg_status slamg_op_spgemm(int32_t nnz, const int32_t* d_rowc, const int32_t* d_colc,
                                        const int32_t* d_lrp, const int32_t* d_lci, const double* d_lv,
                                        const int32_t* d_rtrp, const int32_t* d_rtci, const double* d_rtv,
                                        double* d_out, void* stream) {
  if (nnz < 0) return SLAMG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    launch_spgemm_dot(nnz, d_rowc, d_colc, d_lrp, d_lci, d_lv, d_rtrp, d_rtci, d_rtv, d_out, s);
  });
}

extern "C" slamg_status slamg_op_topsel(int32_t m, const int32_t* d_rp, const int32_t* d_col, const double* d_val,
                                        int32_t s, int32_t* d_out_col, double* d_out_val, void* stream) {
  if (m < 0 || s < 1 || s > 16) return SLAMG_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  return guarded(st, [&] { launch_topsel(0, m, d_rp, 0, d_col, d_val, s, d_out_col, d_out_val, st); });
}

extern "C" slamg_status slamg_op_coarse_gsvd(int32_t spd, int32_t minimal, int32_t mL, int32_t nL, int32_t nb,
                                             const double* h_a, const double* h_b, const double* h_c, double* h_sig,
                                             double* h_u, double* h_v) {
  if (mL < 1 || nL < 1 || nb < 1 || nb > 64 || (spd && mL != nL) || nb > std::min(mL, nL) || mL > 1024 ||
      nL > 1024)
    return SLAMG_E_INVALID;
  hipStream_t s = nullptr;
  return guarded(s, [&] {
    Tmp t;
    const size_t mx = std::max(mL, nL);
    double* A = t.get<double>((size_t)mL * nL);
    double* B = t.get<double>((size_t)mL * mL);
    double* C = t.get<double>((size_t)nL * nL);
    double* work = t.get<double>(3 * mx * mx + 2 * (size_t)mL * nL + 64 * mx + mx);
    double* sig = t.get<double>(nb);
    double* U = t.get<double>((size_t)mL * nb);
    double* V = t.get<double>((size_t)nL * nb);
    int* status = t.get<int>(1);
    OPCHK(hipMemsetAsync(status, 0, sizeof(int), s));
    up(A, h_a, (size_t)mL * nL, s);
    up(B, h_b, (size_t)mL * mL, s);
    if (!spd) up(C, h_c, (size_t)nL * nL, s);
    launch_coarse_gsvd(spd, minimal, mL, nL, nb, A, B, spd ? nullptr : C, work, sig, U, spd ? nullptr : V, status,
                       s);
    int st = 0;
    down(&st, status, 1, s);
    if (st) throw SolverError{ST_E_NUMERIC, "Cholesky breakdown"};
    down(h_sig, sig, nb, s);
    down(h_u, U, (size_t)mL * nb, s);
    if (!spd && h_v) down(h_v, V, (size_t)nL * nb, s);
  });
}

extern "C" slamg_status slamg_op_proj_svd(int32_t minimal, int32_t k, int32_t nb, const double* h_m, double* h_sig,
                                          double* h_y, double* h_z) {
  if (k < 1 || k > 32 || nb < 1 || nb > k || !h_m || !h_sig || !h_y || !h_z) return SLAMG_E_INVALID;
  hipStream_t s = nullptr;
  return guarded(s, [&] {
    Tmp t;
    double* M = t.get<double>((size_t)k * k);
    double* Y = t.get<double>((size_t)k * nb);
    double* Z = t.get<double>((size_t)k * nb);
    double* sig = t.get<double>(nb);
    up(M, h_m, (size_t)k * k, s);
    launch_proj_svd(k, nb, minimal ? 1 : 0, M, Y, Z, sig, s);
    down(h_sig, sig, nb, s);
    down(h_y, Y, (size_t)k * nb, s);
    down(h_z, Z, (size_t)k * nb, s);
  });
}

extern "C" slamg_status slamg_op_coarse_solve(int32_t variant, int32_t N, int32_t nb, const double* h_x,
                                              const double* h_y, const double* h_sig, const double* h_rhs,
                                              double* h_out) {
  if (N < 1 || N > 1024 || nb < 1 || nb > 16 || (variant < 0 || variant > 5)) return SLAMG_E_INVALID;
  hipStream_t s = nullptr;
  return guarded(s, [&] {
    Tmp t;
    double* X = t.get<double>((size_t)N * N);
    double* Y = t.get<double>((size_t)N * N);
    double* sig = t.get<double>(nb);
    double* rhs = t.get<double>((size_t)N * nb);
    double* out = t.get<double>((size_t)N * nb);
    int* status = t.get<int>(1);
    OPCHK(hipMemsetAsync(status, 0, sizeof(int), s));
    up(X, h_x, (size_t)N * N, s);
    up(Y, h_y, (size_t)N * N, s);
    up(sig, h_sig, nb, s);
    up(rhs, h_rhs, (size_t)N * nb, s);
    if (variant != 1) {
      double* work = t.get<double>((size_t)nb * 2 * N * N);
      double* basis = t.get<double>((size_t)nb * N * N);
      const bool warm = variant >= 2;
      if (warm) {
        // warm start: eigenvectors of X - sigma'_j Y at sigma'_j = sigma_j (1 + delta) first
        const double delta = (variant == 2 || variant == 5) ? 1e-6 : variant == 3 ? 1e-12 : 1e-3;
        double* sig2 = t.get<double>(nb);
        std::vector<double> h2(h_sig, h_sig + nb);
        for (auto& v : h2) v *= 1.0 + delta;
        up(sig2, h2.data(), nb, s);
        launch_pinv_solve(N, nb, X, Y, sig2, rhs, out, work, basis, 0, status, s);
      }
      launch_pinv_solve(N, nb, X, Y, sig, rhs, out, work, basis, warm ? (variant == 5 ? 2 : 1) : 0, status, s);
    } else {
      double* mu = t.get<double>(N);
      double* Z = t.get<double>((size_t)N * N);
      double* work = t.get<double>((size_t)2 * N * N);
      launch_pencil_setup(N, X, Y, mu, Z, work, status, s);
      launch_pencil_solve(N, nb, mu, Z, sig, rhs, out, s);
    }
    int st = 0;
    down(&st, status, 1, s);
    if (st) throw SolverError{ST_E_NUMERIC, "Cholesky breakdown"};
    down(h_out, out, (size_t)N * nb, s);
  });
}

// ------------------------------------------------------------------------------------------------
// host graph entry points
// ------------------------------------------------------------------------------------------------
static HCsr host_csr(int m, int n, const int32_t* rp, const int32_t* ci, const double* v) {
  HCsr h;
  h.m = m; h.n = n;
  h.rp.assign(rp, rp + m + 1);
  h.ci.assign(ci, ci + rp[m]);
  if (v) h.v.assign(v, v + rp[m]);
  return h;
}

extern "C" slamg_status slamg_graph_strength(int32_t n, const int32_t* h_rp, const int32_t* h_ci, const double* h_v,
                                             double theta, int32_t rule, int32_t top_s, int32_t* h_sp,
                                             int32_t* h_si) {
  if (n < 0 || !h_rp || !h_sp || rule < 0 || rule > 2) return SLAMG_E_INVALID;
  HCsr N = host_csr(n, n, h_rp, h_ci, h_v);
  std::vector<int> Sp, Si;
  strength_sets(N, theta, rule, top_s, Sp, Si);
  std::copy(Sp.begin(), Sp.end(), h_sp);
  std::copy(Si.begin(), Si.end(), h_si);
  return SLAMG_OK;
}

extern "C" slamg_status slamg_graph_rs(int32_t n, const int32_t* h_sp, const int32_t* h_si, int8_t* h_is_c) {
  if (n < 0 || !h_sp || !h_is_c) return SLAMG_E_INVALID;
  std::vector<int> Sp(h_sp, h_sp + n + 1), Si(h_si, h_si + h_sp[n]);
  auto c = rs_coarsen(Sp, Si, n);
  for (int i = 0; i < n; ++i) h_is_c[i] = c[i];
  return SLAMG_OK;
}

extern "C" slamg_status slamg_graph_interp(int32_t n, const int32_t* h_sp, const int32_t* h_si, const int32_t* h_rp,
                                           const int32_t* h_ci, const double* h_v, const int8_t* h_is_c, int32_t cap,
                                           int32_t* h_ptr, int32_t* h_cols, int32_t* h_capped) {
  if (n < 0 || cap < 1 || !h_ptr || !h_cols) return SLAMG_E_INVALID;
  std::vector<int> Sp(h_sp, h_sp + n + 1), Si(h_si, h_si + h_sp[n]);
  HCsr N = host_csr(n, n, h_rp, h_ci, h_v);
  std::vector<char> isc(h_is_c, h_is_c + n);
  std::vector<int> ptr, cols;
  int capped = 0;
  interp_pattern(Sp, Si, N, isc, cap, ptr, cols, capped);
  std::copy(ptr.begin(), ptr.end(), h_ptr);
  std::copy(cols.begin(), cols.end(), h_cols);
  if (h_capped) *h_capped = capped;
  return SLAMG_OK;
}

extern "C" slamg_status slamg_graph_colour(int32_t m, int32_t n, const int32_t* h_rp, const int32_t* h_ci,
                                           int32_t* h_colour) {
  if (m < 0 || n < 0 || !h_rp || !h_colour) return SLAMG_E_INVALID;
  HCsr A = host_csr(m, n, h_rp, h_ci, nullptr);
  auto c = greedy_row_colouring(A);
  std::copy(c.begin(), c.end(), h_colour);
  return SLAMG_OK;
}
