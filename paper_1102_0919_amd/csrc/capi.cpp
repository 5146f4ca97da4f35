// C ABI of the solver (include/slamg.h): validation, problem preparation (transposition when
// m < n, removal of empty rows and columns), output conventions and the request queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>

#include "../../include/slamg.h"
#include "graph.h"
#include "solver.h"

using namespace slamg;

struct Request {
  uint64_t id = 0;
  slamg_csr A{};
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  slamg_kind kind = SLAMG_SVD;
  slamg_target target = SLAMG_DOMINANT;
  int32_t nb = 1;
  slamg_params p{};
  bool done = false;
  slamg_status status = SLAMG_OK;
  std::vector<double> sigma, U, V;
  slamg_report rep{};
  // serving loop
  size_t est = 0;                                       // admission estimate of the footprint
  std::string err;
  std::chrono::steady_clock::time_point t_submit, t_start;
};

struct slamg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  std::string err;
  uint64_t next_id = 1;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  // serving loop: worker threads, one HIP stream each; queue, reqs and the fields below are
  // guarded by mu once it runs
  std::mutex mu;
  std::condition_variable cv;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> wstreams;
  bool serving = false, stopping = false;
  size_t reserved = 0;     // admission estimates of the running requests
  int running = 0;
};

static slamg_status fail(slamg_ctx* c, slamg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}
static slamg_status fail(std::string& err, slamg_status s, const std::string& msg) {
  err = msg;
  return s;
}

// Where a solve runs: device, stream, device-memory budget of its arena.
struct Exec {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
};
static Exec exec_of(const slamg_ctx* c) { return Exec{c->device, c->stream, c->budget}; }

extern "C" slamg_status slamg_params_init(slamg_params* p, slamg_kind kind, slamg_target target) {
  if (!p) return SLAMG_E_INVALID;
  std::memset(p, 0, sizeof(*p));
  p->theta = kind == SLAMG_SVD ? 0.05 : 0.06;
  p->strength_rule = 0;
  p->top_s = 4;
  p->df_filter = 0.0;
  p->n_t = 8;
  p->mu_t = 4;
  p->mu_b = 4;
  p->omega_J = 0.7;
  p->n_mult = 10;
  p->max_add = 200;
  p->coarse_max = 64;
  p->max_levels = 25;
  p->stall_ratio = 0.9;
  p->tol = 1e-8;
  p->seed = 1102;
  p->precision = SLAMG_FP64;
  p->ritz_in_mult = 1;
  p->coarse_pinv = 0;
  p->graphs = 1;
  p->n_guard = 0;
  p->mu_tJ = 1;
  p->mu_bJ = 1;
  p->kaczmarz_order = 0;
  p->coarse_dense_max = 1024;
  p->redo_p = 0;
  p->redo_tol = 1e-14;
  p->cycle_gamma = 1;
  p->ritz_coarse = 0;
  p->solve_phase = 0;
  p->fmg = 0;
  (void)target;
  return SLAMG_OK;
}

extern "C" slamg_status slamg_create(slamg_ctx** ctx, int device, void* hip_stream, size_t hbm_budget_bytes) {
  if (!ctx) return SLAMG_E_INVALID;
  *ctx = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SLAMG_E_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return SLAMG_E_DEVICE;
  auto* c = new slamg_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return SLAMG_E_DEVICE;
    }
    c->own_stream = true;
  }
  *ctx = c;
  return SLAMG_OK;
}

extern "C" slamg_status slamg_serve_stop(slamg_ctx* ctx);

extern "C" void slamg_destroy(slamg_ctx* ctx) {
  if (!ctx) return;
  (void)slamg_serve_stop(ctx);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

extern "C" const char* slamg_status_string(slamg_status s) {
  switch (s) {
    case SLAMG_OK: return "ok";
    case SLAMG_NOT_CONVERGED: return "not converged";
    case SLAMG_E_INVALID: return "invalid argument";
    case SLAMG_E_OOM: return "out of device memory";
    case SLAMG_E_BUDGET: return "HBM budget exceeded";
    case SLAMG_E_DEVICE: return "device error";
    case SLAMG_E_NUMERIC: return "numerical breakdown";
    case SLAMG_E_BUSY: return "busy";
  }
  return "unknown status";
}

extern "C" const char* slamg_last_error(const slamg_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

// Host copy of a (host or device) CSR with validation.
static slamg_status fetch_csr(slamg_ctx* c, const slamg_csr* A, std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                              std::vector<double>& v) {
  if (!A || A->m <= 0 || A->n <= 0 || A->nnz < 0 || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(c, SLAMG_E_INVALID, "invalid CSR descriptor");
  if (A->nnz >= (int64_t)INT32_MAX || A->m >= INT32_MAX || A->n >= INT32_MAX)
    return fail(c, SLAMG_E_INVALID, "matrix too large for 32-bit indices");
  rp.resize(A->m + 1);
  ci.resize(A->nnz);
  v.resize(A->nnz);
  if (A->on_device) {
    if (hipMemcpy(rp.data(), A->row_ptr, rp.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        (A->nnz && hipMemcpy(ci.data(), A->col_idx, ci.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
        (A->nnz && hipMemcpy(v.data(), A->val, v.size() * 8, hipMemcpyDeviceToHost) != hipSuccess))
      return fail(c, SLAMG_E_DEVICE, "copy of the device CSR failed");
  } else {
    std::memcpy(rp.data(), A->row_ptr, rp.size() * 8);
    if (A->nnz) {
      std::memcpy(ci.data(), A->col_idx, ci.size() * 4);
      std::memcpy(v.data(), A->val, v.size() * 8);
    }
  }
  if (rp[0] != 0 || rp[A->m] != A->nnz) return fail(c, SLAMG_E_INVALID, "row_ptr inconsistent with nnz");
  for (int64_t i = 0; i < A->m; ++i) {
    if (rp[i + 1] < rp[i]) return fail(c, SLAMG_E_INVALID, "row_ptr not monotone");
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= A->n) return fail(c, SLAMG_E_INVALID, "column index out of range");
      if (k > rp[i] && ci[k] <= ci[k - 1]) return fail(c, SLAMG_E_INVALID, "columns not sorted / duplicated");
      if (!std::isfinite(v[k])) return fail(c, SLAMG_E_INVALID, "non-finite value");
    }
  }
  return SLAMG_OK;
}

// Matrix prepared for the solver: m >= n after an optional transposition (SVD), empty rows and
// columns removed (eigenproblems: rows/columns empty in both), with the keep maps back to the
// caller's numbering.
struct Prepared {
  int kind = SLAMG_SVD;
  int64_t m0 = 0, n0 = 0;    // caller's sizes
  bool transposed = false;
  int64_t M = 0, N = 0;      // sizes after the transposition
  std::vector<int> rkeep, ckeep;
  HCsr A;
};

static slamg_status prepare(std::string& err, int64_t m0, int64_t n0, const std::vector<int64_t>& rp,
                            const std::vector<int32_t>& ci, const std::vector<double>& v, slamg_kind kind,
                            Prepared& P) {
  if (kind == SLAMG_SPD_EIG && m0 != n0) return fail(err, SLAMG_E_INVALID, "SPD kind needs a square matrix");
  HCsr A;
  A.m = (int)m0; A.n = (int)n0;
  A.rp.resize(m0 + 1);
  for (int64_t i = 0; i <= m0; ++i) A.rp[i] = (int)rp[i];
  A.ci.assign(ci.begin(), ci.end());
  A.v = v;
  P.kind = kind; P.m0 = m0; P.n0 = n0;
  P.transposed = false;
  if (kind == SLAMG_SVD && m0 < n0) {
    A = transpose(A, nullptr);
    P.transposed = true;
  }
  P.M = A.m; P.N = A.n;
  std::vector<int> colcnt(A.n, 0);
  for (int k = 0; k < A.nnz(); ++k) colcnt[A.ci[k]]++;
  P.rkeep.clear(); P.ckeep.clear();
  if (kind == SLAMG_SPD_EIG) {
    for (int i = 0; i < A.m; ++i)
      if (A.rp[i + 1] > A.rp[i] || colcnt[i] > 0) P.rkeep.push_back(i);
    P.ckeep = P.rkeep;
  } else {
    for (int i = 0; i < A.m; ++i)
      if (A.rp[i + 1] > A.rp[i]) P.rkeep.push_back(i);
    for (int j = 0; j < A.n; ++j)
      if (colcnt[j] > 0) P.ckeep.push_back(j);
  }
  if (P.rkeep.empty() || P.ckeep.empty()) return fail(err, SLAMG_E_INVALID, "matrix has no nonzero entries");
  std::vector<int> cmap(A.n, -1);
  for (size_t j = 0; j < P.ckeep.size(); ++j) cmap[P.ckeep[j]] = (int)j;
  P.A = HCsr();
  P.A.m = (int)P.rkeep.size(); P.A.n = (int)P.ckeep.size();
  P.A.rp.assign(1, 0);
  for (int i : P.rkeep) {
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      P.A.ci.push_back(cmap[A.ci[k]]);
      P.A.v.push_back(A.v[k]);
    }
    P.A.rp.push_back((int)P.A.ci.size());
  }
  if (kind == SLAMG_SPD_EIG) {
    for (int i = 0; i < P.A.m; ++i) {
      bool d = false;
      for (int k = P.A.rp[i]; k < P.A.rp[i + 1]; ++k) d |= P.A.ci[k] == i && P.A.v[k] > 0.0;
      if (!d) return fail(err, SLAMG_E_INVALID, "SPD kind needs a positive diagonal");
    }
  }
  return SLAMG_OK;
}

static slamg_status check_params(std::string& err, const Prepared& P, int32_t nb, const slamg_params& p) {
  if (nb < 1 || nb > 16) return fail(err, SLAMG_E_INVALID, "n_b must be in 1..16");
  if (p.n_guard < 0 || nb + p.n_guard > 16) return fail(err, SLAMG_E_INVALID, "n_b + n_guard must be in 1..16");
  if (p.mu_tJ < 1 || p.mu_bJ < 1) return fail(err, SLAMG_E_INVALID, "mu_tJ and mu_bJ must be at least 1");
  if (p.kaczmarz_order != 0 && p.kaczmarz_order != 1) return fail(err, SLAMG_E_INVALID, "unknown kaczmarz_order");
  if (p.coarse_dense_max < 1 || p.coarse_dense_max > 1024)
    return fail(err, SLAMG_E_INVALID, "coarse_dense_max must lie in 1 .. 1024");
  if (p.redo_p != 0 && p.redo_p != 1) return fail(err, SLAMG_E_INVALID, "redo_p must be 0 or 1");
  if (p.redo_p && !(p.redo_tol > 0.0 && p.redo_tol < 1.0)) return fail(err, SLAMG_E_INVALID, "redo_tol must lie in (0, 1)");
  if (p.cycle_gamma != 1 && p.cycle_gamma != 2) return fail(err, SLAMG_E_INVALID, "cycle_gamma must be 1 or 2");
  if (p.ritz_coarse != 0 && p.ritz_coarse != 1) return fail(err, SLAMG_E_INVALID, "ritz_coarse must be 0 or 1");
  if (p.solve_phase != 0 && p.solve_phase != 1) return fail(err, SLAMG_E_INVALID, "solve_phase must be 0 or 1");
  if (p.fmg != 0 && p.fmg != 1) return fail(err, SLAMG_E_INVALID, "fmg must be 0 or 1");
  if (!(p.tol > 0.0)) return fail(err, SLAMG_E_INVALID, "tol must be positive");
  if (p.n_t < 2 || p.n_t > 16) return fail(err, SLAMG_E_INVALID, "n_t must be in 2..16");
  if (p.mu_t < 0 || p.mu_b < 0 || p.n_mult < 1 || p.max_add < 0) return fail(err, SLAMG_E_INVALID, "bad counts");
  if (p.precision != SLAMG_FP64 && p.precision != SLAMG_MIXED_FP32 && p.precision != SLAMG_MIXED_BF16)
    return fail(err, SLAMG_E_INVALID, "unknown precision");
  if (p.coarse_pinv != 0 && p.coarse_pinv != 1) return fail(err, SLAMG_E_INVALID, "unknown coarse_pinv");
  if (p.square_coarsening != 0 && p.square_coarsening != 1)
    return fail(err, SLAMG_E_INVALID, "square_coarsening must be 0 or 1");
  if (p.square_coarsening && P.kind == SLAMG_SVD && P.A.m != P.A.n)
    return fail(err, SLAMG_E_INVALID, "square coarsening needs a square matrix without empty rows or columns");
  if (p.strength_rule < 0 || p.strength_rule > 2) return fail(err, SLAMG_E_INVALID, "unknown strength rule");
  if (p.strength_rule == 2 && (p.top_s < 1 || p.top_s > 16)) return fail(err, SLAMG_E_INVALID, "top_s must be in 1..16");
  if (nb > std::min(P.m0, P.n0)) return fail(err, SLAMG_E_INVALID, "n_b larger than min(m, n)");
  if (nb > std::min(P.A.m, P.A.n)) return fail(err, SLAMG_E_INVALID, "n_b larger than the nonzero part of A");
  if (nb + p.n_guard > std::min(P.A.m, P.A.n))
    return fail(err, SLAMG_E_INVALID, "n_b + n_guard larger than the nonzero part of A");
  return SLAMG_OK;
}

static slamg_status run_guarded(const Exec& x, std::string& err, Problem& pb, const slamg_params& p,
                                const double* init_tests, SolveOutput& out) {
  try {
    if (hipSetDevice(x.device) != hipSuccess) return fail(err, SLAMG_E_DEVICE, "hipSetDevice failed");
    run_solver(x.stream, x.budget, pb, p, init_tests, out);
  } catch (const SolverError& e) {
    (void)hipStreamSynchronize(x.stream);
    return fail(err, (slamg_status)e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(err, SLAMG_E_OOM, "host allocation failed");
  } catch (const std::length_error& e) {
    return fail(err, SLAMG_E_OOM, std::string("host structure too large: ") + e.what());
  } catch (const std::exception& e) {
    return fail(err, SLAMG_E_DEVICE, std::string("unexpected host error: ") + e.what());
  }
  return SLAMG_OK;
}

static slamg_status solve_host(const Exec& x, std::string& err, int64_t m0, int64_t n0, const std::vector<int64_t>& rp,
                               const std::vector<int32_t>& ci, const std::vector<double>& v, slamg_kind kind,
                               slamg_target target, int32_t nb, const slamg_params& p, const double* init_tests,
                               std::vector<double>& sigma, std::vector<double>& Uc, std::vector<double>& Vc,
                               slamg_report* rep) {
  Prepared P;
  slamg_status s = prepare(err, m0, n0, rp, ci, v, kind, P);
  if (s != SLAMG_OK) return s;
  s = check_params(err, P, nb, p);
  if (s != SLAMG_OK) return s;
  Problem pb;
  pb.kind = kind; pb.target = target; pb.nb = nb;
  pb.A = P.A;
  SolveOutput out;
  s = run_guarded(x, err, pb, p, init_tests, out);
  if (s != SLAMG_OK) return s;
  // scatter back, sign convention on the caller's v_j (x_j), column-major outputs
  const int mp = pb.A.m, np = pb.A.n;
  const int64_t M = P.M, N = P.N;
  std::vector<double> Uf((size_t)M * nb, 0.0), Vf(kind == SLAMG_SVD ? (size_t)N * nb : 0, 0.0);
  for (int r = 0; r < mp; ++r)
    for (int j = 0; j < nb; ++j) Uf[(size_t)P.rkeep[r] + (size_t)j * M] = out.U[(size_t)r * nb + j];
  if (kind == SLAMG_SVD)
    for (int r = 0; r < np; ++r)
      for (int j = 0; j < nb; ++j) Vf[(size_t)P.ckeep[r] + (size_t)j * N] = out.V[(size_t)r * nb + j];
  if (P.transposed) std::swap(Uf, Vf);
  const int64_t lu = P.m0, lv = P.n0;
  for (int j = 0; j < nb; ++j) {
    const std::vector<double>& ref = kind == SLAMG_SVD ? Vf : Uf;
    const int64_t len = kind == SLAMG_SVD ? lv : lu;
    int64_t best = 0;
    for (int64_t r = 1; r < len; ++r)
      if (std::fabs(ref[r + (size_t)j * len]) > std::fabs(ref[best + (size_t)j * len])) best = r;
    if (ref[best + (size_t)j * len] < 0.0) {
      for (int64_t r = 0; r < lu; ++r) Uf[r + (size_t)j * lu] = -Uf[r + (size_t)j * lu];
      if (kind == SLAMG_SVD)
        for (int64_t r = 0; r < lv; ++r) Vf[r + (size_t)j * lv] = -Vf[r + (size_t)j * lv];
    }
  }
  sigma = out.sigma;
  Uc.swap(Uf);
  Vc.swap(Vf);
  if (rep) *rep = out.rep;
  if (out.status == ST_NOT_CONVERGED) {
    err = "tolerance not reached within max_add iterations";
    return SLAMG_NOT_CONVERGED;
  }
  err.clear();
  return SLAMG_OK;
}

// ------------------------------------------------------------------------------------------------
// Prepared, device-resident matrices
// ------------------------------------------------------------------------------------------------
struct slamg_matrix {
  slamg_ctx* ctx = nullptr;
  Prepared P;
  DCsr dA, dAt, dB, dC;
  int* d_rkeep = nullptr;
  int* d_ckeep = nullptr;
  std::vector<void*> allocs;
  ~slamg_matrix() {
    for (void* q : allocs) (void)hipFree(q);
  }
  template <class T>
  T* dalloc(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      throw SolverError{ST_E_OOM, "hipMalloc failed"};
    }
    allocs.push_back(q);
    return (T*)q;
  }
  template <class T>
  void put(T* d, const std::vector<T>& h) {
    if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      throw SolverError{ST_E_DEVICE, "hipMemcpy failed"};
  }
  DCsr upload(const HCsr& h) {
    DCsr d;
    d.m = h.m; d.n = h.n; d.nnz = h.nnz();
    d.rp = dalloc<int>(h.m + 1); d.ci = dalloc<int>(d.nnz); d.v = dalloc<double>(d.nnz);
    put(d.rp, h.rp); put(d.ci, h.ci); put(d.v, h.v);
    return d;
  }
};

extern "C" slamg_status slamg_matrix_create(slamg_ctx* ctx, const slamg_csr* A, slamg_kind kind,
                                            slamg_matrix** out) {
  if (!ctx || !out) return SLAMG_E_INVALID;
  *out = nullptr;
  if (kind != SLAMG_SVD && kind != SLAMG_SPD_EIG) return fail(ctx, SLAMG_E_INVALID, "unknown kind");
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  slamg_status s = fetch_csr(ctx, A, rp, ci, v);
  if (s != SLAMG_OK) return s;
  auto M = std::make_unique<slamg_matrix>();
  M->ctx = ctx;
  s = prepare(ctx->err, A->m, A->n, rp, ci, v, kind, M->P);
  if (s != SLAMG_OK) return s;
  try {
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SLAMG_E_DEVICE, "hipSetDevice failed");
    const HCsr& H = M->P.A;
    M->dA = M->upload(H);
    auto ident = [](int n) {
      HCsr I;
      I.m = I.n = n;
      I.rp.resize(n + 1); I.ci.resize(n); I.v.assign(n, 1.0);
      for (int i = 0; i <= n; ++i) I.rp[i] = i;
      for (int i = 0; i < n; ++i) I.ci[i] = i;
      return I;
    };
    if (kind == SLAMG_SVD) {
      M->dAt = M->upload(transpose(H, nullptr));
      M->dB = M->upload(ident(H.m));
      M->dC = M->upload(ident(H.n));
    } else {
      HCsr Bh = H;   // identity on A's pattern
      for (int i = 0; i < Bh.m; ++i)
        for (int k = Bh.rp[i]; k < Bh.rp[i + 1]; ++k) Bh.v[k] = Bh.ci[k] == i ? 1.0 : 0.0;
      M->dB = M->dA;
      M->dB.v = M->dalloc<double>(Bh.nnz());
      M->put(M->dB.v, Bh.v);
    }
    M->d_rkeep = M->dalloc<int>(M->P.rkeep.size());
    M->put(M->d_rkeep, M->P.rkeep);
    M->d_ckeep = M->dalloc<int>(M->P.ckeep.size());
    M->put(M->d_ckeep, M->P.ckeep);
  } catch (const SolverError& e) {
    return fail(ctx, (slamg_status)e.code, e.msg);
  }
  *out = M.release();
  return SLAMG_OK;
}

extern "C" void slamg_matrix_destroy(slamg_matrix* M) { delete M; }

extern "C" slamg_status slamg_solve_matrix(slamg_ctx* ctx, const slamg_matrix* M, slamg_target target, int32_t n_b,
                                           const slamg_params* p, const double* init_tests, double* sigma, double* U,
                                           double* V, int32_t outputs_on_device, slamg_report* rep) {
  if (!ctx || !M || !sigma) return SLAMG_E_INVALID;
  if (M->ctx != ctx) return fail(ctx, SLAMG_E_INVALID, "matrix belongs to another context");
  if (target != SLAMG_DOMINANT && target != SLAMG_MINIMAL) return fail(ctx, SLAMG_E_INVALID, "unknown target");
  slamg_params prm;
  if (p) prm = *p;
  else slamg_params_init(&prm, (slamg_kind)M->P.kind, target);
  const Prepared& P = M->P;
  slamg_status s = check_params(ctx->err, P, n_b, prm);
  if (s != SLAMG_OK) return s;
  Problem pb;
  pb.kind = P.kind; pb.target = target; pb.nb = n_b;
  pb.A = P.A;
  pb.dA = &M->dA;
  pb.dB = &M->dB;
  if (P.kind == SLAMG_SVD) { pb.dAt = &M->dAt; pb.dC = &M->dC; }
  if (outputs_on_device) {
    pb.outU = U;
    pb.outV = P.kind == SLAMG_SVD ? V : nullptr;
    pb.ldU = P.m0; pb.ldV = P.n0;
    pb.keepU = M->d_rkeep;
    pb.keepV = M->d_ckeep;
    pb.swapUV = P.transposed;
    if (!pb.outU && !pb.outV) pb.outU = nullptr;
  }
  SolveOutput out;
  s = run_guarded(exec_of(ctx), ctx->err, pb, prm, init_tests, out);
  if (s != SLAMG_OK) return s;
  std::copy(out.sigma.begin(), out.sigma.end(), sigma);
  if (!outputs_on_device && (U || V)) {
    // host outputs: same conventions as slamg_solve
    const int64_t Mr = P.M, Nr = P.N;
    std::vector<double> Uf((size_t)Mr * n_b, 0.0), Vf(P.kind == SLAMG_SVD ? (size_t)Nr * n_b : 0, 0.0);
    for (size_t r = 0; r < P.rkeep.size(); ++r)
      for (int j = 0; j < n_b; ++j) Uf[(size_t)P.rkeep[r] + (size_t)j * Mr] = out.U[r * n_b + j];
    if (P.kind == SLAMG_SVD)
      for (size_t r = 0; r < P.ckeep.size(); ++r)
        for (int j = 0; j < n_b; ++j) Vf[(size_t)P.ckeep[r] + (size_t)j * Nr] = out.V[r * n_b + j];
    if (P.transposed) std::swap(Uf, Vf);
    const int64_t lu = P.m0, lv = P.n0;
    for (int j = 0; j < n_b; ++j) {
      const std::vector<double>& ref = P.kind == SLAMG_SVD ? Vf : Uf;
      const int64_t len = P.kind == SLAMG_SVD ? lv : lu;
      int64_t best = 0;
      for (int64_t r = 1; r < len; ++r)
        if (std::fabs(ref[r + (size_t)j * len]) > std::fabs(ref[best + (size_t)j * len])) best = r;
      const double sg = ref[best + (size_t)j * len] < 0.0 ? -1.0 : 1.0;
      if (U) for (int64_t r = 0; r < lu; ++r) U[r + (size_t)j * lu] = sg * Uf[r + (size_t)j * lu];
      if (V && P.kind == SLAMG_SVD) for (int64_t r = 0; r < lv; ++r) V[r + (size_t)j * lv] = sg * Vf[r + (size_t)j * lv];
    }
  }
  if (rep) *rep = out.rep;
  if (out.status == ST_NOT_CONVERGED) {
    ctx->err = "tolerance not reached within max_add iterations";
    return SLAMG_NOT_CONVERGED;
  }
  ctx->err.clear();
  return SLAMG_OK;
}

extern "C" slamg_status slamg_solve(slamg_ctx* ctx, const slamg_csr* A, slamg_kind kind, slamg_target target,
                                    int32_t n_b, const slamg_params* p, const double* init_tests, double* sigma,
                                    double* U, double* V, slamg_report* rep) {
  if (!ctx) return SLAMG_E_INVALID;
  if (!sigma) return fail(ctx, SLAMG_E_INVALID, "sigma output is required");
  if (kind != SLAMG_SVD && kind != SLAMG_SPD_EIG) return fail(ctx, SLAMG_E_INVALID, "unknown kind");
  if (target != SLAMG_DOMINANT && target != SLAMG_MINIMAL) return fail(ctx, SLAMG_E_INVALID, "unknown target");
  slamg_params prm;
  if (p) prm = *p;
  else slamg_params_init(&prm, kind, target);
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  slamg_status s = fetch_csr(ctx, A, rp, ci, v);
  if (s != SLAMG_OK) return s;
  std::vector<double> sg, Uc, Vc;
  s = solve_host(exec_of(ctx), ctx->err, A->m, A->n, rp, ci, v, kind, target, n_b, prm, init_tests, sg, Uc, Vc, rep);
  if (s != SLAMG_OK && s != SLAMG_NOT_CONVERGED) return s;
  std::copy(sg.begin(), sg.end(), sigma);
  if (U) std::copy(Uc.begin(), Uc.end(), U);
  if (V && kind == SLAMG_SVD) std::copy(Vc.begin(), Vc.end(), V);
  return s;
}

// ------------------------------------------------------------------------------------------------
// Request interface.  Without the serving loop, requests are solved first come, first served on
// the context stream when poll / fetch asks for them.  With it (slamg_serve_start), worker threads
// each own a HIP stream and take requests as they arrive: a request is admitted when a worker is
// free and its footprint estimate fits the context's HBM budget next to those already running
// (first fit among the oldest pending requests, so that small requests can pass a large one that
// must wait for memory); its solve then overlaps on the device with the others.  Every solve
// owns all of its device memory, and the kernels use no atomics, so a result does not depend on
// what else runs.
// ------------------------------------------------------------------------------------------------

// Upper bound of a solve's device memory: operators and hierarchy (A, A^t, Galerkin products,
// interpolation: <= 400 B per nonzero of A), the strength products' device chunk, vector blocks of all levels
// (test, boot, ping-pong, residual and scratch blocks, FP64 and FP32), and the dense coarsest
// level (<= 1024 unknowns; X, Y, factors, work, per-column eigenvector stores).
static size_t footprint_estimate(int64_t m, int64_t n, int64_t nnz, slamg_kind kind, int32_t nb,
                                 const slamg_params& p) {
  const double rows = (double)(kind == SLAMG_SVD ? m + n : m);
  const double nc = std::min(1024.0, kind == SLAMG_SVD ? (double)(m + n) : (double)m);
  const int32_t blk = nb + std::max(p.n_guard, 0);   // the block holds the guard pairs too
  const double w = (double)(4 * p.n_t + 12 * blk);
  // SVD: the strength products' entries pass through the device in chunks of 2^25 (16 B each)
  const double strength = kind == SLAMG_SVD ? 16.0 * std::min(33554432.0, 64.0 * (double)nnz) : 0.0;
  // LOBPCG: six further blocks per side
  const double lob = p.solve_phase == 1 ? 48.0 * rows * blk : 0.0;
  const double bytes = 64.0 * 1024 * 1024 + 400.0 * (double)nnz + 8.0 * rows * w * 2.0 +
                       8.0 * (3.0 * blk + 10.0) * nc * nc + strength + lob;
  return (size_t)bytes;
}

extern "C" slamg_status slamg_submit(slamg_ctx* ctx, const slamg_csr* A, slamg_kind kind, slamg_target target,
                                     int32_t n_b, const slamg_params* p, uint64_t* request_id) {
  if (!ctx || !request_id) return SLAMG_E_INVALID;
  auto r = std::make_unique<Request>();
  slamg_status s = fetch_csr(ctx, A, r->rp, r->ci, r->v);
  if (s != SLAMG_OK) return s;
  r->A = *A;
  r->kind = kind; r->target = target; r->nb = n_b;
  if (p) r->p = *p;
  else slamg_params_init(&r->p, kind, target);
  r->est = footprint_estimate(A->m, A->n, A->nnz, kind, n_b, r->p);
  if (ctx->budget && r->est > ctx->budget)
    return fail(ctx, SLAMG_E_BUDGET, "request footprint estimate exceeds the context's HBM budget");
  r->t_submit = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(ctx->mu);
  r->id = ctx->next_id++;
  *request_id = r->id;
  ctx->queue.push_back(r->id);
  ctx->reqs[r->id] = std::move(r);
  ctx->cv.notify_all();
  return SLAMG_OK;
}

static void finish(Request& r) {
  const auto t = std::chrono::steady_clock::now();
  r.rep.t_queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count();
  r.rep.t_latency_ms = std::chrono::duration<double, std::milli>(t - r.t_submit).count();
}

static void process_until(slamg_ctx* ctx, uint64_t id) {
  while (!ctx->queue.empty()) {
    uint64_t head = ctx->queue.front();
    ctx->queue.pop_front();
    auto it = ctx->reqs.find(head);
    if (it == ctx->reqs.end()) continue;
    Request& r = *it->second;
    r.t_start = std::chrono::steady_clock::now();
    r.status = solve_host(exec_of(ctx), ctx->err, r.A.m, r.A.n, r.rp, r.ci, r.v, r.kind, r.target, r.nb, r.p,
                          nullptr, r.sigma, r.U, r.V, &r.rep);
    r.err = ctx->err;
    finish(r);
    r.done = true;
    if (head == id) break;
  }
}

// Worker thread of the serving loop.
static void serve_worker(slamg_ctx* ctx, hipStream_t stream) {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(ctx->mu);
  for (;;) {
    Request* pick = nullptr;
    size_t scanned = 0;
    for (auto it = ctx->queue.begin(); it != ctx->queue.end() && scanned < 64; ++it, ++scanned) {
      Request& r = *ctx->reqs.at(*it);
      if (!ctx->budget || ctx->reserved + r.est <= ctx->budget) {
        pick = &r;
        ctx->queue.erase(it);
        break;
      }
    }
    if (!pick) {
      if (ctx->stopping && ctx->queue.empty()) return;
      ctx->cv.wait(lk);
      continue;
    }
    ctx->reserved += pick->est;
    ctx->running += 1;
    pick->t_start = std::chrono::steady_clock::now();
    lk.unlock();
    Exec x{ctx->device, stream, ctx->budget ? pick->est : 0};
    std::string err;
    const slamg_status st = solve_host(x, err, pick->A.m, pick->A.n, pick->rp, pick->ci, pick->v, pick->kind,
                                       pick->target, pick->nb, pick->p, nullptr, pick->sigma, pick->U, pick->V,
                                       &pick->rep);
    lk.lock();
    pick->status = st;
    pick->err = err;
    finish(*pick);
    pick->done = true;
    ctx->reserved -= pick->est;
    ctx->running -= 1;
    ctx->cv.notify_all();
  }
}

extern "C" slamg_status slamg_serve_start(slamg_ctx* ctx, int32_t slots) {
  if (!ctx || slots < 1 || slots > 64) return SLAMG_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->serving) return fail(ctx, SLAMG_E_INVALID, "the serving loop already runs");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SLAMG_E_DEVICE, "hipSetDevice failed");
  for (int i = 0; i < slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      for (hipStream_t q : ctx->wstreams) (void)hipStreamDestroy(q);
      ctx->wstreams.clear();
      return fail(ctx, SLAMG_E_DEVICE, "stream creation failed");
    }
    ctx->wstreams.push_back(st);
  }
  ctx->stopping = false;
  ctx->serving = true;
  for (int i = 0; i < slots; ++i) ctx->workers.emplace_back(serve_worker, ctx, ctx->wstreams[i]);
  return SLAMG_OK;
}

extern "C" slamg_status slamg_serve_stop(slamg_ctx* ctx) {
  if (!ctx) return SLAMG_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->serving) return SLAMG_OK;
    ctx->stopping = true;
    ctx->cv.notify_all();
  }
  for (auto& t : ctx->workers) t.join();
  ctx->workers.clear();
  for (hipStream_t q : ctx->wstreams) (void)hipStreamDestroy(q);
  ctx->wstreams.clear();
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->serving = false;
  ctx->stopping = false;
  return SLAMG_OK;
}

extern "C" slamg_status slamg_poll(slamg_ctx* ctx, uint64_t request_id, int32_t* done) {
  if (!ctx || !done) return SLAMG_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(request_id);
  if (it == ctx->reqs.end()) return fail(ctx, SLAMG_E_INVALID, "unknown request id");
  if (!it->second->done && !ctx->serving) process_until(ctx, request_id);
  *done = it->second->done ? 1 : 0;
  return SLAMG_OK;
}

extern "C" slamg_status slamg_wait(slamg_ctx* ctx, uint64_t request_id) {
  if (!ctx) return SLAMG_E_INVALID;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(request_id);
  if (it == ctx->reqs.end()) return fail(ctx, SLAMG_E_INVALID, "unknown request id");
  Request& r = *it->second;
  if (!ctx->serving) {
    if (!r.done) process_until(ctx, request_id);
    return SLAMG_OK;
  }
  ctx->cv.wait(lk, [&] { return r.done; });
  return SLAMG_OK;
}

extern "C" slamg_status slamg_fetch(slamg_ctx* ctx, uint64_t request_id, double* sigma, double* U, double* V,
                                    slamg_report* rep) {
  if (!ctx) return SLAMG_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(request_id);
  if (it == ctx->reqs.end()) return fail(ctx, SLAMG_E_INVALID, "unknown request id");
  if (!it->second->done && !ctx->serving) process_until(ctx, request_id);
  Request& r = *it->second;
  if (!r.done) return SLAMG_E_BUSY;
  slamg_status s = r.status;
  if (s == SLAMG_OK || s == SLAMG_NOT_CONVERGED) {
    if (sigma) std::copy(r.sigma.begin(), r.sigma.end(), sigma);
    if (U) std::copy(r.U.begin(), r.U.end(), U);
    if (V && r.kind == SLAMG_SVD) std::copy(r.V.begin(), r.V.end(), V);
  }
  if (rep) *rep = r.rep;
  ctx->err = r.err;
  ctx->reqs.erase(it);
  return s;
}
