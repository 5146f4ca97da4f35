// Device orchestration of the self-learning AMG method: the multiplicative (setup) phase of §3,
// the additive (solve) phase of §4 with the Ritz projection of §4.3, for SVD and SPD-eigen kinds and
// dominant / minimal targets (§5).  Every numeric step is a HIP kernel launched on one stream; the
// host only builds the hierarchy structure in the first cycle (graph.cpp) and reads the residual
// norms once per additive iteration.
#include "solver.h"

#include <cstdio>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>

#include "graph.h"

namespace slamg {

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) throw SolverError{ST_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// ------------------------------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014)
// ------------------------------------------------------------------------------------------------
uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double splitmix64_uniform(uint64_t seed, uint64_t k) {
  uint64_t st = seed + (k - 1) * 0x9E3779B97F4A7C15ull;
  uint64_t z = splitmix64_next(st);
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}
static const uint64_t NORM_SEED_XOR = 0xA5A5A5A5A5A5A5A5ull;

// ------------------------------------------------------------------------------------------------
// Device memory arena (freed when the solve ends); enforces the context's HBM budget
// ------------------------------------------------------------------------------------------------
// Device memory of one solve.  Allocations are stream-ordered (hipMallocAsync / hipFreeAsync on the
// solve's stream): a plain hipFree waits for the whole device, which would stall every other solve
// running concurrently on other streams.
class Arena {
 public:
  Arena(size_t budget, hipStream_t s) : budget_(budget), st_(s) {}
  ~Arena() {
    for (void* p : ptrs_) (void)hipFreeAsync(p, st_);
  }
  template <class T>
  T* alloc(size_t n) {
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    bytes = (bytes + 255) & ~size_t(255);
    if (budget_ && used_ + bytes > budget_)
      throw SolverError{ST_E_BUDGET, "device footprint exceeds the HBM budget of the context"};
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, st_) != hipSuccess) {
      (void)hipGetLastError();
      throw SolverError{ST_E_OOM, "hipMallocAsync failed"};
    }
    ptrs_.push_back(p);
    sizes_.push_back(bytes);
    used_ += bytes;
    peak_ = std::max(peak_, used_);
    return static_cast<T*>(p);
  }
  // Returns one allocation before the solve ends (stream-ordered: work queued on the solve's
  // stream that still reads it completes first); null is ignored.
  void release(const void* p) {
    if (!p) return;
    for (size_t i = ptrs_.size(); i-- > 0;) {
      if (ptrs_[i] != p) continue;
      (void)hipFreeAsync(ptrs_[i], st_);
      used_ -= sizes_[i];
      ptrs_.erase(ptrs_.begin() + (long)i);
      sizes_.erase(sizes_.begin() + (long)i);
      return;
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  size_t budget_, used_ = 0, peak_ = 0;
  hipStream_t st_;
  std::vector<void*> ptrs_;
  std::vector<size_t> sizes_;
};

template <class T>
static void h2d(T* d, const std::vector<T>& h, hipStream_t s) {
  if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
static void d2h(std::vector<T>& h, const T* d, size_t n, hipStream_t s) {
  h.resize(n);
  if (n) HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------------------------
// Hierarchy data
// ------------------------------------------------------------------------------------------------
struct Plan {   // numeric C = L R on a fixed pattern: entry (i, j) = row i of L . row j of Rt
  int nnz = 0;
  int* rowC = nullptr;
  const int* colC = nullptr;
  const DCsr* L = nullptr;
  const DCsr* Rt = nullptr;
  double* out = nullptr;
  void run(hipStream_t s) const {
    launch_spgemm_dot(nnz, rowC, colC, L->rp, L->ci, L->v, Rt->rp, Rt->ci, Rt->v, out, s);
  }
};

struct Side {
  int npts = 0, nc = 0;
  std::vector<char> is_c;
  std::vector<int> cpts;
  int* d_cpts = nullptr;
  HCsr Ppat, Ptpat;
  std::vector<int> perm;   // Pt entry -> P entry
  DCsr P, Pt;
  int* d_perm = nullptr;
  int nF = 0, qmax = 0, capped = 0;
  int* d_F = nullptr;
  int* d_prp = nullptr;
  int* d_fc = nullptr;
};

template <class T>
struct Blocks {
  T *Ut = nullptr, *Vt = nullptr;          // test vectors (mult phase, FP64 only)
  T *Ub = nullptr, *Vb = nullptr;          // boot vectors / additive iterates (contiguous)
  T *Ua = nullptr, *Va = nullptr;          // second contiguous pair: relaxation writes here, then swaps
  T *kap = nullptr, *tau = nullptr;        // restricted residuals (contiguous)
  T *tU = nullptr, *tV = nullptr, *tU2 = nullptr, *tV2 = nullptr;
};
template <class T>
struct Aux {
  T *dinvB = nullptr, *dinvC = nullptr;    // 1 / diag(B), 1 / diag(C)
  T *rnA = nullptr, *rnAab = nullptr, *rnAbb = nullptr, *rnAt = nullptr;   // Kaczmarz row sums
};

// Rows of one side whose walk is far longer than the others' (a frequent term of a term-document
// matrix): a flag per row and their list, on the device.
struct LongRows {
  bool done = false;
  unsigned char* flag = nullptr;
  int* rows = nullptr;
  int n = 0;
};

// Kaczmarz row order of a level's sides, computed on the host (rows of A; SVD: also rows of A^t)
struct ColourJob {
  std::vector<int> rows, cptr, rows2, cptr2;
  std::vector<long> cnnz, cnnz2;
};

struct Level {
  int m = 0, n = 0;
  // the Kaczmarz colouring, computed on a host thread of its own from the level's pattern and
  // uploaded when the level's first Kaczmarz sweep needs it
  std::future<ColourJob> colour_job;
  bool coloured = true;
  LongRows lgu, lgv;        // u-side rows (A, B) and v-side rows (A^t, C)
  HCsr hA, hAt, hB, hC;     // host patterns (hB/hC: SVD only)
  std::vector<int> permAt;
  DCsr A, At, B, C;         // SPD: At aliases A, B lives on A's pattern, C unused
  int* d_permAt = nullptr;
  bool finest = false;
  // Kaczmarz orders (minimal targets)
  int* kA_rows = nullptr;  std::vector<int> kA_cptr;  std::vector<long> kA_cnnz;
  int* kAt_rows = nullptr; std::vector<int> kAt_cptr; std::vector<long> kAt_cnnz;
  int* d_kA_cptr = nullptr;
  int* d_kAt_cptr = nullptr;
  bool kacz_wg = false;     // small level: whole sweeps in one workgroup
  // minimal LS pre-smoothing scales
  double* smU = nullptr;    // 1 / diag(N_u)
  double* smV = nullptr;    // 1 / diag(N_v)
  Blocks<double> bd;
  Blocks<float> bf;
  Aux<double> ad;
  Aux<float> af;
  Side su, sv;
  DCsr S1, S2, S3;
  std::vector<Plan> plans;  // Galerkin numeric products producing level + 1
  Plan pAc, pBc, pCc;
  // A colouring still running reads hA / hAt through pointers.  Members are destroyed in reverse
  // declaration order, so the future's own wait would come after those patterns are freed: a level
  // dropped while its colouring runs (a set-up that ends in an error, a level never relaxed, a level
  // rebuilt) waits for it here, before any member goes.
  ~Level() {
    if (colour_job.valid()) colour_job.wait();
  }
};

template <class T> static const T* vals(const DCsr& a);
template <> const double* vals<double>(const DCsr& a) { return a.v; }
template <> const float* vals<float>(const DCsr& a) { return a.vf; }
template <class T> static Blocks<T>& blocks(Level& L);
template <> Blocks<double>& blocks<double>(Level& L) { return L.bd; }
template <> Blocks<float>& blocks<float>(Level& L) { return L.bf; }
template <class T> static Aux<T>& aux(Level& L);
template <> Aux<double>& aux<double>(Level& L) { return L.ad; }
template <> Aux<float>& aux<float>(Level& L) { return L.af; }

// ------------------------------------------------------------------------------------------------
class Solver {
 public:
  Solver(hipStream_t s, size_t budget, const Problem& pb, const slamg_params& p)
      : st_(s), ar_(budget, s), p_(p), spd_(pb.kind == SLAMG_SPD_EIG), minimal_(pb.target == SLAMG_MINIMAL),
        nb_(pb.nb + p.n_guard), nw_(pb.nb), nt_(p.n_t), mixed_(p.precision == SLAMG_MIXED_FP32 || p.precision == SLAMG_MIXED_BF16),
        bf16_(p.precision == SLAMG_MIXED_BF16),
        square_(pb.kind == SLAMG_SVD && p.square_coarsening != 0), A0_(pb.A), pb_(pb) {}
  ~Solver() {
    if (igx_) (void)hipGraphExecDestroy(igx_);
    if (ig_) (void)hipGraphDestroy(ig_);
  }
  Solver(const Solver&) = delete;
  Solver& operator=(const Solver&) = delete;

  void run(const double* init_tests, SolveOutput& out);

 private:
  // set-up helpers
  DCsr upload(const HCsr& h, bool with_values);
  void alloc_level_buffers(Level& L);
  void finest_level(const double* init_tests);
  void norm_estimate();
  bool build_structure(int l);
  // strength sets of a side, kept while its level's coarsening is decided
  struct Strength {
    std::vector<int> Sp, Si;
  };
  void build_side(Level& L, Side& S, const HCsr& N, int npts, Strength* keep = nullptr);
  void complete_side(Side& S, const HCsr& N, const Strength& st, int need);
  void identity_side(Side& S, int npts);
  void finish_side(Side& S, const std::vector<int>& ptr, const std::vector<int>& fine_cols);
  void make_coarse_level(int l);
  void refresh_level_aux(Level& L);
  void colour(Level& L);
  void ensure_colours(Level& L);
  std::vector<int> row_colours(const HCsr& M) const;
  HCsr strength_operator(Level& L, bool u_side, bool finest);
  // cycle pieces
  void relax_tests(int l);
  void boot_relax_rq(int l);
  void fit_interpolation(int l, int cycle);
  void redo_interpolation(const std::vector<char>& conv);
  template <class T> void cycle_level(int l, const double* sig, T* rhsU, T* rhsV, bool zero_iterate);
  template <class T> void coarsest_additive(const double* sig);
  long coarse_calls_per_iter() const;
  // set-up timing on stderr (verbose >= 2): host time since the previous mark
  std::chrono::steady_clock::time_point vt_ = std::chrono::steady_clock::now();
  void vmark(const char* what, int l) {
    if (p_.verbose < 2) return;
    const auto t = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[slamg]   level %d %s: %.1f ms\n", l, what,
                 std::chrono::duration<double, std::milli>(t - vt_).count());
    std::fflush(stderr);
    vt_ = t;
  }
  void coarse_setup();
  void cast_transfers();
  void galerkin(int l);
  void inject(int l, int cycle);
  void coarsest_mult();
  void mult_cycle(int c);
  template <class T> void boot_relax(int l, const T* kap, const T* tau, const double* sig, int nsweeps = 1,
                                      bool zero_start = false);
  template <class T> void additive_vcycle(const double* sig, T* rhsU, T* rhsV);
  template <class T> void additive_fmg(const double* sig, T* rhsU, T* rhsV);
  template <class T> void additive_cycle(const double* sig, T* rhsU, T* rhsV) {
    if (p_.fmg) additive_fmg<T>(sig, rhsU, rhsV);
    else additive_vcycle<T>(sig, rhsU, rhsV);
  }
  template <class T> void level_residual_restrict(int l, const T* kap, const T* tau, const double* sig);
  void additive_iteration();
  void ritz();
  void ritz_level(int l);
  void lobpcg_setup();
  void lobpcg_iteration();
  void lob_remove(double* Y, int rows, std::initializer_list<const double*> bases);
  bool lob_pcheck(const double* P0, double* Pq, int rows, int nact, std::initializer_list<const double*> bases,
                  double* tmp, const char* side);
  void cholqr2(double* X, int rows, double* tmp, double* out);
  void cholqr2_pair(double* Xa, int rows_a, double* tmpa, double* outa, double* Xb, int rows_b, double* tmpb,
                    double* outb);
  void residuals(std::vector<double>& rho);
  void residual_launch();
  void residual_collect(std::vector<double>& rho);
  void iteration_body();
  void capture_iteration();
  bool lob_replay_ = false;   // the LOBPCG iteration replays the captured additive cycle
  std::vector<void**> block_pointers();
  void check_status();
  void dense_coarsest(double* X, double* Y);
  void sync() { HIPCHK(hipStreamSynchronize(st_)); }
  void lastcheck() { HIPCHK(hipGetLastError()); }

  int rows_u(const Level& L) const { return L.m; }
  int rows_v(const Level& L) const { return spd_ ? L.m : L.n; }
  int size_of(const Level& L) const { return spd_ ? L.m : L.m + L.n; }

  hipStream_t st_;
  Arena ar_;
  slamg_params p_;
  bool spd_, minimal_;
  int nb_;   // block width: the n_b wanted pairs and the guard pairs
  int nw_;   // wanted pairs: the stopping test and the outputs
  int nt_;
  bool mixed_;
  bool bf16_;   // the FP32 V-cycle reads BF16 operator values (their bit patterns in the .vf arrays)
  bool square_; // SVD of a square A with both sides coarsened on A itself (§5.1)
  // low-precision copy of an operator's values for the FP32 V-cycle: FP32, or BF16 bit patterns
  void cast_vals(const DCsr& a) {
    if (!a.vf) return;
    if (bf16_) launch_cast_bf16(a.v, a.vf, a.nnz, st_);
    else launch_copy_cast_df(a.v, a.vf, a.nnz, st_);
  }
  template <class T> int vbf() const { return std::is_same<T, float>::value && bf16_ ? 1 : 0; }
  void long_rows(Level& L);
  template <class T> void attach_long(int l, RowOpArgs<T>& a);
  const HCsr& A0_;
  const Problem& pb_;
  std::vector<std::unique_ptr<Level>> lv_;
  double anorm_ = 0.0;
  double* sig_ = nullptr;       // device sigma_b (nb)
  double* flip_ = nullptr;
  double* partial_ = nullptr;   // reduction partials
  double* partial2_ = nullptr;  // partials of the second reduction of a paired launch
  double* gram2_ = nullptr;     // second Gram matrix / factor of a paired Cholesky-QR
  double* small3_ = nullptr;
  double* r1_ = nullptr;        // small device vectors (>= 64)
  double* r2_ = nullptr;
  double* r3_ = nullptr;
  double* wts_ = nullptr;
  double* gram_ = nullptr;      // 16 x 16
  double* small1_ = nullptr;    // 16 x 16
  double* small2_ = nullptr;
  double* small_work_ = nullptr;
  int* status_ = nullptr;
  // coarsest dense data
  int NL_ = 0;
  double* pbasis_ = nullptr;   // eigenvectors of X - sigma_j Y from the previous coarsest solve
  long pinv_calls_ = 0;
  bool pinv_reortho_ = false;    // the next literal coarsest solve re-orthonormalises its basis
  // redetermined interpolation (§6.3): LS weight factors of the refit, the kept iterate
  double* wscale_ = nullptr;
  bool redo_weights_ = false;
  double* redo_keep_ = nullptr;
  double* pencil_wk_ = nullptr;
  // LOBPCG solve phase (§7): per side the old X, the W, P and projected-P blocks, an operator
  // product and a Cholesky-QR temporary (rows x n_b each), the k x k projected problem
  struct LobSide {
    double *X = nullptr, *W = nullptr, *P = nullptr, *Pq = nullptr, *T = nullptr, *tmp = nullptr;
  };
  LobSide lbu_, lbv_;
  double *lobM_ = nullptr, *lobB_ = nullptr, *lobC_ = nullptr, *lobY_ = nullptr, *lobZ_ = nullptr;
  double *lobwork_ = nullptr, *lobchk_ = nullptr;   // lobchk_: two Gram matrices and a pivot
  int* lobflag_ = nullptr;   // status of the P blocks' factorisations (a failure only drops P)
  bool lob_have_p_ = false;
  double *dX_ = nullptr, *dY_ = nullptr, *dwork_ = nullptr, *dA_ = nullptr, *dB_ = nullptr, *dC_ = nullptr;
  double *mu_ = nullptr, *Zp_ = nullptr;
  bool pencil_ready_ = false;
  slamg_report rep_{};
  // profiling (HIP events around the launches of selected kernel classes)
  struct ProfEv { hipEvent_t a, b; int cls; };
  std::vector<ProfEv> pev_;
  double pbytes_[8] = {};
  long pn_[8] = {};
  int pmask_ = 0;
  template <class F> void prof(int cls, double bytes, F&& f) {
    // launches inside a graph capture are not timed: the eager iterations sample them
    if (capturing_ || !((pmask_ >> cls) & 1)) { f(); return; }
    ProfEv e{event(), event(), cls};
    HIPCHK(hipEventRecord(e.a, st_));
    f();
    HIPCHK(hipEventRecord(e.b, st_));
    pev_.push_back(e);
    pbytes_[cls] += bytes;
    pn_[cls] += 1;
  }
  // HIP graph of one additive iteration
  hipGraph_t ig_ = nullptr;
  hipGraphExec_t igx_ = nullptr;
  bool capturing_ = false, graph_off_ = false;
  void prof_finish();
  // events are reused across solves (creating one per launch would dominate the host time)
  // (one pool per host thread: concurrent solves on several streams each own their events)
  static std::vector<hipEvent_t>& event_pool() {
    thread_local std::vector<hipEvent_t> pool;
    return pool;
  }
  size_t ev_used_ = 0;
  hipEvent_t event() {
    auto& pool = event_pool();
    if (ev_used_ == pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[ev_used_++];
  }
  template <class T> void rowop(int l, const RowOpArgs<T>& a, const DCsr* K, int cls = 0);
  template <class T>
  void rowop2(int l, const RowOpArgs<T>& a, const DCsr* Ka, const RowOpArgs<T>& b, const DCsr* Kb, int cls);
  template <class T> void spmm(int l, const DCsr& K, const T* Kv, int w, const T* x, T* y, double beta);
  template <class T>
  void spmm2(int l, const DCsr& Ka, const T* Kva, const T* xa, T* ya, const DCsr& Kb, const T* Kvb, const T* xb, T* yb,
             double beta);
  template <class T> void dots(int l, const DotArgs<T>& a, const DCsr* K, double* out);
  template <class T> void kacz(int l, const KaczArgs<T>& a, long nnz_colour);
};

// Algorithmic bytes of one launch: every array the launch touches, counted once.
template <class T>
static double rowop_bytes(const RowOpArgs<T>& a, const DCsr* K) {
  const double sz = sizeof(T), vs = a.vbf ? 2.0 : sz, w = a.w, r = a.nrows;
  double b = 0.0;
  if (a.Kv && K) b += 4.0 * (r + 1) + (4.0 + vs) * K->nnz + sz * w * K->n;
  if (a.mmode == M_SHARED && K) b += vs * K->nnz;
  const bool own = a.x || a.mmode == M_IDENT;
  const bool same = a.Kv && (a.z == a.x || a.z == a.y);
  if (own && !same) b += sz * w * r;
  if (a.D) b += sz * r;
  if (a.kap) b += sz * w * r;
  b += sz * w * r;
  return b;
}

template <class T>
void Solver::rowop(int l, const RowOpArgs<T>& a0, const DCsr* K, int cls) {
  RowOpArgs<T> a = a0;
  if (a.nnzK < 0 && K) a.nnzK = K->nnz;
  a.vbf = vbf<T>();
  attach_long(l, a);
  if (l == 0) prof(cls, rowop_bytes(a, K), [&] { launch_rowop(a, st_); });
  else launch_rowop(a, st_);
}

template <class T>
void Solver::rowop2(int l, const RowOpArgs<T>& a0, const DCsr* Ka, const RowOpArgs<T>& b0, const DCsr* Kb, int cls) {
  RowOpArgs<T> a = a0, b = b0;
  if (a.nnzK < 0 && Ka) a.nnzK = Ka->nnz;
  if (b.nnzK < 0 && Kb) b.nnzK = Kb->nnz;
  a.vbf = b.vbf = vbf<T>();
  attach_long(l, a);
  attach_long(l, b);
  if (l == 0) prof(cls, rowop_bytes(a, Ka) + rowop_bytes(b, Kb), [&] { launch_rowop2(a, b, st_); });
  else launch_rowop2(a, b, st_);
}

template <class T>
static double spmm_bytes(const DCsr& K, int w, double beta, int vbf) {
  const double sz = sizeof(T), vs = vbf ? 2.0 : sz;
  return 4.0 * (K.m + 1) + (4.0 + vs) * K.nnz + sz * w * ((double)K.n + K.m * (beta != 0.0 ? 2 : 1));
}

template <class T>
void Solver::spmm(int l, const DCsr& K, const T* Kv, int w, const T* x, T* y, double beta) {
  if (beta == 0.0) {
    // a product with A or A^t whose side has long rows runs as the row kernel (out = K x), which
    // gives each long row a workgroup
    Level& L = *lv_[l];
    const LongRows* g = &K == &L.A ? &L.lgu : (!spd_ && &K == &L.At) ? &L.lgv : nullptr;
    if (g && g->done && g->n > 0) {
      RowOpArgs<T> a;
      a.nrows = K.m; a.w = w; a.Krp = K.rp; a.Kci = K.ci; a.nnzK = K.nnz; a.Kv = Kv; a.z = x;
      a.mmode = M_NONE; a.cmode = C_COPYK; a.out = y;
      rowop(l, a, &K, 5);
      return;
    }
  }
  if (l == 0)
    prof(5, spmm_bytes<T>(K, w, beta, vbf<T>()), [&] { launch_spmm<T>(K.m, w, K.rp, K.ci, Kv, x, y, beta, st_, K.nnz, vbf<T>()); });
  else launch_spmm<T>(K.m, w, K.rp, K.ci, Kv, x, y, beta, st_, K.nnz, vbf<T>());
}

template <class T>
void Solver::spmm2(int l, const DCsr& Ka, const T* Kva, const T* xa, T* ya, const DCsr& Kb, const T* Kvb, const T* xb,
                   T* yb, double beta) {
  SpmmArgs<T> a, b;
  a.m = Ka.m; a.nnz = Ka.nnz; a.rp = Ka.rp; a.ci = Ka.ci; a.v = Kva; a.x = xa; a.y = ya; a.beta = beta;
  b.m = Kb.m; b.nnz = Kb.nnz; b.rp = Kb.rp; b.ci = Kb.ci; b.v = Kvb; b.x = xb; b.y = yb; b.beta = beta;
  a.vbf = b.vbf = vbf<T>();
  if (l == 0) prof(5, spmm_bytes<T>(Ka, nb_, beta, a.vbf) + spmm_bytes<T>(Kb, nb_, beta, b.vbf), [&] { launch_spmm2(a, b, nb_, st_); });
  else launch_spmm2(a, b, nb_, st_);
}

template <class T>
void Solver::dots(int l, const DotArgs<T>& a, const DCsr* K, double* out) {
  const double sz = sizeof(T), w = a.w, r = a.nrows;
  double b = (a.a && a.a != a.z ? sz * w * r : 0.0) + (a.y && a.y != a.z ? sz * w * r : 0.0);
  if (a.Kv && K) b += 4.0 * (r + 1) + (4.0 + sz) * K->nnz + sz * w * K->n;
  else b += sz * w * r;
  if (l == 0 && a.Kv) prof(6, b, [&] { launch_dots(a, partial_, out, st_); });
  else launch_dots(a, partial_, out, st_);
}

template <class T>
void Solver::kacz(int l, const KaczArgs<T>& a0, long nnz_colour) {
  KaczArgs<T> a = a0;
  a.vbf = vbf<T>();
  a.nnz_total = nnz_colour;
  a.nnz_rows = a.nrows;
  const double sz = sizeof(T), vs = a.vbf ? 2.0 : sz, w = a.w, r = a.nrows, z = (double)nnz_colour;
  double b = r * (8.0 + 4.0 + sz) + (4.0 + vs) * z + 2.0 * sz * w * z;
  if (a.bv) b += vs * z;
  if (a.lam) b += 2.0 * sz * r;
  if (a.rmode == M_IDENT) b += sz * w * r;
  if (a.kap) b += sz * w * r;
  if (l == 0) prof(1, b, [&] { launch_kacz(a, st_); });
  else launch_kacz(a, st_);
}

// Long rows of a level's sides: a row is long when its operator row (A or A^t) or its B / C row
// holds more than max(256, 8 x the mean row length) entries.  Built once per level (host copies of
// the row pointers), before the additive phase captures its graph.
void Solver::long_rows(Level& L) {
  auto side = [&](LongRows& g, const DCsr& K, const DCsr* M, int rows) {
    if (g.done) return;
    g.done = true;
    if (!K.rp || rows <= 0) return;
    std::vector<int> kr, mr;
    d2h(kr, K.rp, (size_t)rows + 1, st_);
    if (M && M->rp) d2h(mr, M->rp, (size_t)rows + 1, st_);
    const double tk = std::max(256.0, 8.0 * (double)(kr[rows] - kr[0]) / rows);
    const double tm = mr.empty() ? 0.0 : std::max(256.0, 8.0 * (double)(mr[rows] - mr[0]) / rows);
    std::vector<unsigned char> flag(rows, 0);
    std::vector<int> list;
    for (int i = 0; i < rows; ++i) {
      const bool lng = kr[i + 1] - kr[i] > tk || (!mr.empty() && mr[i + 1] - mr[i] > tm);
      if (lng) { flag[i] = 1; list.push_back(i); }
    }
    if (list.empty()) return;
    g.flag = ar_.alloc<unsigned char>(rows);
    h2d(g.flag, flag, st_);
    g.rows = ar_.alloc<int>(list.size());
    h2d(g.rows, list, st_);
    g.n = (int)list.size();
    sync();
  };
  side(L.lgu, L.A, L.finest ? nullptr : &L.B, L.m);
  if (!spd_) side(L.lgv, L.At, L.finest ? nullptr : &L.C, L.n);
}

template <class T>
void Solver::attach_long(int l, RowOpArgs<T>& a) {
  Level& L = *lv_[l];
  if (!a.Kv && a.mmode != M_CSR) return;   // no walk
  if (!L.lgu.done || (!spd_ && !L.lgv.done)) {
    if (capturing_) return;
    long_rows(L);
  }
  const LongRows* g = nullptr;
  if (a.Krp == L.A.rp && a.nrows == L.m) g = &L.lgu;
  else if (!spd_ && a.Krp == L.At.rp && a.nrows == L.n) g = &L.lgv;
  if (g && g->n > 0) { a.lflag = g->flag; a.lrows = g->rows; a.nlong = g->n; }
}

static double avg_row(const DCsr& M) { return M.m > 0 ? (double)M.nnz / M.m : 0.0; }

static double plan_bytes(const Plan& p) {
  return 12.0 * p.L->nnz + 4.0 * p.L->m + 12.0 * p.Rt->nnz + 4.0 * p.Rt->m + 16.0 * p.nnz;
}

void Solver::prof_finish() {
  if (pev_.empty()) return;
  sync();
  double ms[8] = {};
  for (size_t i = 0; i < pev_.size(); ++i) {
    const ProfEv& e = pev_[i];
    float t = 0.0f;
    const hipError_t er = hipEventElapsedTime(&t, e.a, e.b);
    if (er != hipSuccess)
      throw SolverError{ST_E_DEVICE, std::string("eager event ") + std::to_string(i) + "/" +
                                         std::to_string(pev_.size()) + " (class " + std::to_string(e.cls) +
                                         "): " + hipGetErrorString(er)};
    ms[e.cls] += t;
  }
  pev_.clear();
  ev_used_ = 0;
  for (int c = 0; c < 8; ++c) {
    rep_.prof_ms[c] = ms[c];
    rep_.prof_launches[c] = pn_[c];
    rep_.prof_bytes[c] = pbytes_[c];
  }
}

// ------------------------------------------------------------------------------------------------
DCsr Solver::upload(const HCsr& h, bool with_values) {
  DCsr d;
  d.m = h.m; d.n = h.n; d.nnz = h.nnz();
  d.rp = ar_.alloc<int>(h.m + 1);
  d.ci = ar_.alloc<int>(d.nnz);
  d.v = ar_.alloc<double>(d.nnz);
  h2d(d.rp, h.rp, st_);
  h2d(d.ci, h.ci, st_);
  if (with_values && !h.v.empty()) h2d(d.v, h.v, st_);
  if (mixed_) d.vf = ar_.alloc<float>(d.nnz);
  return d;
}

void Solver::alloc_level_buffers(Level& L) {
  const int mu = rows_u(L), mv = rows_v(L);
  const int wmax = std::max(nt_, nb_);
  auto& b = L.bd;
  // The test blocks hold n_t columns but get the scratch blocks' capacity (max(n_t, n_b) columns):
  // the test relaxation swaps Ut / tU and Vt / tV, and the scratch blocks are later written with n_b
  // columns (Cholesky-QR, residual blocks)
  if (!spd_) {
    b.Ut = ar_.alloc<double>((size_t)mu * wmax);
    b.Vt = ar_.alloc<double>((size_t)mv * wmax);
    double* UV = ar_.alloc<double>((size_t)(mu + mv) * nb_);
    b.Ub = UV; b.Vb = UV + (size_t)mu * nb_;
    double* UV2 = ar_.alloc<double>((size_t)(mu + mv) * nb_);
    b.Ua = UV2; b.Va = UV2 + (size_t)mu * nb_;
    double* KT = ar_.alloc<double>((size_t)(mu + mv) * nb_);
    b.kap = KT; b.tau = KT + (size_t)mu * nb_;
    b.tU = ar_.alloc<double>((size_t)mu * wmax);
    b.tV = ar_.alloc<double>((size_t)mv * wmax);
    b.tU2 = ar_.alloc<double>((size_t)mu * wmax);
    b.tV2 = ar_.alloc<double>((size_t)mv * wmax);
  } else {
    b.Ut = ar_.alloc<double>((size_t)mu * wmax);
    b.Ub = ar_.alloc<double>((size_t)mu * nb_);
    b.Ua = ar_.alloc<double>((size_t)mu * nb_);
    b.kap = ar_.alloc<double>((size_t)mu * nb_);
    b.tU = ar_.alloc<double>((size_t)mu * wmax);
    b.tU2 = ar_.alloc<double>((size_t)mu * wmax);
  }
  L.ad.dinvB = ar_.alloc<double>(mu);
  if (!spd_) L.ad.dinvC = ar_.alloc<double>(mv);
  if (minimal_) {
    L.ad.rnA = ar_.alloc<double>(L.m);
    if (spd_) {
      L.ad.rnAab = ar_.alloc<double>(L.m);
      L.ad.rnAbb = ar_.alloc<double>(L.m);
    } else {
      L.ad.rnAt = ar_.alloc<double>(L.n);
    }
    L.smU = ar_.alloc<double>(mu);
    if (!spd_) L.smV = ar_.alloc<double>(mv);
  }
  if (mixed_) {
    auto& f = L.bf;
    if (!spd_) {
      float* UV = ar_.alloc<float>((size_t)(mu + mv) * nb_);
      f.Ub = UV; f.Vb = UV + (size_t)mu * nb_;
      float* UV2 = ar_.alloc<float>((size_t)(mu + mv) * nb_);
      f.Ua = UV2; f.Va = UV2 + (size_t)mu * nb_;
      float* KT = ar_.alloc<float>((size_t)(mu + mv) * nb_);
      f.kap = KT; f.tau = KT + (size_t)mu * nb_;
      f.tU = ar_.alloc<float>((size_t)mu * nb_);
      f.tV = ar_.alloc<float>((size_t)mv * nb_);
    } else {
      f.Ub = ar_.alloc<float>((size_t)mu * nb_);
      f.Ua = ar_.alloc<float>((size_t)mu * nb_);
      f.kap = ar_.alloc<float>((size_t)mu * nb_);
      f.tU = ar_.alloc<float>((size_t)mu * nb_);
    }
    L.af.dinvB = ar_.alloc<float>(mu);
    if (!spd_) L.af.dinvC = ar_.alloc<float>(mv);
    if (minimal_) {
      L.af.rnA = ar_.alloc<float>(L.m);
      if (spd_) {
        L.af.rnAab = ar_.alloc<float>(L.m);
        L.af.rnAbb = ar_.alloc<float>(L.m);
      } else {
        L.af.rnAt = ar_.alloc<float>(L.n);
      }
    }
  }
}

// Values derived from the level operators: diagonal inverses and Kaczmarz row sums.
void Solver::refresh_level_aux(Level& L) {
  launch_diag_inv(L.B.m, L.B.rp, L.B.ci, L.B.v, L.ad.dinvB, st_);
  if (!spd_) launch_diag_inv(L.C.m, L.C.rp, L.C.ci, L.C.v, L.ad.dinvC, st_);
  if (minimal_) {
    if (spd_) {
      launch_row_sq(L.m, L.A.rp, L.A.v, L.finest ? nullptr : L.B.v, L.ad.rnA, L.ad.rnAab, L.ad.rnAbb, L.A.ci, st_);
      // Jacobi pre-smoothing of the LS fit uses N = A: 1 / diag(A)
      launch_diag_inv(L.m, L.A.rp, L.A.ci, L.A.v, L.smU, st_);
    } else {
      launch_row_sq(L.m, L.A.rp, L.A.v, nullptr, L.ad.rnA, nullptr, nullptr, L.A.ci, st_);
      launch_row_sq(L.n, L.At.rp, L.At.v, nullptr, L.ad.rnAt, nullptr, nullptr, L.At.ci, st_);
      if (square_) {
        // square coarsening measures strength on A itself: the pre-smoothing step uses 1 / diag(A)
        // on both sides
        launch_diag_inv(L.m, L.A.rp, L.A.ci, L.A.v, L.smU, st_);
        launch_diag_inv(L.m, L.A.rp, L.A.ci, L.A.v, L.smV, st_);
      } else {
        launch_recip(L.m, L.ad.rnA, L.smU, st_);    // diag(A A^t) = row norms^2 of A
        launch_recip(L.n, L.ad.rnAt, L.smV, st_);   // diag(A^t A) = column norms^2
      }
    }
  }
  if (mixed_) {
    auto cast = [&](const DCsr& a) { cast_vals(a); };
    cast(L.A);
    if (!spd_) { cast(L.At); cast(L.C); }
    cast(L.B);
    launch_copy_cast_df(L.ad.dinvB, L.af.dinvB, L.B.m, st_);
    if (!spd_) launch_copy_cast_df(L.ad.dinvC, L.af.dinvC, L.C.m, st_);
    if (minimal_) {
      launch_copy_cast_df(L.ad.rnA, L.af.rnA, L.m, st_);
      if (spd_) {
        launch_copy_cast_df(L.ad.rnAab, L.af.rnAab, L.m, st_);
        launch_copy_cast_df(L.ad.rnAbb, L.af.rnAbb, L.m, st_);
      } else {
        launch_copy_cast_df(L.ad.rnAt, L.af.rnAt, L.n, st_);
      }
    }
  }
}

// Levels with at most this many rows run whole Kaczmarz sweeps (all colours) in one workgroup.
static const int KACZ_WG_MAX_ROWS = 4096;

static std::vector<long> colour_nnz(const HCsr& A, const std::vector<int>& rows, const std::vector<int>& cptr) {
  std::vector<long> z(cptr.size() > 0 ? cptr.size() - 1 : 0, 0);
  for (size_t c = 0; c + 1 < cptr.size(); ++c)
    for (int t = cptr[c]; t < cptr[c + 1]; ++t) z[c] += A.rp[rows[t] + 1] - A.rp[rows[t]];
  return z;
}

// Kaczmarz row order (§5.3): multicolour (greedy first-fit colouring of "rows sharing a column"),
// or lexicographic, every row its own colour.
std::vector<int> Solver::row_colours(const HCsr& M) const {
  if (p_.kaczmarz_order == 1) {
    std::vector<int> c(M.m);
    for (int i = 0; i < M.m; ++i) c[i] = i;
    return c;
  }
  return greedy_row_colouring(M);
}

// Starts the colouring of a level's Kaczmarz order on a host thread: it needs the level's pattern
// only (host copies that do not change afterwards), and the set-up of the level's coarsening runs
// meanwhile.
void Solver::colour(Level& L) {
  if (!minimal_) return;
  const HCsr* a = &L.hA;
  const HCsr* at = spd_ ? nullptr : &L.hAt;   // eigenproblems: B_l lives on A_l's pattern
  L.coloured = false;
  L.colour_job = std::async(std::launch::async, [this, a, at] {
    ColourJob j;
    colour_order(row_colours(*a), j.rows, j.cptr);
    j.cnnz = colour_nnz(*a, j.rows, j.cptr);
    if (at) {
      colour_order(row_colours(*at), j.rows2, j.cptr2);
      j.cnnz2 = colour_nnz(*at, j.rows2, j.cptr2);
    }
    return j;
  });
}

// Waits for a level's colouring and uploads it (once).
void Solver::ensure_colours(Level& L) {
  if (L.coloured) return;
  ColourJob j = L.colour_job.get();
  L.coloured = true;
  L.kA_rows = ar_.alloc<int>(j.rows.size());
  h2d(L.kA_rows, j.rows, st_);
  L.kA_cptr = j.cptr;
  L.kA_cnnz = j.cnnz;
  L.d_kA_cptr = ar_.alloc<int>(j.cptr.size());
  h2d(L.d_kA_cptr, j.cptr, st_);
  if (spd_) {
    L.kacz_wg = L.m <= KACZ_WG_MAX_ROWS;
  } else {
    L.kAt_rows = ar_.alloc<int>(j.rows2.size());
    h2d(L.kAt_rows, j.rows2, st_);
    L.kAt_cptr = j.cptr2;
    L.kAt_cnnz = j.cnnz2;
    L.d_kAt_cptr = ar_.alloc<int>(j.cptr2.size());
    h2d(L.d_kAt_cptr, j.cptr2, st_);
    L.kacz_wg = std::max(L.m, L.n) <= KACZ_WG_MAX_ROWS;
  }
  sync();
}

// ------------------------------------------------------------------------------------------------
void Solver::finest_level(const double* init_tests) {
  auto L = std::make_unique<Level>();
  L->finest = true;
  L->m = A0_.m; L->n = A0_.n;
  L->hA = A0_;
  if (pb_.dA) {
    L->A = *pb_.dA;
    if (mixed_) L->A.vf = ar_.alloc<float>(L->A.nnz);
  } else {
    L->A = upload(A0_, true);
  }
  if (spd_) {
    L->At = L->A;
    L->B = L->A;
    if (pb_.dB) {
      L->B.v = pb_.dB->v;
    } else {
      HCsr Bh = A0_;   // identity on A's pattern
      for (int i = 0; i < Bh.m; ++i)
        for (int k = Bh.rp[i]; k < Bh.rp[i + 1]; ++k) Bh.v[k] = Bh.ci[k] == i ? 1.0 : 0.0;
      L->B.v = ar_.alloc<double>(L->A.nnz);
      h2d(L->B.v, Bh.v, st_);
    }
    if (mixed_) L->B.vf = ar_.alloc<float>(L->A.nnz);
  } else if (pb_.dAt) {
    L->hAt = transpose(A0_, &L->permAt);
    L->At = *pb_.dAt;
    if (mixed_) L->At.vf = ar_.alloc<float>(L->At.nnz);
    auto identp = [&](int n) {
      HCsr I;
      I.m = I.n = n;
      I.rp.resize(n + 1); I.ci.resize(n);
      for (int i = 0; i <= n; ++i) I.rp[i] = i;
      for (int i = 0; i < n; ++i) I.ci[i] = i;
      return I;
    };
    L->hB = identp(L->m);
    L->hC = identp(L->n);
    L->B = *pb_.dB;
    L->C = *pb_.dC;
    if (mixed_) { L->B.vf = ar_.alloc<float>(L->B.nnz); L->C.vf = ar_.alloc<float>(L->C.nnz); }
  } else {
    L->hAt = transpose(A0_, &L->permAt);
    L->At = upload(L->hAt, true);
    auto ident = [&](int n) {
      HCsr I;
      I.m = I.n = n;
      I.rp.resize(n + 1); I.ci.resize(n); I.v.assign(n, 1.0);
      for (int i = 0; i <= n; ++i) I.rp[i] = i;
      for (int i = 0; i < n; ++i) I.ci[i] = i;
      return I;
    };
    L->hB = ident(L->m);
    L->hC = ident(L->n);
    L->B = upload(L->hB, true);
    L->C = upload(L->hC, true);
  }
  alloc_level_buffers(*L);
  refresh_level_aux(*L);
  colour(*L);
  // initial test vectors (column-major input -> row-major blocks)
  const int mu = rows_u(*L), mv = rows_v(*L);
  const int rows = spd_ ? mu : mu + mv;
  if (init_tests) {
    std::vector<double> U((size_t)mu * nt_), V(spd_ ? 0 : (size_t)mv * nt_);
    for (int c = 0; c < nt_; ++c)
      for (int r = 0; r < rows; ++r) {
        double x = init_tests[(size_t)c * rows + r];
        if (r < mu) U[(size_t)r * nt_ + c] = x;
        else V[(size_t)(r - mu) * nt_ + c] = x;
      }
    h2d(L->bd.Ut, U, st_);
    if (!spd_) h2d(L->bd.Vt, V, st_);
  } else {
    // SplitMix64 stream, column-major over [U_t; V_t], generated on the device
    launch_splitmix_block(mu, spd_ ? 0 : mv, nt_, p_.seed, L->bd.Ut, spd_ ? nullptr : L->bd.Vt, st_);
  }
  lv_.push_back(std::move(L));
}

// ||A||_2 estimate: 30 power steps on A^t A from a SplitMix64 start vector.
void Solver::norm_estimate() {
  Level& L = *lv_[0];
  const int m = L.m, n = L.n;
  double* x = L.bd.tU2;          // size >= n (n <= m for SVD; equal for SPD)
  double* t = L.bd.tU;           // size >= m
  double* y = spd_ ? L.bd.kap : L.bd.tV;   // size >= n
  launch_splitmix_block(n, 0, 1, p_.seed ^ NORM_SEED_XOR, x, nullptr, st_);
  DotArgs<double> da;
  da.nrows = n; da.w = 1; da.a = x; da.z = x;
  launch_dots<double>(da, partial_, r1_, st_);
  launch_scale_cols<double>(n, 1, x, r1_, 0, st_);
  for (int it = 0; it < 30; ++it) {
    launch_spmm<double>(m, 1, L.A.rp, L.A.ci, L.A.v, x, t, 0.0, st_, L.A.nnz);
    launch_spmm<double>(n, 1, L.At.rp, L.At.ci, L.At.v, t, y, 0.0, st_, L.At.nnz);
    da = DotArgs<double>{};
    da.nrows = n; da.w = 1; da.a = y; da.z = y;
    launch_dots<double>(da, partial_, r1_, st_);
    HIPCHK(hipMemcpyAsync(x, y, sizeof(double) * n, hipMemcpyDeviceToDevice, st_));
    launch_scale_cols<double>(n, 1, x, r1_, 0, st_);
  }
  launch_spmm<double>(m, 1, L.A.rp, L.A.ci, L.A.v, x, t, 0.0, st_, L.A.nnz);
  da = DotArgs<double>{};
  da.nrows = m; da.w = 1; da.a = t; da.z = t;
  launch_dots<double>(da, partial_, r1_, st_);
  std::vector<double> r;
  d2h(r, r1_, 1, st_);
  anorm_ = std::sqrt(r[0]);
  if (!(anorm_ > 0.0)) throw SolverError{ST_E_INVALID, "matrix norm estimate is zero"};
}

// ------------------------------------------------------------------------------------------------
// Hierarchy structure (first multiplicative cycle only)
// ------------------------------------------------------------------------------------------------
// Entries of a strength product computed per device pass (16 bytes each while on the device).
static const size_t STRENGTH_CHUNK = size_t(1) << 25;

HCsr Solver::strength_operator(Level& L, bool u_side, bool finest) {
  // Eigenproblems (§5.2) and square coarsening (§5.1) measure strength on A itself; SVD otherwise
  // on A A^t (u) and A^t A (v) (§3.7).
  HCsr N;
  if (spd_ || square_) {
    N = L.hA;
    if (finest) N.v = A0_.v;
    else d2h(N.v, L.A.v, L.A.nnz, st_);
    return N;
  }
  const bool filt = finest && p_.strength_rule == 2 && p_.df_filter > 0.0;
  HCsr Af = L.hA;
  if (filt) {
    // rows (terms) appearing in more than df_filter * n columns are left out of the strength graph
    HCsr F;
    F.m = Af.m; F.n = Af.n;
    F.rp.assign(Af.m + 1, 0);
    for (int i = 0; i < Af.m; ++i) {
      int len = Af.rp[i + 1] - Af.rp[i];
      bool keep = len <= p_.df_filter * Af.n;
      if (keep) {
        for (int k = Af.rp[i]; k < Af.rp[i + 1]; ++k) {
          F.ci.push_back(Af.ci[k]);
          F.v.push_back(A0_.v[k]);
        }
      }
      F.rp[i + 1] = (int)F.ci.size();
    }
    Af = F;
  }
  HCsr AfT = transpose(Af, nullptr);
  DCsr dAf, dAfT;
  if (filt) {
    dAf = upload(Af, true);
    dAfT = upload(AfT, true);
  } else {
    dAf = L.A;
    dAfT = L.At;
  }
  const int lev = (int)(std::find_if(lv_.begin(), lv_.end(), [&](const auto& q) { return q.get() == &L; }) - lv_.begin());
  vmark(u_side ? "  strength A A^t: copies, transpose" : "  strength A^t A: copies, transpose", lev);
  N = u_side ? symbolic_product(Af, AfT) : symbolic_product(AfT, Af);
  vmark("  strength: symbolic product", lev);
  // numeric on the device: entries are dot products of rows of A (u) or of A^t (v), computed in
  // chunks of at most STRENGTH_CHUNK entries so that the product's device arrays stay bounded; a
  // chunk's row indices are expanded on the device from the row pointers
  int* d_rp = ar_.alloc<int>((size_t)N.m + 1);
  h2d(d_rp, N.rp, st_);
  const DCsr& M = u_side ? dAf : dAfT;
  if (p_.strength_rule == 2) {
    // top-s rule: only the s strongest off-diagonal entries of a row are ever read (strength sets,
    // interpolatory sets), so the device selects them per row and the operator comes back with
    // those entries alone; chunks hold whole rows
    const int ts = p_.top_s;
    std::vector<std::pair<int, int>> ranges;
    size_t maxc = 0;
    for (int r = 0; r < N.m;) {
      int r1 = r + 1;
      while (r1 < N.m && (size_t)(N.rp[r1 + 1] - N.rp[r]) <= STRENGTH_CHUNK) ++r1;
      ranges.push_back({r, r1});
      maxc = std::max(maxc, (size_t)(N.rp[r1] - N.rp[r]));
      r = r1;
    }
    maxc = std::max<size_t>(maxc, 1);
    int* d_row = ar_.alloc<int>(maxc);
    int* d_col = ar_.alloc<int>(maxc);
    double* d_val = ar_.alloc<double>(maxc);
    int* d_sc = ar_.alloc<int>((size_t)N.m * ts);
    double* d_sv = ar_.alloc<double>((size_t)N.m * ts);
    for (const auto& rg : ranges) {
      const long e0 = N.rp[rg.first], cnt = (long)N.rp[rg.second] - e0;
      launch_row_index_range(rg.first, rg.second, d_rp, e0, cnt, d_row, st_);
      if (cnt > 0)
        HIPCHK(hipMemcpyAsync(d_col, N.ci.data() + e0, cnt * sizeof(int), hipMemcpyHostToDevice, st_));
      launch_spgemm_dot((int)cnt, d_row, d_col, M.rp, M.ci, M.v, M.rp, M.ci, M.v, d_val, st_);
      launch_topsel(rg.first, rg.second, d_rp, e0, d_col, d_val, ts, d_sc, d_sv, st_);
    }
    std::vector<int> sc;
    std::vector<double> sv;
    d2h(sc, d_sc, (size_t)N.m * ts, st_);
    d2h(sv, d_sv, (size_t)N.m * ts, st_);
    if (p_.verbose >= 2) {
      std::fprintf(stderr, "[slamg]   strength product of level %d: %d entries, top %d per row kept\n", lev, N.nnz(), ts);
      std::fflush(stderr);
    }
    HCsr R;
    R.m = N.m; R.n = N.n;
    R.rp.assign((size_t)N.m + 1, 0);
    for (int i = 0; i < N.m; ++i) {
      for (int q = 0; q < ts; ++q) {
        const int j = sc[(size_t)i * ts + q];
        if (j < 0) break;
        R.ci.push_back(j);
        R.v.push_back(sv[(size_t)i * ts + q]);
      }
      R.rp[i + 1] = (int)R.ci.size();
    }
    vmark("  strength: device products, top-s selection", lev);
    for (const void* d : {(const void*)d_rp, (const void*)d_row, (const void*)d_col, (const void*)d_val,
                          (const void*)d_sc, (const void*)d_sv})
      ar_.release(d);
    if (filt) {
      for (const DCsr* d : {&dAf, &dAfT}) {
        ar_.release(d->rp);
        ar_.release(d->ci);
        ar_.release(d->v);
      }
    }
    return R;
  }
  const size_t total = (size_t)N.nnz(), chunk = std::min<size_t>(total, STRENGTH_CHUNK);
  int* d_row = ar_.alloc<int>(chunk);
  int* d_col = ar_.alloc<int>(chunk);
  double* d_val = ar_.alloc<double>(chunk);
  N.v.resize(total);
  vmark("  strength: value array", lev);
  for (size_t e0 = 0; e0 < total; e0 += chunk) {
    const size_t cnt = std::min(chunk, total - e0);
    // rows [r0, r1) hold the entries [e0, e0 + cnt)
    const int r0 = (int)(std::upper_bound(N.rp.begin(), N.rp.end(), (int)e0) - N.rp.begin()) - 1;
    const int r1 = (int)(std::lower_bound(N.rp.begin(), N.rp.end(), (int)(e0 + cnt)) - N.rp.begin());
    launch_row_index_range(r0, r1, d_rp, (long)e0, (long)cnt, d_row, st_);
    HIPCHK(hipMemcpyAsync(d_col, N.ci.data() + e0, cnt * sizeof(int), hipMemcpyHostToDevice, st_));
    launch_spgemm_dot((int)cnt, d_row, d_col, M.rp, M.ci, M.v, M.rp, M.ci, M.v, d_val, st_);
    HIPCHK(hipMemcpyAsync(N.v.data() + e0, d_val, cnt * sizeof(double), hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
  }
  if (p_.verbose >= 2) {
    std::fprintf(stderr, "[slamg]   strength product of level %d: %zu entries\n", lev, total);
    std::fflush(stderr);
  }
  vmark("  strength: device products and transfers", lev);
  // the product's entries are on the host now: its device arrays (and the filtered operator's)
  // go back to the solve's budget
  ar_.release(d_rp);
  ar_.release(d_row);
  ar_.release(d_col);
  ar_.release(d_val);
  if (filt) {
    for (const DCsr* d : {&dAf, &dAfT}) {
      ar_.release(d->rp);
      ar_.release(d->ci);
      ar_.release(d->v);
    }
  }
  return N;
}

void Solver::build_side(Level& L, Side& S, const HCsr& N, int npts, Strength* keep) {
  (void)L;
  std::vector<int> Sp, Si;
  strength_sets(N, p_.theta, p_.strength_rule, p_.top_s, Sp, Si);
  S.npts = npts;
  S.is_c = rs_coarsen(Sp, Si, npts);
  std::vector<int> ptr, fine_cols;
  interp_pattern(Sp, Si, N, S.is_c, nt_ - 1, ptr, fine_cols, S.capped);
  finish_side(S, ptr, fine_cols);
  if (keep) {
    keep->Sp = std::move(Sp);
    keep->Si = std::move(Si);
  }
}

// Completed C-set of a side with fewer than `need` C-points: its F-points that strongly influence
// the most points (Algorithm 1's initial measure; lowest index on ties) become C-points until it
// has `need`, and its interpolatory sets are rebuilt on the same strength sets.  A side with at
// most `need` points keeps all of them.
void Solver::complete_side(Side& S, const HCsr& N, const Strength& st, int need) {
  if (S.nc >= need) return;
  if (S.npts <= need) {
    identity_side(S, S.npts);
    return;
  }
  std::vector<int> infl(S.npts, 0);
  for (int k : st.Si) ++infl[k];
  std::vector<int> f;
  for (int i = 0; i < S.npts; ++i)
    if (!S.is_c[i]) f.push_back(i);
  std::stable_sort(f.begin(), f.end(), [&](int a, int b) { return infl[a] > infl[b]; });
  for (int t = 0; t < need - S.nc; ++t) S.is_c[f[t]] = 1;
  std::vector<int> ptr, fine_cols;
  interp_pattern(st.Sp, st.Si, N, S.is_c, nt_ - 1, ptr, fine_cols, S.capped);
  finish_side(S, ptr, fine_cols);
}

// Every point a C-point: the interpolation is the identity (one-sided coarsening of a level).
void Solver::identity_side(Side& S, int npts) {
  S.npts = npts;
  S.is_c.assign(npts, 1);
  S.capped = 0;
  std::vector<int> ptr(npts + 1), fine_cols(npts);
  for (int i = 0; i <= npts; ++i) ptr[i] = i;
  for (int i = 0; i < npts; ++i) fine_cols[i] = i;
  finish_side(S, ptr, fine_cols);
}

void Solver::finish_side(Side& S, const std::vector<int>& ptr, const std::vector<int>& fine_cols) {
  const int npts = S.npts;
  std::vector<int> cidx(npts, -1);
  S.cpts.clear();
  for (int i = 0; i < npts; ++i)
    if (S.is_c[i]) { cidx[i] = (int)S.cpts.size(); S.cpts.push_back(i); }
  S.nc = (int)S.cpts.size();
  S.Ppat = HCsr();
  S.Ppat.m = npts; S.Ppat.n = S.nc;
  S.Ppat.rp = ptr;
  S.Ppat.ci.resize(fine_cols.size());
  S.Ppat.v.assign(fine_cols.size(), 0.0);
  S.qmax = 0;
  int nF = 0;
  for (int i = 0; i < npts; ++i) {
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) S.Ppat.ci[k] = cidx[fine_cols[k]];
    if (S.is_c[i]) S.Ppat.v[ptr[i]] = 1.0;
    else { ++nF; S.qmax = std::max(S.qmax, ptr[i + 1] - ptr[i]); }
  }
  S.nF = nF;
  S.Ptpat = transpose(S.Ppat, &S.perm);
}

// Decide whether level l is coarsened (true) or becomes the coarsest level (false).
bool Solver::build_structure(int l) {
  Level& L = *lv_[l];
  if (size_of(L) <= p_.coarse_max || l + 1 >= p_.max_levels) return false;
  vmark("(before set-up of the level)", l);
  HCsr Nu = strength_operator(L, true, l == 0);
  vmark("strength operator", l);
  Side su, sv;
  Strength stu, stv;
  build_side(L, su, Nu, L.m, &stu);
  vmark("strength sets, Algorithm 1, interpolatory sets", l);
  HCsr Nv;
  if (square_) {
    // §5.1: the v-side takes the u-side's C/F split and interpolatory sets (one pattern for P and
    // Q, square levels); only its LS weights differ
    sv = su;
    sv.capped = 0;
  } else if (!spd_) {
    Nv = strength_operator(L, false, l == 0);
    build_side(L, sv, Nv, L.n, &stv);
  }
  const int need = nb_ + nt_;
  const Side su0 = su, sv0 = sv;
  if (!spd_) {
    // one-sided coarsening: a side that would keep fewer than n_b + n_t points while the other
    // side coarsens keeps all of its points
    if (su.nc < need && sv.nc >= need) identity_side(su, L.m);
    else if (sv.nc < need && su.nc >= need) identity_side(sv, L.n);
  }
  auto coarsens = [&] {
    const int nc = spd_ ? su.nc : su.nc + sv.nc;
    return !(nc > p_.stall_ratio * size_of(L)) && su.nc >= need && (spd_ || sv.nc >= need);
  };
  if (!coarsens()) {
    if (size_of(L) <= p_.coarse_dense_max) return false;
    // completed C-sets of Algorithm 1's split instead of a coarsest level too large for the
    // dense coarsest solves
    su = su0;
    complete_side(su, Nu, stu, need);
    if (square_) {
      sv = su;
      sv.capped = 0;
    } else if (!spd_) {
      sv = sv0;
      complete_side(sv, Nv, stv, need);
    }
    if (!coarsens()) return false;
  }
  // device copies
  auto devside = [&](Side& S) {
    S.P = upload(S.Ppat, true);
    S.Pt = upload(S.Ptpat, false);
    S.d_perm = ar_.alloc<int>(S.perm.size());
    h2d(S.d_perm, S.perm, st_);
    S.d_cpts = ar_.alloc<int>(S.nc);
    h2d(S.d_cpts, S.cpts, st_);
    std::vector<int> F;
    for (int i = 0; i < S.npts; ++i)
      if (!S.is_c[i]) F.push_back(i);
    S.d_F = ar_.alloc<int>(F.size());
    h2d(S.d_F, F, st_);
    S.d_prp = S.P.rp;
    std::vector<int> fc(S.Ppat.ci.size());
    for (int i = 0; i < S.npts; ++i)
      for (int k = S.Ppat.rp[i]; k < S.Ppat.rp[i + 1]; ++k) fc[k] = S.cpts[S.Ppat.ci[k]];
    S.d_fc = ar_.alloc<int>(fc.size());
    h2d(S.d_fc, fc, st_);
    launch_perm_gather(S.Pt.nnz, S.d_perm, S.P.v, S.Pt.v, st_);
  };
  devside(su);
  if (!spd_) devside(sv);
  vmark("transfer uploads", l);
  L.su = std::move(su);
  if (!spd_) L.sv = std::move(sv);
  rep_.capped[l] = L.su.capped + (spd_ ? 0 : L.sv.capped);
  make_coarse_level(l);
  return true;
}

// Symbolic Galerkin products (§3.1) and the coarse level's storage.
void Solver::make_coarse_level(int l) {
  Level& L = *lv_[l];
  auto C = std::make_unique<Level>();
  // a plan over the device copy of its pattern: the row of every entry expanded on the device
  auto mkplan = [&](const DCsr& pat, const DCsr* Lm, const DCsr* Rt, double* out) {
    Plan pl;
    pl.nnz = pat.nnz;
    pl.rowC = ar_.alloc<int>(pl.nnz);
    launch_row_index(pat.m, pat.rp, pl.rowC, st_);
    pl.L = Lm; pl.Rt = Rt; pl.out = out;
    return pl;
  };
  Side& su = L.su;
  if (spd_) {
    HCsr S1 = symbolic_product(su.Ptpat, L.hA);            // P^t A
    HCsr Ac = symbolic_product(S1, su.Ppat);               // P^t A P
    L.S1 = upload(S1, false);
    L.S2 = L.S1;
    L.S2.v = ar_.alloc<double>(L.S1.nnz);                  // P^t B on the same pattern
    C->m = C->n = su.nc;
    C->A = upload(Ac, false);
    C->hA = std::move(Ac);
    C->At = C->A;
    C->B = C->A;
    C->B.v = ar_.alloc<double>(C->A.nnz);
    if (mixed_) C->B.vf = ar_.alloc<float>(C->A.nnz);
    L.plans.clear();
    L.plans.push_back(mkplan(L.S1, &su.Pt, &L.A, L.S1.v));   // rows of P^t . rows of A (= A^t)
    L.plans.push_back(mkplan(L.S1, &su.Pt, &L.B, L.S2.v));   // rows of P^t . rows of B
    // A_c, B_c: rows of S . rows of P^t (columns of P)
    L.pAc = mkplan(C->A, &L.S1, &su.Pt, C->A.v);
    L.pBc = mkplan(C->A, &L.S2, &su.Pt, C->B.v);
    L.pAc.colC = C->A.ci; L.pBc.colC = C->A.ci;
    L.plans[0].colC = L.S1.ci; L.plans[1].colC = L.S1.ci;
  } else {
    Side& sv = L.sv;
    HCsr S1 = symbolic_product(su.Ptpat, L.hA);            // P^t A      (mc x n)
    HCsr Ac = symbolic_product(S1, sv.Ppat);               // P^t A Q    (mc x nc)
    HCsr S2 = symbolic_product(su.Ptpat, L.hB);            // P^t B      (mc x m)
    HCsr Bc = symbolic_product(S2, su.Ppat);               // P^t B P
    HCsr S3 = symbolic_product(sv.Ptpat, L.hC);            // Q^t C      (nc x n)
    HCsr Cc = symbolic_product(S3, sv.Ppat);               // Q^t C Q
    L.S1 = upload(S1, false);
    L.S2 = upload(S2, false);
    L.S3 = upload(S3, false);
    C->m = su.nc; C->n = sv.nc;
    C->hAt = transpose(Ac, &C->permAt);
    C->A = upload(Ac, false);
    C->At = upload(C->hAt, false);
    C->d_permAt = ar_.alloc<int>(C->permAt.size());
    h2d(C->d_permAt, C->permAt, st_);
    C->B = upload(Bc, false);
    C->C = upload(Cc, false);
    C->hA = std::move(Ac);
    C->hB = std::move(Bc);
    C->hC = std::move(Cc);
    L.plans.clear();
    L.plans.push_back(mkplan(L.S1, &su.Pt, &L.At, L.S1.v));  // (P^t A)_{I j} = P^t row I . A^t row j
    L.plans.push_back(mkplan(L.S2, &su.Pt, &L.B, L.S2.v));   // B symmetric
    L.plans.push_back(mkplan(L.S3, &sv.Pt, &L.C, L.S3.v));
    L.plans[0].colC = L.S1.ci; L.plans[1].colC = L.S2.ci; L.plans[2].colC = L.S3.ci;
    L.pAc = mkplan(C->A, &L.S1, &sv.Pt, C->A.v); L.pAc.colC = C->A.ci;
    L.pBc = mkplan(C->B, &L.S2, &su.Pt, C->B.v); L.pBc.colC = C->B.ci;
    L.pCc = mkplan(C->C, &L.S3, &sv.Pt, C->C.v); L.pCc.colC = C->C.ci;
  }
  rep_.rows[l + 1] = C->m;
  rep_.cols[l + 1] = C->n;
  rep_.nnz[l + 1] = C->hA.nnz();
  vmark("Galerkin symbolic products and plans", l);
  alloc_level_buffers(*C);
  colour(*C);
  vmark("coarse buffers and Kaczmarz colouring", l + 1);
  lv_.push_back(std::move(C));
}

// ------------------------------------------------------------------------------------------------
// Relaxation (§3.4, §3.5, §5.3)
// ------------------------------------------------------------------------------------------------
void Solver::relax_tests(int l) {
  Level& L = *lv_[l];
  ensure_colours(L);
  auto& b = L.bd;
  const int mu = rows_u(L), mv = rows_v(L);
  DotArgs<double> da;
  for (int it = 0; it < p_.mu_t; ++it) {
    if (!minimal_) {
      if (spd_) {
        // mu_tJ weighted-Jacobi steps on B x_bar = A x from x_bar = x:
        // x_bar <- x_bar - w D_B^-1 (B x_bar - A x); then x = x_bar / ||x_bar||_B
        RowOpArgs<double> a;
        a.nrows = mu; a.w = nt_;
        a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = L.A.v; a.z = b.Ut;
        a.mmode = L.finest ? M_IDENT : M_SHARED; a.Mv = L.B.v; a.y = b.Ut;
        a.x = b.Ut; a.D = L.ad.dinvB; a.cmode = C_JAC_TEST; a.omega = p_.omega_J; a.out = b.tU;
        rowop(l, a, &L.A);
        if (!L.finest) {   // B x_bar on B's own walk (the shared walk multiplies z only)
          a.mmode = M_CSR; a.Mrp = L.A.rp; a.Mci = L.A.ci; a.avgM = avg_row(L.A);
        }
        for (int j = 1; j < p_.mu_tJ; ++j) {   // A x stays the product with the outer iterate
          a.y = b.tU; a.x = b.tU; a.out = b.tU2;
          rowop(l, a, &L.A);
          std::swap(b.tU, b.tU2);
        }
        std::swap(b.Ut, b.tU);
        da = DotArgs<double>{};
        da.nrows = mu; da.w = nt_; da.a = b.Ut; da.z = b.Ut;
        if (!L.finest) { da.Krp = L.A.rp; da.Kci = L.A.ci; da.nnzK = L.A.nnz; da.Kv = L.B.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mu, nt_, b.Ut, r1_, 0, st_);
      } else {
        // v_bar = v - w D_C^-1 (C v - A^t u), normalised in C; then u likewise with A v and B
        RowOpArgs<double> a;
        a.nrows = mv; a.w = nt_;
        a.Krp = L.At.rp; a.Kci = L.At.ci; a.nnzK = L.At.nnz; a.Kv = L.At.v; a.z = b.Ut;
        a.mmode = L.finest ? M_IDENT : M_CSR; a.Mrp = L.C.rp; a.avgM = avg_row(L.C); a.Mci = L.C.ci; a.Mv = L.C.v; a.y = b.Vt;
        a.x = b.Vt; a.D = L.ad.dinvC; a.cmode = C_JAC_TEST; a.omega = p_.omega_J; a.out = b.tV;
        for (int j = 0; j < p_.mu_tJ; ++j) {   // mu_tJ Jacobi steps on C v_bar = A^t u
          a.y = b.Vt; a.x = b.Vt; a.out = b.tV;
          rowop(l, a, &L.At);
          std::swap(b.Vt, b.tV);
        }
        da = DotArgs<double>{};
        da.nrows = mv; da.w = nt_; da.a = b.Vt; da.z = b.Vt;
        if (!L.finest) { da.Krp = L.C.rp; da.Kci = L.C.ci; da.nnzK = L.C.nnz; da.Kv = L.C.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mv, nt_, b.Vt, r1_, 0, st_);
        RowOpArgs<double> c;
        c.nrows = mu; c.w = nt_;
        c.Krp = L.A.rp; c.Kci = L.A.ci; c.nnzK = L.A.nnz; c.Kv = L.A.v; c.z = b.Vt;
        c.mmode = L.finest ? M_IDENT : M_CSR; c.Mrp = L.B.rp; c.avgM = avg_row(L.B); c.Mci = L.B.ci; c.Mv = L.B.v; c.y = b.Ut;
        c.x = b.Ut; c.D = L.ad.dinvB; c.cmode = C_JAC_TEST; c.omega = p_.omega_J; c.out = b.tU;
        for (int j = 0; j < p_.mu_tJ; ++j) {   // mu_tJ Jacobi steps on B u_bar = A v
          c.y = b.Ut; c.x = b.Ut; c.out = b.tU;
          rowop(l, c, &L.A);
          std::swap(b.Ut, b.tU);
        }
        da = DotArgs<double>{};
        da.nrows = mu; da.w = nt_; da.a = b.Ut; da.z = b.Ut;
        if (!L.finest) { da.Krp = L.B.rp; da.Kci = L.B.ci; da.nnzK = L.B.nnz; da.Kv = L.B.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mu, nt_, b.Ut, r1_, 0, st_);
      }
    } else {
      // Kaczmarz on A v = 0 (rows of A, updates v), then A^t u = 0; or A x = 0; then normalise
      auto sweep = [&](const DCsr& M, const int* rows, const std::vector<int>& cptr, const double* rn, double* x,
                       const std::vector<long>& cnnz) {
        for (size_t c = 0; c + 1 < cptr.size(); ++c) {
          KaczArgs<double> k;
          k.nrows = cptr[c + 1] - cptr[c]; k.rows = rows + cptr[c]; k.w = nt_;
          k.rp = M.rp; k.ci = M.ci; k.av = M.v; k.rn_aa = rn; k.x = x;
          kacz(l, k, cnnz[c]);
        }
      };
      // whole sweeps in one launch: per-column workgroups with the vectors in LDS where they fit,
      // else one workgroup for the block on small levels, else one launch per colour
      bool whole = false;
      {
        KaczArgs<double> h[2];
        const int* cp[2] = {nullptr, nullptr};
        int nc[2] = {0, 0};
        h[0].nnz_total = L.A.nnz; h[0].nnz_rows = L.A.m;
        h[0].rows = L.kA_rows; h[0].w = nt_; h[0].rp = L.A.rp; h[0].ci = L.A.ci; h[0].av = L.A.v;
        h[0].rn_aa = L.ad.rnA; h[0].x = spd_ ? b.Ut : b.Vt;
        cp[0] = L.d_kA_cptr; nc[0] = (int)L.kA_cptr.size() - 1;
        if (!spd_) {
          h[1].nnz_total = L.At.nnz; h[1].nnz_rows = L.At.m;
          h[1].rows = L.kAt_rows; h[1].w = nt_; h[1].rp = L.At.rp; h[1].ci = L.At.ci; h[1].av = L.At.v;
          h[1].rn_aa = L.ad.rnAt; h[1].x = b.Ut;
          cp[1] = L.d_kAt_cptr; nc[1] = (int)L.kAt_cptr.size() - 1;
        }
        const int nx[2] = {spd_ ? L.m : L.n, L.m};
        whole = launch_kacz_lds<double>(h, cp, nc, nx, spd_ ? 1 : 2, 1, st_);
        if (!whole && L.kacz_wg) {
          launch_kacz_wg<double>(h, cp, nc, spd_ ? 1 : 2, 1, st_);
          whole = true;
        }
      }
      if (whole) {
        da = DotArgs<double>{};
        da.nrows = mu; da.w = nt_; da.a = b.Ut; da.z = b.Ut;
        if (!L.finest) { da.Krp = spd_ ? L.A.rp : L.B.rp; da.Kci = spd_ ? L.A.ci : L.B.ci; da.nnzK = spd_ ? L.A.nnz : L.B.nnz; da.Kv = L.B.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mu, nt_, b.Ut, r1_, 0, st_);
        if (!spd_) {
          da = DotArgs<double>{};
          da.nrows = mv; da.w = nt_; da.a = b.Vt; da.z = b.Vt;
          if (!L.finest) { da.Krp = L.C.rp; da.Kci = L.C.ci; da.nnzK = L.C.nnz; da.Kv = L.C.v; }
          launch_dots(da, partial_, r1_, st_);
          launch_scale_cols<double>(mv, nt_, b.Vt, r1_, 0, st_);
        }
      } else if (spd_) {
        sweep(L.A, L.kA_rows, L.kA_cptr, L.ad.rnA, b.Ut, L.kA_cnnz);
        da = DotArgs<double>{};
        da.nrows = mu; da.w = nt_; da.a = b.Ut; da.z = b.Ut;
        if (!L.finest) { da.Krp = L.A.rp; da.Kci = L.A.ci; da.nnzK = L.A.nnz; da.Kv = L.B.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mu, nt_, b.Ut, r1_, 0, st_);
      } else {
        sweep(L.A, L.kA_rows, L.kA_cptr, L.ad.rnA, b.Vt, L.kA_cnnz);
        da = DotArgs<double>{};
        da.nrows = mv; da.w = nt_; da.a = b.Vt; da.z = b.Vt;
        if (!L.finest) { da.Krp = L.C.rp; da.Kci = L.C.ci; da.nnzK = L.C.nnz; da.Kv = L.C.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mv, nt_, b.Vt, r1_, 0, st_);
        sweep(L.At, L.kAt_rows, L.kAt_cptr, L.ad.rnAt, b.Ut, L.kAt_cnnz);
        da = DotArgs<double>{};
        da.nrows = mu; da.w = nt_; da.a = b.Ut; da.z = b.Ut;
        if (!L.finest) { da.Krp = L.B.rp; da.Kci = L.B.ci; da.nnzK = L.B.nnz; da.Kv = L.B.v; }
        launch_dots(da, partial_, r1_, st_);
        launch_scale_cols<double>(mu, nt_, b.Ut, r1_, 0, st_);
      }
    }
  }
}

// One boot relaxation (no sigma update) on level l with right-hand sides kap, tau (null: zero).
// zero_start: the iterate is zero on entry (a coarse correction of the additive cycle), so the
// first Jacobi-type sweep skips the products with it and need not read it.
template <class T>
void Solver::boot_relax(int l, const T* kap, const T* tau, const double* sig, int nsweeps, bool zero_start) {
  Level& L = *lv_[l];
  ensure_colours(L);
  Blocks<T>& b = blocks<T>(L);
  Aux<T>& x = aux<T>(L);
  const int mu = rows_u(L), mv = rows_v(L);
  if (nsweeps <= 0) return;
  if (minimal_) {
    // all nsweeps sweeps, all colours, in one launch: per-column workgroups with the vectors in
    // LDS where they fit, else one workgroup for the block on small levels
    KaczArgs<T> h[2];
    const int* cp[2] = {nullptr, nullptr};
    int nc[2] = {0, 0};
    const int nx[2] = {spd_ ? L.m : L.n, L.m};
    if (spd_) {
      h[0].nnz_total = L.A.nnz; h[0].nnz_rows = L.A.m;
      h[0].rows = L.kA_rows; h[0].w = nb_; h[0].rp = L.A.rp; h[0].ci = L.A.ci; h[0].av = vals<T>(L.A);
      h[0].bv = L.finest ? nullptr : vals<T>(L.B); h[0].lam = sig;
      h[0].rn_aa = x.rnA; h[0].rn_ab = x.rnAab; h[0].rn_bb = x.rnAbb; h[0].kap = kap; h[0].x = b.Ub;
      cp[0] = L.d_kA_cptr; nc[0] = (int)L.kA_cptr.size() - 1;
      h[0].vbf = vbf<T>();
      h[0].nnz_total = L.A.nnz; h[0].nnz_rows = L.A.m;
      if (launch_kacz_lds<T>(h, cp, nc, nx, 1, nsweeps, st_)) return;
      if (L.kacz_wg) {
        launch_kacz_wg<T>(h, cp, nc, 1, nsweeps, st_);
        return;
      }
    } else {
      h[0].nnz_total = L.A.nnz; h[0].nnz_rows = L.A.m;
      h[0].rows = L.kA_rows; h[0].w = nb_; h[0].rp = L.A.rp; h[0].ci = L.A.ci; h[0].av = vals<T>(L.A);
      h[0].rn_aa = x.rnA; h[0].rmode = L.finest ? M_IDENT : M_CSR; h[0].Mrp = L.B.rp; h[0].avgM = avg_row(L.B); h[0].Mci = L.B.ci;
      h[0].Mv = vals<T>(L.B); h[0].y = b.Ub; h[0].rsig = sig; h[0].kap = kap; h[0].x = b.Vb;
      h[1].nnz_total = L.At.nnz; h[1].nnz_rows = L.At.m;
      h[1].rows = L.kAt_rows; h[1].w = nb_; h[1].rp = L.At.rp; h[1].ci = L.At.ci; h[1].av = vals<T>(L.At);
      h[1].rn_aa = x.rnAt; h[1].rmode = L.finest ? M_IDENT : M_CSR; h[1].Mrp = L.C.rp; h[1].avgM = avg_row(L.C); h[1].Mci = L.C.ci;
      h[1].Mv = vals<T>(L.C); h[1].y = b.Vb; h[1].rsig = sig; h[1].kap = tau; h[1].x = b.Ub;
      cp[0] = L.d_kA_cptr; nc[0] = (int)L.kA_cptr.size() - 1;
      cp[1] = L.d_kAt_cptr; nc[1] = (int)L.kAt_cptr.size() - 1;
      h[0].vbf = h[1].vbf = vbf<T>();
      if (launch_kacz_lds<T>(h, cp, nc, nx, 2, nsweeps, st_)) return;
      if (L.kacz_wg) {
        launch_kacz_wg<T>(h, cp, nc, 2, nsweeps, st_);
        return;
      }
    }
  }
  if (nsweeps > 1) {
    for (int it = 0; it < nsweeps; ++it) boot_relax<T>(l, kap, tau, sig, 1, zero_start && it == 0);
    return;
  }
  if (!minimal_) {
    if (spd_) {
      // x <- x - w D_B^-1 (B x - (A x - kappa)/lambda)
      RowOpArgs<T> a;
      a.nrows = mu; a.w = nb_;
      a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = vals<T>(L.A); a.z = b.Ub;
      a.mmode = L.finest ? M_IDENT : M_SHARED; a.Mv = vals<T>(L.B); a.y = b.Ub;
      a.x = b.Ub; a.D = x.dinvB; a.kap = kap; a.sig = sig; a.cmode = C_JAC_BOOT; a.omega = p_.omega_J;
      a.out = b.Ua;
      if (zero_start) { a.Kv = nullptr; a.mmode = M_NONE; a.x = nullptr; }
      rowop(l, a, &L.A);
      if (p_.mu_bJ > 1) {
        // further Jacobi steps on B x_new = (A x - kappa)/lambda, A x from the outer iterate
        // (kept in the scratch block tU)
        T* keep = b.tU;
        if (zero_start) {
          if (std::is_same<T, float>::value) launch_fillf((float*)keep, (size_t)mu * nb_, 0.0f, st_);
          else launch_fill((double*)keep, (size_t)mu * nb_, 0.0, st_);
        } else {
          HIPCHK(hipMemcpyAsync(keep, b.Ub, sizeof(T) * (size_t)mu * nb_, hipMemcpyDeviceToDevice, st_));
        }
        a = RowOpArgs<T>{};
        a.nrows = mu; a.w = nb_;
        a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = vals<T>(L.A); a.z = keep;
        // B x on B's own walk (B_l shares A_l's pattern; the shared walk multiplies z only)
        a.mmode = L.finest ? M_IDENT : M_CSR; a.Mrp = L.A.rp; a.Mci = L.A.ci; a.avgM = avg_row(L.A);
        a.Mv = vals<T>(L.B); a.D = x.dinvB; a.kap = kap; a.sig = sig;
        a.cmode = C_JAC_BOOT; a.omega = p_.omega_J;
        for (int j = 1; j < p_.mu_bJ; ++j) {
          a.y = b.Ua; a.x = b.Ua; a.out = b.Ub;
          rowop(l, a, &L.A);
          std::swap(b.Ub, b.Ua);
        }
      }
      std::swap(b.Ub, b.Ua);
    } else {
      // u <- u - w D_B^-1 (B u - (A v - kappa)/sigma); then v <- v - w D_C^-1 (C v - (A^t u - tau)/sigma)
      RowOpArgs<T> a;
      a.nrows = mu; a.w = nb_;
      a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = vals<T>(L.A); a.z = b.Vb;
      a.mmode = L.finest ? M_IDENT : M_CSR; a.Mrp = L.B.rp; a.avgM = avg_row(L.B); a.Mci = L.B.ci; a.Mv = vals<T>(L.B); a.y = b.Ub;
      a.x = b.Ub; a.D = x.dinvB; a.kap = kap; a.sig = sig; a.cmode = C_JAC_BOOT; a.omega = p_.omega_J;
      a.out = b.Ua;
      if (zero_start) { a.Kv = nullptr; a.mmode = M_NONE; a.x = nullptr; }
      rowop(l, a, &L.A);
      for (int j = 1; j < p_.mu_bJ; ++j) {   // further Jacobi steps on B u = (A v - kappa)/sigma
        a.mmode = L.finest ? M_IDENT : M_CSR; a.y = b.Ua; a.x = b.Ua; a.out = b.Ub;
        rowop(l, a, &L.A);
        std::swap(b.Ub, b.Ua);
      }
      RowOpArgs<T> c;
      c.nrows = mv; c.w = nb_;
      c.Krp = L.At.rp; c.Kci = L.At.ci; c.nnzK = L.At.nnz; c.Kv = vals<T>(L.At); c.z = b.Ua;
      c.mmode = L.finest ? M_IDENT : M_CSR; c.Mrp = L.C.rp; c.avgM = avg_row(L.C); c.Mci = L.C.ci; c.Mv = vals<T>(L.C); c.y = b.Vb;
      c.x = b.Vb; c.D = x.dinvC; c.kap = tau; c.sig = sig; c.cmode = C_JAC_BOOT; c.omega = p_.omega_J;
      c.out = b.Va;
      if (zero_start) { c.mmode = M_NONE; c.x = nullptr; }
      rowop(l, c, &L.At);
      for (int j = 1; j < p_.mu_bJ; ++j) {   // further Jacobi steps on C v = (A^t u - tau)/sigma
        c.mmode = L.finest ? M_IDENT : M_CSR; c.y = b.Va; c.x = b.Va; c.out = b.Vb;
        rowop(l, c, &L.At);
        std::swap(b.Vb, b.Va);
      }
      std::swap(b.Ub, b.Ua);
      std::swap(b.Vb, b.Va);
    }
  } else {
    if (spd_) {
      // Kaczmarz on (A - lambda_j B) x = kappa
      for (size_t c = 0; c + 1 < L.kA_cptr.size(); ++c) {
        KaczArgs<T> k;
        k.nrows = L.kA_cptr[c + 1] - L.kA_cptr[c]; k.rows = L.kA_rows + L.kA_cptr[c]; k.w = nb_;
        k.rp = L.A.rp; k.ci = L.A.ci; k.av = vals<T>(L.A);
        k.bv = L.finest ? nullptr : vals<T>(L.B); k.lam = sig;
        k.rn_aa = x.rnA; k.rn_ab = x.rnAab; k.rn_bb = x.rnAbb;
        k.kap = kap; k.x = b.Ub;
        kacz(l, k, L.kA_cnnz[c]);
      }
    } else {
      // v from A v = sigma B u + kappa (rows of A), then u from A^t u = sigma C v + tau (rows of A^t)
      for (size_t c = 0; c + 1 < L.kA_cptr.size(); ++c) {
        KaczArgs<T> k;
        k.nrows = L.kA_cptr[c + 1] - L.kA_cptr[c]; k.rows = L.kA_rows + L.kA_cptr[c]; k.w = nb_;
        k.rp = L.A.rp; k.ci = L.A.ci; k.av = vals<T>(L.A); k.rn_aa = x.rnA;
        k.rmode = L.finest ? M_IDENT : M_CSR; k.Mrp = L.B.rp; k.avgM = avg_row(L.B); k.Mci = L.B.ci; k.Mv = vals<T>(L.B);
        k.y = b.Ub; k.rsig = sig; k.kap = kap; k.x = b.Vb;
        kacz(l, k, L.kA_cnnz[c]);
      }
      for (size_t c = 0; c + 1 < L.kAt_cptr.size(); ++c) {
        KaczArgs<T> k;
        k.nrows = L.kAt_cptr[c + 1] - L.kAt_cptr[c]; k.rows = L.kAt_rows + L.kAt_cptr[c]; k.w = nb_;
        k.rp = L.At.rp; k.ci = L.At.ci; k.av = vals<T>(L.At); k.rn_aa = x.rnAt;
        k.rmode = L.finest ? M_IDENT : M_CSR; k.Mrp = L.C.rp; k.avgM = avg_row(L.C); k.Mci = L.C.ci; k.Mv = vals<T>(L.C);
        k.y = b.Vb; k.rsig = sig; k.kap = tau; k.x = b.Ub;
        kacz(l, k, L.kAt_cnnz[c]);
      }
    }
  }
}

// Multiplicative-phase boot relaxation: mu_b steps, each followed by the Rayleigh quotient (3.31)
// and the sign check of §5.3.
void Solver::boot_relax_rq(int l) {
  Level& L = *lv_[l];
  auto& b = L.bd;
  const int mu = rows_u(L), mv = rows_v(L);
  for (int it = 0; it < p_.mu_b; ++it) {
    boot_relax<double>(l, nullptr, nullptr, sig_);
    DotArgs<double> d1, d2, d3;
    if (spd_) {
      d1.nrows = mu; d1.w = nb_; d1.a = b.Ub; d1.Krp = L.A.rp; d1.Kci = L.A.ci; d1.nnzK = L.A.nnz; d1.Kv = L.A.v; d1.z = b.Ub;
      dots(l, d1, &L.A, r1_);
      d2.nrows = mu; d2.w = nb_; d2.a = b.Ub; d2.z = b.Ub;
      if (!L.finest) { d2.Krp = L.A.rp; d2.Kci = L.A.ci; d2.nnzK = L.A.nnz; d2.Kv = L.B.v; }
      launch_dots(d2, partial_, r2_, st_);
      launch_rq_update(nb_, r1_, r2_, nullptr, sig_, flip_, st_);
    } else {
      d1.nrows = mu; d1.w = nb_; d1.a = b.Ub; d1.Krp = L.A.rp; d1.Kci = L.A.ci; d1.nnzK = L.A.nnz; d1.Kv = L.A.v; d1.z = b.Vb;
      dots(l, d1, &L.A, r1_);
      d2.nrows = mu; d2.w = nb_; d2.a = b.Ub; d2.z = b.Ub;
      if (!L.finest) { d2.Krp = L.B.rp; d2.Kci = L.B.ci; d2.nnzK = L.B.nnz; d2.Kv = L.B.v; }
      launch_dots(d2, partial_, r2_, st_);
      d3.nrows = mv; d3.w = nb_; d3.a = b.Vb; d3.z = b.Vb;
      if (!L.finest) { d3.Krp = L.C.rp; d3.Kci = L.C.ci; d3.nnzK = L.C.nnz; d3.Kv = L.C.v; }
      launch_dots(d3, partial_, r3_, st_);
      launch_rq_update(nb_, r1_, r2_, r3_, sig_, flip_, st_);
    }
    launch_scale_cols<double>(mu, nb_, b.Ub, flip_, 1, st_);
  }
}

// ------------------------------------------------------------------------------------------------
// LS interpolation (§3.8), Galerkin operators (§3.1), injection (§3.3)
// ------------------------------------------------------------------------------------------------
void Solver::fit_interpolation(int l, int cycle) {
  Level& L = *lv_[l];
  auto& b = L.bd;
  const int mu = rows_u(L), mv = rows_v(L);
  const bool boots = cycle >= 2;
  const int nf = nt_ + (boots ? nb_ : 0);
  // Rayleigh-quotient weights of the fitted pairs (test pairs, then boot pairs)
  auto rq_parts = [&](const double* U, const double* V, int w, int off) {
    DotArgs<double> d1, d2, d3;
    if (spd_) {
      d1.nrows = mu; d1.w = w; d1.a = U; d1.Krp = L.A.rp; d1.Kci = L.A.ci; d1.nnzK = L.A.nnz; d1.Kv = L.A.v; d1.z = U;
      d2.nrows = mu; d2.w = w; d2.a = U; d2.z = U;
      if (!L.finest) { d2.Krp = L.A.rp; d2.Kci = L.A.ci; d2.nnzK = L.A.nnz; d2.Kv = L.B.v; }
      launch_dots(d1, partial_, r1_ + off, st_);
      launch_dots(d2, partial_, r2_ + off, st_);
    } else {
      d1.nrows = mu; d1.w = w; d1.a = U; d1.Krp = L.A.rp; d1.Kci = L.A.ci; d1.nnzK = L.A.nnz; d1.Kv = L.A.v; d1.z = V;
      d2.nrows = mu; d2.w = w; d2.a = U; d2.z = U;
      if (!L.finest) { d2.Krp = L.B.rp; d2.Kci = L.B.ci; d2.nnzK = L.B.nnz; d2.Kv = L.B.v; }
      d3.nrows = mv; d3.w = w; d3.a = V; d3.z = V;
      if (!L.finest) { d3.Krp = L.C.rp; d3.Kci = L.C.ci; d3.nnzK = L.C.nnz; d3.Kv = L.C.v; }
      launch_dots(d1, partial_, r1_ + off, st_);
      launch_dots(d2, partial_, r2_ + off, st_);
      launch_dots(d3, partial_, r3_ + off, st_);
    }
  };
  rq_parts(b.Ut, b.Vt, nt_, 0);
  if (boots) rq_parts(b.Ub, b.Vb, nb_, nt_);
  launch_rq_weights(nf, r1_, r2_, spd_ ? nullptr : r3_, minimal_ ? 1 : 0, 1e-12 * anorm_,
                    redo_weights_ ? wscale_ : nullptr, wts_, st_);
  // values fitted at the F-points: the vectors themselves, or (minimal) one Jacobi step on N z = 0
  auto smooth = [&](bool u_side, const double* X, int w, double* tmp, double* out) {
    RowOpArgs<double> a;
    a.w = w; a.x = X; a.cmode = C_SMOOTH; a.omega = p_.omega_J; a.out = out;
    if (spd_ || square_) {
      // N = A (eigenproblems; both sides of a square-coarsened SVD)
      a.nrows = mu; a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = L.A.v; a.z = X;
      a.D = u_side ? L.smU : L.smV;
    } else if (u_side) {
      launch_spmm<double>(L.n, w, L.At.rp, L.At.ci, L.At.v, X, tmp, 0.0, st_, L.At.nnz);   // A^t u
      a.nrows = mu; a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = L.A.v; a.z = tmp; a.D = L.smU;
    } else {
      launch_spmm<double>(L.m, w, L.A.rp, L.A.ci, L.A.v, X, tmp, 0.0, st_, L.A.nnz);      // A v
      a.nrows = mv; a.Krp = L.At.rp; a.Kci = L.At.ci; a.nnzK = L.At.nnz; a.Kv = L.At.v; a.z = tmp; a.D = L.smV;
    }
    launch_rowop(a, st_);
  };
  auto fit_side = [&](Side& S, const double* Tb, const double* Bb, double* tmp_other, double* sm1, double* sm2,
                      bool u_side) {
    const double* B1 = Tb;
    const double* B2 = Bb;
    if (minimal_) {
      smooth(u_side, Tb, nt_, tmp_other, sm1);
      B1 = sm1;
      if (boots) { smooth(u_side, Bb, nb_, tmp_other, sm2); B2 = sm2; }
    }
    launch_ls_fit(S.nF, S.d_F, S.d_prp, S.d_fc, nt_, Tb, boots ? nb_ : 0, Bb, B1, B2, wts_, S.P.v, S.qmax, st_);
    launch_perm_gather(S.Pt.nnz, S.d_perm, S.P.v, S.Pt.v, st_);
  };
  if (spd_) {
    fit_side(L.su, b.Ut, b.Ub, nullptr, b.tU, b.tU2, true);
  } else {
    fit_side(L.su, b.Ut, b.Ub, b.tV, b.tU, b.tU2, true);
    fit_side(L.sv, b.Vt, b.Vb, b.tU, b.tV, b.tV2, false);
  }
}

void Solver::galerkin(int l) {
  Level& L = *lv_[l];
  Level& C = *lv_[l + 1];
  for (auto& pl : L.plans) prof(3, plan_bytes(pl), [&] { pl.run(st_); });
  prof(3, plan_bytes(L.pAc), [&] { L.pAc.run(st_); });
  prof(3, plan_bytes(L.pBc), [&] { L.pBc.run(st_); });
  if (!spd_) {
    prof(3, plan_bytes(L.pCc), [&] { L.pCc.run(st_); });
    launch_perm_gather(C.At.nnz, C.d_permAt, C.A.v, C.At.v, st_);
  }
  refresh_level_aux(C);
}

void Solver::inject(int l, int cycle) {
  Level& L = *lv_[l];
  Level& C = *lv_[l + 1];
  launch_gather_rows<double>(L.su.nc, nt_, L.su.d_cpts, L.bd.Ut, C.bd.Ut, st_);
  if (!spd_) launch_gather_rows<double>(L.sv.nc, nt_, L.sv.d_cpts, L.bd.Vt, C.bd.Vt, st_);
  if (cycle >= 2) {
    launch_gather_rows<double>(L.su.nc, nb_, L.su.d_cpts, L.bd.Ub, C.bd.Ub, st_);
    if (!spd_) launch_gather_rows<double>(L.sv.nc, nb_, L.sv.d_cpts, L.bd.Vb, C.bd.Vb, st_);
  }
}

// ------------------------------------------------------------------------------------------------
// Coarsest level (§3.6) and the dense additive solve (§4.2)
// ------------------------------------------------------------------------------------------------
void Solver::coarsest_mult() {
  Level& L = *lv_.back();
  const int m = L.m, n = L.n;
  if (spd_) {
    launch_fill(dA_, (size_t)m * m, 0.0, st_);
    launch_fill(dB_, (size_t)m * m, 0.0, st_);
    launch_csr_to_dense(m, L.A.rp, L.A.ci, L.A.v, dA_, m, 0, 0, false, st_);
    launch_csr_to_dense(m, L.A.rp, L.A.ci, L.B.v, dB_, m, 0, 0, false, st_);
    launch_coarse_gsvd(1, minimal_, m, m, nb_, dA_, dB_, nullptr, dwork_, sig_, L.bd.Ub, nullptr, status_, st_);
  } else {
    launch_fill(dA_, (size_t)m * n, 0.0, st_);
    launch_fill(dB_, (size_t)m * m, 0.0, st_);
    launch_fill(dC_, (size_t)n * n, 0.0, st_);
    launch_csr_to_dense(m, L.A.rp, L.A.ci, L.A.v, dA_, n, 0, 0, false, st_);
    launch_csr_to_dense(m, L.B.rp, L.B.ci, L.B.v, dB_, m, 0, 0, false, st_);
    launch_csr_to_dense(n, L.C.rp, L.C.ci, L.C.v, dC_, n, 0, 0, false, st_);
    launch_coarse_gsvd(0, minimal_, m, n, nb_, dA_, dB_, dC_, dwork_, sig_, L.bd.Ub, L.bd.Vb, status_, st_);
  }
}

// Dense X = [[0, A], [A^t, 0]] and Y = diag(B, C) (SVD) or A and B (eigen) of the coarsest level.
void Solver::dense_coarsest(double* X, double* Y) {
  Level& L = *lv_.back();
  const int N = NL_;
  launch_fill(X, (size_t)N * N, 0.0, st_);
  launch_fill(Y, (size_t)N * N, 0.0, st_);
  if (spd_) {
    launch_csr_to_dense(L.m, L.A.rp, L.A.ci, L.A.v, X, N, 0, 0, false, st_);
    launch_csr_to_dense(L.m, L.A.rp, L.A.ci, L.B.v, Y, N, 0, 0, false, st_);
  } else {
    launch_csr_to_dense(L.m, L.A.rp, L.A.ci, L.A.v, X, N, 0, L.m, false, st_);
    launch_csr_to_dense(L.m, L.A.rp, L.A.ci, L.A.v, X, N, L.m, 0, true, st_);
    launch_csr_to_dense(L.m, L.B.rp, L.B.ci, L.B.v, Y, N, 0, 0, false, st_);
    launch_csr_to_dense(L.n, L.C.rp, L.C.ci, L.C.v, Y, N, L.m, L.m, false, st_);
  }
}

// ------------------------------------------------------------------------------------------------
// Multiplicative cycle (§3.3)
// ------------------------------------------------------------------------------------------------
void Solver::mult_cycle(int c) {
  int l = 0;
  while (true) {
    if (c == 1) {
      if (!build_structure(l)) break;
    } else if (l == (int)lv_.size() - 1) {
      break;
    }
    relax_tests(l);
    if (c >= 2) boot_relax_rq(l);
    fit_interpolation(l, c);
    galerkin(l);
    inject(l, c);
    ++l;
    lastcheck();
  }
  if (c == 1) {
    // the coarsest level is now known: dense workspaces
    Level& L = *lv_.back();
    const int m = L.m, n = L.n;
    NL_ = spd_ ? m : m + n;
    if (NL_ > 1024) {
      std::string sizes;
      for (const auto& Lv : lv_) sizes += " " + std::to_string(Lv->m) + (spd_ ? "" : "x" + std::to_string(Lv->n));
      throw SolverError{ST_E_NUMERIC, "coarsest level larger than 1024 unknowns (coarsening stalled); levels:" + sizes};
    }
    if ((spd_ ? m : std::min(m, n)) < nb_) throw SolverError{ST_E_NUMERIC, "coarsest level smaller than n_b"};
    const size_t mx = std::max(m, n);
    dA_ = ar_.alloc<double>((size_t)m * std::max(m, n));
    dB_ = ar_.alloc<double>((size_t)m * m);
    dC_ = ar_.alloc<double>((size_t)n * n);
    size_t wk = std::max<size_t>(3 * mx * mx + 2 * (size_t)m * n + 64 * mx + mx, (size_t)nb_ * 2 * NL_ * NL_);
    wk = std::max(wk, (size_t)2 * NL_ * NL_);
    dwork_ = ar_.alloc<double>(wk);
    dX_ = ar_.alloc<double>((size_t)NL_ * NL_);
    dY_ = ar_.alloc<double>((size_t)NL_ * NL_);
    mu_ = ar_.alloc<double>(NL_);
    Zp_ = ar_.alloc<double>((size_t)NL_ * NL_);
    pbasis_ = ar_.alloc<double>((size_t)nb_ * NL_ * NL_);
    rep_.levels = (int)lv_.size();
  }
  coarsest_mult();
  for (int k = (int)lv_.size() - 2; k >= 0; --k) {
    Level& L = *lv_[k];
    Level& C = *lv_[k + 1];
    launch_spmm<double>(L.su.npts, nb_, L.su.P.rp, L.su.P.ci, L.su.P.v, C.bd.Ub, L.bd.Ub, 0.0, st_);
    if (!spd_) launch_spmm<double>(L.sv.npts, nb_, L.sv.P.rp, L.sv.P.ci, L.sv.P.v, C.bd.Vb, L.bd.Vb, 0.0, st_);
    boot_relax_rq(k);
    if (p_.ritz_coarse && k >= 1) ritz_level(k);
  }
  if (p_.ritz_in_mult) ritz();
  lastcheck();
}

// ------------------------------------------------------------------------------------------------
// Additive V-cycle (§4.1-4.2), all n_b columns at once with sigma_j fixed.  rhsU / rhsV: finest
// right-hand sides (null: zero).  On return the finest level's Ub/Vb hold the new iterate (or, in
// the refinement form, the correction).
// ------------------------------------------------------------------------------------------------
template <class T>
void Solver::additive_vcycle(const double* sig, T* rhsU, T* rhsV) {
  const int nl = (int)lv_.size();
  // a single level is solved exactly by the coarsest generalized SVD of the multiplicative phase;
  // there is no coarse correction to add
  if (nl < 2) return;
  cycle_level<T>(0, sig, rhsU, rhsV, false);
}

// One visit of level l (above the coarsest) in the additive cycle: pre-relaxation, residual and
// restriction, the coarse correction (the coarsest solve, or p_.cycle_gamma visits of level l + 1:
// 1 a V-cycle, 2 a W-cycle), prolongation and post-relaxation.  zero_iterate: level l's correction is
// zero on entry (first visit of a coarse level).
template <class T>
void Solver::cycle_level(int l, const double* sig, T* rhsU, T* rhsV, bool zero_iterate) {
  const int nl = (int)lv_.size();
  const bool zero_start_ok = !minimal_ && p_.mu_b > 0;
  Level& L = *lv_[l];
  Level& C = *lv_[l + 1];
  Blocks<T>& b = blocks<T>(L);
  Blocks<T>& cb = blocks<T>(C);
  const T* kap = l == 0 ? rhsU : b.kap;
  const T* tau = l == 0 ? rhsV : b.tau;
  boot_relax<T>(l, kap, tau, sig, p_.mu_b, zero_iterate && zero_start_ok);
  level_residual_restrict<T>(l, kap, tau, sig);
  // zero initial coarse correction: written explicitly for Kaczmarz (it updates in place); the
  // Jacobi-type relaxation starts from zero without reading it, and the coarsest solve writes it
  if (!zero_start_ok) {
    if constexpr (std::is_same<T, double>::value) {
      launch_fill(cb.Ub, (size_t)(rows_u(C) + (spd_ ? 0 : rows_v(C))) * nb_, 0.0, st_);
    } else {
      launch_fillf(cb.Ub, (size_t)(rows_u(C) + (spd_ ? 0 : rows_v(C))) * nb_, 0.0f, st_);
    }
  }
  if (l + 2 == nl) {
    coarsest_additive<T>(sig);
  } else {
    for (int v = 0; v < p_.cycle_gamma; ++v) cycle_level<T>(l + 1, sig, rhsU, rhsV, v == 0);
  }
  if (spd_) spmm<T>(l, L.su.P, vals<T>(L.su.P), nb_, cb.Ub, b.Ub, 1.0);
  else spmm2<T>(l, L.su.P, vals<T>(L.su.P), cb.Ub, b.Ub, L.sv.P, vals<T>(L.sv.P), cb.Vb, b.Vb, 1.0);
  boot_relax<T>(l, kap, tau, sig, p_.mu_b);
}

// Residuals of level l's blocks, r = kappa - (A v - sigma B u) and s = tau - (A^t u - sigma C v),
// restricted into level l + 1's kappa and tau (§4.1, §4.2).
template <class T>
void Solver::level_residual_restrict(int l, const T* kap, const T* tau, const double* sig) {
  Level& L = *lv_[l];
  Level& C = *lv_[l + 1];
  Blocks<T>& b = blocks<T>(L);
  Blocks<T>& cb = blocks<T>(C);
  {
    const int mu = rows_u(L), mv = rows_v(L);
    RowOpArgs<T> a;
    a.nrows = mu; a.w = nb_; a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = vals<T>(L.A);
    a.z = spd_ ? b.Ub : b.Vb;
    if (spd_) { a.mmode = L.finest ? M_IDENT : M_SHARED; a.Mv = vals<T>(L.B); }
    else { a.mmode = L.finest ? M_IDENT : M_CSR; a.Mrp = L.B.rp; a.avgM = avg_row(L.B); a.Mci = L.B.ci; a.Mv = vals<T>(L.B); }
    a.y = b.Ub; a.kap = kap; a.sig = sig; a.cmode = C_RESID; a.out = b.tU;
    if (spd_) {
      rowop(l, a, &L.A, 7);
      spmm<T>(l, L.su.Pt, vals<T>(L.su.Pt), nb_, b.tU, cb.kap, 0.0);
    } else {
      // the two residuals, then the two restrictions, each pair in one launch
      RowOpArgs<T> s;
      s.nrows = mv; s.w = nb_; s.Krp = L.At.rp; s.Kci = L.At.ci; s.nnzK = L.At.nnz; s.Kv = vals<T>(L.At); s.z = b.Ub;
      s.mmode = L.finest ? M_IDENT : M_CSR; s.Mrp = L.C.rp; s.avgM = avg_row(L.C); s.Mci = L.C.ci; s.Mv = vals<T>(L.C);
      s.y = b.Vb; s.kap = tau; s.sig = sig; s.cmode = C_RESID; s.out = b.tV;
      rowop2(l, a, &L.A, s, &L.At, 7);
      spmm2<T>(l, L.su.Pt, vals<T>(L.su.Pt), b.tU, cb.kap, L.sv.Pt, vals<T>(L.sv.Pt), b.tV, cb.tau, 0.0);
    }
  }
}

// FMG cycle of the additive phase (§3.3 names FMG): the finest block's residual restricted through
// every level, the coarsest solve, then upwards: each coarse level starts from the prolonged
// correction of the level below it and runs one cycle against its restricted residual; the finest
// block adds the prolonged correction and runs one cycle.
template <class T>
void Solver::additive_fmg(const double* sig, T* rhsU, T* rhsV) {
  const int nl = (int)lv_.size();
  if (nl < 2) return;
  level_residual_restrict<T>(0, rhsU, rhsV, sig);
  for (int l = 1; l + 1 < nl; ++l) {
    Level& L = *lv_[l];
    Blocks<T>& b = blocks<T>(L);
    Blocks<T>& cb = blocks<T>(*lv_[l + 1]);
    if (spd_) spmm<T>(l, L.su.Pt, vals<T>(L.su.Pt), nb_, b.kap, cb.kap, 0.0);
    else spmm2<T>(l, L.su.Pt, vals<T>(L.su.Pt), b.kap, cb.kap, L.sv.Pt, vals<T>(L.sv.Pt), b.tau, cb.tau, 0.0);
  }
  coarsest_additive<T>(sig);
  for (int l = nl - 2; l >= 0; --l) {
    Level& L = *lv_[l];
    Blocks<T>& b = blocks<T>(L);
    Blocks<T>& cb = blocks<T>(*lv_[l + 1]);
    const double beta = l == 0 ? 1.0 : 0.0;   // coarse levels start from the prolonged correction
    if (spd_) spmm<T>(l, L.su.P, vals<T>(L.su.P), nb_, cb.Ub, b.Ub, beta);
    else spmm2<T>(l, L.su.P, vals<T>(L.su.P), cb.Ub, b.Ub, L.sv.P, vals<T>(L.sv.P), cb.Vb, b.Vb, beta);
    cycle_level<T>(l, sig, rhsU, rhsV, false);
  }
}

// Coarsest level of the additive cycle: [u; v] = pinv(X - sigma_j Y) [kappa; tau] (FP64), from and
// into the coarsest level's blocks.
template <class T>
void Solver::coarsest_additive(const double* sig) {
  Level& L = *lv_.back();
  Blocks<T>& b = blocks<T>(L);
  const size_t n = (size_t)NL_ * nb_;
  double* rhs = L.bd.kap;
  double* sol = L.bd.Ub;
  T* rk = b.kap;
  if constexpr (std::is_same<T, float>::value) {
    launch_copy_cast_fd(rk, L.bd.kap, n, st_);
  } else {
    if (rk != L.bd.kap) HIPCHK(hipMemcpyAsync(rhs, rk, n * sizeof(double), hipMemcpyDeviceToDevice, st_));
  }
  if (p_.coarse_pinv == 0) {
    // the eigenvectors of the previous call start the next one; the first call of the additive
    // phase starts cold, and the first call of every eagerly run iteration (every 32nd)
    // re-orthonormalises the basis, so that captured iterations (plain warm start) and eager ones
    // take the same steps whatever the number of coarsest solves per iteration
    const long c = pinv_calls_++;
    const int warm = c == 0 ? 0 : pinv_reortho_ ? 2 : 1;
    pinv_reortho_ = false;
    prof(4, 0.0, [&] { launch_pinv_solve(NL_, nb_, dX_, dY_, sig, rhs, sol, dwork_, pbasis_, warm, status_, st_); });
  }
  else prof(4, 0.0, [&] { launch_pencil_solve(NL_, nb_, mu_, Zp_, sig, rhs, sol, st_); });
  if constexpr (std::is_same<T, float>::value) launch_copy_cast_df(sol, b.Ub, n, st_);
}

void Solver::additive_iteration() {
  if (!mixed_) {
    additive_cycle<double>(sig_, nullptr, nullptr);
    return;
  }
  // Refinement form: FP64 residual of the current iterate, FP32 V-cycle on the error equation
  // with zero initial correction, FP64 update.  For fixed sigma every relaxation is affine, so in
  // exact arithmetic this equals the additive V-cycle applied to the iterate.
  Level& L = *lv_[0];
  const int mu = rows_u(L), mv = rows_v(L);
  RowOpArgs<double> a;
  a.nrows = mu; a.w = nb_; a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = L.A.v; a.z = spd_ ? L.bd.Ub : L.bd.Vb;
  a.mmode = M_IDENT; a.y = L.bd.Ub; a.sig = sig_; a.cmode = C_RESID; a.out = L.bd.tU;
  if (spd_) {
    rowop(0, a, &L.A, 7);
    launch_copy_cast_df(L.bd.tU, L.bf.kap, (size_t)mu * nb_, st_);
  } else {
    RowOpArgs<double> s;
    s.nrows = mv; s.w = nb_; s.Krp = L.At.rp; s.Kci = L.At.ci; s.nnzK = L.At.nnz; s.Kv = L.At.v; s.z = L.bd.Ub;
    s.mmode = M_IDENT; s.y = L.bd.Vb; s.sig = sig_; s.cmode = C_RESID; s.out = L.bd.tV;
    rowop2(0, a, &L.A, s, &L.At, 7);
    launch_copy_cast_df(L.bd.tU, L.bf.kap, (size_t)mu * nb_, st_);
    launch_copy_cast_df(L.bd.tV, L.bf.tau, (size_t)mv * nb_, st_);
  }
  launch_fillf(L.bf.Ub, (size_t)(mu + (spd_ ? 0 : mv)) * nb_, 0.0f, st_);
  additive_cycle<float>(sig_, L.bf.kap, spd_ ? nullptr : L.bf.tau);
  launch_axpy_fd(L.bf.Ub, L.bd.Ub, (size_t)mu * nb_, st_);
  if (!spd_) launch_axpy_fd(L.bf.Vb, L.bd.Vb, (size_t)mv * nb_, st_);
}

// ------------------------------------------------------------------------------------------------
// Ritz projection on the finest level (§4.3): Cholesky-QR2 of the boot blocks (MFMA Gram), the
// projected n_b x n_b problem, rotation of the bases.
// ------------------------------------------------------------------------------------------------
void Solver::cholqr2(double* X, int rows, double* tmp, double* out) {
  prof(2, 8.0 * rows * nb_, [&] { launch_gram(rows, nb_, X, X, partial_, gram_, st_); });
  launch_chol_inv_upper(nb_, gram_, small1_, status_, st_);
  launch_rotate<double>(rows, nb_, nb_, X, small1_, tmp, st_);
  prof(2, 8.0 * rows * nb_, [&] { launch_gram(rows, nb_, tmp, tmp, partial_, gram_, st_); });
  launch_chol_inv_upper(nb_, gram_, small1_, status_, st_);
  launch_rotate<double>(rows, nb_, nb_, tmp, small1_, out, st_);
}

// The U- and V-side Cholesky-QR2 are independent: each of their steps runs both in one launch.
void Solver::cholqr2_pair(double* Xa, int rows_a, double* tmpa, double* outa, double* Xb, int rows_b, double* tmpb,
                          double* outb) {
  const double bytes = 8.0 * ((double)rows_a + rows_b) * nb_;
  prof(2, bytes, [&] {
    launch_gram2(nb_, rows_a, Xa, Xa, partial_, gram_, rows_b, Xb, Xb, partial2_, gram2_, st_);
  });
  launch_chol_inv_upper2(nb_, gram_, small1_, gram2_, small3_, status_, st_);
  launch_rotate2<double>(nb_, rows_a, Xa, small1_, tmpa, rows_b, Xb, small3_, tmpb, st_);
  prof(2, bytes, [&] {
    launch_gram2(nb_, rows_a, tmpa, tmpa, partial_, gram_, rows_b, tmpb, tmpb, partial2_, gram2_,
                 st_);
  });
  launch_chol_inv_upper2(nb_, gram_, small1_, gram2_, small3_, status_, st_);
  launch_rotate2<double>(nb_, rows_a, tmpa, small1_, outa, rows_b, tmpb, small3_, outb, st_);
}

void Solver::ritz() {
  Level& L = *lv_[0];
  auto& b = L.bd;
  const int mu = rows_u(L), mv = rows_v(L);
  if (!spd_) {
    cholqr2_pair(b.Ub, mu, b.tU, b.tU2, b.Vb, mv, b.tV, b.tV2);   // U_hat in tU2, V_hat in tV2
    spmm<double>(0, L.A, L.A.v, nb_, b.tV2, b.tU, 0.0);   // W = A V_hat
    prof(2, 16.0 * mu * nb_, [&] { launch_gram(mu, nb_, b.tU2, b.tU, partial_, gram_, st_); });                      // M = U_hat^t W
    launch_small_ritz(nb_, 0, minimal_, gram_, small1_, small2_, sig_, small_work_, status_, st_);
    launch_rotate2<double>(nb_, mu, b.tU2, small1_, b.Ub, mv, b.tV2, small2_, b.Vb, st_);
  } else {
    cholqr2(b.Ub, mu, b.tU, b.tU2);               // U_hat in tU2
    spmm<double>(0, L.A, L.A.v, nb_, b.tU2, b.tU, 0.0);   // A X_hat
    prof(2, 16.0 * mu * nb_, [&] { launch_gram(mu, nb_, b.tU2, b.tU, partial_, gram_, st_); });
    launch_small_ritz(nb_, 1, minimal_, gram_, small1_, small2_, sig_, small_work_, status_, st_);
    launch_rotate<double>(mu, nb_, nb_, b.tU2, small1_, b.Ub, st_);
  }
}

// §4.3's Ritz step on coarse level l: bases of span(U_b) and span(V_b) orthonormal in the B and
// C metrics (Cholesky-QR2 on X^t M X), the projected n_b x n_b problem, and the rotated blocks.
void Solver::ritz_level(int l) {
  Level& L = *lv_[l];
  auto& b = L.bd;
  const int mu = rows_u(L), mv = rows_v(L);
  auto orth = [&](const DCsr& M, double* X, int rows, double* tmp, double* mx, double* out) {
    spmm<double>(l, M, M.v, nb_, X, mx, 0.0);
    launch_gram(rows, nb_, X, mx, partial_, gram_, st_);
    launch_chol_inv_upper(nb_, gram_, small1_, status_, st_);
    launch_rotate<double>(rows, nb_, nb_, X, small1_, tmp, st_);
    spmm<double>(l, M, M.v, nb_, tmp, mx, 0.0);
    launch_gram(rows, nb_, tmp, mx, partial_, gram_, st_);
    launch_chol_inv_upper(nb_, gram_, small1_, status_, st_);
    launch_rotate<double>(rows, nb_, nb_, tmp, small1_, out, st_);
  };
  if (spd_) {
    orth(L.B, b.Ub, mu, b.tU, b.Ua, b.tU2);                  // X_hat in tU2 (B on A's pattern)
    spmm<double>(l, L.A, L.A.v, nb_, b.tU2, b.tU, 0.0);      // A X_hat
    launch_gram(mu, nb_, b.tU2, b.tU, partial_, gram_, st_);
    launch_small_ritz(nb_, 1, minimal_, gram_, small1_, small2_, sig_, small_work_, status_, st_);
    launch_rotate<double>(mu, nb_, nb_, b.tU2, small1_, b.Ub, st_);
  } else {
    orth(L.B, b.Ub, mu, b.tU, b.Ua, b.tU2);                  // U_hat in tU2
    orth(L.C, b.Vb, mv, b.tV, b.Va, b.tV2);                  // V_hat in tV2
    spmm<double>(l, L.A, L.A.v, nb_, b.tV2, b.tU, 0.0);      // A V_hat
    launch_gram(mu, nb_, b.tU2, b.tU, partial_, gram_, st_);
    launch_small_ritz(nb_, 0, minimal_, gram_, small1_, small2_, sig_, small_work_, status_, st_);
    launch_rotate2<double>(nb_, mu, b.tU2, small1_, b.Ub, mv, b.tV2, small2_, b.Vb, st_);
  }
}

// ------------------------------------------------------------------------------------------------
// LOBPCG solve phase on the learned hierarchy (§7 names it as a replacement of the multigrid-Ritz
// additive phase).  The preconditioned direction of a column is the change the additive cycle
// makes to it, W = C(X) - X; the Ritz step runs on span[X, W, P] with P the previous search
// direction.  Bases block by block: Cholesky-QR2 of X; W with its X components removed (two
// passes), Cholesky-QR2; P with its X and W components removed (two passes).  A column of P (a
// part of a unit Ritz vector) below 1e-10 on either side is left out (its Ritz vector no longer
// moves: the others come first, zero columns after them); the block of the others is kept only
// when one remains, every column keeps at least 1e-8 of its norm and the unshifted Cholesky factorisation of its
// column-scaled Gram matrix has no pivot below 1e-10 (a condition number below about 1e5, so that
// rounding does not decide).  SVD: both sides, P kept on both or neither; for minimal
// targets the left blocks are those of A Q_v (a two-sided projection of the enlarged spaces has
// singular values below sigma_min(A)).  The k x k projected problem (k = 2 n_b or 3 n_b) goes to
// the dense solver of the coarsest level with identity metrics; the new P is the part of each
// new Ritz vector in the W and P blocks.
// ------------------------------------------------------------------------------------------------
void Solver::lobpcg_setup() {
  Level& L = *lv_[0];
  const size_t nu = (size_t)rows_u(L) * nb_, nv = (size_t)rows_v(L) * nb_;
  auto side = [&](LobSide& b, size_t n) {
    for (double** f : {&b.X, &b.W, &b.P, &b.Pq, &b.T, &b.tmp}) *f = ar_.alloc<double>(n);
  };
  side(lbu_, nu);
  if (!spd_) side(lbv_, nv);
  const int kmax = 3 * nb_;
  lobM_ = ar_.alloc<double>((size_t)kmax * kmax);
  lobB_ = ar_.alloc<double>((size_t)kmax * kmax);
  lobC_ = ar_.alloc<double>((size_t)kmax * kmax);
  lobY_ = ar_.alloc<double>((size_t)kmax * nb_);
  lobZ_ = ar_.alloc<double>((size_t)kmax * nb_);
  lobwork_ = ar_.alloc<double>((size_t)8 * kmax * kmax + 64 * kmax + 64);
  lobchk_ = ar_.alloc<double>(512);
  lobflag_ = ar_.alloc<int>(4);
  HIPCHK(hipMemsetAsync(lobchk_, 0, 512 * sizeof(double), st_));
  lob_have_p_ = false;
}

// Y minus its components along the orthonormal blocks, two passes
void Solver::lob_remove(double* Y, int rows, std::initializer_list<const double*> bases) {
  for (int pass = 0; pass < 2; ++pass)
    for (const double* Q : bases) {
      launch_gram(rows, nb_, Q, Y, partial_, gram_, st_);   // Q^t Y
      launch_rotate_acc(rows, nb_, Q, gram_, -1.0, Y, Y, st_);
    }
}

// Pq (a copy of P0, nact leading columns, zero columns after them) projected and orthonormalised;
// returns whether the P block is kept
bool Solver::lob_pcheck(const double* P0, double* Pq, int rows, int nact, std::initializer_list<const double*> bases,
                        double* tmp, const char* side) {
  const size_t w2 = (size_t)nb_ * nb_;
  launch_gram(rows, nb_, P0, P0, partial_, gram_, st_);
  HIPCHK(hipMemcpyAsync(lobchk_, gram_, w2 * sizeof(double), hipMemcpyDeviceToDevice, st_));
  lob_remove(Pq, rows, bases);
  launch_gram(rows, nb_, Pq, Pq, partial_, gram_, st_);
  HIPCHK(hipMemcpyAsync(lobchk_ + 256, gram_, w2 * sizeof(double), hipMemcpyDeviceToDevice, st_));
  // Cholesky-QR2; a failed factorisation only drops the block (status into lobflag_)
  launch_chol_inv_upper_pivot(nb_, nact, gram_, small1_, lobflag_, lobchk_ + 511, st_);
  launch_rotate<double>(rows, nb_, nb_, Pq, small1_, tmp, st_);
  launch_gram(rows, nb_, tmp, tmp, partial_, gram_, st_);
  launch_chol_inv_upper(nb_, gram_, small1_, lobflag_, st_);
  launch_rotate<double>(rows, nb_, nb_, tmp, small1_, Pq, st_);
  std::vector<double> h;
  d2h(h, lobchk_, 512, st_);
  double ratio = 1.0;
  for (int j = 0; j < nact; ++j) {
    const double g0 = h[(size_t)j * nb_ + j], g = h[256 + (size_t)j * nb_ + j];
    ratio = g > 0.0 ? std::min(ratio, std::sqrt(g / g0)) : 0.0;
    if (!(g > 0.0)) break;
  }
  const double piv = h[511];
  const bool keep = ratio >= 1e-8 && piv >= 1e-10;
  if (p_.verbose >= 2) {
    std::fprintf(stderr, "[slamg] LOBPCG %s-side search directions: smallest kept norm fraction %.3e, smallest pivot %.3e%s\n",
                 side, ratio, piv, keep ? "" : ", left out");
    std::fflush(stderr);
  }
  return keep;
}

void Solver::lobpcg_iteration() {
  Level& L = *lv_[0];
  auto& b = L.bd;
  const int mu = rows_u(L), mv = rows_v(L);
  const size_t nu = (size_t)mu * nb_, nv = (size_t)mv * nb_;
  const bool svd = !spd_, one_sided = svd && minimal_;
  HIPCHK(hipMemcpyAsync(lbu_.X, b.Ub, nu * sizeof(double), hipMemcpyDeviceToDevice, st_));
  if (svd) HIPCHK(hipMemcpyAsync(lbv_.X, b.Vb, nv * sizeof(double), hipMemcpyDeviceToDevice, st_));
  if (lob_replay_) {
    HIPCHK(hipGraphLaunch(igx_, st_));
    if (p_.coarse_pinv == 0) pinv_calls_ += coarse_calls_per_iter();
    ++rep_.graph_iters;
  } else {
    additive_iteration();
  }
  launch_axpby(nu, 1.0, b.Ub, -1.0, lbu_.X, lbu_.W, st_);   // W = C(X) - X
  if (svd) {
    launch_axpby(nv, 1.0, b.Vb, -1.0, lbv_.X, lbv_.W, st_);
    cholqr2(lbv_.X, mv, lbv_.tmp, lbv_.X);
    lob_remove(lbv_.W, mv, {lbv_.X});
    cholqr2(lbv_.W, mv, lbv_.tmp, lbv_.W);
  }
  if (one_sided) {
    spmm<double>(0, L.A, L.A.v, nb_, lbv_.X, lbu_.X, 0.0);
    spmm<double>(0, L.A, L.A.v, nb_, lbv_.W, lbu_.W, 0.0);
  }
  cholqr2(lbu_.X, mu, lbu_.tmp, lbu_.X);
  lob_remove(lbu_.W, mu, {lbu_.X});
  cholqr2(lbu_.W, mu, lbu_.tmp, lbu_.W);
  bool keep = false;
  int act[16] = {}, nact = 0;
  if (lob_have_p_) {
    // columns of P at least 1e-10 on each side (a smaller one: a Ritz vector that no longer moves)
    const size_t w2 = (size_t)nb_ * nb_;
    launch_gram(mu, nb_, lbu_.P, lbu_.P, partial_, gram_, st_);
    HIPCHK(hipMemcpyAsync(lobchk_, gram_, w2 * sizeof(double), hipMemcpyDeviceToDevice, st_));
    if (svd) {
      launch_gram(mv, nb_, lbv_.P, lbv_.P, partial_, gram_, st_);
      HIPCHK(hipMemcpyAsync(lobchk_ + 256, gram_, w2 * sizeof(double), hipMemcpyDeviceToDevice, st_));
    }
    std::vector<double> h;
    d2h(h, lobchk_, 512, st_);
    // the columns that still move, in column order; their blocks (P0 in T) lead, zeros after
    for (int j = 0; j < nb_; ++j) {
      bool m = h[(size_t)j * nb_ + j] >= 1e-20;
      if (svd) m = m && h[256 + (size_t)j * nb_ + j] >= 1e-20;
      if (m) act[nact++] = j;
    }
    bool okv = nact > 0;
    if (svd && okv) {
      launch_gather_cols(mv, nb_, act, nact, lbv_.P, lbv_.T, st_);
      HIPCHK(hipMemcpyAsync(lbv_.Pq, lbv_.T, nv * sizeof(double), hipMemcpyDeviceToDevice, st_));
      okv = lob_pcheck(lbv_.T, lbv_.Pq, mv, nact, {lbv_.X, lbv_.W}, lbv_.tmp, "V");
    }
    if (okv) {
      if (one_sided) spmm<double>(0, L.A, L.A.v, nb_, lbv_.Pq, lbu_.T, 0.0);
      else launch_gather_cols(mu, nb_, act, nact, lbu_.P, lbu_.T, st_);
      HIPCHK(hipMemcpyAsync(lbu_.Pq, lbu_.T, nu * sizeof(double), hipMemcpyDeviceToDevice, st_));
      keep = lob_pcheck(lbu_.T, lbu_.Pq, mu, nact, {lbu_.X, lbu_.W}, lbu_.tmp, svd ? "U" : "X");
    }
    if (!keep) ++rep_.p_dropped;
  }
  const int nblk = keep ? 3 : 2, k = 2 * nb_ + (keep ? nact : 0);
  const double* Qu[3] = {lbu_.X, lbu_.W, lbu_.Pq};
  const double* Qv[3] = {svd ? lbv_.X : lbu_.X, svd ? lbv_.W : lbu_.W, svd ? lbv_.Pq : lbu_.Pq};
  for (int c = 0; c < nblk; ++c) {
    spmm<double>(0, L.A, L.A.v, nb_, Qv[c], lbu_.T, 0.0);   // A Q_c
    for (int a = 0; a < nblk; ++a) {
      if (!svd && a > c) continue;   // symmetric: block (c, a) is the transpose of (a, c)
      launch_gram(mu, nb_, Qu[a], lbu_.T, partial_, gram_, st_);
      launch_place_block(nb_, a == 2 ? nact : nb_, c == 2 ? nact : nb_, gram_, lobM_, k, a * nb_, c * nb_,
                         !svd && a != c, st_);
    }
  }
  launch_eye(k, lobB_, st_);
  if (svd) launch_eye(k, lobC_, st_);
  // rows of the Ritz coefficients beyond k stay zero (they meet the zero columns of the P basis)
  launch_fill(lobY_, (size_t)3 * nb_ * nb_, 0.0, st_);
  if (svd) launch_fill(lobZ_, (size_t)3 * nb_ * nb_, 0.0, st_);
  if (svd && k <= 32) {
    // one-sided Jacobi on the projected matrix itself (orthonormal bases: identity metrics)
    launch_proj_svd(k, nb_, minimal_, lobM_, lobY_, lobZ_, sig_, st_);
  } else {
    launch_coarse_gsvd(spd_, minimal_, k, k, nb_, lobM_, lobB_, svd ? lobC_ : nullptr, lobwork_, sig_, lobY_,
                       svd ? lobZ_ : nullptr, status_, st_);
  }
  // new Ritz vectors Q Y and search directions (the W and P block parts)
  const size_t w2 = (size_t)nb_ * nb_;
  auto update = [&](const double* const* Q, const double* Y, int rows, double* X, double* P) {
    launch_rotate<double>(rows, nb_, nb_, Q[0], Y, X, st_);
    launch_rotate<double>(rows, nb_, nb_, Q[1], Y + w2, P, st_);
    if (nblk == 3) launch_rotate_acc(rows, nb_, Q[2], Y + 2 * w2, 1.0, P, P, st_);
    launch_axpby((size_t)rows * nb_, 1.0, X, 1.0, P, X, st_);
  };
  update(Qu, lobY_, mu, b.Ub, lbu_.P);
  if (svd) update(Qv, lobZ_, mv, b.Vb, lbv_.P);
  lob_have_p_ = true;
  residual_launch();
}

// rho_j = max(||A v_j - s_j u_j||, ||A^t u_j - s_j v_j||) / ||A||_est  (unit vectors after Ritz)
void Solver::residual_launch() {
  Level& L = *lv_[0];
  auto& b = L.bd;
  DotArgs<double> d1, d2;
  d1.nrows = L.m; d1.w = nb_; d1.Krp = L.A.rp; d1.Kci = L.A.ci; d1.nnzK = L.A.nnz; d1.Kv = L.A.v;
  d1.z = spd_ ? b.Ub : b.Vb; d1.y = b.Ub; d1.sig = sig_;
  if (L.lgu.n > 0 || L.lgv.n > 0) {
    // sides with long rows: the residual blocks by the row kernel (a workgroup per long row), then
    // their column norms
    RowOpArgs<double> a, c;
    a.nrows = L.m; a.w = nb_; a.Krp = L.A.rp; a.Kci = L.A.ci; a.nnzK = L.A.nnz; a.Kv = L.A.v;
    a.z = spd_ ? b.Ub : b.Vb; a.mmode = M_IDENT; a.y = b.Ub; a.sig = sig_; a.cmode = C_RESID; a.out = b.tU;
    DotArgs<double> e1, e2;
    e1.nrows = L.m; e1.w = nb_; e1.z = b.tU;
    if (spd_) {
      rowop(0, a, &L.A, 7);
      launch_dots(e1, partial_, r1_, st_);
    } else {
      c.nrows = L.n; c.w = nb_; c.Krp = L.At.rp; c.Kci = L.At.ci; c.nnzK = L.At.nnz; c.Kv = L.At.v;
      c.z = b.Ub; c.mmode = M_IDENT; c.y = b.Vb; c.sig = sig_; c.cmode = C_RESID; c.out = b.tV;
      rowop2(0, a, &L.A, c, &L.At, 7);
      e2.nrows = L.n; e2.w = nb_; e2.z = b.tV;
      launch_dots2(e1, partial_, r1_, e2, partial2_, r2_, st_);
    }
    return;
  }
  if (spd_) {
    dots(0, d1, &L.A, r1_);
  } else {
    d2.nrows = L.n; d2.w = nb_; d2.Krp = L.At.rp; d2.Kci = L.At.ci; d2.nnzK = L.At.nnz; d2.Kv = L.At.v;
    d2.z = b.Ub; d2.y = b.Vb; d2.sig = sig_;
    launch_dots2(d1, partial_, r1_, d2, partial2_, r2_, st_);
  }
}

void Solver::residual_collect(std::vector<double>& rho) {
  std::vector<double> h;
  d2h(h, r1_, spd_ ? (size_t)nb_ : (size_t)64 + nb_, st_);   // r1_[0..nb) and r2_ = r1_ + 64
  rho.resize(nb_);
  for (int j = 0; j < nb_; ++j) {
    double r = std::sqrt(std::max(h[j], 0.0));
    if (!spd_) r = std::max(r, std::sqrt(std::max(h[64 + j], 0.0)));
    rho[j] = r / anorm_;
    if (!std::isfinite(rho[j])) throw SolverError{ST_E_NUMERIC, "non-finite residual"};
  }
}

void Solver::residuals(std::vector<double>& rho) {
  residual_launch();
  residual_collect(rho);
}

// One additive iteration on the device: V-cycle, Ritz step, residual reductions (no host sync).
void Solver::iteration_body() {
  additive_iteration();
  ritz();
  residual_launch();
}

// Every block pointer the cycles may swap (relaxation ping-pong pairs).
std::vector<void**> Solver::block_pointers() {
  std::vector<void**> v;
  auto add = [&](auto& b) {
    for (auto* f : {&b.Ut, &b.Vt, &b.Ub, &b.Vb, &b.Ua, &b.Va, &b.kap, &b.tau, &b.tU, &b.tV, &b.tU2, &b.tV2})
      v.push_back(reinterpret_cast<void**>(f));
  };
  for (auto& L : lv_) {
    add(L->bd);
    add(L->bf);
  }
  return v;
}

// Capture one iteration into a graph (the LOBPCG phase: its additive cycle only, the rest of its
// iteration decides on P on the host).  The capture runs the host side of the iteration without
// executing anything; the graph is kept only if the iteration leaves every block pointer where it
// found it (an even number of swaps per pair), so that replays chain.
void Solver::capture_iteration() {
  auto ptrs = block_pointers();
  std::vector<void*> before;
  for (auto* p : ptrs) before.push_back(*p);
  const long calls = pinv_calls_;
  hipGraph_t g = nullptr;
  bool ok = true;
  capturing_ = true;
  try {
    HIPCHK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    try {
      if (p_.solve_phase == 1) additive_iteration();
      else iteration_body();
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(st_, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    HIPCHK(hipStreamEndCapture(st_, &g));
  } catch (const SolverError&) {
    ok = false;
  }
  capturing_ = false;
  (void)hipGetLastError();
  pinv_calls_ = calls;
  for (size_t i = 0; i < ptrs.size(); ++i) {
    if (*ptrs[i] != before[i]) ok = false;
    *ptrs[i] = before[i];
  }
  hipGraphExec_t x = nullptr;
  if (ok && g && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    ok = false;
  }
  if (!ok) {
    if (g) (void)hipGraphDestroy(g);
    graph_off_ = true;
    return;
  }
  ig_ = g;
  igx_ = x;
}

void Solver::check_status() {
  std::vector<int> st;
  d2h(st, status_, 1, st_);
  if (st[0] != 0) throw SolverError{ST_E_NUMERIC, "dense factorisation breakdown on the device"};
}

// Coarsest solves per additive iteration: cycle_gamma^(levels - 2).
long Solver::coarse_calls_per_iter() const {
  // a cycle from level l solves the coarsest level gamma^(levels - 2 - l) times
  const int nl = (int)lv_.size();
  auto from = [&](int l) {
    long c = 1;
    for (int k = l + 2; k < nl; ++k) c *= p_.cycle_gamma;
    return c;
  };
  if (!p_.fmg) return from(0);
  long c = 1;   // FMG: the first coarsest solve, then one cycle from every level above it
  for (int l = nl - 2; l >= 0; --l) c += from(l);
  return c;
}

// The additive phase's coarsest-level structures: dense X, Y (and the pencil eigenbasis).
void Solver::coarse_setup() {
  dense_coarsest(dX_, dY_);
  pinv_calls_ = 0;
  if (p_.coarse_pinv == 1) {
    double* Xc = dwork_;
    double* Yc = dwork_ + (size_t)NL_ * NL_;
    HIPCHK(hipMemcpyAsync(Xc, dX_, sizeof(double) * NL_ * NL_, hipMemcpyDeviceToDevice, st_));
    HIPCHK(hipMemcpyAsync(Yc, dY_, sizeof(double) * NL_ * NL_, hipMemcpyDeviceToDevice, st_));
    if (!pencil_wk_) pencil_wk_ = ar_.alloc<double>((size_t)2 * NL_ * NL_);
    launch_pencil_setup(NL_, Xc, Yc, mu_, Zp_, pencil_wk_, status_, st_);
  }
}

// FP32 copies of the transfer operators' values (mixed precision)
void Solver::cast_transfers() {
  for (auto& L : lv_) {
    cast_vals(L->su.P);
    cast_vals(L->su.Pt);
    if (!spd_) {
      cast_vals(L->sv.P);
      cast_vals(L->sv.Pt);
    }
  }
}

// Redetermined interpolation during the additive phase (§6.3): one downward sweep of the
// multiplicative phase (test and boot relaxations, LS fits, Galerkin products, injection) refits
// P, Q and the coarse operators, with the LS weights of the test vectors and of the pairs marked in
// conv multiplied by 1e-3.  The sweep relaxes a copy of the iterate: the finest boot block and
// sigma are restored afterwards.
void Solver::redo_interpolation(const std::vector<char>& conv) {
  Level& F = *lv_[0];
  const size_t nu = (size_t)rows_u(F) * nb_, nv = spd_ ? 0 : (size_t)rows_v(F) * nb_;
  if (!redo_keep_) {
    redo_keep_ = ar_.alloc<double>(nu + nv + 64);
    wscale_ = ar_.alloc<double>(64);
  }
  double* kU = redo_keep_;
  double* kV = redo_keep_ + nu;
  double* kS = redo_keep_ + nu + nv;
  HIPCHK(hipMemcpyAsync(kU, F.bd.Ub, nu * sizeof(double), hipMemcpyDeviceToDevice, st_));
  if (nv) HIPCHK(hipMemcpyAsync(kV, F.bd.Vb, nv * sizeof(double), hipMemcpyDeviceToDevice, st_));
  HIPCHK(hipMemcpyAsync(kS, sig_, nb_ * sizeof(double), hipMemcpyDeviceToDevice, st_));
  std::vector<double> sc(nt_ + nb_, 1.0);
  for (int i = 0; i < nt_; ++i) sc[i] = 1e-3;
  for (int j = 0; j < nb_; ++j)
    if (conv[j]) sc[nt_ + j] = 1e-3;
  h2d(wscale_, sc, st_);
  redo_weights_ = true;
  for (int l = 0; l + 1 < (int)lv_.size(); ++l) {
    relax_tests(l);
    boot_relax_rq(l);
    fit_interpolation(l, 2);
    galerkin(l);
    inject(l, 2);
  }
  redo_weights_ = false;
  HIPCHK(hipMemcpyAsync(F.bd.Ub, kU, nu * sizeof(double), hipMemcpyDeviceToDevice, st_));
  if (nv) HIPCHK(hipMemcpyAsync(F.bd.Vb, kV, nv * sizeof(double), hipMemcpyDeviceToDevice, st_));
  HIPCHK(hipMemcpyAsync(sig_, kS, nb_ * sizeof(double), hipMemcpyDeviceToDevice, st_));
  coarse_setup();
  if (mixed_) cast_transfers();
  check_status();
}

// ------------------------------------------------------------------------------------------------
void Solver::run(const double* init_tests, SolveOutput& out) {
  using clk = std::chrono::steady_clock;
  auto t0 = clk::now();
  std::memset(&rep_, 0, sizeof(rep_));
  (void)hipGetLastError();   // an earlier failed call's error was reported by that call
  if (nb_ > 16 || nt_ > 16) throw SolverError{ST_E_INVALID, "n_b and n_t must be at most 16"};
  sig_ = ar_.alloc<double>(64);
  flip_ = ar_.alloc<double>(64);
  partial_ = ar_.alloc<double>(PARTIAL_DOUBLES);
  // r1_, r2_, r3_ adjacent: the residual norms of both sides come back in one copy
  r1_ = ar_.alloc<double>(3 * 64); r2_ = r1_ + 64; r3_ = r1_ + 128;
  wts_ = ar_.alloc<double>(64);
  gram_ = ar_.alloc<double>(256);
  small1_ = ar_.alloc<double>(256);
  small2_ = ar_.alloc<double>(256);
  small_work_ = ar_.alloc<double>(4 * 32 * 32);
  status_ = ar_.alloc<int>(4);
  HIPCHK(hipMemsetAsync(status_, 0, 4 * sizeof(int), st_));
  partial2_ = ar_.alloc<double>(PARTIAL_DOUBLES);
  gram2_ = ar_.alloc<double>(256);
  small3_ = ar_.alloc<double>(256);
  HIPCHK(hipMemsetAsync(sig_, 0, 64 * sizeof(double), st_));
  rep_.rows[0] = A0_.m; rep_.cols[0] = A0_.n; rep_.nnz[0] = A0_.nnz();
  pmask_ = p_.profile_mask;
  vt_ = std::chrono::steady_clock::now();
  finest_level(init_tests);
  vmark("finest level (uploads, transpose, colouring)", 0);
  norm_estimate();
  vmark("norm estimate", 0);
  rep_.anorm = anorm_;
  std::vector<double> rho;
  std::vector<double> hs;
  for (int c = 1; c <= p_.n_mult; ++c) {
    mult_cycle(c);
    rep_.mult_cycles = c;
    d2h(hs, sig_, nb_, st_);
    if (c <= 32)
      for (int j = 0; j < nb_; ++j) rep_.mult_sigma[c - 1][j] = hs[j];
    // a breakdown ends the solve here, before non-finite values reach the next cycle
    for (int j = 0; j < nb_; ++j)
      if (!std::isfinite(hs[j]))
        throw SolverError{ST_E_NUMERIC, "non-finite singular value estimate after multiplicative cycle " +
                                            std::to_string(c)};
    check_status();
    if (p_.verbose > 0) {
      std::fprintf(stderr, "[slamg] multiplicative cycle %d: %zu levels, %.1f ms\n", c, lv_.size(),
                   std::chrono::duration<double, std::milli>(clk::now() - t0).count());
      std::fflush(stderr);
    }
  }
  if (!p_.ritz_in_mult) ritz();
  check_status();
  for (size_t l = 0; l < lv_.size(); ++l) {
    ensure_colours(*lv_[l]);
    rep_.rows[l] = lv_[l]->m;
    rep_.cols[l] = lv_[l]->n;
    rep_.nnz[l] = lv_[l]->hA.nnz();
    rep_.colours[l] = (int)(lv_[l]->kA_cptr.empty() ? 0 : lv_[l]->kA_cptr.size() - 1);
  }
  residuals(rho);
  double rmax = *std::max_element(rho.begin(), rho.begin() + nw_);
  rep_.rho_history[0] = rmax;
  auto t1 = clk::now();
  // additive phase: frozen operators (dense coarsest matrices built once, and again after a
  // redetermined interpolation)
  coarse_setup();
  if (mixed_) cast_transfers();
  for (auto& Lp : lv_) long_rows(*Lp);   // before any capture
  int it = 0, it0 = 0;
  graph_off_ = !p_.graphs;
  if (p_.solve_phase == 1) lobpcg_setup();
  // redetermined interpolation (§6.3): pairs whose sigma has settled, and the previous sigma
  std::vector<char> conv(nb_, 0);
  std::vector<double> sprev, snow;
  if (p_.redo_p) d2h(sprev, sig_, nb_, st_);
  while (rmax > p_.tol && it < p_.max_add) {
    // every 32nd iteration (counted from the additive phase's start or its last redetermined
    // interpolation) runs eagerly: the literal coarsest solve re-orthonormalises its eigenvector
    // basis there (starts cold in the first), and the profiled kernel classes are timed there; the
    // other iterations replay the graph (captured with the plain warm start)
    const bool eager = ((it - it0) % 32) == 0;
    pinv_reortho_ = eager;
    if (!eager && !graph_off_ && !igx_) capture_iteration();
    const bool replay = !eager && igx_ != nullptr;
    if (p_.solve_phase == 1) {
      lob_replay_ = replay;
      lobpcg_iteration();
    } else if (replay) {
      HIPCHK(hipGraphLaunch(igx_, st_));
      if (p_.coarse_pinv == 0) pinv_calls_ += coarse_calls_per_iter();
      ++rep_.graph_iters;
    } else {
      iteration_body();
    }
    residual_collect(rho);
    rmax = *std::max_element(rho.begin(), rho.begin() + nw_);
    ++it;
    if (it < 256) rep_.rho_history[it] = rmax;
    if (p_.redo_p) {
      d2h(snow, sig_, nb_, st_);
      bool grew = false, all = true;
      for (int j = 0; j < nb_; ++j) {
        const bool now = std::fabs(snow[j] - sprev[j]) <= p_.redo_tol * std::fabs(snow[j]);
        all = all && now;
        grew = grew || (now && !conv[j]);
      }
      if (grew && !all && rmax > p_.tol) {
        for (int j = 0; j < nb_; ++j)
          if (std::fabs(snow[j] - sprev[j]) <= p_.redo_tol * std::fabs(snow[j])) conv[j] = 1;
        redo_interpolation(conv);
        ++rep_.redo_count;
        // the captured iteration used the old coarsest solve: capture again, cold start first
        if (igx_) (void)hipGraphExecDestroy(igx_);
        if (ig_) (void)hipGraphDestroy(ig_);
        igx_ = nullptr;
        ig_ = nullptr;
        pinv_calls_ = 0;
        it0 = it;
      }
      sprev = snow;
    }
    if (p_.verbose > 0 && it % p_.verbose == 0) {
      std::fprintf(stderr, "[slamg] additive iteration %d: max relative residual %.3e, %.1f ms\n", it, rmax,
                   std::chrono::duration<double, std::milli>(clk::now() - t1).count());
      std::fflush(stderr);
    }
  }
  check_status();
  auto t2 = clk::now();
  rep_.add_iters = it;
  rep_.converged = rmax <= p_.tol ? 1 : 0;
  rep_.device_bytes = (int64_t)ar_.peak();
  rep_.t_setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  rep_.t_solve_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
  for (int j = 0; j < nw_ && j < 16; ++j) {
    rep_.resid[j] = rho[j];
    rep_.err_bound[j] = rho[j] * anorm_;
  }
  prof_finish();
  // outputs
  Level& L = *lv_[0];
  if (pb_.outU || pb_.outV) {
    // device outputs: sign convention and scatter into the caller's column-major arrays
    // reference column: the caller's v_j (x_j for eigenproblems)
    const bool refU = spd_ || pb_.swapUV;
    const double* ref = refU ? L.bd.Ub : L.bd.Vb;
    const int rref = refU ? rows_u(L) : rows_v(L);
    launch_sign_argmax(rref, nw_, nb_, ref, flip_, st_);
    double* dstU = pb_.swapUV ? pb_.outV : pb_.outU;
    double* dstV = pb_.swapUV ? pb_.outU : pb_.outV;
    long ldu = pb_.swapUV ? pb_.ldV : pb_.ldU, ldv = pb_.swapUV ? pb_.ldU : pb_.ldV;
    if (dstU) {
      launch_fill(dstU, (size_t)ldu * nw_, 0.0, st_);
      launch_scatter_out(rows_u(L), nw_, nb_, L.bd.Ub, pb_.keepU, flip_, dstU, ldu, st_);
    }
    if (!spd_ && dstV) {
      launch_fill(dstV, (size_t)ldv * nw_, 0.0, st_);
      launch_scatter_out(rows_v(L), nw_, nb_, L.bd.Vb, pb_.keepV, flip_, dstV, ldv, st_);
    }
    d2h(out.sigma, sig_, nw_, st_);
  } else {
    // the wanted columns of the row-major blocks (the guard pairs are dropped)
    auto wanted = [&](std::vector<double>& dst, const double* X, int rows) {
      std::vector<double> h;
      d2h(h, X, (size_t)rows * nb_, st_);
      dst.resize((size_t)rows * nw_);
      for (int r = 0; r < rows; ++r)
        for (int j = 0; j < nw_; ++j) dst[(size_t)r * nw_ + j] = h[(size_t)r * nb_ + j];
    };
    d2h(out.sigma, sig_, nw_, st_);
    wanted(out.U, L.bd.Ub, rows_u(L));
    if (!spd_) wanted(out.V, L.bd.Vb, rows_v(L));
  }
  out.rep = rep_;
  out.status = rep_.converged ? ST_OK : ST_NOT_CONVERGED;
}

void run_solver(hipStream_t stream, size_t budget, const Problem& pb, const slamg_params& p,
                const double* init_tests, SolveOutput& out) {
  Solver s(stream, budget, pb, p);
  s.run(init_tests, out);
}

}  // namespace slamg
