// Host-side graph work of the first multiplicative cycle (§3.7): strength of connection,
// Algorithm 1 (one-pass Ruge-Stueben coarsening), interpolatory sets and the sparsity patterns of
// P and Q, plus the symbolic sparse products of the Galerkin operators, transposes and the greedy
// multicolouring that orders the Kaczmarz sweeps.  They run once per level; every numeric step runs
// in the HIP kernels.  Algorithm 1 and the colouring are sequential (the solver colours a level on
// a host thread of its own while it builds the level's coarsening); the strength sets and the
// symbolic products are built row by row on several host threads (identical results).
#include "graph.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdint>
#include <exception>
#include <functional>
#include <memory>
#include <queue>
#include <stdexcept>
#include <thread>

namespace slamg {

// Row-parallel construction of a CSR pattern: rows [0, n) in contiguous chunks, one host thread
// per chunk.  make_row() gives each chunk its own row builder (with its own scratch), and
// row(i, out) appends row i's entries to the chunk's list.  The chunks are joined in row order, so
// the result does not depend on the number of threads.
// A pattern holds at most MAX_PATTERN_ENTRIES entries (int32 row pointers); a larger one (the
// strength graph of a matrix with nearly dense A^t A, say) ends the build with std::length_error.
static constexpr size_t MAX_PATTERN_ENTRIES = (size_t)2147483647;

template <class M>
static void build_rows(int n, std::vector<int>& rp, std::vector<int>& ci, M make_row) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nt = n >= 8192 ? (int)hw : 1;
  std::vector<std::vector<int>> part(nt), len(nt);
  std::atomic<size_t> built{0};
  std::atomic<bool> too_large{false};
  std::vector<std::exception_ptr> err(nt);
  auto work = [&](int t) {
    try {
      const int r0 = (int)((long)n * t / nt), r1 = (int)((long)n * (t + 1) / nt);
      auto row_fn = make_row();
      len[t].resize(r1 - r0);
      // the shared entry count is updated every 4096 rows (a per-row atomic on one cache line
      // serialises the threads)
      size_t pending = 0;
      for (int i = r0; i < r1; ++i) {
        const size_t before = part[t].size();
        row_fn(i, part[t]);
        const size_t got = part[t].size() - before;
        len[t][i - r0] = (int)got;
        pending += got;
        if (((i - r0) & 4095) == 4095 || i + 1 == r1 || pending > MAX_PATTERN_ENTRIES) {
          if (built.fetch_add(pending, std::memory_order_relaxed) + pending > MAX_PATTERN_ENTRIES) too_large = true;
          pending = 0;
          if (too_large.load(std::memory_order_relaxed)) break;
        }
      }
    } catch (...) {
      err[t] = std::current_exception();
    }
  };
  if (nt == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  if (too_large) throw std::length_error("sparsity pattern with more than 2^31 - 1 entries");
  rp.assign(n + 1, 0);
  size_t total = 0;
  for (int t = 0; t < nt; ++t) total += part[t].size();
  ci.clear();
  ci.reserve(total);
  int i = 0;
  for (int t = 0; t < nt; ++t) {
    for (int l : len[t]) { rp[i + 1] = rp[i] + l; ++i; }
    ci.insert(ci.end(), part[t].begin(), part[t].end());
  }
}

// S_i = { j != i : |n_ij| > 0 and the rule holds }, returned as a CSR pattern (sorted).
//  rule 0: |n_ij| >= theta * sum_k |n_ik|   (the row-sum condition of §3.7, all k)
//  rule 1: |n_ij| >= theta * max_{k != i} |n_ik|
//  rule 2: the top_s largest off-diagonal |n_ij| (ties to the lower j)
void strength_sets(const HCsr& N, double theta, int rule, int top_s, std::vector<int>& Sp, std::vector<int>& Si) {
  auto make_row = [&] {
    return [&, cand = std::vector<std::pair<double, int>>()](int i, std::vector<int>& out) mutable {
      const int b = N.rp[i], e = N.rp[i + 1];
      if (rule == 0) {
        double sum = 0.0;
        for (int k = b; k < e; ++k) sum += std::fabs(N.v[k]);
        const double thr = theta * sum;
        for (int k = b; k < e; ++k) {
          const double a = std::fabs(N.v[k]);
          if (N.ci[k] != i && a > 0.0 && a >= thr) out.push_back(N.ci[k]);
        }
      } else if (rule == 1) {
        double mx = 0.0;
        for (int k = b; k < e; ++k)
          if (N.ci[k] != i) mx = std::max(mx, std::fabs(N.v[k]));
        const double thr = theta * mx;
        for (int k = b; k < e; ++k) {
          const double a = std::fabs(N.v[k]);
          if (N.ci[k] != i && a > 0.0 && a >= thr) out.push_back(N.ci[k]);
        }
      } else {
        // the top_s smallest (-|n_ij|, j) pairs: distinct j make the order total, so the partial
        // sort selects exactly the entries a full sort would put first
        cand.clear();
        for (int k = b; k < e; ++k) {
          const double a = std::fabs(N.v[k]);
          if (N.ci[k] != i && a > 0.0) cand.push_back({-a, N.ci[k]});
        }
        const int take = std::min<int>(top_s, (int)cand.size());
        std::partial_sort(cand.begin(), cand.begin() + take, cand.end());
        const size_t at = out.size();
        for (int t = 0; t < take; ++t) out.push_back(cand[t].second);
        std::sort(out.begin() + at, out.end());
      }
    };
  };
  build_rows(N.m, Sp, Si, make_row);
}

// Algorithm 1.  "i strongly influences j" <=> i in S_j.  lambda_i = #points i influences; the
// undecided point of maximal lambda (lowest index on ties) becomes C, the undecided points it
// influences become F, and every undecided point influencing a new F-point gets lambda + 1.
std::vector<char> rs_coarsen(const std::vector<int>& Sp, const std::vector<int>& Si, int n) {
  std::vector<int> Tp(n + 1, 0), Ti(Si.size());
  for (int j : Si) Tp[j + 1]++;
  for (int i = 0; i < n; ++i) Tp[i + 1] += Tp[i];
  {
    std::vector<int> pos(Tp.begin(), Tp.end() - 1);
    for (int j = 0; j < n; ++j)
      for (int k = Sp[j]; k < Sp[j + 1]; ++k) Ti[pos[Si[k]]++] = j;
  }
  std::vector<int> lam(n);
  int lmax = 0;
  for (int i = 0; i < n; ++i) {
    lam[i] = Tp[i + 1] - Tp[i];
    lmax = std::max(lmax, lam[i]);
  }
  std::vector<char> state(n, 0);   // 0 undecided, 1 C, 2 F
  // Buckets by lambda.  Bucket l holds the points whose lambda started at l, in index order (a
  // counting sort, consumed through a cursor), and a min-heap of the points whose lambda grew to
  // l.  An entry is valid while its point is undecided and still has that lambda; the next C-point
  // is the lowest valid index of the highest bucket with a valid entry, the order a max-heap on
  // (lambda, -index) gives.
  std::vector<int> bstart(lmax + 2, 0), members(n);
  for (int i = 0; i < n; ++i) bstart[lam[i] + 1]++;
  for (int l = 0; l <= lmax; ++l) bstart[l + 1] += bstart[l];
  std::vector<int> cursor(bstart.begin(), bstart.end() - 1);
  {
    std::vector<int> pos(cursor);
    for (int i = 0; i < n; ++i) members[pos[lam[i]]++] = i;
  }
  using MinHeap = std::priority_queue<int, std::vector<int>, std::greater<int>>;
  std::vector<MinHeap> grown(lmax + 1);
  auto valid = [&](int i, int l) { return state[i] == 0 && lam[i] == l; };
  int top = lmax;
  while (top >= 0) {
    const int l = top;
    const int cend = l + 1 < (int)bstart.size() ? bstart[l + 1] : 0;
    int& cur = cursor[l];   // buckets above lmax start empty
    while (l <= lmax && cur < cend && !valid(members[cur], l)) ++cur;
    MinHeap& hp = grown[l];
    while (!hp.empty() && !valid(hp.top(), l)) hp.pop();
    const bool from_init = l <= lmax && cur < cend;
    if (!from_init && hp.empty()) {
      --top;
      continue;
    }
    int i;
    if (from_init && (hp.empty() || members[cur] < hp.top())) i = members[cur++];
    else { i = hp.top(); hp.pop(); }
    state[i] = 1;
    for (int t = Tp[i]; t < Tp[i + 1]; ++t) {
      const int j = Ti[t];
      if (state[j] != 0) continue;
      state[j] = 2;
      for (int k = Sp[j]; k < Sp[j + 1]; ++k) {
        const int kk = Si[k];
        if (state[kk] == 0) {
          const int nl = ++lam[kk];
          if (nl >= (int)grown.size()) {
            grown.resize(nl + 1);
            cursor.resize(nl + 1, 0);
          }
          grown[nl].push(kk);
          top = std::max(top, nl);
        }
      }
    }
  }
  std::vector<char> is_c(n);
  for (int i = 0; i < n; ++i) is_c[i] = state[i] == 1;
  return is_c;
}

// Interpolatory sets C^i = S_i intersected with C (a C-point interpolates from itself), capped to
// the `cap` strongest connections |n_ij| (ties to the lower j); fine ids, ascending.
void interp_pattern(const std::vector<int>& Sp, const std::vector<int>& Si, const HCsr& N,
                    const std::vector<char>& is_c, int cap, std::vector<int>& ptr, std::vector<int>& fine_cols,
                    int& capped) {
  const int n = (int)is_c.size();
  ptr.assign(n + 1, 0);
  fine_cols.clear();
  capped = 0;
  std::vector<int> sel;
  std::vector<std::pair<double, int>> mag;
  for (int i = 0; i < n; ++i) {
    sel.clear();
    if (is_c[i]) {
      sel.push_back(i);
    } else {
      for (int k = Sp[i]; k < Sp[i + 1]; ++k)
        if (is_c[Si[k]]) sel.push_back(Si[k]);
      if ((int)sel.size() > cap) {
        ++capped;
        mag.clear();
        for (int j : sel) {
          auto it = std::lower_bound(N.ci.begin() + N.rp[i], N.ci.begin() + N.rp[i + 1], j);
          double a = std::fabs(N.v[it - N.ci.begin()]);
          mag.push_back({-a, j});
        }
        std::sort(mag.begin(), mag.end());
        sel.clear();
        for (int t = 0; t < cap; ++t) sel.push_back(mag[t].second);
        std::sort(sel.begin(), sel.end());
      }
    }
    fine_cols.insert(fine_cols.end(), sel.begin(), sel.end());
    ptr[i + 1] = (int)fine_cols.size();
  }
}

// Transpose of a pattern; perm[e] = index in A of the e-th entry of A^t (rows of A^t sorted).
HCsr transpose(const HCsr& A, std::vector<int>* perm, bool values) {
  HCsr T;
  T.m = A.n; T.n = A.m;
  T.rp.assign(A.n + 1, 0);
  const int nnz = A.nnz();
  for (int k = 0; k < nnz; ++k) T.rp[A.ci[k] + 1]++;
  for (int i = 0; i < A.n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(nnz);
  const bool vals = values && !A.v.empty();
  if (vals) T.v.resize(nnz);
  if (perm) perm->resize(nnz);
  std::vector<int> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.m; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int d = pos[A.ci[k]]++;
      T.ci[d] = i;
      if (vals) T.v[d] = A.v[k];
      if (perm) (*perm)[d] = k;
    }
  return T;
}

// Structural pattern of L R (no cancellation pruning), rows sorted.
HCsr symbolic_product(const HCsr& L, const HCsr& R) {
  HCsr C;
  C.m = L.m; C.n = R.n;
  auto make_row = [&] {
    return [&, mark = std::vector<int>(R.n, -1)](int i, std::vector<int>& out) mutable {
      const size_t at = out.size();
      for (int k = L.rp[i]; k < L.rp[i + 1]; ++k) {
        const int j = L.ci[k];
        for (int t = R.rp[j]; t < R.rp[j + 1]; ++t) {
          const int c = R.ci[t];
          if (mark[c] != i) { mark[c] = i; out.push_back(c); }
        }
      }
      // a dense row (more than 1/16 of the columns) comes out in column order from a scan of the
      // marks, a sparse one from a sort: the same entries in the same order
      const size_t cnt = out.size() - at;
      if (cnt * 16 > (size_t)R.n) {
        out.resize(at);
        for (int c = 0; c < R.n; ++c)
          if (mark[c] == i) out.push_back(c);
      } else {
        std::sort(out.begin() + at, out.end());
      }
    };
  };
  build_rows(L.m, C.rp, C.ci, make_row);
  return C;
}

// Greedy first-fit colouring of the rows of A in index order; rows conflict when they share a
// column.  Returns the colour of every row; colours ascending, rows ascending within a colour
// give the Kaczmarz order.
std::vector<int> greedy_row_colouring(const HCsr& A) {
  HCsr T = transpose(A, nullptr, false);
  std::vector<int> colour(A.m, -1);
  std::vector<int> stamp;
  for (int i = 0; i < A.m; ++i) {
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int c = A.ci[k];
      // the rows of a column come in ascending order: only those before i are coloured
      for (int t = T.rp[c]; t < T.rp[c + 1]; ++t) {
        const int r = T.ci[t];
        if (r >= i) break;
        const int col = colour[r];
        if (col >= (int)stamp.size()) stamp.resize(col + 1, -1);
        stamp[col] = i;
      }
    }
    int c = 0;
    while (c < (int)stamp.size() && stamp[c] == i) ++c;
    colour[i] = c;
  }
  return colour;
}

void colour_order(const std::vector<int>& colour, std::vector<int>& rows, std::vector<int>& cptr) {
  int nc = 0;
  for (int c : colour) nc = std::max(nc, c + 1);
  cptr.assign(nc + 1, 0);
  for (int c : colour) cptr[c + 1]++;
  for (int c = 0; c < nc; ++c) cptr[c + 1] += cptr[c];
  rows.resize(colour.size());
  std::vector<int> pos(cptr.begin(), cptr.end() - 1);
  for (int i = 0; i < (int)colour.size(); ++i) rows[pos[colour[i]]++] = i;
}

HCsr union_pattern(const HCsr& A, const HCsr& B) {
  HCsr C;
  C.m = A.m; C.n = A.n;
  C.rp.assign(A.m + 1, 0);
  for (int i = 0; i < A.m; ++i) {
    int a = A.rp[i], ae = A.rp[i + 1], b = B.rp[i], be = B.rp[i + 1];
    while (a < ae || b < be) {
      int ca = a < ae ? A.ci[a] : INT32_MAX, cb = b < be ? B.ci[b] : INT32_MAX;
      if (ca == cb) { C.ci.push_back(ca); ++a; ++b; }
      else if (ca < cb) { C.ci.push_back(ca); ++a; }
      else { C.ci.push_back(cb); ++b; }
    }
    C.rp[i + 1] = (int)C.ci.size();
  }
  return C;
}

}  // namespace slamg
