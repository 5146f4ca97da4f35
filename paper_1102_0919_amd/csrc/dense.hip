// Small dense FP64 procedures run by one workgroup each: Cholesky factorisation, triangular
// solves, a parallel-order two-sided Jacobi eigensolver, the coarsest-level generalized SVD /
// eigenproblem (§3.6 with Theorem 3.1's change of variables), the additive coarsest solves
// (§4.2: pseudo-inverse of X - sigma Y without its smallest singular component, and the pencil
// variant), and the n_b x n_b Ritz problems (§4.3).  Matrices are row-major in global memory
// (they are small and stay in L2); rotation parameters live in LDS.
#include "common.h"

#include <algorithm>

namespace slamg {

static constexpr int DBLK = 256;
static constexpr int MAXPAIR = 512;   // matrices up to 1024 x 1024

__device__ static void wg_sync() { __syncthreads(); }

// Visits every (i, j), 0 <= i < R, 0 <= j < n, with the workgroup's threads: consecutive threads take
// consecutive j (coalesced rows), and the loop carries no integer division.
template <int BS = DBLK, class F>
__device__ __forceinline__ void wg_for2(int R, int n, F&& f) {
  if (n <= 0 || R <= 0) return;
  if (n <= BS) {
    const int G = BS / n, j = (int)threadIdx.x % n, g = (int)threadIdx.x / n;
    if (g < G) {
#pragma unroll 4
      for (int i = g; i < R; i += G) f(i, j);
    }
  } else {
    for (int j = threadIdx.x; j < n; j += BS) {
#pragma unroll 4
      for (int i = 0; i < R; ++i) f(i, j);
    }
  }
}

// A (n x n, ld) <- L (lower), A = L L^t.  Returns (in *info) 0 or the first failing pivot + 1;
// a failing pivot is replaced by a tiny positive value so the factor stays finite.
template <int BS = DBLK>
__device__ static void wg_chol(double* A, int n, int ld, int* info) {
  __shared__ double dk_s;
  for (int k = 0; k < n; ++k) {
    wg_sync();
    if (threadIdx.x == 0) {
      double d = A[(long)k * ld + k];
      if (!(d > 0.0)) {
        if (*info == 0) *info = k + 1;
        d = 1e-300;
      }
      d = sqrt(d);
      A[(long)k * ld + k] = d;
      dk_s = d;
    }
    wg_sync();
    const double dk = dk_s;
    for (int i = k + 1 + threadIdx.x; i < n; i += BS) A[(long)i * ld + k] /= dk;
    wg_sync();
    const int nt = n - k - 1;
    for (long t = threadIdx.x; t < (long)nt * nt; t += BS) {
      int i = k + 1 + (int)(t / nt), j = k + 1 + (int)(t % nt);
      if (j <= i) A[(long)i * ld + j] -= A[(long)i * ld + k] * A[(long)j * ld + k];
    }
  }
  wg_sync();
  for (long t = threadIdx.x; t < (long)n * n; t += BS) {
    int i = (int)(t / n), j = (int)(t % n);
    if (j > i) A[(long)i * ld + j] = 0.0;
  }
  wg_sync();
}

// Solve L X = B in place (B: n x nc, ldb), L lower; one thread per right-hand side column.
template <int BS = DBLK>
__device__ static void wg_trsm_lower(const double* L, int n, int ld, double* B, int nc, int ldb) {
  wg_sync();
  for (int c = threadIdx.x; c < nc; c += BS) {
    for (int i = 0; i < n; ++i) {
      double s = B[(long)i * ldb + c];
      for (int k = 0; k < i; ++k) s -= L[(long)i * ld + k] * B[(long)k * ldb + c];
      B[(long)i * ldb + c] = s / L[(long)i * ld + i];
    }
  }
  wg_sync();
}

// Solve L^t X = B in place (B: n x nc), L lower.
template <int BS = DBLK>
__device__ static void wg_trsm_lower_t(const double* L, int n, int ld, double* B, int nc, int ldb) {
  wg_sync();
  for (int c = threadIdx.x; c < nc; c += BS) {
    for (int i = n - 1; i >= 0; --i) {
      double s = B[(long)i * ldb + c];
      for (int k = i + 1; k < n; ++k) s -= L[(long)k * ld + i] * B[(long)k * ldb + c];
      B[(long)i * ldb + c] = s / L[(long)i * ld + i];
    }
  }
  wg_sync();
}

template <int BS = DBLK>
__device__ static void wg_transpose(const double* A, int r, int c, int lda, double* B, int ldb) {
  wg_sync();
  for (long t = threadIdx.x; t < (long)r * c; t += BS) {
    int i = (int)(t / c), j = (int)(t % c);
    B[(long)j * ldb + i] = A[(long)i * lda + j];
  }
  wg_sync();
}

// Two-sided cyclic Jacobi with the round-robin parallel ordering: A (n x n symmetric) is reduced to
// diagonal form in place; V accumulates the rotations (A_in = V diag V^t; with init_v false, V
// holds an orthogonal start basis and receives V J_1 J_2 ...).  A pair is rotated
// when |a_pq| > 1e-15 sqrt(|a_pp a_qq|) and |a_pq| > 2^-53 ||A||_F; the sweeps stop after one that
// rotated nothing or only by angles with |tan| <= 2^-26.  The absolute floor is the backward-stable accuracy of any symmetric eigensolver
// in double precision: below it the off-diagonal entries are rounding noise of earlier rotations,
// and an indefinite matrix would keep producing such noise under the relative test alone.
// Inlined at each call so that the compiler sees where A and V live (LDS or global memory) and
// emits LDS instructions for LDS-resident matrices; the procedure is latency-bound.
template <int BS = DBLK, bool VGLOBAL = false>
__device__ static __forceinline__ void wg_jacobi(double* A, int n, int ld, double* V, int ldv, int maxsweep,
                                                 bool init_v = true) {
  __shared__ int P[MAXPAIR], Q[MAXPAIR];
  __shared__ double Cs[MAXPAIR], Sn[MAXPAIR];
  __shared__ double red[BS];
  __shared__ int rotated, large;
  if (init_v) wg_for2<BS>(n, n, [&](int i, int j) { V[(long)i * ldv + j] = i == j ? 1.0 : 0.0; });
  const int N = n + (n & 1);
  const int npair = N / 2;
  if (n <= 1) { wg_sync(); return; }
  double tot = 0.0;
  wg_for2<BS>(n, n, [&](int i, int j) {
    const double a = A[(long)i * ld + j];
    tot += a * a;
  });
  red[threadIdx.x] = tot;
  wg_sync();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    wg_sync();
  }
  const double floor_abs = 0x1p-53 * sqrt(red[0]);
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    if (threadIdx.x == 0) { rotated = 0; large = 0; }
    wg_sync();
    for (int r = 0; r < N - 1; ++r) {
      for (int k = threadIdx.x; k < npair; k += BS) {
        // round-robin schedule: index 0 stays, the others rotate by r (a - 1 + r < 2 (N - 1))
        const int a = k, b = N - 1 - k;
        int p = a - 1 + r, q = b - 1 + r;
        p = a == 0 ? 0 : (p >= N - 1 ? p - (N - 1) : p) + 1;
        q = b == 0 ? 0 : (q >= N - 1 ? q - (N - 1) : q) + 1;
        if (p > q) { int tmp = p; p = q; q = tmp; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[(long)p * ld + q];
          const double app = A[(long)p * ld + p], aqq = A[(long)q * ld + q];
          // |a_pq| > 1e-15 sqrt(|a_pp a_qq|), compared in squares
          if (apq * apq > 1e-30 * fabs(app * aqq) && fabs(apq) > floor_abs && fabs(apq) > 1e-300) {
            double tau = (aqq - app) / (2.0 * apq);
            double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            rotated = 1;
            if (fabs(tt) > 0x1p-26) large = 1;
          }
        }
        // the pair with the padding index n (odd n) becomes (p, p) with the identity rotation, so the
        // updates below need no branch
        if (q >= n) q = p;
        P[k] = p; Q[k] = q; Cs[k] = c; Sn[k] = s;
      }
      wg_sync();
      // A <- R A R^t for the block-diagonal rotation R of this round: every 2 x 2 block (rows of
      // pair a, columns of pair b) is independent, so one phase suffices: rotate the block's rows,
      // then its columns (the same operations, in the same order, as a row pass followed by a
      // column pass).  The padding pair is (p, p) with the identity rotation.
      wg_for2<BS>(npair, npair, [&](int a, int b) {
        const int pa = P[a], qa = Q[a], pb = P[b], qb = Q[b];
        const double ca = Cs[a], sa = Sn[a], cb = Cs[b], sb = Sn[b];
        const double x00 = A[(long)pa * ld + pb], x01 = A[(long)pa * ld + qb];
        const double x10 = A[(long)qa * ld + pb], x11 = A[(long)qa * ld + qb];
        const double r00 = ca * x00 - sa * x10, r10 = sa * x00 + ca * x10;   // rows, column pb
        const double r01 = ca * x01 - sa * x11, r11 = sa * x01 + ca * x11;   // rows, column qb
        A[(long)pa * ld + pb] = cb * r00 - sb * r01;
        A[(long)pa * ld + qb] = sb * r00 + cb * r01;
        A[(long)qa * ld + pb] = cb * r10 - sb * r11;
        A[(long)qa * ld + qb] = sb * r10 + cb * r11;
      });
      // V <- V R^t.  A round's pairs are disjoint, so a thread's updates are independent; with V in
      // global memory (VGLOBAL) its loads go out first, four pairs at a time, then the updates, where
      // a load -> store chain per pair would serialise the round.
      if (VGLOBAL && n <= BS) {
        const int gv = BS / n, i = (int)threadIdx.x % n, g = (int)threadIdx.x / n;
        if (g < gv) {
          for (int b0 = g; b0 < npair; b0 += 4 * gv) {
            int pb[4], qb[4];
            double vp[4], vq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int b = b0 + u * gv;
              pb[u] = qb[u] = -1;
              vp[u] = vq[u] = 0.0;
              if (b < npair) {
                pb[u] = P[b];
                qb[u] = Q[b];
                vp[u] = V[(long)i * ldv + pb[u]];
                vq[u] = V[(long)i * ldv + qb[u]];
              }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int b = b0 + u * gv;
              if (b < npair) {
                const double cb = Cs[b], sb = Sn[b];
                V[(long)i * ldv + pb[u]] = cb * vp[u] - sb * vq[u];
                V[(long)i * ldv + qb[u]] = sb * vp[u] + cb * vq[u];
              }
            }
          }
        }
      } else {
        wg_for2<BS>(npair, n, [&](int b, int i) {
          const int pb = P[b], qb = Q[b];
          const double cb = Cs[b], sb = Sn[b];
          const double vip = V[(long)i * ldv + pb], viq = V[(long)i * ldv + qb];
          V[(long)i * ldv + pb] = cb * vip - sb * viq;
          V[(long)i * ldv + qb] = sb * vip + cb * viq;
        });
      }
      wg_sync();
    }
    const int any = rotated, big = large;
    wg_sync();
    // done after a sweep that rotated nothing, or whose rotations all had |tan| <= 2^-26: the
    // entries such a sweep leaves off the diagonal are second order in those angles, below the
    // 2^-53 ||A||_F floor, so a further sweep would rotate nothing
    if (!any || !big) break;
  }
  wg_sync();
}

// Ranking key: a NaN ranks after every other value (NaN compares false with everything, so ranking
// it directly would give several entries one rank and leave output positions unwritten).
__device__ __forceinline__ double rank_key(double x, bool desc) {
  return x == x ? x : (desc ? -INFINITY : INFINITY);
}

// indices of the k extremal values of lam[0..n) (largest first if desc, else smallest first); ties
// to the lower index.  Each thread ranks its own entries (the rank is the output position); every
// entry gets a distinct rank in [0, n), so out[0..k) is always filled with indices below n.
template <int BS = DBLK>
__device__ static void select_extremal(const double* lam, int n, int k, bool desc, int* out) {
  wg_sync();
  for (int i = threadIdx.x; i < n; i += BS) {
    const double li = rank_key(lam[i], desc);
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = rank_key(lam[j], desc);
      rank += (desc ? lj > li : lj < li) || (lj == li && j < i);
    }
    if (rank < k) out[rank] = i;
  }
  wg_sync();
}

// ------------------------------------------------------------------------------------------------
// Cholesky-QR step: G = R^t R, T = R^{-1} (upper), row-major w x w, computed on the column-scaled
// Gram matrix.  A non-positive pivot retries once with a diagonal shift of 1e-14 trace; a second
// failure sets *status.  With pivot_min given, it receives the smallest of the first wpiv pivots
// L_ii^2 of the unshifted factorisation of the column-scaled matrix, or -1 when that factorisation
// failed within them (a failure at a later pivot leaves the first wpiv unchanged).
// ------------------------------------------------------------------------------------------------
// The Cholesky-QR factor of the n_b x n_b Gram matrix runs on one wavefront: its steps are short
// chains of LDS updates, and a barrier of a one-wave workgroup costs next to nothing.
static constexpr int SB = 64;

// workgroup b of the launch factors G_b into T_b (b = 0, 1: the U- and V-side passes of a pair)
__global__ __launch_bounds__(SB) void k_chol_inv_upper(int w, const double* G0, double* T0, const double* G1, double* T1,
                                                       int* status, double* pivot_min, int wpiv) {
  const double* G = blockIdx.x == 0 ? G0 : G1;
  double* T = blockIdx.x == 0 ? T0 : T1;
  // Columns are first scaled to unit norm (D G D with D = diag(G)^-1/2, T = D R^-1): the span,
  // and hence the Ritz step, is unchanged, and the factorisation then depends on the angles between
  // the columns only, not on their norms (relaxations can grow some columns by many orders).
  __shared__ double L[16 * 16], Ts[16 * 16], Gs[16 * 16];
  __shared__ double dsc[16];
  __shared__ int info;
  for (int t = threadIdx.x; t < w * w; t += SB) Gs[t] = G[t];
  wg_sync();
  for (int i = threadIdx.x; i < w; i += SB) {
    const double g = Gs[i * w + i];
    dsc[i] = g > 0.0 ? 1.0 / sqrt(g) : 1.0;
  }
  wg_sync();
  for (int attempt = 0; attempt < 2; ++attempt) {
    double tr = 0.0;
    for (int i = 0; i < w; ++i) tr += Gs[i * w + i] * dsc[i] * dsc[i];
    for (int t = threadIdx.x; t < w * w; t += SB) {
      int i = t / w, j = t % w;
      L[i * 16 + j] = Gs[t] * dsc[i] * dsc[j] + (attempt && i == j ? 1e-14 * tr : 0.0);
    }
    if (threadIdx.x == 0) info = 0;
    wg_sync();
    wg_chol<SB>(L, w, 16, &info);
    if (pivot_min && attempt == 0 && threadIdx.x == 0) {
      const bool failed = info != 0 && info <= wpiv;
      double pm = failed ? -1.0 : L[0] * L[0];
      for (int i = 1; !failed && i < wpiv; ++i) pm = fmin(pm, L[i * 16 + i] * L[i * 16 + i]);
      *pivot_min = pm;
    }
    if (info == 0) break;
    if (attempt == 1 && threadIdx.x == 0) *status = ST_E_NUMERIC;
    wg_sync();
  }
  // T = D L^{-t}: solve L^t T' = I, then scale the rows
  for (int t = threadIdx.x; t < w * w; t += SB) Ts[t] = (t / w == t % w) ? 1.0 : 0.0;
  wg_trsm_lower_t<SB>(L, w, 16, Ts, w, w);
  for (int t = threadIdx.x; t < w * w; t += SB) T[t] = Ts[t] * dsc[t / w];
}
void launch_chol_inv_upper(int w, const double* G, double* T, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv_upper, dim3(1), dim3(SB), 0, s, w, G, T, G, T, status, (double*)nullptr, w);
}
void launch_chol_inv_upper_pivot(int w, int wpiv, const double* G, double* T, int* status, double* pivot_min,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv_upper, dim3(1), dim3(SB), 0, s, w, G, T, G, T, status, pivot_min, wpiv);
}
void launch_chol_inv_upper2(int w, const double* G0, double* T0, const double* G1, double* T1, int* status,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv_upper, dim3(2), dim3(SB), 0, s, w, G0, T0, G1, T1, status, (double*)nullptr, w);
}

// ------------------------------------------------------------------------------------------------
// Ritz problem on the finest level (§4.3).  Eigenproblem: M = V diag V^t (M symmetrised), Y = V
// sorted; order descending (dominant) or ascending (minimal).
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(DBLK) void k_small_eig(int w, int minimal, const double* M, double* Y, double* sig) {
  __shared__ int ord[32];
  __shared__ double lam[32];
  __shared__ double A[16 * 16], V[16 * 16];
  for (int t = threadIdx.x; t < w * w; t += DBLK) {
    int i = t / w, j = t % w;
    A[t] = 0.5 * (M[i * w + j] + M[j * w + i]);
  }
  wg_jacobi(A, w, w, V, w, 60);
  for (int i = threadIdx.x; i < w; i += DBLK) lam[i] = A[i * w + i];
  wg_sync();
  select_extremal(lam, w, w, !minimal, ord);
  for (int t = threadIdx.x; t < w * w; t += DBLK) {
    int i = t / w, k = t % w;
    Y[i * w + k] = V[i * w + ord[k]];
  }
  for (int k = threadIdx.x; k < w; k += DBLK) sig[k] = lam[ord[k]];
}

// SVD of the n_b x n_b Ritz matrix (§4.3) by one-sided (Hestenes) Jacobi on one wavefront: pairs of
// columns of M, and of V (from I), are rotated until every pair is orthogonal to 1e-15 relative;
// then sigma_k = ||M e_k||, z_k = V e_k, y_k = M z_k / sigma_k (so y_k^t M z_k = sigma_k >= 0).  An
// n_b-column problem takes n_b - 1 rounds per sweep (the augmented 2 n_b form takes 2 n_b - 1).  Lane
// l serves pair slot l / 8 on rows l % 8 and l % 8 + 8; the three sums of a pair meet by lane
// shuffles.  Numerically zero sigma (<= 1e-13 sigma_max) get y completed to an orthonormal set.
// Output: Y, Z (w x w row-major, column k the k-th triplet), sig; order descending (dominant) or
// ascending (minimal).
__global__ __launch_bounds__(64) void k_small_svd(int w, int minimal, const double* M, double* Y, double* Z,
                                                  double* sig) {
  __shared__ double Ms[16 * 16], Vs[16 * 16];   // row-major, ld 16, zero beyond w
  __shared__ double Ys[16 * 16], Zs[16 * 16], ss[16], sg[16];
  __shared__ int ord[32], tinyk[16];
  const int lane = threadIdx.x;
  for (int t = lane; t < 256; t += 64) {
    const int i = t >> 4, j = t & 15;
    Ms[t] = (i < w && j < w) ? M[i * w + j] : 0.0;
    Vs[t] = (i == j && i < w) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int W = w + (w & 1), np = W / 2;
  const int slot = lane >> 3, r = lane & 7;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rotated = 0;
    for (int rr = 0; rr < W - 1; ++rr) {
      int p = 0, q = 0;
      if (slot < np) {
        const int a = slot, b = W - 1 - slot;
        int pp = a - 1 + rr, qq = b - 1 + rr;
        pp = a == 0 ? 0 : (pp >= W - 1 ? pp - (W - 1) : pp) + 1;
        qq = b == 0 ? 0 : (qq >= W - 1 ? qq - (W - 1) : qq) + 1;
        p = pp < qq ? pp : qq;
        q = pp < qq ? qq : pp;
      }
      const bool act = slot < np && q < w;   // the padding column (odd w) pairs with nothing
      double mp0 = 0.0, mq0 = 0.0, mp1 = 0.0, mq1 = 0.0, vp0 = 0.0, vq0 = 0.0, vp1 = 0.0, vq1 = 0.0;
      if (act) {
        mp0 = Ms[r * 16 + p]; mq0 = Ms[r * 16 + q]; mp1 = Ms[(r + 8) * 16 + p]; mq1 = Ms[(r + 8) * 16 + q];
        vp0 = Vs[r * 16 + p]; vq0 = Vs[r * 16 + q]; vp1 = Vs[(r + 8) * 16 + p]; vq1 = Vs[(r + 8) * 16 + q];
      }
      double al = mp0 * mp0 + mp1 * mp1, be = mq0 * mq0 + mq1 * mq1, ga = mp0 * mq0 + mp1 * mq1;
#pragma unroll
      for (int m = 1; m < 8; m <<= 1) {
        al += __shfl_xor(al, m);
        be += __shfl_xor(be, m);
        ga += __shfl_xor(ga, m);
      }
      if (act && ga * ga > 1e-30 * al * be && fabs(ga) > 1e-300) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        rotated = 1;
        Ms[r * 16 + p] = c * mp0 - sn * mq0;
        Ms[r * 16 + q] = sn * mp0 + c * mq0;
        Ms[(r + 8) * 16 + p] = c * mp1 - sn * mq1;
        Ms[(r + 8) * 16 + q] = sn * mp1 + c * mq1;
        Vs[r * 16 + p] = c * vp0 - sn * vq0;
        Vs[r * 16 + q] = sn * vp0 + c * vq0;
        Vs[(r + 8) * 16 + p] = c * vp1 - sn * vq1;
        Vs[(r + 8) * 16 + q] = sn * vp1 + c * vq1;
      }
      __syncthreads();
    }
    if (__ballot(rotated) == 0) break;
  }
  if (lane < w) {
    double s2 = 0.0;
    for (int i = 0; i < w; ++i) s2 += Ms[i * 16 + lane] * Ms[i * 16 + lane];
    sg[lane] = sqrt(s2);
  }
  select_extremal<64>(sg, w, w, true, ord);   // descending
  const double smax = sg[ord[0]];
  if (lane < w) {
    const int src = ord[lane], dst = minimal ? (w - 1 - lane) : lane;
    const double sk = sg[src];
    const bool tiny = !(sk > 1e-13 * smax);
    for (int i = 0; i < w; ++i) {
      Zs[i * w + dst] = Vs[i * 16 + src];
      Ys[i * w + dst] = tiny ? 0.0 : Ms[i * 16 + src] / sk;
    }
    ss[dst] = sk;
    tinyk[dst] = tiny ? 1 : 0;
  }
  __syncthreads();
  // zero sigma: y_k from the unit vector e_e with the largest remainder after projection onto the
  // columns already set (orthonormal, so the remainder is 1 - sum_k2 Y[e][k2]^2, at least 1/w while
  // the complement is not empty; ties to the lower e), then two Gram-Schmidt passes against them
  // (column order)
  if (lane == 0) {
    for (int k = 0; k < w; ++k) {
      if (!tinyk[k]) continue;
      int eb = 0;
      double best = -1.0;
      for (int e = 0; e < w; ++e) {
        double rem = 1.0;
        for (int k2 = 0; k2 < w; ++k2)
          if (k2 != k && !(tinyk[k2] && k2 > k)) rem -= Ys[e * w + k2] * Ys[e * w + k2];
        if (rem > best) {
          best = rem;
          eb = e;
        }
      }
      for (int i = 0; i < w; ++i) Ys[i * w + k] = i == eb ? 1.0 : 0.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int k2 = 0; k2 < w; ++k2) {
          if (k2 == k || (tinyk[k2] && k2 > k)) continue;
          double d = 0.0;
          for (int i = 0; i < w; ++i) d += Ys[i * w + k] * Ys[i * w + k2];
          for (int i = 0; i < w; ++i) Ys[i * w + k] -= d * Ys[i * w + k2];
        }
      double nrm = 0.0;
      for (int i = 0; i < w; ++i) nrm += Ys[i * w + k] * Ys[i * w + k];
      nrm = sqrt(nrm);
      for (int i = 0; i < w; ++i) Ys[i * w + k] /= nrm;
    }
  }
  __syncthreads();
  for (int t = lane; t < w * w; t += 64) {
    Y[t] = Ys[t];
    Z[t] = Zs[t];
  }
  if (lane < w) sig[lane] = ss[lane];
}

// SVD of the k x k projected matrix of the LOBPCG step (k <= 32) by one-sided (Hestenes) Jacobi, as
// k_small_svd: columns of M and of V (from I) rotated in pairs until every pair is orthogonal to
// 1e-15 relative; sigma_j = ||M e_j||, z_j = V e_j, y_j = M z_j / sigma_j, zero sigma (<= 1e-13
// sigma_max) completed to an orthonormal set.  A pair slot of 8 lanes holds rows r, r + 8, r + 16,
// r + 24 of its two columns; 16 slots rotate the 16 pairs of a round.  Output: the nb triplets in
// target order (descending for dominant, ascending for minimal), Y, Z (k x nb row-major), sig (nb).
constexpr int PSB = 128;
__global__ __launch_bounds__(PSB) void k_proj_svd(int k, int nb, int minimal, const double* M, double* Y, double* Z,
                                                  double* sig) {
  __shared__ double Ms[32 * 32], Vs[32 * 32];   // row-major, ld 32, zero beyond k
  __shared__ double Ys[32 * 32], Zs[32 * 32];   // sorted triplets, ld 32
  __shared__ double sg[32], ss[32];
  __shared__ int ord[32], tinyk[32];
  __shared__ int rot;
  const int t = threadIdx.x;
  for (int q = t; q < 1024; q += PSB) {
    const int i = q >> 5, j = q & 31;
    Ms[q] = (i < k && j < k) ? M[i * k + j] : 0.0;
    Vs[q] = (i == j && i < k) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int W = k + (k & 1), np = W / 2;
  const int slot = t >> 3, r = t & 7;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) rot = 0;
    __syncthreads();
    for (int rr = 0; rr < W - 1; ++rr) {
      int p = 0, q = 0;
      if (slot < np) {
        const int a = slot, b = W - 1 - slot;
        int pp = a - 1 + rr, qq = b - 1 + rr;
        pp = a == 0 ? 0 : (pp >= W - 1 ? pp - (W - 1) : pp) + 1;
        qq = b == 0 ? 0 : (qq >= W - 1 ? qq - (W - 1) : qq) + 1;
        p = pp < qq ? pp : qq;
        q = pp < qq ? qq : pp;
      }
      const bool act = slot < np && q < k;   // the padding column (odd k) pairs with nothing
      double mp[4], mq[4], vp[4], vq[4];
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = r + 8 * u;
        mp[u] = act ? Ms[row * 32 + p] : 0.0;
        mq[u] = act ? Ms[row * 32 + q] : 0.0;
        vp[u] = act ? Vs[row * 32 + p] : 0.0;
        vq[u] = act ? Vs[row * 32 + q] : 0.0;
        al += mp[u] * mp[u];
        be += mq[u] * mq[u];
        ga += mp[u] * mq[u];
      }
#pragma unroll
      for (int m = 1; m < 8; m <<= 1) {
        al += __shfl_xor(al, m);
        be += __shfl_xor(be, m);
        ga += __shfl_xor(ga, m);
      }
      if (act && ga * ga > 1e-30 * al * be && fabs(ga) > 1e-300) {
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), sn = tt * c;
        if (r == 0) rot = 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = r + 8 * u;
          Ms[row * 32 + p] = c * mp[u] - sn * mq[u];
          Ms[row * 32 + q] = sn * mp[u] + c * mq[u];
          Vs[row * 32 + p] = c * vp[u] - sn * vq[u];
          Vs[row * 32 + q] = sn * vp[u] + c * vq[u];
        }
      }
      __syncthreads();
    }
    const int any = rot;
    __syncthreads();
    if (any == 0) break;
  }
  if (t < k) {
    double s2 = 0.0;
    for (int i = 0; i < k; ++i) s2 += Ms[i * 32 + t] * Ms[i * 32 + t];
    sg[t] = sqrt(s2);
  }
  select_extremal<PSB>(sg, k, k, true, ord);   // descending
  const double smax = sg[ord[0]];
  if (t < k) {
    const int src = ord[t], dst = minimal ? (k - 1 - t) : t;
    const double sk = sg[src];
    const bool tiny = !(sk > 1e-13 * smax);
    for (int i = 0; i < k; ++i) {
      Zs[i * 32 + dst] = Vs[i * 32 + src];
      Ys[i * 32 + dst] = tiny ? 0.0 : Ms[i * 32 + src] / sk;
    }
    ss[dst] = sk;
    tinyk[dst] = tiny ? 1 : 0;
  }
  __syncthreads();
  // zero sigma: y from the unit vector e_e with the largest remainder after projection onto the
  // columns already set (orthonormal, so the remainder is 1 - sum_c2 Y[e][c2]^2, at least 1/k while
  // the complement is not empty; ties to the lower e), then two Gram-Schmidt passes against them
  // (column order)
  if (t == 0) {
    for (int c = 0; c < k; ++c) {
      if (!tinyk[c]) continue;
      int eb = 0;
      double best = -1.0;
      for (int e = 0; e < k; ++e) {
        double rem = 1.0;
        for (int c2 = 0; c2 < k; ++c2)
          if (c2 != c && !(tinyk[c2] && c2 > c)) rem -= Ys[e * 32 + c2] * Ys[e * 32 + c2];
        if (rem > best) {
          best = rem;
          eb = e;
        }
      }
      for (int i = 0; i < k; ++i) Ys[i * 32 + c] = i == eb ? 1.0 : 0.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int c2 = 0; c2 < k; ++c2) {
          if (c2 == c || (tinyk[c2] && c2 > c)) continue;
          double d = 0.0;
          for (int i = 0; i < k; ++i) d += Ys[i * 32 + c] * Ys[i * 32 + c2];
          for (int i = 0; i < k; ++i) Ys[i * 32 + c] -= d * Ys[i * 32 + c2];
        }
      double nrm = 0.0;
      for (int i = 0; i < k; ++i) nrm += Ys[i * 32 + c] * Ys[i * 32 + c];
      nrm = sqrt(nrm);
      for (int i = 0; i < k; ++i) Ys[i * 32 + c] /= nrm;
    }
  }
  __syncthreads();
  for (int q = t; q < k * nb; q += PSB) {
    const int i = q / nb, d = q % nb;
    Y[q] = Ys[i * 32 + d];
    Z[q] = Zs[i * 32 + d];
  }
  if (t < nb) sig[t] = ss[t];
}
// the caller keeps 1 <= nb <= k <= 32; other sizes launch nothing
void launch_proj_svd(int k, int nb, int minimal, const double* M, double* Y, double* Z, double* sig, hipStream_t s) {
  if (k < 1 || k > 32 || nb < 1 || nb > k) return;
  hipLaunchKernelGGL(k_proj_svd, dim3(1), dim3(PSB), 0, s, k, nb, minimal, M, Y, Z, sig);
}

void launch_small_ritz(int w, int spd, int minimal, const double* M, double* Y, double* Z, double* sig, double* work,
                       int* status, hipStream_t s) {
  (void)work;
  (void)status;
  if (spd) hipLaunchKernelGGL(k_small_eig, dim3(1), dim3(DBLK), 0, s, w, minimal, M, Y, sig);
  else hipLaunchKernelGGL(k_small_svd, dim3(1), dim3(64), 0, s, w, minimal, M, Y, Z, sig);
}

// ------------------------------------------------------------------------------------------------
// Coarsest generalized SVD / eigenproblem (§3.6).  A, B, C dense row-major (C unused for spd);
// B and C are overwritten by their Cholesky factors.
// spd:  D = L^-1 A L^-t, D = W diag W^t, x = L^-t w; the n_b smallest / largest.
// svd:  D = L_B^-1 A L_C^-t, D^t D = W diag(s^2) W^t, t = D w / s, u = L_B^-t t, v = L_C^-t w.
//       A zero s gets t completed to an orthonormal set by Gram-Schmidt on unit vectors.
// Output U (mL x nb), V (nL x nb) row-major, sig (nb).
// work: >= 3 max(mL,nL)^2 + 2 mL nL + 2 max doubles.
// ------------------------------------------------------------------------------------------------
// The coarsest generalized SVD runs on 1024 threads: its Jacobi rounds and its O(n) factorisation
// steps are chains of dependent updates, and only one workgroup runs.
static constexpr int GB = 1024;

// Jacobi on the n x n matrix S (row-major, global memory), eigenvectors into V; with LDSJ the
// rotations run on an LDS copy of S, which is written back.
template <bool LDSJ>
__device__ __forceinline__ void jacobi_lds(double* S, int n, double* V) {
  if constexpr (LDSJ) {
    extern __shared__ double jdyn[];
    wg_sync();
    for (long t = threadIdx.x; t < (long)n * n; t += GB) jdyn[t] = S[t];
    wg_sync();
    wg_jacobi<GB, true>(jdyn, n, n, V, n, 60);
    for (long t = threadIdx.x; t < (long)n * n; t += GB) S[t] = jdyn[t];
    wg_sync();
  } else {
    wg_jacobi<GB, true>(S, n, n, V, n, 60);
  }
}

template <bool LDSJ>
__global__ __launch_bounds__(GB) void k_coarse_gsvd(int spd, int minimal, int mL, int nL, int nb, double* A,
                                                      double* B, double* C, double* work, double* sig, double* U,
                                                      double* V, int* status) {
  __shared__ int info;
  __shared__ int ord[64];
  if (threadIdx.x == 0) info = 0;
  wg_sync();
  if (spd) {
    const int n = nL;
    double* T1 = work;                 // n x n
    double* D = work + (long)n * n;    // n x n
    double* W = work + 2L * n * n;     // n x n
    double* lam = work + 3L * n * n;   // n
    wg_chol<GB>(B, n, n, &info);
    for (long t = threadIdx.x; t < (long)n * n; t += GB) T1[t] = A[t];
    wg_trsm_lower<GB>(B, n, n, T1, n, n);           // T1 = L^-1 A
    wg_transpose<GB>(T1, n, n, n, D, n);           // D = (L^-1 A)^t = A L^-t
    wg_trsm_lower<GB>(B, n, n, D, n, n);            // D = L^-1 A L^-t
    for (long t = threadIdx.x; t < (long)n * n; t += GB) {
      int i = (int)(t / n), j = (int)(t % n);
      if (j > i) {
        double s = 0.5 * (D[(long)i * n + j] + D[(long)j * n + i]);
        D[(long)i * n + j] = s; D[(long)j * n + i] = s;
      }
    }
    jacobi_lds<LDSJ>(D, n, W);
    for (int i = threadIdx.x; i < n; i += GB) {
      lam[i] = D[(long)i * n + i];
      if (!isfinite(lam[i])) info = 1;
    }
    wg_sync();
    select_extremal<GB>(lam, n, nb, !minimal, ord);
    for (long t = threadIdx.x; t < (long)n * nb; t += GB) {
      int i = (int)(t / nb), k = (int)(t % nb);
      U[t] = W[(long)i * n + ord[k]];
    }
    wg_trsm_lower_t<GB>(B, n, n, U, nb, nb);        // x = L^-t w
    for (int k = threadIdx.x; k < nb; k += GB) sig[k] = lam[ord[k]];
    if (threadIdx.x == 0 && info) *status = ST_E_NUMERIC;
    return;
  }
  // D = L_B^-1 A L_C^-t has l = min(m, n) singular values (§3.1, Theorem 3.2).  X is D or D^t,
  // whichever is tall (L x l, L = max(m, n)); the eigen-decomposition of X^t X gives the short-side
  // vectors w, and the long-side vectors are X w / ||X w||.  A (numerically) zero sigma
  // takes a unit long-side vector in the null space of X^t instead, orthogonal to the other ones.
  const int m = mL, n = nL;
  const bool tall = m >= n;
  const int l = tall ? n : m, Lr = tall ? m : n;
  double* Dt = work;                       // n x m   (D^t)
  double* G = Dt + (long)m * n;            // l x l
  double* W = G + (long)l * l;             // l x l
  double* Y = W + (long)l * l;             // Lr x l  (long-side vectors of every non-zero sigma)
  double* Tm = Y + (long)Lr * l;           // Lr x nb (long-side vectors of the selected triplets)
  double* lam = Tm + (long)Lr * 64;        // l
  double* score = lam + l;                 // Lr
  // X(r, c), r < Lr, c < l
  auto X = [&](int r, int c) -> double { return tall ? Dt[(long)c * m + r] : Dt[(long)r * m + c]; };
  wg_chol<GB>(B, m, m, &info);
  wg_chol<GB>(C, n, n, &info);
  wg_trsm_lower<GB>(B, m, m, A, n, n);             // A <- L_B^-1 A   (m x n)
  wg_transpose<GB>(A, m, n, n, Dt, m);             // Dt = (L_B^-1 A)^t   (n x m)
  wg_trsm_lower<GB>(C, n, n, Dt, m, m);            // Dt = L_C^-1 A^t L_B^-t = D^t
  for (long t = threadIdx.x; t < (long)l * l; t += GB) {
    int i = (int)(t / l), j = (int)(t % l);
    double s = 0.0;
    for (int r = 0; r < Lr; ++r) s += X(r, i) * X(r, j);
    G[t] = s;
  }
  wg_sync();
  for (long t = threadIdx.x; t < (long)l * l; t += GB) {
    int i = (int)(t / l), j = (int)(t % l);
    if (j > i) {
      double s = 0.5 * (G[(long)i * l + j] + G[(long)j * l + i]);
      G[(long)i * l + j] = s; G[(long)j * l + i] = s;
    }
  }
  jacobi_lds<LDSJ>(G, l, W);
  for (int i = threadIdx.x; i < l; i += GB) {
    lam[i] = sqrt(fmax(G[(long)i * l + i], 0.0));
    if (!isfinite(G[(long)i * l + i])) info = 1;
  }
  wg_sync();
  select_extremal<GB>(lam, l, nb, !minimal, ord);
  double smax = 0.0;
  for (int i = 0; i < l; ++i) smax = fmax(smax, lam[i]);
  const double thr = 1e-12 * smax;
  // sigma_k = ||X w_k||: accurate to about eps sigma_max, where the square root of X^t X's
  // eigenvalue is only accurate to about sqrt(eps) sigma_max
  __shared__ double nu[64];
  for (long t = threadIdx.x; t < (long)Lr * nb; t += GB) {
    int r = (int)(t / nb), k = (int)(t % nb);
    double s = 0.0;
    for (int c = 0; c < l; ++c) s += X(r, c) * W[(long)c * l + ord[k]];
    Tm[t] = s;
  }
  wg_sync();
  for (int k = threadIdx.x; k < nb; k += GB) {
    double s = 0.0;
    for (int r = 0; r < Lr; ++r) s += Tm[(long)r * nb + k] * Tm[(long)r * nb + k];
    nu[k] = sqrt(s);
  }
  wg_sync();
  bool any_zero = false;
  for (int k = 0; k < nb; ++k) any_zero = any_zero || !(nu[k] > thr);
  for (long t = threadIdx.x; t < (long)Lr * nb; t += GB) {
    const int k = (int)(t % nb);
    Tm[t] = nu[k] > thr ? Tm[t] / nu[k] : 0.0;
  }
  if (any_zero) {
    // the range of X: unit vectors X w_i / sigma_i of every non-zero sigma_i
    for (long t = threadIdx.x; t < (long)Lr * l; t += GB) {
      int r = (int)(t / l), i = (int)(t % l);
      double s = 0.0;
      for (int c = 0; c < l; ++c) s += X(r, c) * W[(long)c * l + i];
      Y[t] = s;
    }
    wg_sync();
    for (int i = threadIdx.x; i < l; i += GB) {
      double s = 0.0;
      for (int r = 0; r < Lr; ++r) s += Y[(long)r * l + i] * Y[(long)r * l + i];
      lam[i] = sqrt(s);    // lam is not read again: the selected sigma_k are in nu
    }
    wg_sync();
    for (long t = threadIdx.x; t < (long)Lr * l; t += GB) {
      const int i = (int)(t % l);
      Y[t] = lam[i] > thr ? Y[t] / lam[i] : 0.0;
    }
    wg_sync();
    // each zero sigma: the projection of e_e onto null(X^t), minus the vectors already completed,
    // for the e with the largest remainder ||P e_e||^2 = 1 - sum_i Y[e][i]^2 - sum_q T[e][q]^2
    __shared__ int ebest;
    __shared__ double nbest;
    for (int k = 0; k < nb; ++k) {
      if (nu[k] > thr) continue;
      for (int e = threadIdx.x; e < Lr; e += GB) {
        double s = 1.0;
        for (int i = 0; i < l; ++i) s -= Y[(long)e * l + i] * Y[(long)e * l + i];
        for (int q = 0; q < k; ++q)
          if (!(nu[q] > thr)) s -= Tm[(long)e * nb + q] * Tm[(long)e * nb + q];
        score[e] = s;
      }
      wg_sync();
      if (threadIdx.x == 0) {
        int eb = 0;
        for (int e = 1; e < Lr; ++e)
          if (score[e] > score[eb]) eb = e;
        ebest = eb;
      }
      wg_sync();
      const int e = ebest;
      for (int r = threadIdx.x; r < Lr; r += GB) {
        double s = r == e ? 1.0 : 0.0;
        for (int i = 0; i < l; ++i) s -= Y[(long)r * l + i] * Y[(long)e * l + i];
        for (int q = 0; q < k; ++q)
          if (!(nu[q] > thr)) s -= Tm[(long)r * nb + q] * Tm[(long)e * nb + q];
        score[r] = s;
      }
      wg_sync();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int r = 0; r < Lr; ++r) s += score[r] * score[r];
        nbest = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
      }
      wg_sync();
      for (int r = threadIdx.x; r < Lr; r += GB) Tm[(long)r * nb + k] = score[r] * nbest;
      wg_sync();
    }
  }
  wg_sync();
  double* Ul = tall ? U : V;    // long side
  double* Us = tall ? V : U;    // short side
  for (long t = threadIdx.x; t < (long)Lr * nb; t += GB) Ul[t] = Tm[t];
  for (long t = threadIdx.x; t < (long)l * nb; t += GB) {
    int i = (int)(t / nb), k = (int)(t % nb);
    Us[t] = W[(long)i * l + ord[k]];
  }
  wg_trsm_lower_t<GB>(B, m, m, U, nb, nb);
  wg_trsm_lower_t<GB>(C, n, n, V, nb, nb);
  for (int k = threadIdx.x; k < nb; k += GB) sig[k] = nu[k];
  if (threadIdx.x == 0 && info) *status = ST_E_NUMERIC;
}
void launch_coarse_gsvd(int spd, int minimal, int mL, int nL, int nb, double* A, double* B, double* C, double* work,
                        double* sig, double* U, double* V, int* status, hipStream_t s) {
  // the rotated n x n matrix in LDS when it fits the workgroup's share beside the static arrays
  static const int max_dyn = [] {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void*)k_coarse_gsvd<true>) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    int m = v - (int)fa.sharedSizeBytes;
    if (m > 0 && hipFuncSetAttribute((const void*)k_coarse_gsvd<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     m) != hipSuccess) {
      (void)hipGetLastError();
      m = 0;
    }
    return m < 0 ? 0 : m;
  }();
  const size_t lds = (size_t)nL * nL * sizeof(double);
  if (lds <= (size_t)max_dyn)
    hipLaunchKernelGGL(k_coarse_gsvd<true>, dim3(1), dim3(GB), lds, s, spd, minimal, mL, nL, nb, A, B, C, work, sig,
                       U, V, status);
  else
    hipLaunchKernelGGL(k_coarse_gsvd<false>, dim3(1), dim3(GB), 0, s, spd, minimal, mL, nL, nb, A, B, C, work, sig,
                       U, V, status);
}

// ------------------------------------------------------------------------------------------------
// Additive coarsest solve (§4.2), one workgroup per column j: M = X - sigma_j Y is symmetric, so
// its SVD is its eigen-decomposition with |eigenvalues|; the pseudo-inverse without the smallest
// singular component is sum_{i != i*} q_i q_i^t / lambda_i, i* = argmin |lambda_i|.
// basis (nb N^2) holds each column's eigenvectors Q_j.  warm = 0 (cold): Jacobi on M from the
// identity.  warm = 1: sigma_j moved little since Q_j was computed, so Q_j^t M Q_j is nearly
// diagonal; the updates below finish it and Q_j <- Q_j V.  warm = 2: as 1 after re-orthonormalising
// Q_j (cold where the fourth LDS array is not available).  All give the eigen-decomposition of M to
// rounding.  rhs / out: N x nb row-major.  work: nb * 2 N^2 doubles.
//
// The workgroup has 1024 threads: a Jacobi round is a chain of dependent LDS updates, and only nb
// workgroups run, so four times the threads of the other dense kernels shorten each round's chain.
// ------------------------------------------------------------------------------------------------
static constexpr int PB = 1024;
typedef double v4d __attribute__((ext_vector_type(4)));

// C = op(A) op(B) for N x N row-major matrices in LDS, N <= 64, on the FP64 matrix cores: wave w of
// the 16 computes the 16 x 16 tile (w / 4, w % 4) of the product padded to 64 x 64, four k per
// instruction (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of the 16 x 4 and 4 x 16
// slices; the tile's D[l / 16 + 4 v][l % 16] comes back in register v).  C aliases neither input;
// the caller synchronises before and after.
template <bool TA, bool TB>
__device__ __forceinline__ void wg_mm64(const double* A, const double* B, double* C, int N) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ti = w >> 2, tj = w & 3;
  const int r = ti * 16 + (lane & 15), c = tj * 16 + (lane & 15), kk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < N; k0 += 4) {
    const int k = k0 + kk;
    double a = 0.0, b = 0.0;
    if (r < N && k < N) a = TA ? A[k * N + r] : A[r * N + k];
    if (c < N && k < N) b = TB ? B[c * N + k] : B[k * N + c];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = ti * 16 + kk + 4 * v;
    if (row < N && c < N) C[row * N + c] = acc[v];
  }
}

// C = op(A) op(B), N x N row-major, any N: one output per thread per pass, k ascending
template <bool TA, bool TB>
__device__ __forceinline__ void wg_mm(const double* A, const double* B, double* C, int N) {
  wg_for2<PB>(N, N, [&](int i, int c) {
    double acc = 0.0;
    for (int r = 0; r < N; ++r) acc += (TA ? A[(long)r * N + i] : A[(long)i * N + r]) * (TB ? B[(long)c * N + r] : B[(long)r * N + c]);
    C[(long)i * N + c] = acc;
  });
}

template <int LDSMODE>
__global__ __launch_bounds__(PB) void k_pinv_solve(int N, int nb, const double* X, const double* Y,
                                                   const double* sig, const double* rhs, double* out,
                                                   double* work, double* basis, int warm, int lds4) {
  // LDSMODE 0: everything in global memory (L2); 1: M in LDS; 2: M, the rotation accumulator and
  // the eigenvector copy in LDS (Q is read from / written back to `basis`), and for N <= 64 the
  // dense products on the matrix cores
  constexpr int lds_mode = LDSMODE;
  extern __shared__ double dyn[];
  const int j = blockIdx.x;
  const long NN = (long)N * N;
  const bool mm = lds_mode == 2 && N <= 64;
  double* Qg = basis + (long)j * NN;
  double* M;
  double* W2;
  double* Q;
  if constexpr (lds_mode >= 1) M = dyn; else M = work + (long)j * 2 * NN;
  if constexpr (lds_mode == 2) { W2 = dyn + NN; Q = dyn + 2 * NN; }
  else { W2 = work + (long)j * 2 * NN + NN; Q = Qg; }
  // fourth LDS array for the Newton-type steps (matrix-core products only)
  double* Tm = (lds_mode == 2 && mm && lds4) ? dyn + 3 * NN : nullptr;
  // the three N-vectors (eigenvalues, coefficients, right-hand side) follow the LDS matrices
  const int narr = lds_mode == 2 ? (lds4 ? 4 : 3) : lds_mode == 1 ? 1 : 0;
  double* lam = dyn + (long)narr * NN;
  double* cf = lam + N;
  double* rj = cf + N;
  __shared__ double red[PB];
  __shared__ int imin;
  const double s = sig[j];
  if (!warm || (warm == 2 && !Tm)) {
    for (long t = threadIdx.x; t < NN; t += PB) M[t] = X[t] - s * Y[t];
    wg_jacobi<PB, lds_mode < 2>(M, N, N, Q, N, 60);
    for (int i = threadIdx.x; i < N; i += PB) lam[i] = M[(long)i * N + i];
  } else {
    if constexpr (lds_mode == 2)
      for (long t = threadIdx.x; t < NN; t += PB) Q[t] = Qg[t];
    if (warm == 2) {
      // one Newton-Schulz step Q <- Q (3 I - Q^t Q) / 2: the products of many warm updates leave Q
      // orthogonal only to rounding accumulated over the calls; this takes it back to rounding
      wg_sync();
      wg_mm64<true, false>(Q, Q, Tm, N);
      wg_sync();
      wg_for2<PB>(N, N, [&](int i, int c) {
        Tm[(long)i * N + c] = (i == c ? 1.5 : 0.0) - 0.5 * Tm[(long)i * N + c];
      });
      wg_sync();
      wg_mm64<false, false>(Q, Tm, W2, N);
      wg_sync();
      for (long t = threadIdx.x; t < NN; t += PB) Q[t] = W2[t];
    }
    // M = X - s Y ; W2 = M Q ; M = Q^t W2 (symmetrised)
    for (long t = threadIdx.x; t < NN; t += PB) M[t] = X[t] - s * Y[t];
    wg_sync();
    if (mm) wg_mm64<false, false>(M, Q, W2, N);
    else wg_mm<false, false>(M, Q, W2, N);
    wg_sync();
    if (mm) wg_mm64<true, false>(Q, W2, M, N);
    else wg_mm<true, false>(Q, W2, M, N);
    wg_sync();
    wg_for2<PB>(N, N, [&](int i, int c) {
      if (c <= i) return;
      const double v = 0.5 * (M[(long)i * N + c] + M[(long)c * N + i]);
      M[(long)i * N + c] = v;
      M[(long)c * N + i] = v;
    });
    wg_sync();
    // M = D + E with E off the diagonal, K_pq = E_pq / (d_q - d_p) (zero where a Jacobi sweep would
    // not rotate the pair), kmax = max |K_pq|.
    //  * kmax <= 2^-26: every rotation of a sweep would have |tan| <= 2^-26 (the sweep after which
    //    the eigensolver stops); first-order perturbation gives the eigenvectors to the same accuracy
    //    in one step: W2 = I + K + K^2 / 2, eigenvalues d_q + sum_p E_pq K_pq.
    //  * kmax <= 1e-4 (and a fourth N x N array in LDS): a Newton-type step M <- W^t M W, Q <- Q W
    //    with W = I + K + K^2 / 2 (W^t W = I + K^4 / 4: orthogonal to rounding) leaves off-diagonal
    //    entries of order kmax^2 relative to the gaps; repeat.
    //  * kmax > 1e-4 (with the fourth array): one Jacobi sweep, then test again.
    //  * without the fourth array, or after three steps: Jacobi sweeps to convergence.
    double fro = 0.0;
    wg_for2<PB>(N, N, [&](int i, int c) {
      const double a = M[(long)i * N + c];
      fro += a * a;
    });
    red[threadIdx.x] = fro;
    wg_sync();
    for (int h = PB / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      wg_sync();
    }
    const double floor_abs = 0x1p-53 * sqrt(red[0]);
    wg_sync();
    for (int step = 0;; ++step) {
      // K into W2 (diagonal zero) and kmax
      double kl = 0.0;
      wg_for2<PB>(N, N, [&](int p, int q) {
        double k = 0.0;
        if (p != q) {
          const double apq = M[(long)p * N + q], app = M[(long)p * N + p], aqq = M[(long)q * N + q];
          if (apq * apq > 1e-30 * fabs(app * aqq) && fabs(apq) > floor_abs && fabs(apq) > 1e-300) {
            const double g = aqq - app;
            if (fabs(apq) < 0.25 * fabs(g)) k = apq / g;
            kl = fmax(kl, fabs(apq) < 0.25 * fabs(g) ? fabs(k) : 1.0);
          }
        }
        W2[(long)p * N + q] = k;
      });
      red[threadIdx.x] = kl;
      wg_sync();
      for (int h = PB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        wg_sync();
      }
      const double kmax = red[0];
      wg_sync();
      if (kmax <= 0x1p-26) {
        for (int q = threadIdx.x; q < N; q += PB) {
          double l = M[(long)q * N + q];
          for (int p = 0; p < N; ++p) l += M[(long)p * N + q] * W2[(long)p * N + q];
          lam[q] = l;
        }
        wg_sync();
        // M <- K^2, then W2 <- I + K + K^2 / 2
        if (mm) wg_mm64<false, false>(W2, W2, M, N);
        else wg_mm<false, false>(W2, W2, M, N);
        wg_sync();
        wg_for2<PB>(N, N, [&](int i, int c) {
          W2[(long)i * N + c] += 0.5 * M[(long)i * N + c] + (i == c ? 1.0 : 0.0);
        });
        break;
      }
      if (!Tm || step == 3) {
        wg_jacobi<PB, lds_mode < 2>(M, N, N, W2, N, 60);
        for (int i = threadIdx.x; i < N; i += PB) lam[i] = M[(long)i * N + i];
        break;
      }
      if (kmax > 1e-4) {
        // one Jacobi sweep (roughly squares max |K|), Q <- Q W2, then test again
        wg_jacobi<PB, lds_mode < 2>(M, N, N, W2, N, 1);
        wg_mm64<false, false>(Q, W2, Tm, N);
        wg_sync();
        for (long t = threadIdx.x; t < NN; t += PB) Q[t] = Tm[t];
        wg_sync();
        continue;
      }
      // W2 <- W = I + K + K^2 / 2 ; M <- W^t (M W) (symmetrised) ; Q <- Q W
      wg_mm64<false, false>(W2, W2, Tm, N);
      wg_sync();
      wg_for2<PB>(N, N, [&](int i, int c) {
        W2[(long)i * N + c] += 0.5 * Tm[(long)i * N + c] + (i == c ? 1.0 : 0.0);
      });
      wg_sync();
      wg_mm64<false, false>(M, W2, Tm, N);
      wg_sync();
      wg_mm64<true, false>(W2, Tm, M, N);
      wg_sync();
      wg_for2<PB>(N, N, [&](int i, int c) {
        if (c <= i) return;
        const double v = 0.5 * (M[(long)i * N + c] + M[(long)c * N + i]);
        M[(long)i * N + c] = v;
        M[(long)c * N + i] = v;
      });
      wg_mm64<false, false>(Q, W2, Tm, N);
      wg_sync();
      for (long t = threadIdx.x; t < NN; t += PB) Q[t] = Tm[t];
      wg_sync();
    }
    wg_sync();
    // Q <- Q W2, through M as the temporary
    if (mm) wg_mm64<false, false>(Q, W2, M, N);
    else wg_mm<false, false>(Q, W2, M, N);
    wg_sync();
    for (long t = threadIdx.x; t < NN; t += PB) Q[t] = M[t];
  }
  wg_sync();
  if constexpr (lds_mode == 2)
    for (long t = threadIdx.x; t < NN; t += PB) Qg[t] = Q[t];
  if (threadIdx.x == 0) {
    int best = 0;
    for (int i = 1; i < N; ++i)
      if (fabs(lam[i]) < fabs(lam[best])) best = i;
    imin = best;
  }
  for (int r = threadIdx.x; r < N; r += PB) rj[r] = rhs[(long)r * nb + j];
  wg_sync();
  for (int i = threadIdx.x; i < N; i += PB) {
    double d = 0.0;
    for (int r = 0; r < N; ++r) d += Q[(long)r * N + i] * rj[r];
    const double l = lam[i];
    cf[i] = (i == imin || l == 0.0) ? 0.0 : d / l;
  }
  wg_sync();
  for (int r = threadIdx.x; r < N; r += PB) {
    double z = 0.0;
    for (int i = 0; i < N; ++i) z += Q[(long)r * N + i] * cf[i];
    out[(long)r * nb + j] = z;
  }
}

// The eigensolve of X - sigma_j Y keeps its working matrices in LDS when they fit the workgroup's
// share (gfx950: 160 KB per CU) beside the kernel's static arrays: all three N x N arrays for small
// N, else the matrix alone.
static int pinv_max_dyn_lds() {
  // initialised once per process (thread-safe static initialisation)
  static const int max_dyn = [] {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
    hipFuncAttributes fa0{}, fa1{}, fa2{};
    if (hipFuncGetAttributes(&fa0, (const void*)k_pinv_solve<0>) != hipSuccess ||
        hipFuncGetAttributes(&fa1, (const void*)k_pinv_solve<1>) != hipSuccess ||
        hipFuncGetAttributes(&fa2, (const void*)k_pinv_solve<2>) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    const int static_lds = (int)std::max(fa0.sharedSizeBytes, std::max(fa1.sharedSizeBytes, fa2.sharedSizeBytes));
    int m = v - static_lds;
    if (m > 0 &&
        (hipFuncSetAttribute((const void*)k_pinv_solve<0>, hipFuncAttributeMaxDynamicSharedMemorySize, m) !=
             hipSuccess ||
         hipFuncSetAttribute((const void*)k_pinv_solve<1>, hipFuncAttributeMaxDynamicSharedMemorySize, m) !=
             hipSuccess ||
         hipFuncSetAttribute((const void*)k_pinv_solve<2>, hipFuncAttributeMaxDynamicSharedMemorySize, m) !=
             hipSuccess)) {
      (void)hipGetLastError();
      m = 0;
    }
    return m < 0 ? 0 : m;
  }();
  return max_dyn;
}

void launch_pinv_solve(int N, int nb, const double* X, const double* Y, const double* sig, const double* rhs,
                       double* out, double* work, double* basis, int warm, int* status, hipStream_t s) {
  (void)status;
  const size_t one = (size_t)N * N * sizeof(double), vec = 3 * (size_t)N * sizeof(double);
  const size_t max_dyn = (size_t)pinv_max_dyn_lds();
  const int mode = 3 * one + vec <= max_dyn ? 2 : one + vec <= max_dyn ? 1 : 0;
  const int lds4 = (mode == 2 && N <= 64 && 4 * one + vec <= max_dyn) ? 1 : 0;
  const size_t lds = (mode == 2 ? (lds4 ? 4 : 3) * one : mode == 1 ? one : 0) + vec;
  if (mode == 2)
    hipLaunchKernelGGL(k_pinv_solve<2>, dim3(nb), dim3(PB), lds, s, N, nb, X, Y, sig, rhs, out, work, basis, warm,
                       lds4);
  else if (mode == 1)
    hipLaunchKernelGGL(k_pinv_solve<1>, dim3(nb), dim3(PB), lds, s, N, nb, X, Y, sig, rhs, out, work, basis, warm,
                       0);
  else
    hipLaunchKernelGGL(k_pinv_solve<0>, dim3(nb), dim3(PB), lds, s, N, nb, X, Y, sig, rhs, out, work, basis, warm,
                       0);
}

// Pencil variant, set-up once per additive phase: Y = L L^t, K = L^-1 X L^-t = W diag(mu) W^t,
// Z = L^-t W (Y-orthonormal eigenvectors of X z = mu Y z).  X and Y are overwritten.
// work: >= 2 N^2 doubles.
__global__ __launch_bounds__(DBLK) void k_pencil_setup(int N, double* X, double* Y, double* mu, double* Z,
                                                       double* work, int* status) {
  __shared__ int info;
  if (threadIdx.x == 0) info = 0;
  wg_sync();
  double* K = work;
  wg_chol(Y, N, N, &info);
  wg_trsm_lower(Y, N, N, X, N, N);         // X <- L^-1 X
  wg_transpose(X, N, N, N, K, N);          // K = X L^-t (X symmetric)
  wg_trsm_lower(Y, N, N, K, N, N);         // K = L^-1 X L^-t
  for (long t = threadIdx.x; t < (long)N * N; t += DBLK) {
    int i = (int)(t / N), j = (int)(t % N);
    if (j > i) {
      double s = 0.5 * (K[(long)i * N + j] + K[(long)j * N + i]);
      K[(long)i * N + j] = s; K[(long)j * N + i] = s;
    }
  }
  wg_jacobi(K, N, N, Z, N, 60);
  for (int i = threadIdx.x; i < N; i += DBLK) mu[i] = K[(long)i * N + i];
  wg_trsm_lower_t(Y, N, N, Z, N, N);
  if (threadIdx.x == 0 && info) *status = ST_E_NUMERIC;
}
void launch_pencil_setup(int N, double* X, double* Y, double* mu, double* Z, double* work, int* status,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_pencil_setup, dim3(1), dim3(DBLK), 0, s, N, X, Y, mu, Z, work, status);
}

__global__ __launch_bounds__(DBLK) void k_pencil_solve(int N, int nb, const double* mu, const double* Z,
                                                       const double* sig, const double* rhs, double* out) {
  const int j = blockIdx.x;
  __shared__ double cf[1024];
  __shared__ int imin;
  const double s = sig[j];
  if (threadIdx.x == 0) {
    int best = 0;
    for (int i = 1; i < N; ++i)
      if (fabs(mu[i] - s) < fabs(mu[best] - s)) best = i;
    imin = best;
  }
  wg_sync();
  for (int i = threadIdx.x; i < N; i += DBLK) {
    double d = 0.0;
    for (int r = 0; r < N; ++r) d += Z[(long)r * N + i] * rhs[(long)r * nb + j];
    double den = mu[i] - s;
    cf[i] = (i == imin || den == 0.0) ? 0.0 : d / den;
  }
  wg_sync();
  for (int r = threadIdx.x; r < N; r += DBLK) {
    double z = 0.0;
    for (int i = 0; i < N; ++i) z += Z[(long)r * N + i] * cf[i];
    out[(long)r * nb + j] = z;
  }
}
void launch_pencil_solve(int N, int nb, const double* mu, const double* Z, const double* sig, const double* rhs,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pencil_solve, dim3(nb), dim3(DBLK), 0, s, N, nb, mu, Z, sig, rhs, out);
}

// Plain symmetric eigen-decomposition (used by the step-level test entry point).
__global__ __launch_bounds__(DBLK) void k_dense_sym_eig(int n, double* A, double* V, double* lam) {
  wg_jacobi(A, n, n, V, n, 60);
  for (int i = threadIdx.x; i < n; i += DBLK) lam[i] = A[(long)i * n + i];
}
void launch_dense_sym_eig(int n, double* A, double* V, double* lam, int* status, hipStream_t s) {
  (void)status;
  hipLaunchKernelGGL(k_dense_sym_eig, dim3(1), dim3(DBLK), 0, s, n, A, V, lam);
}

}  // namespace slamg
