// Streaming kernels of the multilevel cycles: block SpMM, fused relaxation / residual row kernels,
// multicolour Kaczmarz sweeps, deterministic column reductions, the MFMA FP64 Gram product,
// block rotations, transfers, the merge-based numeric SpGEMM of the Galerkin products and the
// per-F-point least-squares interpolation fit.
//
// Blocks of vectors are row-major (row i holds its w <= 16 columns contiguously), so one row of an
// 8-column FP64 block is one 64-byte line.  A row of a sparse operator is handled by a group of
// LPR lanes of a 64-wide wavefront; lane l of the group owns columns [CPL*l, CPL*l + CPL).  The
// column loads of a gathered vector row are therefore contiguous across the group.
#include "common.h"
#include "solver.h"

#include <algorithm>
#include <type_traits>

namespace slamg {

static constexpr int BLK = 256;

static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
static inline int cpl_of(int w) { return w >= 2 ? 2 : 1; }
static inline int lshift_of(int w) {
  int lanes = (w + cpl_of(w) - 1) / cpl_of(w);
  int s = 0;
  while ((1 << s) < lanes) ++s;
  return s;
}

// Rows with many nonzeros (coarse Galerkin levels) are split over SPLIT lane groups of the same
// wavefront; each group takes every SPLIT-th nonzero and the partial sums meet by lane shuffles.
// Lane layout of a row's group: lane = split * LPRc + column lane (LPRc = 1 << lshift).
static inline int log2i(int v) { int s = 0; while ((1 << s) < v) ++s; return s; }
static inline int split_of(long nnz, long rows, int lshift, double avg_other = 0.0) {
  double avg = (nnz < 0 || rows <= 0) ? 0.0 : (double)nnz / (double)rows;
  if (avg_other > avg) avg = avg_other;
  // Short rows: one lane group.  Otherwise enough groups that each lane walks a few nonzeros (the
  // walk is a chain of dependent index / value loads, so its length sets the latency) -- unless the
  // rows alone already give the chip enough wavefronts (>= 4 per SIMD), where splitting only adds
  // shuffles.
  const bool many = (rows << lshift) >= (1L << 18);
  int sp = many ? (avg < 12.0 ? 1 : avg < 48.0 ? 4 : 16) : (avg < 3.0 ? 1 : avg < 12.0 ? 4 : 16);
  while (sp > 1 && ((1 << lshift) * sp) > 64) sp >>= 1;
  return sp;
}

template <int SPLIT, typename T>
__device__ __forceinline__ T split_sum(T v, int lprc) {
#pragma unroll
  for (int m = 1; m < SPLIT; m <<= 1) v += __shfl_xor(v, lprc * m);
  return v;
}

// Workgroups are dispatched to the 8 XCDs round-robin (XCD = id mod 8), and each XCD has its own L2.
// The logical workgroup index gives XCD x one contiguous range of the grid, so that neighbouring
// rows, and the rows they gather, meet in one L2.  A bijection of [0, gridDim.x).  Used by the
// Kaczmarz sweep, whose updates re-read what neighbouring rows just wrote (5% faster on a 7-point
// operator); the gather-only kernels measured 5% slower with it.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <typename T, int CPL>
__device__ __forceinline__ void ldrow(const T* __restrict__ p, int c0, int w, T (&v)[CPL]) {
  if constexpr (CPL == 2) {
    if (!(w & 1)) {
      typedef T T2 __attribute__((ext_vector_type(2)));
      T2 t = *reinterpret_cast<const T2*>(p + c0);
      v[0] = t.x; v[1] = t.y;
      return;
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) v[c] = (c0 + c < w) ? p[c0 + c] : T(0);
}

template <typename T, int CPL>
__device__ __forceinline__ void strow(T* __restrict__ p, int c0, int w, const T (&v)[CPL]) {
  if constexpr (CPL == 2) {
    if (!(w & 1)) {
      typedef T T2 __attribute__((ext_vector_type(2)));
      T2 t; t.x = v[0]; t.y = v[1];
      *reinterpret_cast<T2*>(p + c0) = t;
      return;
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
    if (c0 + c < w) p[c0 + c] = v[c];
}

// Operator value k.  With BF (FP32 V-cycles with BF16 operator values) the array holds BF16 bit
// patterns: the value is those 16 bits as the high half of an FP32 word.  BF is a template argument
// so that each kernel's loop carries one load form and no branch per load.
template <typename T, bool BF>
__device__ __forceinline__ T ldval(const T* __restrict__ p, long k) {
  if constexpr (BF) {
    static_assert(std::is_same<T, float>::value, "BF16 values feed FP32 arithmetic only");
    return __uint_as_float((unsigned)reinterpret_cast<const unsigned short*>(p)[k] << 16);
  } else {
    return p[k];
  }
}

// One lane's walk over the nonzeros k, k + SPLIT, k + 2 SPLIT, ... < ke of a CSR row, summing
// a_k z(j_k) (and b_k z(j_k) when TWO).  Each step takes four nonzeros (two when TWO, to bound the
// registers): their index and value loads are issued together, then their row gathers, so a lane
// with at most four nonzeros waits for one index -> row chain.  Slots past the row's end load
// nothing and add zero, which leaves the sums bitwise equal to the one-by-one walk.
template <typename T, int CPL, int SPLIT, bool TWO, bool BF = false>
__device__ __forceinline__ void walk_row(int k, int ke, const int* __restrict__ ci, const T* __restrict__ av,
                                         const T* __restrict__ bv, const T* __restrict__ z, int w, int c0,
                                         T (&s1)[CPL], T (&s2)[CPL]) {
  constexpr int U = TWO ? 2 : 4;
  for (; k < ke; k += U * SPLIT) {
    int j[U];
    T a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k + u * SPLIT;
      j[u] = -1;
      a[u] = T(0);
      b[u] = T(0);
      if (kk < ke) {
        j[u] = ci[kk];
        a[u] = ldval<T, BF>(av, kk);
        if constexpr (TWO) b[u] = ldval<T, BF>(bv, kk);
      }
    }
    T zr[U][CPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] >= 0) ldrow<T, CPL>(z + (long)j[u] * w, c0, w, zr[u]);
      else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) zr[u][c] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        s1[c] += a[u] * zr[u][c];
        if constexpr (TWO) s2[c] += b[u] * zr[u][c];
      }
  }
}

// The same walk with a run-time stride between a lane group's nonzeros (a whole workgroup on one
// long row: nonzeros k, k + stride, k + 2 stride, ...).
template <typename T, int CPL, bool TWO, bool BF = false>
__device__ __forceinline__ void walk_row_strided(int k, int ke, int stride, const int* __restrict__ ci,
                                                 const T* __restrict__ av, const T* __restrict__ bv,
                                                 const T* __restrict__ z, int w, int c0, T (&s1)[CPL],
                                                 T (&s2)[CPL]) {
  constexpr int U = TWO ? 2 : 4;
  for (; k < ke; k += U * stride) {
    int j[U];
    T a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k + u * stride;
      j[u] = -1;
      a[u] = T(0);
      b[u] = T(0);
      if (kk < ke) {
        j[u] = ci[kk];
        a[u] = ldval<T, BF>(av, kk);
        if constexpr (TWO) b[u] = ldval<T, BF>(bv, kk);
      }
    }
    T zr[U][CPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] >= 0) ldrow<T, CPL>(z + (long)j[u] * w, c0, w, zr[u]);
      else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) zr[u][c] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        s1[c] += a[u] * zr[u][c];
        if constexpr (TWO) s2[c] += b[u] * zr[u][c];
      }
  }
}

// ------------------------------------------------------------------------------------------------
// Block SpMM  y = A x (+ beta y)
// ------------------------------------------------------------------------------------------------
template <typename T>
struct SpmmPOD {
  int m, w;
  const int* rp; const int* ci; const T* v; const T* x; T* y; T beta;
};

// thread t of the product's own grid
template <typename T, int CPL, int SPLIT, bool BF>
__device__ __forceinline__ void spmm_body(const SpmmPOD<T>& a, int lshift, long t) {
  constexpr int LS = SPLIT == 1 ? 0 : SPLIT == 4 ? 2 : SPLIT == 8 ? 3 : 4;
  const int m = a.m, w = a.w;
  const int* __restrict__ rp = a.rp;
  const int* __restrict__ ci = a.ci;
  const T* __restrict__ v = a.v;
  const T* __restrict__ x = a.x;
  T* __restrict__ y = a.y;
  const T beta = a.beta;
  const int gl = lshift + LS;
  int row = (int)(t >> gl);
  const int lane = (int)(t & ((1 << gl) - 1));
  const int sidx = lane >> lshift;
  int c0 = (lane & ((1 << lshift) - 1)) * CPL;
  if (row >= m || c0 >= w) return;
  T* yr = y + (long)row * w;
  T old[CPL];
  if (beta != T(0) && sidx == 0) ldrow<T, CPL>(yr, c0, w, old);
  T acc[CPL], unused[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = T(0);
  walk_row<T, CPL, SPLIT, false, BF>(rp[row] + sidx, rp[row + 1], ci, v, nullptr, x, w, c0, acc, unused);
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = split_sum<SPLIT>(acc[c], 1 << lshift);
  if (sidx != 0) return;
  if (beta != T(0)) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] += beta * old[c];
  }
  strow<T, CPL>(yr, c0, w, acc);
}

template <typename T, int CPL, int SPLIT, bool BF>
__global__ __launch_bounds__(BLK) void k_spmm(SpmmPOD<T> a, int lshift) {
  spmm_body<T, CPL, SPLIT, BF>(a, lshift, (long)blockIdx.x * BLK + threadIdx.x);
}

// Two independent products in one launch (the u- and v-side transfers of a level): workgroups
// [0, nb0) run the first, the others the second, so the two latency chains overlap.
template <typename T, int CPL, int SPLIT, bool BF>
__global__ __launch_bounds__(BLK) void k_spmm2(SpmmPOD<T> a, SpmmPOD<T> b, int lshift, int nb0) {
  const int bk = (int)blockIdx.x;
  if (bk < nb0) spmm_body<T, CPL, SPLIT, BF>(a, lshift, (long)bk * BLK + threadIdx.x);
  else spmm_body<T, CPL, SPLIT, BF>(b, lshift, (long)(bk - nb0) * BLK + threadIdx.x);
}

#define SLAMG_DISPATCH_SPLIT(KER, T, CPL, SP, GRID, ...)                                        \
  do {                                                                                      \
    if (SP == 1) hipLaunchKernelGGL((KER<T, CPL, 1>), dim3(GRID), dim3(BLK), 0, __VA_ARGS__);  \
    else if (SP == 4) hipLaunchKernelGGL((KER<T, CPL, 4>), dim3(GRID), dim3(BLK), 0, __VA_ARGS__); \
    else if (SP == 8) hipLaunchKernelGGL((KER<T, CPL, 8>), dim3(GRID), dim3(BLK), 0, __VA_ARGS__); \
    else hipLaunchKernelGGL((KER<T, CPL, 16>), dim3(GRID), dim3(BLK), 0, __VA_ARGS__);        \
  } while (0)

// The same over kernels that read operator values, with their value form as the last template
// argument: BF16 bit patterns (VBF != 0, FP32 kernels only) or T.
#define SLAMG_DISPATCH_SPLIT_BF(KER, T, CPL, BF, SP, GRID, NT, ...)                                \
  do {                                                                                           \
    if (SP == 1) hipLaunchKernelGGL((KER<T, CPL, 1, BF>), dim3(GRID), dim3(NT), 0, __VA_ARGS__);     \
    else if (SP == 4) hipLaunchKernelGGL((KER<T, CPL, 4, BF>), dim3(GRID), dim3(NT), 0, __VA_ARGS__); \
    else if (SP == 8) hipLaunchKernelGGL((KER<T, CPL, 8, BF>), dim3(GRID), dim3(NT), 0, __VA_ARGS__); \
    else hipLaunchKernelGGL((KER<T, CPL, 16, BF>), dim3(GRID), dim3(NT), 0, __VA_ARGS__);           \
  } while (0)
#define SLAMG_DISPATCH_VALS(KER, T, VBF, SP, W, GRID, NT, ...)                                     \
  do {                                                                                           \
    if constexpr (std::is_same<T, float>::value) {                                               \
      if (VBF) {                                                                                 \
        if (cpl_of(W) == 2) SLAMG_DISPATCH_SPLIT_BF(KER, T, 2, true, SP, GRID, NT, __VA_ARGS__); \
        else SLAMG_DISPATCH_SPLIT_BF(KER, T, 1, true, SP, GRID, NT, __VA_ARGS__);               \
        break;                                                                                   \
      }                                                                                          \
    }                                                                                            \
    if (cpl_of(W) == 2) SLAMG_DISPATCH_SPLIT_BF(KER, T, 2, false, SP, GRID, NT, __VA_ARGS__);   \
    else SLAMG_DISPATCH_SPLIT_BF(KER, T, 1, false, SP, GRID, NT, __VA_ARGS__);                  \
  } while (0)

template <typename T>
void launch_spmm(int m, int w, const int* rp, const int* ci, const T* v, const T* x, T* y, double beta,
                 hipStream_t s, int nnz, int vbf) {
  if (m <= 0) return;
  int sh = lshift_of(w);
  int sp = split_of(nnz, m, sh);
  int grid = ceil_div((long)m << (sh + log2i(sp)), BLK);
  SpmmPOD<T> p{m, w, rp, ci, v, x, y, (T)beta};
  SLAMG_DISPATCH_VALS(k_spmm, T, vbf, sp, w, grid, BLK, s, p, sh);
}

template <typename T>
void launch_spmm2(const SpmmArgs<T>& a, const SpmmArgs<T>& b, int w, hipStream_t s) {
  if (a.m <= 0) { launch_spmm<T>(b.m, w, b.rp, b.ci, b.v, b.x, b.y, b.beta, s, b.nnz, b.vbf); return; }
  if (b.m <= 0) { launch_spmm<T>(a.m, w, a.rp, a.ci, a.v, a.x, a.y, a.beta, s, a.nnz, a.vbf); return; }
  const int sh = lshift_of(w);
  const int sp = std::max(split_of(a.nnz, a.m, sh), split_of(b.nnz, b.m, sh));
  const int g0 = ceil_div((long)a.m << (sh + log2i(sp)), BLK), g1 = ceil_div((long)b.m << (sh + log2i(sp)), BLK);
  SpmmPOD<T> pa{a.m, w, a.rp, a.ci, a.v, a.x, a.y, (T)a.beta}, pb{b.m, w, b.rp, b.ci, b.v, b.x, b.y, (T)b.beta};
  SLAMG_DISPATCH_VALS(k_spmm2, T, a.vbf, sp, w, g0 + g1, BLK, s, pa, pb, sh, g0);
}

// ------------------------------------------------------------------------------------------------
// Generic fused row kernel:
//   out_ic = x_ic + D_i * ( ca_c (K z)_ic + cb_c (M y)_ic + ce_c kap_ic )
// covering the weighted-Jacobi test and boot relaxations (power-method and block Gauss-Seidel
// steps), the additive residuals and the Jacobi pre-smoothing of the minimal LS fit.
// ------------------------------------------------------------------------------------------------
template <typename T>
struct RowOpPOD {
  int nrows, w;
  const int* Krp; const int* Kci; const T* Kv; const T* z;
  int mmode;
  const int* Mrp; const int* Mci; const T* Mv; const T* y;
  const T* x; const T* D; const T* kap; const double* sig;
  int cmode; double omega;
  T* out;
  // rows with very many nonzeros (lflag[row] = 1) are skipped by the row-per-lane-group blocks
  // [0, gmain) and handled one per workgroup by blocks gmain + i (row lrows[i])
  const unsigned char* lflag; const int* lrows; int gmain;
};

template <typename T>
__device__ __forceinline__ void coefs(int cmode, double om, double s, T& ca, T& cb, T& ce) {
  switch (cmode) {
    case C_JAC_TEST: ca = (T)om; cb = (T)(-om); ce = T(0); break;
    case C_JAC_BOOT: ca = (T)(om / s); cb = (T)(-om); ce = (T)(-om / s); break;
    case C_RESID: ca = T(-1); cb = (T)s; ce = T(1); break;
    case C_SMOOTH: ca = (T)(-om); cb = T(0); ce = T(0); break;
    default: ca = T(1); cb = T(0); ce = T(0); break;
  }
}

// thread t of the row operation's own grid
template <typename T, int CPL, int SPLIT, bool BF>
__device__ __forceinline__ void rowop_body(const RowOpPOD<T>& a, int lshift, long t) {
  constexpr int LS = SPLIT == 1 ? 0 : SPLIT == 4 ? 2 : SPLIT == 8 ? 3 : 4;
  const int gl = lshift + LS;
  int row = (int)(t >> gl);
  const int lane = (int)(t & ((1 << gl) - 1));
  const int sidx = lane >> lshift;
  int c0 = (lane & ((1 << lshift) - 1)) * CPL;
  const int w = a.w;
  if (row >= a.nrows || c0 >= w) return;
  if (a.lflag && a.lflag[row]) return;
  // the row's own operands first: their loads overlap the walks.  With M = I the row of y goes
  // into the M-sum of the first lane group (the other groups add zeros to it, exactly).
  double sg[CPL];
  T kp[CPL], xv[CPL], kz[CPL], my[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    sg[c] = (a.sig && c0 + c < w) ? a.sig[c0 + c] : 1.0;
    kp[c] = T(0); xv[c] = T(0); kz[c] = T(0); my[c] = T(0);
  }
  T d = T(1);
  if (sidx == 0) {
    if (a.kap) ldrow<T, CPL>(a.kap + (long)row * w, c0, w, kp);
    if (a.x) ldrow<T, CPL>(a.x + (long)row * w, c0, w, xv);
    if (a.mmode == M_IDENT) ldrow<T, CPL>(a.y + (long)row * w, c0, w, my);
    if (a.D) d = a.D[row];
  }
  if (a.Kv) {
    if (a.mmode == M_SHARED)
      walk_row<T, CPL, SPLIT, true, BF>(a.Krp[row] + sidx, a.Krp[row + 1], a.Kci, a.Kv, a.Mv, a.z, w, c0, kz, my);
    else
      walk_row<T, CPL, SPLIT, false, BF>(a.Krp[row] + sidx, a.Krp[row + 1], a.Kci, a.Kv, nullptr, a.z, w, c0, kz, my);
  }
  if (a.mmode == M_CSR) {
    T unused[CPL];
    walk_row<T, CPL, SPLIT, false, BF>(a.Mrp[row] + sidx, a.Mrp[row + 1], a.Mci, a.Mv, nullptr, a.y, w, c0, my, unused);
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    kz[c] = split_sum<SPLIT>(kz[c], 1 << lshift);
    my[c] = split_sum<SPLIT>(my[c], 1 << lshift);
  }
  if (sidx != 0) return;
  T r[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    T ca, cb, ce;
    coefs<T>(a.cmode, a.omega, sg[c], ca, cb, ce);
    r[c] = d * (ca * kz[c] + cb * my[c] + ce * kp[c]);
  }
  if (a.x) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) r[c] += xv[c];
  }
  strow<T, CPL>(a.out + (long)row * w, c0, w, r);
}

// One long row in one workgroup: the 1 << lshift column lanes repeat over BLK >> lshift groups,
// each walking every (BLK >> lshift)-th nonzero; the groups' sums meet by lane shuffles within a
// wavefront, then in LDS across the wavefronts (fixed order), and the row's first lanes finish it
// as rowop_body does.
static constexpr int LONG_MAX_LANES = 8;   // w <= 16 with two columns per lane
template <typename T, int CPL>
using LongRed = T[BLK / 64][LONG_MAX_LANES][2][CPL];

template <typename T, int CPL, bool BF>
__device__ __forceinline__ void rowop_long(const RowOpPOD<T>& a, int lshift, int row, LongRed<T, CPL>& red) {
  const int L = 1 << lshift, t = threadIdx.x;
  const int lane = t & (L - 1), grp = t >> lshift, G = BLK >> lshift;
  const int w = a.w, c0 = lane * CPL;
  T kz[CPL], my[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) { kz[c] = T(0); my[c] = T(0); }
  if (c0 < w) {
    if (a.Kv) {
      const int kb = a.Krp[row], ke = a.Krp[row + 1];
      if (a.mmode == M_SHARED)
        walk_row_strided<T, CPL, true, BF>(kb + grp, ke, G, a.Kci, a.Kv, a.Mv, a.z, w, c0, kz, my);
      else
        walk_row_strided<T, CPL, false, BF>(kb + grp, ke, G, a.Kci, a.Kv, nullptr, a.z, w, c0, kz, my);
    }
    if (a.mmode == M_CSR) {
      T unused[CPL];
      walk_row_strided<T, CPL, false, BF>(a.Mrp[row] + grp, a.Mrp[row + 1], G, a.Mci, a.Mv, nullptr, a.y, w, c0,
                                          my, unused);
    }
  }
  for (int m = L; m < 64; m <<= 1) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      kz[c] += __shfl_xor(kz[c], m);
      my[c] += __shfl_xor(my[c], m);
    }
  }
  const int wave = t >> 6;
  if ((t & 63) < L) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) { red[wave][lane][0][c] = kz[c]; red[wave][lane][1][c] = my[c]; }
  }
  __syncthreads();
  if (t >= L || c0 >= w) return;
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    kz[c] = red[0][lane][0][c];
    my[c] = red[0][lane][1][c];
  }
  for (int v = 1; v < BLK / 64; ++v) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) { kz[c] += red[v][lane][0][c]; my[c] += red[v][lane][1][c]; }
  }
  T kp[CPL], xv[CPL], yv[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) { kp[c] = T(0); xv[c] = T(0); yv[c] = T(0); }
  if (a.kap) ldrow<T, CPL>(a.kap + (long)row * w, c0, w, kp);
  if (a.x) ldrow<T, CPL>(a.x + (long)row * w, c0, w, xv);
  if (a.mmode == M_IDENT) {
    ldrow<T, CPL>(a.y + (long)row * w, c0, w, yv);
#pragma unroll
    for (int c = 0; c < CPL; ++c) my[c] += yv[c];
  }
  const T d = a.D ? a.D[row] : T(1);
  T r[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const double sg = (a.sig && c0 + c < w) ? a.sig[c0 + c] : 1.0;
    T ca, cb, ce;
    coefs<T>(a.cmode, a.omega, sg, ca, cb, ce);
    r[c] = d * (ca * kz[c] + cb * my[c] + ce * kp[c]);
    if (a.x) r[c] += xv[c];
  }
  strow<T, CPL>(a.out + (long)row * w, c0, w, r);
}

// block bk of one row operation's own grid
template <typename T, int CPL, int SPLIT, bool BF>
__device__ __forceinline__ void rowop_block(const RowOpPOD<T>& a, int lshift, int bk, LongRed<T, CPL>& red) {
  if (a.lrows && bk >= a.gmain) rowop_long<T, CPL, BF>(a, lshift, a.lrows[bk - a.gmain], red);
  else rowop_body<T, CPL, SPLIT, BF>(a, lshift, (long)bk * BLK + threadIdx.x);
}

template <typename T, int CPL, int SPLIT, bool BF>
__global__ __launch_bounds__(BLK) void k_rowop(RowOpPOD<T> a, int lshift) {
  __shared__ LongRed<T, CPL> red;
  rowop_block<T, CPL, SPLIT, BF>(a, lshift, (int)blockIdx.x, red);
}

// Two independent row operations in one launch (the u- and v-side residuals of a level):
// workgroups [0, nb0) run the first, the others the second.
template <typename T, int CPL, int SPLIT, bool BF>
__global__ __launch_bounds__(BLK) void k_rowop2(RowOpPOD<T> a, RowOpPOD<T> b, int lshift, int nb0) {
  __shared__ LongRed<T, CPL> red;
  const int bk = (int)blockIdx.x;
  if (bk < nb0) rowop_block<T, CPL, SPLIT, BF>(a, lshift, bk, red);
  else rowop_block<T, CPL, SPLIT, BF>(b, lshift, bk - nb0, red);
}

// POD of a row operation whose row-per-lane-group part takes gmain blocks; its long rows (if any,
// and if a row's lanes fit the long-row reduction) follow as one block each.  Returns the blocks.
template <typename T>
static int rowop_pod(const RowOpArgs<T>& a, int gmain, RowOpPOD<T>& p) {
  const bool lng = a.nlong > 0 && a.lflag && a.lrows && (1 << lshift_of(a.w)) <= LONG_MAX_LANES;
  p = RowOpPOD<T>{a.nrows, a.w, a.Krp, a.Kci, a.Kv, a.z, a.mmode, a.Mrp, a.Mci, a.Mv, a.y,
                  a.x, a.D, a.kap, a.sig, a.cmode, a.omega, a.out,
                  lng ? a.lflag : nullptr, lng ? a.lrows : nullptr, gmain};
  return gmain + (lng ? a.nlong : 0);
}

template <typename T>
void launch_rowop(const RowOpArgs<T>& a, hipStream_t s) {
  if (a.nrows <= 0) return;
  int sh = lshift_of(a.w);
  int sp = split_of(a.Kv ? a.nnzK : -1, a.nrows, sh, a.mmode == M_CSR ? a.avgM : 0.0);
  RowOpPOD<T> p;
  const int grid = rowop_pod(a, ceil_div((long)a.nrows << (sh + log2i(sp)), BLK), p);
  SLAMG_DISPATCH_VALS(k_rowop, T, a.vbf, sp, a.w, grid, BLK, s, p, sh);
}

template <typename T>
void launch_rowop2(const RowOpArgs<T>& a, const RowOpArgs<T>& b, hipStream_t s) {
  if (a.nrows <= 0) { launch_rowop(b, s); return; }
  if (b.nrows <= 0) { launch_rowop(a, s); return; }
  const int sh = lshift_of(a.w);
  const int sp = std::max(split_of(a.Kv ? a.nnzK : -1, a.nrows, sh, a.mmode == M_CSR ? a.avgM : 0.0),
                          split_of(b.Kv ? b.nnzK : -1, b.nrows, sh, b.mmode == M_CSR ? b.avgM : 0.0));
  RowOpPOD<T> pa, pb;
  const int g0 = rowop_pod(a, ceil_div((long)a.nrows << (sh + log2i(sp)), BLK), pa);
  const int g1 = rowop_pod(b, ceil_div((long)b.nrows << (sh + log2i(sp)), BLK), pb);
  SLAMG_DISPATCH_VALS(k_rowop2, T, a.vbf, sp, a.w, g0 + g1, BLK, s, pa, pb, sh, g0);
}

// ------------------------------------------------------------------------------------------------
// Kaczmarz sweep over the rows of one colour.  Rows of a colour share no column, so their updates
// touch disjoint entries of x and the result equals the row-by-row sweep in any order.
//   res_c = rhs_rc - a_r(c) . x_c ;  x_c += res_c / ||a_r(c)||^2 * a_r(c)
// with a_r(c) = A_r - lam_c B_r (shared pattern; bv == nullptr and lam != nullptr means B = I).
// ------------------------------------------------------------------------------------------------
template <typename T>
struct KaczPOD {
  int nrows; const int* rows; int w;
  const int* rp; const int* ci; const T* av; const T* bv; const double* lam;
  const T* rn_aa; const T* rn_ab; const T* rn_bb;
  int rmode; const int* Mrp; const int* Mci; const T* Mv; const T* y; const double* rsig; const T* kap;
  T* x;
};

template <typename T, int CPL, int SPLIT, bool BF>
__device__ __forceinline__ void kacz_row(const KaczPOD<T>& a, int r, int c0, int sidx, int lprc) {
  const int w = a.w;
  T lam[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) lam[c] = (a.lam && c0 + c < w) ? (T)a.lam[c0 + c] : T(0);
  const bool shifted = a.lam != nullptr;
  // operands that do not depend on the walks, loaded first so that their latency overlaps them
  T yid[CPL], kp[CPL], rs[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    yid[c] = T(0);
    kp[c] = T(0);
    rs[c] = (a.rmode != M_NONE && c0 + c < w) ? (T)a.rsig[c0 + c] : T(0);
  }
  if (a.rmode == M_IDENT) ldrow<T, CPL>(a.y + (long)r * w, c0, w, yid);
  if (a.kap) ldrow<T, CPL>(a.kap + (long)r * w, c0, w, kp);
  const T aa = a.rn_aa[r];
  const T ab = shifted ? a.rn_ab[r] : T(0), bb = shifted ? a.rn_bb[r] : T(0);
  const int kb = a.rp[r], ke = a.rp[r + 1];
  // right-hand side
  T rhs[CPL];
  if (a.rmode == M_CSR) {
    T my[CPL], unused[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) my[c] = T(0);
    walk_row<T, CPL, SPLIT, false, BF>(a.Mrp[r] + sidx, a.Mrp[r + 1], a.Mci, a.Mv, nullptr, a.y, w, c0, my, unused);
#pragma unroll
    for (int c = 0; c < CPL; ++c) rhs[c] = rs[c] * split_sum<SPLIT>(my[c], lprc) + kp[c];
  } else {
#pragma unroll
    for (int c = 0; c < CPL; ++c) rhs[c] = rs[c] * yid[c] + kp[c];
  }
  // residual of the row: eight nonzeros per step; a lane whose nonzeros fit one step (a 7-point
  // row on one lane, rows of up to 32 nonzeros on four) keeps their x rows in registers for the
  // update instead of gathering them again
  constexpr int U = 8;
  int j[U];
  T av[U], bv[U], xr[U][CPL];
  T dot[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) dot[c] = T(0);
#pragma unroll
  for (int u = 0; u < U; ++u) j[u] = -1;
  const bool one = kb + sidx + U * SPLIT >= ke;
  for (int k = kb + sidx; k < ke; k += U * SPLIT) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k + u * SPLIT;
      j[u] = -1;
      av[u] = T(0);
      bv[u] = T(0);
      if (kk < ke) {
        j[u] = a.ci[kk];
        av[u] = ldval<T, BF>(a.av, kk);
        if (shifted) bv[u] = a.bv ? ldval<T, BF>(a.bv, kk) : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (shifted && !a.bv && j[u] == r) bv[u] = T(1);
      if (j[u] >= 0) ldrow<T, CPL>(a.x + (long)j[u] * w, c0, w, xr[u]);
      else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) xr[u][c] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CPL; ++c) dot[c] += (shifted ? av[u] - lam[c] * bv[u] : av[u]) * xr[u][c];
  }
  T coef[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    T res = rhs[c] - split_sum<SPLIT>(dot[c], lprc);
    T nr = shifted ? aa - T(2) * lam[c] * ab + lam[c] * lam[c] * bb : aa;
    coef[c] = nr > T(0) ? res / nr : T(0);
  }
  // update x on the row's pattern (the colour's rows share no column, so the rows held in
  // registers are still current)
  if (one) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] < 0) continue;
#pragma unroll
      for (int c = 0; c < CPL; ++c) xr[u][c] += coef[c] * (shifted ? av[u] - lam[c] * bv[u] : av[u]);
      strow<T, CPL>(a.x + (long)j[u] * w, c0, w, xr[u]);
    }
    return;
  }
  #pragma unroll 4
  for (int k = kb + sidx; k < ke; k += SPLIT) {
    int jj = a.ci[k];
    T* xp = a.x + (long)jj * w;
    T xv[CPL];
    ldrow<T, CPL>(xp, c0, w, xv);
    T avk = ldval<T, BF>(a.av, k);
    if (shifted) {
      T bvk = a.bv ? ldval<T, BF>(a.bv, k) : (jj == r ? T(1) : T(0));
#pragma unroll
      for (int c = 0; c < CPL; ++c) xv[c] += coef[c] * (avk - lam[c] * bvk);
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) xv[c] += coef[c] * avk;
    }
    strow<T, CPL>(xp, c0, w, xv);
  }
}

template <typename T, int CPL, int SPLIT, bool BF>
__global__ __launch_bounds__(BLK) void k_kacz(KaczPOD<T> a, int lshift) {
  constexpr int LS = SPLIT == 1 ? 0 : SPLIT == 4 ? 2 : SPLIT == 8 ? 3 : 4;
  const int gl = lshift + LS;
  long t = (long)xcd_block() * BLK + threadIdx.x;
  int idx = (int)(t >> gl);
  const int lane = (int)(t & ((1 << gl) - 1));
  const int sidx = lane >> lshift;
  int c0 = (lane & ((1 << lshift) - 1)) * CPL;
  if (idx >= a.nrows || c0 >= a.w) return;
  kacz_row<T, CPL, SPLIT, BF>(a, a.rows[idx], c0, sidx, 1 << lshift);
}

// Whole sweeps in one workgroup (small levels): for each of `nsweeps` sweeps, each half-sweep
// (SVD: rows of A updating v, then rows of A^t updating u), each colour in order; a barrier
// separates colours, so the result equals the colour-by-colour launches exactly.
template <typename T>
struct KaczWgPOD {
  KaczPOD<T> h[2];
  const int* cptr[2];     // device colour pointers of each half-sweep
  int ncol[2];
  int nhalf, nsweeps;
};

static constexpr int WGB = 1024;

template <typename T, int CPL, int SPLIT, bool BF>
__global__ __launch_bounds__(WGB) void k_kacz_wg(KaczWgPOD<T> a, int lshift) {
  constexpr int LS = SPLIT == 1 ? 0 : SPLIT == 4 ? 2 : SPLIT == 8 ? 3 : 4;
  const int gl = lshift + LS;
  const int per = WGB >> gl;
  const int my = threadIdx.x >> gl;
  const int lane = threadIdx.x & ((1 << gl) - 1);
  const int sidx = lane >> lshift;
  const int c0 = (lane & ((1 << lshift) - 1)) * CPL;
  for (int s = 0; s < a.nsweeps; ++s) {
    for (int h = 0; h < 2; ++h) {
      if (h >= a.nhalf) break;
      const KaczPOD<T> k = h == 0 ? a.h[0] : a.h[1];
      const int* cp = h == 0 ? a.cptr[0] : a.cptr[1];
      const int nc = h == 0 ? a.ncol[0] : a.ncol[1];
      for (int c = 0; c < nc; ++c) {
        const int rb = cp[c], re = cp[c + 1];
        if (c0 < k.w)
          for (int idx = rb + my; idx < re; idx += per) kacz_row<T, CPL, SPLIT, BF>(k, k.rows[idx], c0, sidx, 1 << lshift);
        __syncthreads();
      }
    }
  }
}

template <typename T>
void launch_kacz_wg(const KaczArgs<T>* halves, const int* const* cptr, const int* ncol, int nhalf, int nsweeps,
                    hipStream_t s) {
  KaczWgPOD<T> p{};
  long nnz = 0, rows = 0;
  double avgM = 0.0;
  for (int h = 0; h < nhalf; ++h) {
    const KaczArgs<T>& a = halves[h];
    p.h[h] = KaczPOD<T>{0, a.rows, a.w, a.rp, a.ci, a.av, a.bv, a.lam, a.rn_aa, a.rn_ab, a.rn_bb,
                        a.rmode, a.Mrp, a.Mci, a.Mv, a.y, a.rsig, a.kap, a.x};
    p.cptr[h] = cptr[h];
    p.ncol[h] = ncol[h];
    if (a.nnz_rows > 0 && (double)a.nnz_total / a.nnz_rows > (rows ? (double)nnz / rows : 0.0)) {
      nnz = a.nnz_total; rows = a.nnz_rows;
    }
    if (a.rmode == M_CSR && a.avgM > avgM) avgM = a.avgM;
  }
  p.nhalf = nhalf;
  p.nsweeps = nsweeps;
  const int w = halves[0].w;
  int sh = lshift_of(w);
  int sp = split_of(rows ? nnz : -1, rows, sh, avgM);
  SLAMG_DISPATCH_VALS(k_kacz_wg, T, halves[0].vbf, sp, w, 1, WGB, s, p, sh);
}

// Whole sweeps with one workgroup per column j of the block.  The Kaczmarz update of column j
// reads only column j of x and of y, and sigma_j / lambda_j (§5.3), so the columns are independent
// and need no synchronisation across workgroups; a barrier separates the colours inside the
// workgroup.  The workgroup keeps its column of every updated vector in LDS (SVD: v and u, each
// also the other half-sweep's y), so a colour's gathers and updates never leave the CU; the
// operator rows stream from L2.  The arithmetic per row is kacz_row's: the same lane split, the
// same per-lane order of the nonzeros and the same butterfly reduction.
template <typename T>
struct KaczLdsPOD {
  KaczPOD<T> h[2];
  const int* cptr[2];
  int ncol[2];
  int nx[2];              // length of each half-sweep's updated vector
  int nhalf, nsweeps;
};

static constexpr int KLB = 1024;

template <typename T, int SPLIT, bool BF>
__device__ __forceinline__ T kacz_coef(const KaczPOD<T>& a, int k, int r, T lam, bool shifted) {
  T v = ldval<T, BF>(a.av, k);
  if (shifted) v = v - lam * (a.bv ? ldval<T, BF>(a.bv, k) : (a.ci[k] == r ? T(1) : T(0)));
  return v;
}

template <typename T, int SPLIT, bool BF>
__device__ __forceinline__ void kacz_row_lds(const KaczPOD<T>& a, int r, int j, int sidx, T lam, T rs,
                                             bool shifted, T* __restrict__ xs, const T* __restrict__ ys) {
  const T kp = a.kap ? a.kap[(long)r * a.w + j] : T(0);
  T rhs;
  if (a.rmode == M_CSR) {
    T my = T(0);
    for (int k = a.Mrp[r] + sidx; k < a.Mrp[r + 1]; k += SPLIT) my += ldval<T, BF>(a.Mv, k) * ys[a.Mci[k]];
    rhs = rs * split_sum<SPLIT>(my, 1) + kp;
  } else if (a.rmode == M_IDENT) {
    rhs = rs * ys[r] + kp;
  } else {
    rhs = kp;
  }
  const int kb = a.rp[r], ke = a.rp[r + 1];
  // a lane's first eight nonzeros stay in registers for the update
  constexpr int U = 8;
  int jc[U];
  T cv[U];
  T dot = T(0);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = kb + sidx + u * SPLIT;
    jc[u] = -1;
    cv[u] = T(0);
    if (k < ke) {
      jc[u] = a.ci[k];
      cv[u] = kacz_coef<T, SPLIT, BF>(a, k, r, lam, shifted);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (jc[u] >= 0) dot += cv[u] * xs[jc[u]];
  for (int k = kb + sidx + U * SPLIT; k < ke; k += SPLIT) dot += kacz_coef<T, SPLIT, BF>(a, k, r, lam, shifted) * xs[a.ci[k]];
  dot = split_sum<SPLIT>(dot, 1);
  T nr = a.rn_aa[r];
  if (shifted) nr = nr - T(2) * lam * a.rn_ab[r] + lam * lam * a.rn_bb[r];
  const T coef = nr > T(0) ? (rhs - dot) / nr : T(0);
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (jc[u] >= 0) xs[jc[u]] += coef * cv[u];
  for (int k = kb + sidx + U * SPLIT; k < ke; k += SPLIT) xs[a.ci[k]] += coef * kacz_coef<T, SPLIT, BF>(a, k, r, lam, shifted);
}

template <typename T, int SPLIT, bool BF>
__global__ __launch_bounds__(KLB) void k_kacz_lds(KaczLdsPOD<T> a) {
  extern __shared__ __align__(16) unsigned char kl_smem[];
  T* xs0 = reinterpret_cast<T*>(kl_smem);
  T* xs1 = xs0 + a.nx[0];
  const int j = blockIdx.x;
  const int w = a.h[0].w;
  for (int h = 0; h < a.nhalf; ++h) {
    T* xs = h ? xs1 : xs0;
    const T* xg = a.h[h].x;
    for (int r = threadIdx.x; r < a.nx[h]; r += KLB) xs[r] = xg[(long)r * w + j];
  }
  __syncthreads();
  const int grp = threadIdx.x / SPLIT, sidx = threadIdx.x % SPLIT;
  constexpr int NG = KLB / SPLIT;
  for (int s = 0; s < a.nsweeps; ++s) {
    for (int h = 0; h < a.nhalf; ++h) {
      const KaczPOD<T> k = h == 0 ? a.h[0] : a.h[1];
      T* xs = h ? xs1 : xs0;
      const T* ys = h ? xs0 : xs1;
      const bool shifted = k.lam != nullptr;
      const T lam = shifted ? (T)k.lam[j] : T(0);
      const T rs = k.rmode != M_NONE ? (T)k.rsig[j] : T(0);
      const int* cp = h == 0 ? a.cptr[0] : a.cptr[1];
      const int nc = h == 0 ? a.ncol[0] : a.ncol[1];
      for (int c = 0; c < nc; ++c) {
        const int rb = cp[c], re = cp[c + 1];
        for (int idx = rb + grp; idx < re; idx += NG)
          kacz_row_lds<T, SPLIT, BF>(k, k.rows[idx], j, sidx, lam, rs, shifted, xs, ys);
        __syncthreads();
      }
    }
  }
  for (int h = 0; h < a.nhalf; ++h) {
    const T* xs = h ? xs1 : xs0;
    T* xg = a.h[h].x;
    for (int r = threadIdx.x; r < a.nx[h]; r += KLB) xg[(long)r * w + j] = xs[r];
  }
}

// Largest dynamic LDS one workgroup of k_kacz_lds may take (the device limit; the kernel has no
// static LDS), and the opt-in above the default limit, once per instantiation.
static int kacz_lds_max() {
  static const int v = [] {
    int dev = 0, x = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
      (void)hipGetLastError();
      x = 65536;
    }
    return x;
  }();
  return v;
}

template <typename T, int SPLIT, bool BF>
static bool kacz_lds_optin() {
  static const bool ok = [] {
    if (hipFuncSetAttribute((const void*)k_kacz_lds<T, SPLIT, BF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kacz_lds_max()) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  }();
  return ok;
}

// Every instantiation opts in on the first launch of any, which the multiplicative phase makes
// eagerly, so that no attribute call falls inside a captured iteration.  Every launch, whatever its
// LDS size, passes through this one-time initialisation first: solves on other host threads (the
// serving loop) then never launch a kernel while its attributes are being set.
template <typename T>
static bool kacz_lds_optin_all() {
  static const bool ok = [] {
    bool r = kacz_lds_optin<T, 4, false>() & kacz_lds_optin<T, 8, false>() & kacz_lds_optin<T, 16, false>() &
             kacz_lds_optin<T, 32, false>();
    if constexpr (std::is_same<T, float>::value)
      r = r & kacz_lds_optin<T, 4, true>() & kacz_lds_optin<T, 8, true>() & kacz_lds_optin<T, 16, true>() &
          kacz_lds_optin<T, 32, true>();
    return r;
  }();
  return ok;
}

template <typename T, int SPLIT, bool BF>
static bool kacz_lds_go(const KaczLdsPOD<T>& p, int w, size_t lds, hipStream_t s) {
  const bool optin = kacz_lds_optin_all<T>();
  if (lds > 65536 && !optin) return false;
  hipLaunchKernelGGL((k_kacz_lds<T, SPLIT, BF>), dim3(w), dim3(KLB), lds, s, p);
  return true;
}

template <typename T, bool BF>
static bool kacz_lds_split(const KaczLdsPOD<T>& p, int sp, int w, size_t lds, hipStream_t s) {
  if (sp == 4) return kacz_lds_go<T, 4, BF>(p, w, lds, s);
  if (sp == 8) return kacz_lds_go<T, 8, BF>(p, w, lds, s);
  if (sp == 16) return kacz_lds_go<T, 16, BF>(p, w, lds, s);
  return kacz_lds_go<T, 32, BF>(p, w, lds, s);
}

template <typename T>
bool launch_kacz_lds(const KaczArgs<T>* halves, const int* const* cptr, const int* ncol, const int* nx, int nhalf,
                     int nsweeps, hipStream_t s) {
  size_t lds = 0;
  for (int h = 0; h < nhalf; ++h) lds += (size_t)nx[h] * sizeof(T);
  if (lds == 0 || lds > (size_t)kacz_lds_max() || halves[0].w <= 0) return false;
  // a right-hand side operator reads the other half-sweep's vector, which must be the one in LDS
  for (int h = 0; h < nhalf; ++h) {
    if (halves[h].rmode == M_NONE) continue;
    if (nhalf != 2 || halves[h].y != halves[1 - h].x) return false;
  }
  KaczLdsPOD<T> p{};
  double avg = 0.0;
  for (int h = 0; h < nhalf; ++h) {
    const KaczArgs<T>& a = halves[h];
    p.h[h] = KaczPOD<T>{0, a.rows, a.w, a.rp, a.ci, a.av, a.bv, a.lam, a.rn_aa, a.rn_ab, a.rn_bb,
                        a.rmode, a.Mrp, a.Mci, a.Mv, a.y, a.rsig, a.kap, a.x};
    p.cptr[h] = cptr[h];
    p.ncol[h] = ncol[h];
    p.nx[h] = nx[h];
    if (a.nnz_rows > 0) avg = std::max(avg, (double)a.nnz_total / (double)a.nnz_rows);
    if (a.rmode == M_CSR) avg = std::max(avg, a.avgM);
  }
  p.nhalf = nhalf;
  p.nsweeps = nsweeps;
  // lanes per row: about four nonzeros per lane (a lane keeps up to eight in registers)
  const int sp = avg <= 16.0 ? 4 : avg <= 32.0 ? 8 : avg <= 64.0 ? 16 : 32;
  const int w = halves[0].w;
  if constexpr (std::is_same<T, float>::value) {
    if (halves[0].vbf) return kacz_lds_split<T, true>(p, sp, w, lds, s);
  }
  return kacz_lds_split<T, false>(p, sp, w, lds, s);
}

template <typename T>
void launch_kacz(const KaczArgs<T>& a, hipStream_t s) {
  if (a.nrows <= 0) return;
  KaczPOD<T> p{a.nrows, a.rows, a.w, a.rp, a.ci, a.av, a.bv, a.lam, a.rn_aa, a.rn_ab, a.rn_bb,
               a.rmode, a.Mrp, a.Mci, a.Mv, a.y, a.rsig, a.kap, a.x};
  int sh = lshift_of(a.w);
  int sp = split_of(a.nnz_rows > 0 ? a.nnz_total : -1, a.nnz_rows, sh, a.rmode == M_CSR ? a.avgM : 0.0);
  int grid = ceil_div((long)a.nrows << (sh + log2i(sp)), BLK);
  SLAMG_DISPATCH_VALS(k_kacz, T, a.vbf, sp, a.w, grid, BLK, s, p, sh);
}

// ------------------------------------------------------------------------------------------------
// Column reductions (fixed grid + fixed-order finalisation: bitwise reproducible)
// ------------------------------------------------------------------------------------------------
template <typename T>
struct DotPOD {
  int nrows, w;
  const T* a; const int* Krp; const int* Kci; const T* Kv; const T* z; const T* y; const double* sig;
  double* partial;
};

// Fixed-order finalisation of one or two reductions (bitwise reproducible): one workgroup per
// output entry q; thread t sums partials t, t + 256, ... of entry q in ascending order, then a fixed
// tree.  Workgroups [0, a.nq) finish the first reduction, the rest the second.  gw > 0: a Gram
// product's 16 x 16 tiles (entry (i, j) of the gw x gw result at i * 16 + j of each tile); gw == 0:
// column sums (entry q at q).
struct FinPOD {
  int nparts, nq, gw;
  long stride;
  const double* partial;
  double* out;
};

__global__ __launch_bounds__(BLK) void k_finalize(FinPOD a, FinPOD b) {
  __shared__ double red[BLK];
  const bool first = (int)blockIdx.x < a.nq;
  const FinPOD& f = first ? a : b;
  const int q = first ? (int)blockIdx.x : (int)blockIdx.x - a.nq;
  const long off = f.gw > 0 ? (long)(q / f.gw) * 16 + q % f.gw : (long)q;
  double s = 0.0;
  for (int b = threadIdx.x; b < f.nparts; b += BLK) s += f.partial[(long)b * f.stride + off];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = BLK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) f.out[q] = red[0];
}

static void launch_finalize(const FinPOD& a, const FinPOD* b, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(a.nq + (b ? b->nq : 0)), dim3(BLK), 0, s, a, b ? *b : a);
}

int dots_grid(int nrows, int w) {
  int sh = lshift_of(w);
  return std::max(1, std::min(DOTS_MAX_GRID, ceil_div((long)nrows << sh, BLK)));
}

template <typename T, int CPL, int SPLIT>
__device__ __forceinline__ void dots_body(const DotPOD<T>& a, int lshift, int blk, int nblk, double* red) {
  constexpr int LS = SPLIT == 1 ? 0 : SPLIT == 4 ? 2 : SPLIT == 8 ? 3 : 4;
  double* partial = a.partial;
  const int gl = lshift + LS;
  const int w = a.w;
  const int lane = threadIdx.x & ((1 << gl) - 1);
  const int sidx = lane >> lshift;
  int c0 = (lane & ((1 << lshift) - 1)) * CPL;
  double acc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
  // workgroup blk takes the contiguous rows [r0, r1), BLK >> gl rows per pass
  const int per = BLK >> gl;
  const long chunk = (((long)a.nrows + nblk - 1) / nblk + per - 1) / per * per;
  const int r0 = (int)std::min((long)a.nrows, (long)blk * chunk), r1 = (int)std::min((long)a.nrows, (long)r0 + chunk);
  if (c0 < w) {
    double sc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) sc[c] = (a.sig && c0 + c < w) ? a.sig[c0 + c] : 0.0;
    for (int row = r0 + (int)(threadIdx.x >> gl); row < r1; row += per) {
      T yv[CPL], av[CPL];
      if (sidx == 0) {
        if (a.y) ldrow<T, CPL>(a.y + (long)row * w, c0, w, yv);
        if (a.a) ldrow<T, CPL>(a.a + (long)row * w, c0, w, av);
      }
      T val[CPL];
      if (a.Kv) {
        T unused[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) val[c] = T(0);
        walk_row<T, CPL, SPLIT, false>(a.Krp[row] + sidx, a.Krp[row + 1], a.Kci, a.Kv, nullptr, a.z, w, c0, val,
                                       unused);
#pragma unroll
        for (int c = 0; c < CPL; ++c) val[c] = split_sum<SPLIT>(val[c], 1 << lshift);
      } else {
        ldrow<T, CPL>(a.z + (long)row * w, c0, w, val);
      }
      if (sidx != 0) continue;
      if (a.y) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) val[c] -= (T)sc[c] * yv[c];
      }
      if (a.a) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] += (double)av[c] * (double)val[c];
      } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] += (double)val[c] * (double)val[c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) red[threadIdx.x * CPL + c] = acc[c];
  __syncthreads();
  if ((int)threadIdx.x < w) {
    int col = threadIdx.x;
    int ln = col / CPL, sub = col % CPL;
    double s = 0.0;
    for (int tt = ln; tt < BLK; tt += (1 << lshift)) s += red[tt * CPL + sub];
    partial[(long)blk * w + col] = s;
  }
}

template <typename T, int CPL, int SPLIT>
__global__ __launch_bounds__(BLK) void k_dots(DotPOD<T> a, int lshift) {
  __shared__ double red[BLK * 2];
  dots_body<T, CPL, SPLIT>(a, lshift, (int)blockIdx.x, gridDim.x, red);
}

// two independent reductions (same w) in one launch: workgroups [0, nb0) take the first
template <typename T, int CPL, int SPLIT>
__global__ __launch_bounds__(BLK) void k_dots2(DotPOD<T> a, DotPOD<T> b, int lshift, int nb0) {
  __shared__ double red[BLK * 2];
  const int bk = (int)blockIdx.x;
  if (bk < nb0) dots_body<T, CPL, SPLIT>(a, lshift, bk, nb0, red);
  else dots_body<T, CPL, SPLIT>(b, lshift, bk - nb0, gridDim.x - nb0, red);
}

template <typename T>
void launch_dots(const DotArgs<T>& a, double* partial, double* out, hipStream_t s) {
  int grid = dots_grid(a.nrows, a.w);
  if (a.nrows <= 0) {
    launch_fill(out, a.w, 0.0, s);
    return;
  }
  DotPOD<T> p{a.nrows, a.w, a.a, a.Krp, a.Kci, a.Kv, a.z, a.y, a.sig, partial};
  int sh = lshift_of(a.w);
  int sp = split_of(a.Kv ? a.nnzK : -1, a.nrows, sh);
  if (cpl_of(a.w) == 2) SLAMG_DISPATCH_SPLIT(k_dots, T, 2, sp, grid, s, p, sh);
  else SLAMG_DISPATCH_SPLIT(k_dots, T, 1, sp, grid, s, p, sh);
  launch_finalize(FinPOD{grid, a.w, 0, a.w, partial, out}, nullptr, s);
}

template <typename T>
void launch_dots2(const DotArgs<T>& a, double* pa, double* oa, const DotArgs<T>& b, double* pb, double* ob,
                  hipStream_t s) {
  if (a.nrows <= 0 || b.nrows <= 0) {
    launch_dots(a, pa, oa, s);
    launch_dots(b, pb, ob, s);
    return;
  }
  const int g0 = dots_grid(a.nrows, a.w), g1 = dots_grid(b.nrows, b.w);
  DotPOD<T> qa{a.nrows, a.w, a.a, a.Krp, a.Kci, a.Kv, a.z, a.y, a.sig, pa};
  DotPOD<T> qb{b.nrows, b.w, b.a, b.Krp, b.Kci, b.Kv, b.z, b.y, b.sig, pb};
  const int sh = lshift_of(a.w);
  const int sp = std::max(split_of(a.Kv ? a.nnzK : -1, a.nrows, sh), split_of(b.Kv ? b.nnzK : -1, b.nrows, sh));
  if (cpl_of(a.w) == 2) SLAMG_DISPATCH_SPLIT(k_dots2, T, 2, sp, g0 + g1, s, qa, qb, sh, g0);
  else SLAMG_DISPATCH_SPLIT(k_dots2, T, 1, sp, g0 + g1, s, qa, qb, sh, g0);
  const FinPOD fb{g1, b.w, 0, b.w, pb, ob};
  launch_finalize(FinPOD{g0, a.w, 0, a.w, pa, oa}, &fb, s);
}

// ------------------------------------------------------------------------------------------------
// Tall-skinny Gram G = X^t Y (rows x w, w <= 16) on the FP64 matrix cores.
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16]; the 16x16 result has
// D[l/16 + 4v][l%16] in register v of lane l.  Four rows of X and Y feed one instruction.
// ------------------------------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

// one 64-row pass per workgroup (4 waves x 16 rows) up to GRAM_MAX_GRID workgroups
int gram_grid(int rows) { return std::max(1, std::min(GRAM_MAX_GRID, ceil_div(rows, 64))); }

struct GramPOD {
  int rows, w;
  const double* X; const double* Y; double* partial;
};

__device__ __forceinline__ void gram_body(const GramPOD& a, int blk, int nblk, double (*red)[256]) {
  const int rows = a.rows, w = a.w;
  const double* __restrict__ X = a.X;
  const double* __restrict__ Y = a.Y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  // workgroup blk takes the contiguous rows [b0, b1) in passes of 64 (16 per wave)
  const long chunk = (((long)rows + nblk - 1) / nblk + 63) / 64 * 64;
  const long b0 = std::min((long)rows, (long)blk * chunk), b1 = std::min((long)rows, b0 + chunk);
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (long r0 = b0 + wv * 16; r0 < b1; r0 += 64) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      long r = r0 + u * 4 + kk;
      double av = 0.0, bv = 0.0;
      if (r < b1 && i < w) { av = X[r * w + i]; bv = Y[r * w + i]; }
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][(kk + 4 * v) * 16 + i] = acc[v];
  __syncthreads();
  int tt = threadIdx.x;
  a.partial[(long)blk * 256 + tt] = ((red[0][tt] + red[1][tt]) + red[2][tt]) + red[3][tt];
}

__global__ __launch_bounds__(BLK) void k_gram(GramPOD a) {
  __shared__ double red[4][256];
  gram_body(a, (int)blockIdx.x, gridDim.x, red);
}

// two independent Gram products in one launch: workgroups [0, nb0) take the first
__global__ __launch_bounds__(BLK) void k_gram2(GramPOD a, GramPOD b, int nb0) {
  __shared__ double red[4][256];
  const int bk = (int)blockIdx.x;
  if (bk < nb0) gram_body(a, bk, nb0, red);
  else gram_body(b, bk - nb0, gridDim.x - nb0, red);
}

void launch_gram(int rows, int w, const double* X, const double* Y, double* partial, double* G, hipStream_t s) {
  int grid = gram_grid(rows);
  hipLaunchKernelGGL(k_gram, dim3(grid), dim3(BLK), 0, s, GramPOD{rows, w, X, Y, partial});
  launch_finalize(FinPOD{grid, w * w, w, 256, partial, G}, nullptr, s);
}

void launch_gram2(int w, int rows_a, const double* Xa, const double* Ya, double* pa, double* Ga, int rows_b,
                  const double* Xb, const double* Yb, double* pb, double* Gb, hipStream_t s) {
  const int g0 = gram_grid(rows_a), g1 = gram_grid(rows_b);
  hipLaunchKernelGGL(k_gram2, dim3(g0 + g1), dim3(BLK), 0, s, GramPOD{rows_a, w, Xa, Ya, pa},
                     GramPOD{rows_b, w, Xb, Yb, pb}, g0);
  const FinPOD fb{g1, w * w, w, 256, pb, Gb};
  launch_finalize(FinPOD{g0, w * w, w, 256, pa, Ga}, &fb, s);
}

// ------------------------------------------------------------------------------------------------
// Rotation out = X S (S: win x wout, row-major), gather, column scaling
// ------------------------------------------------------------------------------------------------
// one output entry per thread; t < rows * wout < 2^31 (checked by the launcher)
template <typename T>
__device__ __forceinline__ void rotate_body(int rows, int win, int wout, const T* __restrict__ X,
                                            const double* __restrict__ S, T* __restrict__ out, int blk,
                                            double* Ss) {
  for (int t = threadIdx.x; t < win * wout; t += BLK) Ss[t] = S[t];
  __syncthreads();
  const unsigned t = (unsigned)blk * BLK + threadIdx.x;
  const unsigned row = t / (unsigned)wout;
  const int c = (int)(t - row * (unsigned)wout);
  if (row >= (unsigned)rows) return;
  const T* xr = X + (long)row * win;
  double acc = 0.0;
  for (int k = 0; k < win; ++k) acc += (double)xr[k] * Ss[k * wout + c];
  out[(long)row * wout + c] = (T)acc;
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_rotate(int rows, int win, int wout, const T* __restrict__ X,
                                                const double* __restrict__ S, T* __restrict__ out) {
  __shared__ double Ss[16 * 16];
  rotate_body<T>(rows, win, wout, X, S, out, (int)blockIdx.x, Ss);
}

// the U- and V-side rotations (w x w) in one launch: workgroups [0, nb0) take the first
template <typename T>
__global__ __launch_bounds__(BLK) void k_rotate2(int w, int rows_a, const T* __restrict__ Xa,
                                                 const double* __restrict__ Sa, T* __restrict__ outa, int rows_b,
                                                 const T* __restrict__ Xb, const double* __restrict__ Sb,
                                                 T* __restrict__ outb, int nb0) {
  __shared__ double Ss[16 * 16];
  const int bk = (int)blockIdx.x;
  if (bk < nb0) rotate_body<T>(rows_a, w, w, Xa, Sa, outa, bk, Ss);
  else rotate_body<T>(rows_b, w, w, Xb, Sb, outb, bk - nb0, Ss);
}

template <typename T>
void launch_rotate(int rows, int win, int wout, const T* X, const double* S, T* out, hipStream_t s) {
  if (rows <= 0) return;
  if ((long)rows * wout >= (1L << 31)) throw SolverError{ST_E_INVALID, "rotation too large"};
  hipLaunchKernelGGL((k_rotate<T>), dim3(ceil_div((long)rows * wout, BLK)), dim3(BLK), 0, s, rows, win,
                     wout, X, S, out);
}

template <typename T>
void launch_rotate2(int w, int rows_a, const T* Xa, const double* Sa, T* outa, int rows_b, const T* Xb,
                    const double* Sb, T* outb, hipStream_t s) {
  if (rows_a <= 0 || rows_b <= 0) {
    launch_rotate<T>(rows_a, w, w, Xa, Sa, outa, s);
    launch_rotate<T>(rows_b, w, w, Xb, Sb, outb, s);
    return;
  }
  if ((long)rows_a * w >= (1L << 31) || (long)rows_b * w >= (1L << 31))
    throw SolverError{ST_E_INVALID, "rotation too large"};
  const int g0 = ceil_div((long)rows_a * w, BLK), g1 = ceil_div((long)rows_b * w, BLK);
  hipLaunchKernelGGL((k_rotate2<T>), dim3(g0 + g1), dim3(BLK), 0, s, w, rows_a, Xa, Sa, outa, rows_b, Xb, Sb,
                     outb, g0);
}

template <typename T>
__global__ void k_gather_rows(int nout, int w, const int* __restrict__ idx, const T* __restrict__ X,
                              T* __restrict__ out) {
  long t = (long)blockIdx.x * BLK + threadIdx.x;
  long r = t / w;
  int c = (int)(t % w);
  if (r >= nout) return;
  out[r * w + c] = X[(long)idx[r] * w + c];
}
template <typename T>
void launch_gather_rows(int nout, int w, const int* idx, const T* X, T* out, hipStream_t s) {
  if (nout <= 0) return;
  hipLaunchKernelGGL((k_gather_rows<T>), dim3(ceil_div((long)nout * w, BLK)), dim3(BLK), 0, s, nout, w,
                     idx, X, out);
}

// mode 0: X[:,c] /= sqrt(d[c]) (d > 0);  mode 1: X[:,c] *= d[c]
template <typename T>
__global__ void k_scale_cols(int rows, int w, T* X, const double* __restrict__ d, int mode) {
  long t = (long)blockIdx.x * BLK + threadIdx.x;
  long r = t / w;
  int c = (int)(t % w);
  if (r >= rows) return;
  double f = mode == 0 ? (d[c] > 0.0 ? 1.0 / sqrt(d[c]) : 1.0) : d[c];
  X[r * w + c] = (T)((double)X[r * w + c] * f);
}
template <typename T>
void launch_scale_cols(int rows, int w, T* X, const double* d, int mode, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL((k_scale_cols<T>), dim3(ceil_div((long)rows * w, BLK)), dim3(BLK), 0, s, rows, w, X,
                     d, mode);
}

// Rayleigh quotient update with the sign check: sig = num / sqrt(nu * nv) (nv == null: num / nu);
// a negative quotient flips u (flip = -1) and keeps |sig|.
__global__ void k_rq_update(int w, const double* num, const double* nu, const double* nv, double* sig,
                            double* flip) {
  int c = threadIdx.x;
  if (c >= w) return;
  double q = nv ? num[c] / sqrt(nu[c] * nv[c]) : num[c] / nu[c];
  flip[c] = q < 0.0 ? -1.0 : 1.0;
  sig[c] = fabs(q);
}
void launch_rq_update(int w, const double* num, const double* nu, const double* nv, double* sig, double* flip,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_rq_update, dim3(1), dim3(64), 0, s, w, num, nu, nv, sig, flip);
}

// LS weights from Rayleigh quotients: |rq| (dominant) or 1 / max(|rq|, floor) (minimal)
__global__ void k_rq_weights(int nf, const double* num, const double* nu, const double* nv, int minimal,
                             double floor_abs, const double* scale, double* w) {
  int c = threadIdx.x;
  if (c >= nf) return;
  double q = nv ? num[c] / sqrt(nu[c] * nv[c]) : num[c] / nu[c];
  q = fabs(q);
  w[c] = (minimal ? 1.0 / fmax(q, floor_abs) : q) * (scale ? scale[c] : 1.0);
}
void launch_rq_weights(int nf, const double* num, const double* nu, const double* nv, int minimal,
                       double floor_abs, const double* scale, double* w, hipStream_t s) {
  hipLaunchKernelGGL(k_rq_weights, dim3(1), dim3(64), 0, s, nf, num, nu, nv, minimal, floor_abs, scale, w);
}

template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
  size_t t = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (t < n) p[t] = v;
}
void launch_fill(double* p, size_t n, double val, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_fill<double>), dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, p, n, val);
}
void launch_fillf(float* p, size_t n, float val, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_fill<float>), dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, p, n, val);
}

// out = a x + b y, elementwise
__global__ void k_axpby(size_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out) {
  size_t t = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (t < n) out[t] = a * x[t] + b * y[t];
}
void launch_axpby(size_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_axpby, dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, n, a, x, b, y, out);
}

// out = Y + alpha X S for rows x w blocks (S: w x w row-major, w <= 16); out may be Y, not X
__global__ __launch_bounds__(BLK) void k_rotate_acc(int rows, int w, const double* __restrict__ X,
                                                    const double* __restrict__ S, double alpha, const double* Y,
                                                    double* out) {
  __shared__ double Ss[16 * 16];
  for (int t = threadIdx.x; t < w * w; t += BLK) Ss[t] = S[t];
  __syncthreads();
  const unsigned t = (unsigned)blockIdx.x * BLK + threadIdx.x;
  const unsigned row = t / (unsigned)w;
  const int c = (int)(t - row * (unsigned)w);
  if (row >= (unsigned)rows) return;
  const double* xr = X + (long)row * w;
  double acc = 0.0;
  for (int k = 0; k < w; ++k) acc += xr[k] * Ss[k * w + c];
  const long o = (long)row * w + c;
  out[o] = Y[o] + alpha * acc;
}
void launch_rotate_acc(int rows, int w, const double* X, const double* S, double alpha, const double* Y, double* out,
                       hipStream_t s) {
  if (rows <= 0) return;
  if (w < 1 || w > 16 || (long)rows * w >= (1L << 31)) throw SolverError{ST_E_INVALID, "rotation shape"};
  hipLaunchKernelGGL(k_rotate_acc, dim3(ceil_div((long)rows * w, BLK)), dim3(BLK), 0, s, rows, w, X, S, alpha, Y,
                     out);
}

// M[r0 + i][c0 + j] = G[i][j] (i < wr, j < wc) from a w x w block G into the ld-wide row-major M;
// sym also writes M[c0 + j][r0 + i]
__global__ void k_place_block(int w, int wr, int wc, const double* __restrict__ G, double* __restrict__ M, int ld,
                              int r0, int c0, int sym) {
  const int t = (int)threadIdx.x;
  if (t >= w * w) return;
  const int i = t / w, j = t % w;
  if (i >= wr || j >= wc) return;
  M[(long)(r0 + i) * ld + c0 + j] = G[t];
  if (sym) M[(long)(c0 + j) * ld + r0 + i] = G[t];
}
void launch_place_block(int w, int wr, int wc, const double* G, double* M, int ld, int r0, int c0, int sym,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_place_block, dim3(1), dim3(256), 0, s, w, wr, wc, G, M, ld, r0, c0, sym);
}

// dst (rows x w) = the columns idx[0..n) of src (rows x w) in that order, then zero columns
struct ColSel {
  int idx[16];
  int n;
};
__global__ void k_gather_cols(int rows, int w, ColSel sel, const double* __restrict__ src, double* __restrict__ dst) {
  const long t = (long)blockIdx.x * BLK + threadIdx.x;
  if (t >= (long)rows * w) return;
  const long r = t / w;
  const int c = (int)(t - r * w);
  dst[t] = c < sel.n ? src[r * w + sel.idx[c]] : 0.0;
}
void launch_gather_cols(int rows, int w, const int* idx, int n, const double* src, double* dst, hipStream_t s) {
  if (w < 1 || w > 16 || n < 0 || n > w) throw SolverError{ST_E_INVALID, "column selection"};
  ColSel sel{};
  for (int q = 0; q < n; ++q) sel.idx[q] = idx[q];
  sel.n = n;
  if (rows > 0) hipLaunchKernelGGL(k_gather_cols, dim3(ceil_div((long)rows * w, BLK)), dim3(BLK), 0, s, rows, w, sel, src, dst);
}

// rowC[k] = i for every entry k of row i of a CSR pattern (one thread per row)
__global__ void k_row_index(int m, const int* __restrict__ rp, int* __restrict__ rowC) {
  const int i = (int)(blockIdx.x * BLK + threadIdx.x);
  if (i >= m) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) rowC[k] = i;
}
void launch_row_index(int m, const int* rp, int* rowC, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_row_index, dim3(ceil_div((long)m, BLK)), dim3(BLK), 0, s, m, rp, rowC);
}

// rowC[k] = the row of entry e0 + k of a CSR pattern, k < cnt, for the rows [r0, r1) that hold
// those entries (one thread per entry, a binary search of the row pointers)
__global__ void k_row_index_range(int r0, int r1, const int* __restrict__ rp, long e0, long cnt,
                                  int* __restrict__ rowC) {
  const long k = (long)blockIdx.x * BLK + threadIdx.x;
  if (k >= cnt) return;
  const long g = e0 + k;
  int lo = r0, hi = r1 - 1;   // the last row i in [r0, r1) with rp[i] <= g
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if ((long)rp[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  rowC[k] = lo;
}
void launch_row_index_range(int r0, int r1, const int* rp, long e0, long cnt, int* rowC, hipStream_t s) {
  if (cnt > 0 && r1 > r0)
    hipLaunchKernelGGL(k_row_index_range, dim3(ceil_div(cnt, BLK)), dim3(BLK), 0, s, r0, r1, rp, e0, cnt, rowC);
}

// The top-s rule of §3.7 on a strength operator held in chunks: for each row i of [r0, r0 + grid)
// (entries rp[i] - e0 .. rp[i + 1] - e0 of col / val) the top_s off-diagonal entries with
// |n_ij| > 0 in the order (-|n_ij|, j), written as (j, n_ij) ascending in j, -1 after the last.
// One workgroup per row: each thread keeps its best top_s of a strided share, then the lists are
// merged in pairs through LDS.
constexpr int TOPS_MAX = 16;
__device__ __forceinline__ bool tops_better(double a1, int j1, double a2, int j2) {
  return a1 > a2 || (a1 == a2 && j1 < j2);
}
__global__ __launch_bounds__(256) void k_topsel(int r0, const int* __restrict__ rp, long e0,
                                                const int* __restrict__ col, const double* __restrict__ val, int s,
                                                int* __restrict__ out_col, double* __restrict__ out_val) {
  __shared__ int sj[256 * TOPS_MAX];      // 16 KB
  __shared__ double sv[256 * TOPS_MAX];   // 32 KB (|n_ij| compared as fabs of it)
  __shared__ int sn[256];
  const int i = r0 + (int)blockIdx.x, t = (int)threadIdx.x;
  const long b = (long)rp[i] - e0, e = (long)rp[i + 1] - e0;
  double la[TOPS_MAX], lv[TOPS_MAX];
  int lj[TOPS_MAX];
  int n = 0;
  for (long k = b + t; k < e; k += 256) {
    const int j = col[k];
    const double v = val[k], a = fabs(v);
    if (j == i || !(a > 0.0)) continue;
    if (n == s && !tops_better(a, j, la[s - 1], lj[s - 1])) continue;
    int q = n < s ? n++ : s - 1;
    while (q > 0 && tops_better(a, j, la[q - 1], lj[q - 1])) {
      la[q] = la[q - 1]; lj[q] = lj[q - 1]; lv[q] = lv[q - 1];
      --q;
    }
    la[q] = a; lj[q] = j; lv[q] = v;
  }
  for (int q = 0; q < n; ++q) {
    sj[t * TOPS_MAX + q] = lj[q]; sv[t * TOPS_MAX + q] = lv[q];
  }
  sn[t] = n;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h) {
      // merge list t + h into list t (both ordered best first), keeping the best s
      const int o = t + h, n1 = sn[t], n2 = sn[o];
      int p1 = 0, p2 = 0, m = 0;
      while (m < s && (p1 < n1 || p2 < n2)) {
        const bool take1 = p2 >= n2 || (p1 < n1 && tops_better(fabs(sv[t * TOPS_MAX + p1]), sj[t * TOPS_MAX + p1],
                                                               fabs(sv[o * TOPS_MAX + p2]), sj[o * TOPS_MAX + p2]));
        if (take1) { lj[m] = sj[t * TOPS_MAX + p1]; lv[m] = sv[t * TOPS_MAX + p1]; ++p1; }
        else { lj[m] = sj[o * TOPS_MAX + p2]; lv[m] = sv[o * TOPS_MAX + p2]; ++p2; }
        ++m;
      }
      for (int q = 0; q < m; ++q) {
        sj[t * TOPS_MAX + q] = lj[q]; sv[t * TOPS_MAX + q] = lv[q];
      }
      sn[t] = m;
    }
    __syncthreads();
  }
  if (t == 0) {
    const int m = sn[0];
    for (int q = 0; q < m; ++q) { lj[q] = sj[q]; lv[q] = sv[q]; }
    for (int q = 1; q < m; ++q) {   // ascending in j
      const int j = lj[q];
      const double v = lv[q];
      int r = q;
      while (r > 0 && lj[r - 1] > j) { lj[r] = lj[r - 1]; lv[r] = lv[r - 1]; --r; }
      lj[r] = j; lv[r] = v;
    }
    for (int q = 0; q < s; ++q) {
      out_col[(long)i * s + q] = q < m ? lj[q] : -1;
      out_val[(long)i * s + q] = q < m ? lv[q] : 0.0;
    }
  }
}
void launch_topsel(int r0, int r1, const int* rp, long e0, const int* col, const double* val, int s, int* out_col,
                   double* out_val, hipStream_t st) {
  if (s < 1 || s > TOPS_MAX) throw SolverError{ST_E_INVALID, "top_s outside 1..16"};
  if (r1 > r0) hipLaunchKernelGGL(k_topsel, dim3(r1 - r0), dim3(256), 0, st, r0, rp, e0, col, val, s, out_col, out_val);
}

// k x k identity, row-major
__global__ void k_eye(int k, double* M) {
  const long t = (long)blockIdx.x * BLK + threadIdx.x;
  if (t < (long)k * k) M[t] = (t / k == t % k) ? 1.0 : 0.0;
}
void launch_eye(int k, double* M, hipStream_t s) {
  if (k > 0) hipLaunchKernelGGL(k_eye, dim3(ceil_div((long)k * k, BLK)), dim3(BLK), 0, s, k, M);
}

template <typename A, typename B>
__global__ void k_cast(const A* in, B* out, size_t n) {
  size_t t = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (t < n) out[t] = (B)in[t];
}
// FP64 -> BF16 bit patterns: rounded to FP32, then to the nearest BF16 (ties to even)
__global__ void k_cast_bf16(const double* __restrict__ in, unsigned short* __restrict__ out, size_t n) {
  size_t t = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (t >= n) return;
  const unsigned u = __float_as_uint((float)in[t]);
  const bool nan = (u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu);
  out[t] = nan ? (unsigned short)((u >> 16) | 0x40u) : (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
void launch_cast_bf16(const double* in, void* out, size_t n, hipStream_t s) {
  if (n)
    hipLaunchKernelGGL(k_cast_bf16, dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, in, (unsigned short*)out, n);
}

void launch_copy_cast_df(const double* in, float* out, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_cast<double, float>), dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, in, out, n);
}
void launch_copy_cast_fd(const float* in, double* out, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_cast<float, double>), dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, in, out, n);
}
__global__ void k_axpy_fd(const float* in, double* out, size_t n) {
  size_t t = (size_t)blockIdx.x * BLK + threadIdx.x;
  if (t < n) out[t] += (double)in[t];
}
void launch_axpy_fd(const float* in, double* out, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_axpy_fd, dim3(ceil_div((long)n, BLK)), dim3(BLK), 0, s, in, out, n);
}

template <typename A, typename B>
__global__ void k_recip(int n, const A* in, B* out) {
  int t = blockIdx.x * BLK + threadIdx.x;
  if (t < n) out[t] = in[t] != A(0) ? (B)(1.0 / (double)in[t]) : B(0);
}
void launch_recip(int n, const double* in, double* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_recip<double, double>), dim3(ceil_div(n, BLK)), dim3(BLK), 0, s, n, in, out);
}

__global__ void k_perm_gather(int n, const int* __restrict__ perm, const double* __restrict__ in,
                              double* __restrict__ out) {
  int t = blockIdx.x * BLK + threadIdx.x;
  if (t < n) out[t] = in[perm[t]];
}
void launch_perm_gather(int n, const int* perm, const double* in, double* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_perm_gather, dim3(ceil_div(n, BLK)), dim3(BLK), 0, s, n, perm, in, out);
}

// ------------------------------------------------------------------------------------------------
// Numeric SpGEMM on a known pattern: entry (i, j) of L R is the merge of row i of L with row j of
// R^t (both sorted), summed in increasing inner index.  One thread per output entry.  Each product is
// rounded before it is added (no fused multiply-add): the strength sets of §3.7 compare these
// values, ties included, and this is the textbook order of a sparse product, so the same matrix
// gives bitwise the same strength operator and the same C/F split wherever it is formed.
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLK) void k_spgemm_dot(int nnz, const int* __restrict__ rowC,
                                                    const int* __restrict__ colC, const int* __restrict__ rpL,
                                                    const int* __restrict__ ciL, const double* __restrict__ vL,
                                                    const int* __restrict__ rpR, const int* __restrict__ ciR,
                                                    const double* __restrict__ vR, double* __restrict__ out) {
  int e = blockIdx.x * BLK + threadIdx.x;
  if (e >= nnz) return;
  int i = rowC[e], j = colC[e];
  int a = rpL[i], ae = rpL[i + 1], b = rpR[j], be = rpR[j + 1];
  double s = 0.0;
  while (a < ae && b < be) {
    int ca = ciL[a], cb = ciR[b];
    if (ca == cb) {
#pragma clang fp contract(off)
      const double prod = vL[a] * vR[b];
      s = s + prod;
      ++a; ++b;
    } else if (ca < cb) {
      ++a;
    } else {
      ++b;
    }
  }
  out[e] = s;
}
void launch_spgemm_dot(int nnz, const int* rowC, const int* colC, const int* rpL, const int* ciL, const double* vL,
                       const int* rpR, const int* ciR, const double* vR, double* out, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_spgemm_dot, dim3(ceil_div(nnz, BLK)), dim3(BLK), 0, s, nnz, rowC, colC, rpL, ciL, vL, rpR,
                       ciR, vR, out);
}

__global__ void k_diag_inv(int m, const int* rp, const int* ci, const double* v, double* dinv) {
  int r = blockIdx.x * BLK + threadIdx.x;
  if (r >= m) return;
  double d = 0.0;
  for (int k = rp[r]; k < rp[r + 1]; ++k)
    if (ci[k] == r) d = v[k];
  dinv[r] = d != 0.0 ? 1.0 / d : 0.0;
}
void launch_diag_inv(int m, const int* rp, const int* ci, const double* v, double* dinv, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_diag_inv, dim3(ceil_div(m, BLK)), dim3(BLK), 0, s, m, rp, ci, v, dinv);
}

// Per-row sums for Kaczmarz norms: aa = sum a^2, ab = sum a b, bb = sum b^2 (b on the same pattern;
// bv == nullptr means B = I).  ab and bb may be null.
__global__ void k_row_sq(int m, const int* rp, const int* ci, const double* v, const double* bv, double* aa,
                         double* ab, double* bb) {
  int r = blockIdx.x * BLK + threadIdx.x;
  if (r >= m) return;
  double s_aa = 0.0, s_ab = 0.0, s_bb = 0.0;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    double a = v[k];
    double b = bv ? bv[k] : (ci[k] == r ? 1.0 : 0.0);
    s_aa += a * a; s_ab += a * b; s_bb += b * b;
  }
  aa[r] = s_aa;
  if (ab) ab[r] = s_ab;
  if (bb) bb[r] = s_bb;
}
void launch_row_sq(int m, const int* rp, const double* v, const double* bv, double* aa, double* ab, double* bb,
                   const int* ci, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_row_sq, dim3(ceil_div(m, BLK)), dim3(BLK), 0, s, m, rp, ci, v, bv, aa, ab, bb);
}

__global__ void k_csr_to_dense(int m, const int* rp, const int* ci, const double* v, double* D, int ld, int roff,
                               int coff, int transpose) {
  int r = blockIdx.x * BLK + threadIdx.x;
  if (r >= m) return;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    int c = ci[k];
    if (transpose) D[(long)(roff + c) * ld + coff + r] = v[k];
    else D[(long)(roff + r) * ld + coff + c] = v[k];
  }
}
void launch_csr_to_dense(int m, const int* rp, const int* ci, const double* v, double* D, int ld, int roff, int coff,
                         bool transpose, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(k_csr_to_dense, dim3(ceil_div(m, BLK)), dim3(BLK), 0, s, m, rp, ci, v, D, ld, roff, coff,
                       transpose ? 1 : 0);
}

// ------------------------------------------------------------------------------------------------
// Least-squares interpolation weights, one thread per F-point:
//   (G^t W G + eps I) p = G^t W b,  eps = 1e-13 trace / q,  Cholesky in registers.
// G_{k,a} = value of fitted vector k at the a-th interpolating C-point, b_k = (smoothed) value at
// the F-point.  The fitted vectors are the columns of U1 (w1) followed by those of U2 (w2).
// ------------------------------------------------------------------------------------------------
template <int QM>
__global__ __launch_bounds__(BLK) void k_ls_fit(int nF, const int* __restrict__ Fpts, const int* __restrict__ prp,
                                                const int* __restrict__ fine_cols, int w1,
                                                const double* __restrict__ U1, int w2,
                                                const double* __restrict__ U2, const double* __restrict__ B1,
                                                const double* __restrict__ B2, const double* __restrict__ wts,
                                                double* __restrict__ pval) {
  int f = blockIdx.x * BLK + threadIdx.x;
  if (f >= nF) return;
  const int i = Fpts[f];
  const int p0 = prp[i];
  const int q = prp[i + 1] - p0;
  int J[QM];
  double Nm[QM * (QM + 1) / 2];
  double rhs[QM];
#pragma unroll
  for (int a = 0; a < QM; ++a) {
    J[a] = a < q ? fine_cols[p0 + a] : 0;
    rhs[a] = 0.0;
  }
#pragma unroll
  for (int t = 0; t < QM * (QM + 1) / 2; ++t) Nm[t] = 0.0;
  for (int blk = 0; blk < 2; ++blk) {
    const int wb = blk == 0 ? w1 : w2;
    const double* U = blk == 0 ? U1 : U2;
    const double* Bv = blk == 0 ? B1 : B2;
    const int woff = blk == 0 ? 0 : w1;
    for (int k = 0; k < wb; ++k) {
      const double wk = wts[woff + k];
      const double bk = Bv[(long)i * wb + k];
      double g[QM];
#pragma unroll
      for (int a = 0; a < QM; ++a) g[a] = a < q ? U[(long)J[a] * wb + k] : 0.0;
#pragma unroll
      for (int a = 0; a < QM; ++a) {
        rhs[a] += wk * g[a] * bk;
#pragma unroll
        for (int b = 0; b <= a; ++b) Nm[a * (a + 1) / 2 + b] += wk * g[a] * g[b];
      }
    }
  }
  double tr = 0.0;
#pragma unroll
  for (int a = 0; a < QM; ++a) tr += a < q ? Nm[a * (a + 1) / 2 + a] : 0.0;
  const double eps = q > 0 ? 1e-13 * tr / q : 0.0;
#pragma unroll
  for (int a = 0; a < QM; ++a) Nm[a * (a + 1) / 2 + a] += a < q ? eps : 1.0;
  // Cholesky (lower, packed), padding rows are identity
#pragma unroll
  for (int a = 0; a < QM; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      double s = Nm[a * (a + 1) / 2 + b];
#pragma unroll
      for (int k = 0; k < b; ++k) s -= Nm[a * (a + 1) / 2 + k] * Nm[b * (b + 1) / 2 + k];
      if (a == b) Nm[a * (a + 1) / 2 + a] = sqrt(fmax(s, 1e-300));
      else Nm[a * (a + 1) / 2 + b] = s / Nm[b * (b + 1) / 2 + b];
    }
  }
  // forward / backward substitution
#pragma unroll
  for (int a = 0; a < QM; ++a) {
    double s = rhs[a];
#pragma unroll
    for (int k = 0; k < a; ++k) s -= Nm[a * (a + 1) / 2 + k] * rhs[k];
    rhs[a] = s / Nm[a * (a + 1) / 2 + a];
  }
#pragma unroll
  for (int a = QM - 1; a >= 0; --a) {
    double s = rhs[a];
#pragma unroll
    for (int k = a + 1; k < QM; ++k) s -= Nm[k * (k + 1) / 2 + a] * rhs[k];
    rhs[a] = s / Nm[a * (a + 1) / 2 + a];
  }
#pragma unroll
  for (int a = 0; a < QM; ++a)
    if (a < q) pval[p0 + a] = rhs[a];
}

void launch_ls_fit(int nF, const int* Fpts, const int* prp, const int* fine_cols, int w1, const double* U1, int w2,
                   const double* U2, const double* B1, const double* B2, const double* wts, double* pval, int qmax,
                   hipStream_t s) {
  if (nF <= 0) return;
  int grid = ceil_div(nF, BLK);
  if (qmax <= 4)
    hipLaunchKernelGGL(k_ls_fit<4>, dim3(grid), dim3(BLK), 0, s, nF, Fpts, prp, fine_cols, w1, U1, w2, U2, B1, B2,
                       wts, pval);
  else if (qmax <= 8)
    hipLaunchKernelGGL(k_ls_fit<8>, dim3(grid), dim3(BLK), 0, s, nF, Fpts, prp, fine_cols, w1, U1, w2, U2, B1, B2,
                       wts, pval);
  else
    hipLaunchKernelGGL(k_ls_fit<16>, dim3(grid), dim3(BLK), 0, s, nF, Fpts, prp, fine_cols, w1, U1, w2, U2, B1,
                       B2, wts, pval);
}

// ------------------------------------------------------------------------------------------------
// Seeded initial vectors on the device: SplitMix64 (Steele, Lea & Flood 2014) output k+1 of the
// stream started at `seed`, mapped to [-1, 1) as 2 (z >> 11) 2^-53 - 1.  Value k (column-major over
// the stacked [U; V] of `rows = ru + rv` rows) goes to row-major U (ru x w) or V (rv x w).
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double splitmix_uniform(unsigned long long seed, unsigned long long k) {
  unsigned long long z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}
__global__ void k_splitmix_block(long ru, long rv, int w, unsigned long long seed, double* U, double* V) {
  long t = (long)blockIdx.x * BLK + threadIdx.x;
  long rows = ru + rv;
  if (t >= rows * w) return;
  long c = t / rows, r = t % rows;
  double x = splitmix_uniform(seed, (unsigned long long)t + 1ull);
  if (r < ru) U[r * w + c] = x;
  else V[(r - ru) * w + c] = x;
}
void launch_splitmix_block(long ru, long rv, int w, unsigned long long seed, double* U, double* V, hipStream_t s) {
  long n = (ru + rv) * w;
  if (n > 0) hipLaunchKernelGGL(k_splitmix_block, dim3(ceil_div(n, BLK)), dim3(BLK), 0, s, ru, rv, w, seed, U, V);
}

// Output convention: sgn_j = -1 when the entry of largest magnitude of column j (lowest index on
// ties) is negative.  One workgroup per column.
__global__ __launch_bounds__(BLK) void k_sign_argmax(int rows, int w, const double* __restrict__ X, double* sgn) {
  // column j of the row-major block X with row stride w
  __shared__ double bv[BLK];
  __shared__ int bi[BLK];
  const int j = blockIdx.x;
  double best = -1.0;
  int bidx = 0x7fffffff;
  for (int r = threadIdx.x; r < rows; r += BLK) {
    double a = fabs(X[(long)r * w + j]);
    if (a > best) { best = a; bidx = r; }
  }
  bv[threadIdx.x] = best; bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int s2 = BLK / 2; s2 > 0; s2 >>= 1) {
    if ((int)threadIdx.x < s2) {
      double a = bv[threadIdx.x + s2];
      int ia = bi[threadIdx.x + s2];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ia < bi[threadIdx.x])) {
        bv[threadIdx.x] = a; bi[threadIdx.x] = ia;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sgn[j] = (bi[0] < rows && X[(long)bi[0] * w + j] < 0.0) ? -1.0 : 1.0;
}
void launch_sign_argmax(int rows, int ncols, int w, const double* X, double* sgn, hipStream_t s) {
  hipLaunchKernelGGL(k_sign_argmax, dim3(ncols), dim3(BLK), 0, s, rows, w, X, sgn);
}

// out[keep[r] + j ld] = sgn_j X[r][j] for the first ncols columns of the row-major block X (row
// stride w); column-major output with leading dimension ld
__global__ void k_scatter_out(int rows, int ncols, int w, const double* __restrict__ X, const int* __restrict__ keep,
                              const double* __restrict__ sgn, double* __restrict__ out, long ld) {
  long t = (long)blockIdx.x * BLK + threadIdx.x;
  long r = t / ncols;
  int j = (int)(t % ncols);
  if (r >= rows) return;
  out[(long)keep[r] + (long)j * ld] = sgn[j] * X[r * w + j];
}
void launch_scatter_out(int rows, int ncols, int w, const double* X, const int* keep, const double* sgn, double* out,
                        long ld, hipStream_t s) {
  if (rows > 0 && ncols > 0)
    hipLaunchKernelGGL(k_scatter_out, dim3(ceil_div((long)rows * ncols, BLK)), dim3(BLK), 0, s, rows, ncols, w, X,
                       keep, sgn, out, ld);
}

// explicit instantiations
template void launch_spmm<double>(int, int, const int*, const int*, const double*, const double*, double*, double,
                                  hipStream_t, int, int);
template void launch_spmm<float>(int, int, const int*, const int*, const float*, const float*, float*, double,
                                 hipStream_t, int, int);
template void launch_rowop<double>(const RowOpArgs<double>&, hipStream_t);
template void launch_rowop<float>(const RowOpArgs<float>&, hipStream_t);
template void launch_rowop2<double>(const RowOpArgs<double>&, const RowOpArgs<double>&, hipStream_t);
template void launch_rowop2<float>(const RowOpArgs<float>&, const RowOpArgs<float>&, hipStream_t);
template void launch_spmm2<double>(const SpmmArgs<double>&, const SpmmArgs<double>&, int, hipStream_t);
template void launch_spmm2<float>(const SpmmArgs<float>&, const SpmmArgs<float>&, int, hipStream_t);
template void launch_kacz<double>(const KaczArgs<double>&, hipStream_t);
template void launch_kacz<float>(const KaczArgs<float>&, hipStream_t);
template void launch_kacz_wg<double>(const KaczArgs<double>*, const int* const*, const int*, int, int, hipStream_t);
template void launch_kacz_wg<float>(const KaczArgs<float>*, const int* const*, const int*, int, int, hipStream_t);
template bool launch_kacz_lds<double>(const KaczArgs<double>*, const int* const*, const int*, const int*, int, int,
                                      hipStream_t);
template bool launch_kacz_lds<float>(const KaczArgs<float>*, const int* const*, const int*, const int*, int, int,
                                     hipStream_t);
template void launch_dots<double>(const DotArgs<double>&, double*, double*, hipStream_t);
template void launch_dots<float>(const DotArgs<float>&, double*, double*, hipStream_t);
template void launch_dots2<double>(const DotArgs<double>&, double*, double*, const DotArgs<double>&, double*,
                                   double*, hipStream_t);
template void launch_rotate<double>(int, int, int, const double*, const double*, double*, hipStream_t);
template void launch_rotate<float>(int, int, int, const float*, const double*, float*, hipStream_t);
template void launch_rotate2<double>(int, int, const double*, const double*, double*, int, const double*,
                                    const double*, double*, hipStream_t);
template void launch_gather_rows<double>(int, int, const int*, const double*, double*, hipStream_t);
template void launch_gather_rows<float>(int, int, const int*, const float*, float*, hipStream_t);
template void launch_scale_cols<double>(int, int, double*, const double*, int, hipStream_t);
template void launch_scale_cols<float>(int, int, float*, const double*, int, hipStream_t);

}  // namespace slamg
