"""Plain FP64 CPU oracle of the self-learning AMG method for extremal singular triplets and
eigenpairs (H. De Sterck, "A Self-learning Algebraic Multigrid Method for Extremal Singular
Triplets and Eigenpairs", arXiv:1102.0919).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference that the HIP
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it; the library never calls it and shares no code with it.

Everything is float64 and uses NumPy / SciPy primitives (sparse products, dense SVD, eigh,
Cholesky) as single steps; the method's steps are taken in the paper's order.  Where the paper is
silent or ambiguous, the reading taken is stated at the function (the same readings are listed in
the design notes of the repository):

  R1  initial test vectors: uniform[-1,1) SplitMix64 stream, column-major over [U_t; V_t].
  R2  empty rows / columns of A are removed before solving and re-inserted as zeros.
  R3  strength rule: row-sum rule of §3.7 with the sum over all k (diagonal included);
      alternatives: max-based rule of §3.7, and a top-s rule (s largest off-diagonal magnitudes)
      on the strength operator built from A with high-document-frequency rows ignored.
  R4  C/F split and interpolation patterns are built in the first multiplicative cycle only;
      later cycles refit the weights and rebuild the Galerkin operators on fixed patterns.
  R5  Alg. 1 tie-break: lowest index among maximal lambda; lambda only increases.
  R6  Kaczmarz-relaxed test vectors are normalised in the B/C norm after each outer sweep.
  R7  minimal boot relaxation: v from the rows of (3.27) A v = s B u + kappa, then u from the
      rows of (3.28) A^t u = s C v + tau, each by one Kaczmarz sweep.
  R8  Kaczmarz order: greedy first-fit multicolouring of the row-conflict graph (rows sharing a
      column) in index order; colours ascending, rows ascending in a colour; weight 1.
      (lexicographic order is available as the literal variant).
  R9  additive V-cycle: mu_b pre- and mu_b post-relaxations on every level but the coarsest.
  R10 coarsest generalized SVD: Theorem 3.1's change of variables with Cholesky factors of B, C.
  R11 coarsest vectors scaled so that u^t B u = v^t C v = 1.
  R12 LS normal equations: (G^t W G + eps I) p = G^t W b with eps = 1e-13 trace / n_ci.
  R13 interpolatory sets larger than n_t - 1 are capped to the n_t - 1 strongest connections.
  R14 parameters per problem follow the nearest experiment of §6.
  R15 coarsening stops when the level size (n for eigenproblems, m+n for SVD) is at most
      ``coarse_max``, when the coarse level would keep more than ``stall_ratio`` of the points,
      when it would have fewer than n_b + n_t points on a side, or at ``max_levels``.
  R16 no test-vector relaxation on the coarsest level.
  R17 additive coarsest solve: pseudo-inverse from the SVD of X - sigma Y without its smallest
      singular component (§4.2).  Variant 1 drops the component of the pencil (X, Y)
      eigenvector whose eigenvalue is nearest sigma instead.
  R18 convergence: rho_j = max(||A v - s u||, ||A^t u - s v||) / ||A||_est with unit vectors;
      ||A||_est from 30 power steps on A^t A started from a SplitMix64 vector.
  R19 the LS weight of pair k is |RQ_k| (dominant) or 1 / max(|RQ_k|, 1e-12 ||A||_est) (minimal).
  R20 all n_b triplets iterate until all have converged (no locking).
  R21 after a boot relaxation in the multiplicative phase, a negative Rayleigh quotient flips the
      sign of u and of sigma (§5.3), for both targets.
  R23 minimal SVD targets: after each Ritz step, u_j <- A v_j / ||A v_j|| for sigma_j > 1e-8 ||A||_est.
  R22 the extra F-point Jacobi step of the minimal LS fit (§3.8) uses weight omega_J on the
      operator strength is measured on (A for eigenproblems, A A^t and A^t A for SVD, A for both
      sides under square coarsening); rows with a zero diagonal keep their values.
  R27 one-sided coarsening: on an SVD level where one side would keep fewer than n_b + n_t
      C-points while the other coarsens, that side keeps all its points (identity interpolation).
  R28 square coarsening (§5.1, optional): strength on A itself, and the v-side takes the u-side's
      C/F split and interpolatory sets, so P and Q share one pattern and every level is square.
  R29 guard pairs (optional): the method runs with a block of n_b + n_guard pairs (coarsest
      selection, boot vectors, V-cycles, Ritz step all on the larger block); the stopping test and
      the outputs take the n_b extremal ones.
  R30 completed C-sets: where the rules above would stop coarsening at a level larger than
      ``coarse_dense_max`` unknowns (more than the dense coarsest solves take), each side with
      fewer than n_b + n_t C-points of Algorithm 1's split gets more: its F-points that strongly
      influence the most points (lowest index on ties) become C-points until it has n_b + n_t
      (a side with at most n_b + n_t points keeps them all), the interpolatory sets follow, and
      coarsening continues.
  R33 redetermined interpolation (§6.3, optional): in the additive phase a pair counts as converged
      once its Ritz value changes by at most ``redo_tol`` (1e-14) relative from one iteration to
      the next (the observable stand-in for the relative error the paper plots).  Whenever that
      set grows while some pair of the block is not converged, one downward sweep of the
      multiplicative phase refits P (and Q) and the coarse operators: the test vectors, and copies
      of the current iterates, are relaxed (mu_t; mu_b with Rayleigh quotients) and injected as in
      a cycle, and the LS weights of the test vectors and of the converged pairs are multiplied by
      1e-3.  The iterates themselves are not changed.
  R34 W-cycles (§3.3, optional): with cycle_gamma 2 every level of the additive cycle but the
      last one above the coarsest visits its next coarser level twice per visit of its own (the
      second visit starts from the first one's correction, with the same restricted residual);
      the last one above the coarsest solves the coarsest level once per visit.
  R35 Ritz on coarse levels (§4.3, optional): in the upward sweep of a multiplicative cycle, after
      the boot relaxation of a level below the finest, the level's boot triplets are replaced by
      the Ritz triplets of their span: a B-orthonormal basis of span(U_b) and a C-orthonormal one
      of span(V_b) (eigenproblems: a B-orthonormal basis of span(X_b)), the n_b x n_b projected
      problem, ordered by the target.
  R36 LOBPCG solve phase (§7 names it as a replacement of the multigrid-Ritz additive phase,
      optional): the preconditioned residual of a column is the change the additive cycle makes to
      it, W = C(X) - X, with C the cycle of the additive phase at the current Ritz values.  The
      Ritz step then runs on span[X, W, P] instead of span[C(X)], P the previous iteration's
      search direction (none in the first iteration).  The basis is built block by block: X
      orthonormalised; W with the components along X removed (two passes) and orthonormalised;
      P with the components along X and W removed (two passes).  A column of P (a part of a unit
      Ritz vector) with norm below 1e-10 on either side (a Ritz vector that no longer moves) is
      left out; the block of the others is dropped for that iteration when none remains, when a
      column keeps less than 1e-8 of its norm or the Cholesky factorisation of its
      column-scaled Gram matrix fails or has a pivot below 1e-10 (a condition number of the
      scaled block above about 1e5: a decision well inside FP64's range, so that rounding does
      not decide it).  SVD: the same on
      both sides (P dropped on both when either fails), Ritz triplets from the SVD of
      Q_u^t A Q_v.  For minimal SVD targets the left blocks are the blocks of A Q_v, so that the
      Ritz values are the singular values of A Q_v and none lies below sigma_min(A) (a two-sided
      projection of the enlarged spaces has spurious singular values below it); u_j is then
      A v_j / sigma_j, which makes R23 redundant.  The n_b triplets ordered by the target are
      kept; the new P is the part of each new Ritz vector in the W and P blocks (orthogonal to
      the old X).
  R37 FMG cycles (§3.3 names them, optional): the finest block's residual of (4.1) is restricted
      through every level (no relaxation in between), the coarsest level is solved (§4.2), and
      from the coarsest upwards every coarse level starts from the prolonged correction of the
      level below it and runs one additive cycle (V or W) against its restricted residual; the
      finest block adds the prolonged correction and runs one cycle.
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

SPD = "spd"
SVD = "svd"
DOMINANT = "dominant"
MINIMAL = "minimal"


# ----------------------------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------------------------
@dataclass
class Params:
    theta: float = 0.06
    strength_rule: int = 0        # 0 row-sum, 1 max-based, 2 top-s
    top_s: int = 4
    df_filter: float = 0.0        # rule 2: ignore rows with more than df_filter * n nonzeros
    n_t: int = 8
    mu_t: int = 4
    mu_b: int = 4
    omega: float = 0.7            # omega_J, §3.4
    n_mult: int = 10
    max_add: int = 200
    coarse_max: int = 64
    max_levels: int = 25
    stall_ratio: float = 0.9
    tol: float = 1e-8
    seed: int = 1102
    kaczmarz_order: int = 0       # 0 multicolour, 1 lexicographic
    coarse_pinv: int = 0          # 0 Euclidean SVD pseudo-inverse (literal), 1 pencil variant
    ritz_in_mult: int = 1
    u_from_v: int = 0             # R23: minimal SVD, u_j <- A v_j / ||A v_j|| after each Ritz step
    square_coarsening: int = 0    # §5.1: square A, both sides coarsened on A itself (R28)
    n_guard: int = 0              # R29: extra pairs iterated in the block beyond the n_b wanted
    mu_tJ: int = 1                # inner weighted-Jacobi steps of a test relaxation (§3.4)
    mu_bJ: int = 1                # inner weighted-Jacobi steps of a boot relaxation (§3.5)
    coarse_dense_max: int = 1024  # R30: largest level (unknowns) a coarsening may stop at
    redo_p: int = 0               # R33: redetermine P, Q in the additive phase (§6.3)
    redo_tol: float = 1e-14       # R33: relative change of a Ritz value that counts as converged
    cycle_gamma: int = 1          # R34: coarse visits per level in the additive cycle (1 V, 2 W)
    ritz_coarse: int = 0          # R35: Ritz step on the coarse levels of the multiplicative phase
    solve_phase: int = 0          # R36: 0 multigrid-Ritz additive phase (§4), 1 LOBPCG (§7)
    fmg: int = 0                  # R37: FMG cycles in the additive phase (§3.3)


REDO_DOWN = 1e-3                  # §6.3: LS weight factor of test vectors and converged pairs


NORM_SEED_XOR = 0xA5A5A5A5A5A5A5A5


# ----------------------------------------------------------------------------------------------
# SplitMix64 (Steele, Lea & Flood 2014), written out independently of any other module
# ----------------------------------------------------------------------------------------------
def _splitmix_uniform(seed: int, count: int) -> np.ndarray:
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0


def initial_test_vectors(kind, m, n, n_t, seed):
    """R1: uniform[-1,1) values, column-major over [U_t; V_t] (SVD) or X_t (eigenproblem)."""
    rows = n if kind == SPD else m + n
    blk = _splitmix_uniform(seed, rows * n_t).reshape(n_t, rows).T
    if kind == SPD:
        return blk.copy(), None
    return blk[:m].copy(), blk[m:].copy()


# ----------------------------------------------------------------------------------------------
# sparse helpers (structural patterns: Galerkin products keep every structurally present entry)
# ----------------------------------------------------------------------------------------------
def _ones(M):
    M = sp.csr_matrix(M)
    return sp.csr_matrix((np.ones(M.nnz), M.indices.copy(), M.indptr.copy()), shape=M.shape)


def structural_product(*mats):
    """Product of sparse matrices on the structural pattern of the product (no cancellation
    pruning): values of the numeric product placed on the pattern of the all-ones product."""
    pat = _ones(mats[0])
    val = sp.csr_matrix(mats[0])
    for M in mats[1:]:
        pat = (pat @ _ones(M)).tocsr()
        val = (val @ sp.csr_matrix(M)).tocsr()
    pat.sort_indices(); val.sort_indices()
    nr, nc = pat.shape
    kp = np.repeat(np.arange(nr, dtype=np.int64), np.diff(pat.indptr)) * nc + pat.indices
    kv = np.repeat(np.arange(nr, dtype=np.int64), np.diff(val.indptr)) * nc + val.indices
    data = np.zeros(pat.nnz)
    data[np.searchsorted(kp, kv)] = val.data
    return sp.csr_matrix((data, pat.indices.copy(), pat.indptr.copy()), shape=pat.shape)


def _diag(M):
    return np.asarray(M.diagonal()).ravel()


# ----------------------------------------------------------------------------------------------
# §3.7: strength of connection and Algorithm 1 (one-pass Ruge-Stueben coarsening)
# ----------------------------------------------------------------------------------------------
def strength_sets(N, theta, rule=0, top_s=4):
    """S_i = set of j (j != i) that strongly influence i, as CSR (indptr, indices).

    rule 0: |n_ij| >= theta * sum_k |n_ik| (the row-sum condition of §3.7, sum over all k).
    rule 1: |n_ij| >= theta * max_{k != i} |n_ik| (the max-based condition mentioned in §3.7).
    rule 2: the top_s largest off-diagonal |n_ij| of row i (ties to the lower j).
    Entries with n_ij = 0 are never strong.
    """
    N = sp.csr_matrix(N)
    nr = N.shape[0]
    ind, data = N.indices, np.abs(N.data)
    rows = np.repeat(np.arange(nr), np.diff(N.indptr))
    off = (ind != rows) & (data > 0)
    if rule == 0:
        rowsum = np.add.reduceat(data, N.indptr[:-1]) if N.nnz else np.zeros(nr)
        rowsum[np.diff(N.indptr) == 0] = 0.0
        strong = off & (data >= theta * rowsum[rows])
    elif rule == 1:
        offv = np.where(off, data, 0.0)
        mx = np.zeros(nr)
        np.maximum.at(mx, rows, offv)
        strong = off & (data >= theta * mx[rows])
    else:
        strong = np.zeros(N.nnz, dtype=bool)
        for i in range(nr):
            a, b = N.indptr[i], N.indptr[i + 1]
            cand = np.nonzero(off[a:b])[0]
            if cand.size == 0:
                continue
            order = np.lexsort((ind[a:b][cand], -data[a:b][cand]))
            strong[a + cand[order[:top_s]]] = True
    counts = np.bincount(rows[strong], minlength=nr)
    indptr = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return indptr, ind[strong].astype(np.int64)


def rs_coarsen(S_indptr, S_indices, npts):
    """Algorithm 1 (one-pass Ruge-Stueben).  Returns a bool array, True for C-points.

    "i strongly influences j" means i is in S_j.  lambda_i starts as the number of points that i
    strongly influences; the undecided point with maximal lambda (lowest index on ties, R5) becomes
    C; the undecided points it strongly influences become F; every undecided point that strongly
    influences one of the new F-points has its lambda incremented.
    """
    # influence lists: T_i = { j : i in S_j }
    cnt = np.bincount(S_indices, minlength=npts)
    T_ptr = np.zeros(npts + 1, dtype=np.int64)
    np.cumsum(cnt, out=T_ptr[1:])
    rows = np.repeat(np.arange(npts), np.diff(S_indptr))
    order = np.argsort(S_indices, kind="stable")
    T_idx = rows[order]
    lam = cnt.astype(np.int64).copy()
    state = np.zeros(npts, dtype=np.int8)       # 0 undecided, 1 C, 2 F
    heap = [(-int(lam[i]), i) for i in range(npts)]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if state[i] != 0 or -negl != lam[i]:
            continue
        state[i] = 1
        for j in T_idx[T_ptr[i]:T_ptr[i + 1]]:
            if state[j] == 0:
                state[j] = 2
                for k in S_indices[S_indptr[j]:S_indptr[j + 1]]:
                    if state[k] == 0:
                        lam[k] += 1
                        heapq.heappush(heap, (-int(lam[k]), int(k)))
    return state == 1


def interp_pattern(S_indptr, S_indices, N, is_c, cap):
    """Coarse interpolatory sets C^i = S_i intersected with C (§3.7), capped (R13).

    Returns (ptr, fine_cols, n_capped): for every fine point i, the fine ids of the C-points that
    interpolate to it (for a C-point: itself), sorted ascending.
    """
    N = sp.csr_matrix(N)
    npts = is_c.size
    ptr = np.zeros(npts + 1, dtype=np.int64)
    cols = []
    capped = 0
    for i in range(npts):
        if is_c[i]:
            sel = np.array([i], dtype=np.int64)
        else:
            s = S_indices[S_indptr[i]:S_indptr[i + 1]]
            sel = s[is_c[s]]
            if sel.size > cap:
                capped += 1
                a, b = N.indptr[i], N.indptr[i + 1]
                rowc, rowv = N.indices[a:b], np.abs(N.data[a:b])
                mag = rowv[np.searchsorted(rowc, sel)]
                keep = np.lexsort((sel, -mag))[:cap]
                sel = np.sort(sel[keep])
        cols.append(sel)
        ptr[i + 1] = ptr[i] + sel.size
    return ptr, (np.concatenate(cols) if cols else np.zeros(0, np.int64)), capped


# ----------------------------------------------------------------------------------------------
# §3.8: least-squares interpolation weights
# ----------------------------------------------------------------------------------------------
def ls_interpolation(ptr, fine_cols, is_c, Uf, Ub_values, w):
    """Interpolation matrix P (npts x n_c) with unit rows at C-points and LS weights at F-points.

    For each F-point i:  minimise sum_k w_k (b_k^i - sum_{j in C^i} p_ij u_k^j)^2  over p_i
    (eq. (LS) of §3.8, rows weighted by w_k, R19), where u_k^j are the values of the fitted vectors
    at the interpolating C-points (their injected coarse values) and b_k^i the values at i
    (``Ub_values``: the vectors themselves, or their Jacobi-smoothed values for minimal targets).
    Normal equations with the R12 regularisation, solved per F-point.
    """
    npts = is_c.size
    cidx = np.cumsum(is_c) - 1                     # alpha(i): coarse index of a C-point
    n_c = int(is_c.sum())
    sizes = np.diff(ptr)
    data = np.zeros(fine_cols.size)
    data[ptr[:-1][is_c]] = 1.0
    F = np.nonzero(~is_c)[0]
    for q in np.unique(sizes[F]):
        if q == 0:
            continue
        Fi = F[sizes[F] == q]
        idx = ptr[Fi][:, None] + np.arange(q)[None, :]
        J = fine_cols[idx]                         # (nF, q) fine ids of interpolating C-points
        G = Uf[J]                                  # (nF, q, nf)
        G = np.transpose(G, (0, 2, 1))             # (nF, nf, q)
        b = Ub_values[Fi]                          # (nF, nf)
        GtW = np.transpose(G, (0, 2, 1)) * w[None, None, :]
        Nm = GtW @ G                               # (nF, q, q)
        rhs = np.einsum("fqk,fk->fq", GtW, b)
        eps = 1e-13 * np.trace(Nm, axis1=1, axis2=2) / q
        Nm = Nm + eps[:, None, None] * np.eye(q)[None]
        p = np.linalg.solve(Nm, rhs[..., None])[..., 0]
        data[idx] = p
    P = sp.csr_matrix((data, cidx[fine_cols], ptr), shape=(npts, n_c))
    return P


# ----------------------------------------------------------------------------------------------
# Multicolour ordering for Kaczmarz (R8)
# ----------------------------------------------------------------------------------------------
def greedy_row_colouring(M):
    """Greedy first-fit colouring in row order of the graph 'rows sharing a column'."""
    M = sp.csr_matrix(M)
    MT = M.T.tocsr()
    nr = M.shape[0]
    colour = np.full(nr, -1, dtype=np.int64)
    for i in range(nr):
        cols = M.indices[M.indptr[i]:M.indptr[i + 1]]
        used = set()
        for k in cols:
            for r in MT.indices[MT.indptr[k]:MT.indptr[k + 1]]:
                if r < i:
                    used.add(int(colour[r]))
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


def colour_groups(colour):
    """Rows of each colour, colours ascending, rows ascending."""
    if colour.size == 0:
        return []
    return [np.nonzero(colour == c)[0] for c in range(int(colour.max()) + 1)]


def row_groups(M, groups):
    """(rows, M[rows], M[rows]^t) for each group of rows."""
    out = []
    for rows in groups:
        Mr = sp.csr_matrix(M[rows])
        out.append((rows, Mr, Mr.T.tocsr()))
    return out


def kaczmarz_sweep(M, x, rhs, groups, rownorm2=None, parts=None):
    """One Kaczmarz sweep on M x = rhs (weight 1), row by row in the order of ``groups``.

    Rows of one group share no column, so processing a group at once equals processing its rows
    one after another.  Rows with zero norm are skipped.  x is (n, k), rhs is (nrows, k) or None;
    ``rownorm2`` (nrows,) or (nrows, k) defaults to the squared row norms of M.  ``parts`` may hold
    ``row_groups(M, groups)`` computed beforehand.
    """
    M = sp.csr_matrix(M)
    if rownorm2 is None:
        rownorm2 = np.asarray(M.multiply(M).sum(axis=1)).ravel()
    x = x.copy()
    for rows, Mr, MrT in (parts if parts is not None else row_groups(M, groups)):
        r = (rhs[rows] if rhs is not None else 0.0) - Mr @ x
        rn = rownorm2[rows]
        rn = rn[:, None] if rn.ndim == 1 else rn
        coef = np.where(rn > 0, r / np.where(rn > 0, rn, 1.0), 0.0)
        x += MrT @ coef
    return x


# ----------------------------------------------------------------------------------------------
# Level data
# ----------------------------------------------------------------------------------------------
@dataclass
class Side:
    """Coarsening data of one set of variables (u or v; x for eigenproblems)."""
    is_c: np.ndarray
    cpts: np.ndarray
    ptr: np.ndarray
    fine_cols: np.ndarray
    capped: int
    P: sp.csr_matrix | None = None


@dataclass
class Level:
    A: sp.csr_matrix
    B: sp.csr_matrix
    C: sp.csr_matrix | None
    groups_A: list = field(default_factory=list)     # Kaczmarz order over rows of A
    groups_At: list = field(default_factory=list)    # over rows of A^t (SVD only)
    _parts: dict = field(default_factory=dict)       # row_groups of the current operators

    def kacz_parts(self, which):
        """row_groups of A ("A"), A^t ("At") or B ("B", eigenproblems) in their Kaczmarz order,
        kept while the level's operator objects stay the same."""
        src = self.B if which == "B" else self.A
        got = self._parts.get(which)
        if got is None or got[0] is not src:
            if which == "At":
                got = (src, row_groups(self.A.T.tocsr(), self.groups_At))
            else:
                got = (src, row_groups(src, self.groups_A))
            self._parts[which] = got
        return got[1]
    su: Side | None = None
    sv: Side | None = None

    @property
    def At(self):
        return self.A.T.tocsr()


def _colourings(lev, kind, params):
    order = (lambda M: [np.array([i]) for i in range(M.shape[0])]) if params.kaczmarz_order == 1 \
        else (lambda M: colour_groups(greedy_row_colouring(M)))
    if kind == SPD:
        lev.groups_A = order(_ones(lev.A) + _ones(lev.B))
    else:
        lev.groups_A = order(lev.A)
        lev.groups_At = order(lev.At)


# ----------------------------------------------------------------------------------------------
# Relaxation (§3.4, §3.5, §5.3)
# ----------------------------------------------------------------------------------------------
def _bnorm(M, X):
    return np.sqrt(np.maximum(np.sum(X * (M @ X), axis=0), 0.0))


def relax_test_dominant(lev, kind, U, V, omega, inner=1):
    """One outer power-method step with ``inner`` weighted-Jacobi steps (mu_tJ, §3.4).

    SVD: solve C v_bar = A^t u by v_bar <- v_bar - omega D_C^-1 (C v_bar - A^t u) from v_bar = v,
         v = v_bar / ||v_bar||_C; then B u_bar = A v likewise, u = u_bar / ||u_bar||_B.
    Eigenproblem: B x_bar = A x from x_bar = x, x = x_bar / ||x_bar||_B.
    """
    A, B, C = lev.A, lev.B, lev.C
    if kind == SPD:
        rhs = A @ U
        Xb = U
        for _ in range(inner):
            Xb = Xb - omega * (B @ Xb - rhs) / _diag(B)[:, None]
        return Xb / _bnorm(B, Xb), None
    rhs = A.T @ U
    Vb = V
    for _ in range(inner):
        Vb = Vb - omega * (C @ Vb - rhs) / _diag(C)[:, None]
    V = Vb / _bnorm(C, Vb)
    rhs = A @ V
    Ub = U
    for _ in range(inner):
        Ub = Ub - omega * (B @ Ub - rhs) / _diag(B)[:, None]
    U = Ub / _bnorm(B, Ub)
    return U, V


def relax_test_minimal(lev, kind, U, V):
    """One Kaczmarz sweep on A v = 0 then on A^t u = 0 (SVD) or on A x = 0, then B/C-normalise
    (§5.3, R6, R8)."""
    if kind == SPD:
        X = kaczmarz_sweep(lev.A, U, None, lev.groups_A, parts=lev.kacz_parts("A"))
        return X / _bnorm(lev.B, X), None
    V = kaczmarz_sweep(lev.A, V, None, lev.groups_A, parts=lev.kacz_parts("A"))
    V = V / _bnorm(lev.C, V)
    U = kaczmarz_sweep(lev.At, U, None, lev.groups_At, parts=lev.kacz_parts("At"))
    U = U / _bnorm(lev.B, U)
    return U, V


def relax_boot_dominant(lev, kind, U, V, sig, kap, tau, omega, inner=1):
    """Block Gauss-Seidel with ``inner`` weighted-Jacobi steps per block (mu_bJ, §3.5):
    u <- u - omega D_B^-1 (B u - (A v - kappa)/sigma) with v fixed, then
    v <- v - omega D_C^-1 (C v - (A^t u - tau)/sigma) with the new u fixed.
    Eigenproblem: x <- x - omega D_B^-1 (B x - (A x0 - kappa)/lambda), x0 the outer iterate."""
    A, B, C = lev.A, lev.B, lev.C
    if kind == SPD:
        rhs = (A @ U - kap) / sig[None, :]
        X = U
        for _ in range(inner):
            X = X - omega * (B @ X - rhs) / _diag(B)[:, None]
        return X, None
    rhs = (A @ V - kap) / sig[None, :]
    for _ in range(inner):
        U = U - omega * (B @ U - rhs) / _diag(B)[:, None]
    rhs = (A.T @ U - tau) / sig[None, :]
    for _ in range(inner):
        V = V - omega * (C @ V - rhs) / _diag(C)[:, None]
    return U, V


def relax_boot_minimal(lev, kind, U, V, sig, kap, tau):
    """Block Gauss-Seidel with Kaczmarz blocks (§5.3, R7): v from A v = sigma B u + kappa, then u
    from A^t u = sigma C v + tau.  Eigenproblem: Kaczmarz on (A - lambda_j B) x = kappa."""
    A, B, C = lev.A, lev.B, lev.C
    if kind == SPD:
        # row i of A - lambda_j B is a_i - lambda_j b_i: its residual is
        # kappa_i - (a_i x - lambda_j b_i x) and its squared norm
        # a_i.a_i - 2 lambda_j a_i.b_i + lambda_j^2 b_i.b_i, for every column j at once
        X = U.copy()
        for (rows, Ar, ArT), (_, Br, BrT) in zip(lev.kacz_parts("A"), lev.kacz_parts("B")):
            aa = np.asarray(Ar.multiply(Ar).sum(axis=1)).ravel()[:, None]
            ab = np.asarray(Ar.multiply(Br).sum(axis=1)).ravel()[:, None]
            bb = np.asarray(Br.multiply(Br).sum(axis=1)).ravel()[:, None]
            r = kap[rows] - (Ar @ X - (Br @ X) * sig[None, :])
            rn = aa - 2.0 * sig[None, :] * ab + sig[None, :] ** 2 * bb
            coef = np.where(rn > 0, r / np.where(rn > 0, rn, 1.0), 0.0)
            X += ArT @ coef - BrT @ (coef * sig[None, :])
        return X, None
    V = kaczmarz_sweep(A, V, sig[None, :] * (B @ U) + kap, lev.groups_A, parts=lev.kacz_parts("A"))
    U = kaczmarz_sweep(lev.At, U, sig[None, :] * (C @ V) + tau, lev.groups_At, parts=lev.kacz_parts("At"))
    return U, V


def rayleigh(lev, kind, U, V):
    """Rayleigh quotient (3.31) per column: u^t A v / (||u||_B ||v||_C), or x^t A x / x^t B x."""
    if kind == SPD:
        return np.sum(U * (lev.A @ U), axis=0) / np.sum(U * (lev.B @ U), axis=0)
    return np.sum(U * (lev.A @ V), axis=0) / (_bnorm(lev.B, U) * _bnorm(lev.C, V))


def relax_boot_with_rq(lev, kind, target, U, V, sig, params):
    """Multiplicative-phase boot relaxation: mu_b outer steps, each followed by a Rayleigh-quotient
    update of sigma_b (§3.5) and the sign check of §5.3 (R21)."""
    z_u = np.zeros_like(U)
    z_v = None if V is None else np.zeros_like(V)
    for _ in range(params.mu_b):
        if target == DOMINANT:
            U, V = relax_boot_dominant(lev, kind, U, V, sig, z_u, z_v, params.omega, params.mu_bJ)
        else:
            U, V = relax_boot_minimal(lev, kind, U, V, sig, z_u, z_v)
        sig = rayleigh(lev, kind, U, V)
        neg = sig < 0
        if np.any(neg):
            U = U.copy(); U[:, neg] *= -1.0
            sig = np.abs(sig)
    return U, V, sig


# ----------------------------------------------------------------------------------------------
# Coarsest level (§3.6, Theorem 3.1 / 3.2) and additive coarsest solve (§4.2)
# ----------------------------------------------------------------------------------------------
def coarsest_gsvd(lev, kind, target, n_b):
    """n_b extremal generalized singular triplets of (A, B, C), or eigenpairs of (A, B) (R10, R11)."""
    A = lev.A.toarray(); B = lev.B.toarray()
    if kind == SPD:
        lam, X = sla.eigh(A, B)                          # ascending, B-orthonormal
        idx = np.arange(n_b) if target == MINIMAL else np.arange(lam.size - 1, lam.size - 1 - n_b, -1)
        return lam[idx].copy(), X[:, idx].copy(), None
    C = lev.C.toarray()
    LB = np.linalg.cholesky(B); LC = np.linalg.cholesky(C)
    D = sla.solve_triangular(LB, sla.solve_triangular(LC, A.T, lower=True).T, lower=True)
    T, s, Wt = np.linalg.svd(D, full_matrices=True)      # descending
    l = s.size
    idx = np.arange(n_b) if target == DOMINANT else np.arange(l - 1, l - 1 - n_b, -1)
    U = sla.solve_triangular(LB.T, T[:, idx], lower=False)
    V = sla.solve_triangular(LC.T, Wt.T[:, idx], lower=False)
    return s[idx].copy(), U, V


def pencil_matrices(lev, kind):
    """Dense X and Y of (3.10)-(3.11) (SVD) or A and B (eigenproblem) on the coarsest level."""
    if kind == SPD:
        return lev.A.toarray(), lev.B.toarray()
    m, n = lev.A.shape
    X = np.zeros((m + n, m + n)); Y = np.zeros((m + n, m + n))
    Ad = lev.A.toarray()
    X[:m, m:] = Ad; X[m:, :m] = Ad.T
    Y[:m, :m] = lev.B.toarray(); Y[m:, m:] = lev.C.toarray()
    return X, Y


def coarse_pinv_solve(X, Y, sig, rhs):
    """Per column j: pseudo-inverse of X - sigma_j Y from its SVD with the smallest singular
    component left out, applied to rhs[:, j] (§4.2, R17 literal)."""
    out = np.zeros_like(rhs)
    for j in range(rhs.shape[1]):
        W, s, Zt = np.linalg.svd(X - sig[j] * Y)
        k = s.size - 1
        out[:, j] = Zt[:k].T @ ((W[:, :k].T @ rhs[:, j]) / s[:k])
    return out


def coarse_pencil_solve(X, Y, sig, rhs):
    """R17 variant 1: with the Y-orthonormal pencil eigenbasis X z = mu Y z, apply
    sum_{i != i*} z_i z_i^t / (mu_i - sigma_j), i* = argmin |mu_i - sigma_j|."""
    mu, Z = sla.eigh(X, Y)
    out = np.zeros_like(rhs)
    for j in range(rhs.shape[1]):
        d = mu - sig[j]
        keep = np.ones(mu.size, dtype=bool); keep[np.argmin(np.abs(d))] = False
        out[:, j] = Z[:, keep] @ ((Z[:, keep].T @ rhs[:, j]) / d[keep])
    return out


# ----------------------------------------------------------------------------------------------
# §4.3: Ritz projection on the finest level (B = I, C = I)
# ----------------------------------------------------------------------------------------------
def ritz(A, kind, target, U, V, u_from_v=False, anorm=1.0):
    if kind == SPD:
        Xh, _ = np.linalg.qr(U)
        M = Xh.T @ (A @ Xh)
        M = 0.5 * (M + M.T)
        lam, Yv = np.linalg.eigh(M)
        order = np.argsort(lam) if target == MINIMAL else np.argsort(-lam)
        return lam[order], Xh @ Yv[:, order], None
    Uh, _ = np.linalg.qr(U)
    Vh, _ = np.linalg.qr(V)
    M = Uh.T @ (A @ Vh)
    Y, s, Zt = np.linalg.svd(M)
    order = np.argsort(s) if target == MINIMAL else np.argsort(-s)
    s, U, V = s[order], Uh @ Y[:, order], Vh @ Zt.T[:, order]
    if u_from_v:
        # R23: left vectors of non-zero Ritz values taken from A v_j, which removes the components
        # in the null space of A^t that relaxation never changes.
        AV = A @ V
        nrm = np.linalg.norm(AV, axis=0)
        ok = s > 1e-8 * anorm
        U[:, ok] = AV[:, ok] / nrm[ok]
    return s, U, V


def metric_orthonormal(M, X):
    """A basis of span(X) orthonormal in the inner product of the SPD matrix M: X L^-t with
    L L^t = X^t M X (§4.3)."""
    L = np.linalg.cholesky(X.T @ (M @ X))
    return sla.solve_triangular(L, X.T, lower=True).T


def ritz_level(lev, kind, target, U, V):
    """§4.3's Ritz step on a level with its B and C (R35): the extremal triplets of the projected
    problem on span(U) x span(V) in the B and C metrics, ordered by the target."""
    if kind == SPD:
        Xh = metric_orthonormal(lev.B, U)
        M = Xh.T @ (lev.A @ Xh)
        lam, Yv = np.linalg.eigh(0.5 * (M + M.T))
        order = np.argsort(lam) if target == MINIMAL else np.argsort(-lam)
        return lam[order], Xh @ Yv[:, order], None
    Uh = metric_orthonormal(lev.B, U)
    Vh = metric_orthonormal(lev.C, V)
    Y, s, Zt = np.linalg.svd(Uh.T @ (lev.A @ Vh))
    order = np.argsort(s) if target == MINIMAL else np.argsort(-s)
    return s[order], Uh @ Y[:, order], Vh @ Zt.T[:, order]


def remove_components(Y, bases):
    """Y with its components along the orthonormal blocks in ``bases`` removed, two passes (R36)."""
    for _ in range(2):
        for Q in bases:
            Y = Y - Q @ (Q.T @ Y)
    return Y


def keep_direction(Y0, Y):
    """R36's test for keeping the P block Y0, Y what is left of it after the components along the
    X and W blocks are removed: every column keeps at least 1e-8 of its norm, and the Gram matrix
    of Y with its columns scaled to unit norm has a Cholesky factorisation L L^t whose pivots
    L_ii^2 are all at least 1e-10."""
    d = np.linalg.norm(Y, axis=0)
    if np.any(d < 1e-8 * np.linalg.norm(Y0, axis=0)) or np.any(d == 0.0):
        return False
    Ys = Y / d[None, :]
    try:
        L = np.linalg.cholesky(Ys.T @ Ys)
    except np.linalg.LinAlgError:
        return False
    return bool(np.min(np.diag(L)) ** 2 >= 1e-10)


def orthonormal_basis(Y):
    """An orthonormal basis of span(Y) (Householder QR of the column-scaled block)."""
    d = np.linalg.norm(Y, axis=0)
    d[d == 0.0] = 1.0
    Q, _ = np.linalg.qr(Y / d[None, :])
    return Q


def lobpcg_ritz(A, kind, target, n_b, X, W, P):
    """R36's Rayleigh-Ritz step on span[X, W, P] (§7): X, W, P are (U, V) pairs of blocks (V None
    for eigenproblems), P None when there is no search direction.  Returns sigma, the new Ritz
    pair, the new search direction and whether the P block was kept."""
    one_sided = kind == SVD and target == MINIMAL
    QV = None
    if kind == SVD:
        QV = [orthonormal_basis(X[1])]
        QV.append(orthonormal_basis(remove_components(W[1], QV)))
    left = [A @ Q for Q in QV] if one_sided else [X[0], W[0]]
    QU = [orthonormal_basis(left[0])]
    QU.append(orthonormal_basis(remove_components(left[1], QU)))
    kept = False
    if P is not None:
        # columns of P that still move (1e-10 on each side), in column order
        act = np.ones(P[0].shape[1], dtype=bool)
        for B in P:
            if B is not None:
                act &= np.linalg.norm(B, axis=0) >= 1e-10
        P = (P[0][:, act], None if P[1] is None else P[1][:, act]) if act.any() else None
    if P is not None:
        PV = None if kind == SPD else remove_components(P[1], QV)
        okv = kind == SPD or keep_direction(P[1], PV)
        PU0 = A @ orthonormal_basis(PV) if one_sided and okv else P[0]
        PU = remove_components(PU0, QU)
        if okv and keep_direction(PU0, PU):
            QU.append(orthonormal_basis(PU))
            if kind == SVD:
                QV.append(orthonormal_basis(PV))
            kept = True
    Qu = np.hstack(QU)
    if kind == SPD:
        M = Qu.T @ (A @ Qu)
        lam, Yv = np.linalg.eigh(0.5 * (M + M.T))
        order = np.argsort(lam) if target == MINIMAL else np.argsort(-lam)
        sel = order[:n_b]
        Ysel = Yv[:, sel]
        Xn = Qu @ Ysel
        Pn = Qu[:, n_b:] @ Ysel[n_b:, :]
        return lam[sel], (Xn, None), (Pn, None), kept
    Qv = np.hstack(QV)
    Yl, s, Zt = np.linalg.svd(Qu.T @ (A @ Qv))
    order = np.argsort(s) if target == MINIMAL else np.argsort(-s)
    sel = order[:n_b]
    Ysel, Zsel = Yl[:, sel], Zt.T[:, sel]
    Un, Vn = Qu @ Ysel, Qv @ Zsel
    Pn = (Qu[:, n_b:] @ Ysel[n_b:, :], Qv[:, n_b:] @ Zsel[n_b:, :])
    return s[sel], (Un, Vn), Pn, kept


def residuals(A, kind, U, V, sig, anorm):
    """R18: rho_j (unit vectors assumed)."""
    if kind == SPD:
        return np.linalg.norm(A @ U - U * sig[None, :], axis=0) / anorm
    r1 = np.linalg.norm(A @ V - U * sig[None, :], axis=0)
    r2 = np.linalg.norm(A.T @ U - V * sig[None, :], axis=0)
    return np.maximum(r1, r2) / anorm


def norm_estimate(A, seed, steps=30):
    """R18: ||A||_2 estimate from power steps on A^t A started from a SplitMix64 vector."""
    x = _splitmix_uniform(seed ^ NORM_SEED_XOR, A.shape[1])
    x /= np.linalg.norm(x)
    for _ in range(steps):
        y = A.T @ (A @ x)
        ny = np.linalg.norm(y)
        if ny == 0:
            return 0.0
        x = y / ny
    return float(np.linalg.norm(A @ x))


# ----------------------------------------------------------------------------------------------
# Hierarchy construction pieces
# ----------------------------------------------------------------------------------------------
def strength_operators(lev, kind, params, finest=True):
    """Operators strength is measured on (§3.7, §5.1-5.2): A (eigenproblem), A A^t and A^t A (SVD).
    The document-frequency filter of rule 2 applies on the finest level only (R3)."""
    if kind == SPD:
        return lev.A, None
    A = lev.A
    if finest and params.strength_rule == 2 and params.df_filter > 0:
        df = np.diff(A.indptr)
        keep = (df <= params.df_filter * A.shape[1]).astype(np.float64)
        A = sp.diags(keep) @ A
        A = sp.csr_matrix(A)
    At = A.T.tocsr()
    return structural_product(A, At), structural_product(At, A)


def shared_side(su):
    """§5.1 (R28): the v-side takes the u-side's C/F split and interpolatory sets; only the LS
    weights (fitted to V instead of U) differ, so P and Q share one pattern and every A_l is
    square."""
    return Side(su.is_c.copy(), su.cpts.copy(), su.ptr.copy(), su.fine_cols.copy(), 0)


def build_side(N, params, n_t):
    Sp, Si = strength_sets(N, params.theta, params.strength_rule, params.top_s)
    is_c = rs_coarsen(Sp, Si, N.shape[0])
    ptr, cols, capped = interp_pattern(Sp, Si, N, is_c, n_t - 1)
    side = Side(is_c, np.nonzero(is_c)[0], ptr, cols, capped)
    side.strength = (N, Sp, Si)
    return side


def complete_c_set(side, need, n_t):
    """R30: a side with fewer than ``need`` C-points gets its F-points that strongly influence the
    most points (the initial lambda of Algorithm 1; lowest index on ties) as further C-points until
    it has ``need``; its interpolatory sets are rebuilt on the same strength sets.  A side with at
    most ``need`` points keeps all of them."""
    npts = side.is_c.size
    if int(side.is_c.sum()) >= need:
        return side
    if npts <= need:
        return identity_side(npts)
    N, Sp, Si = side.strength
    influence = np.bincount(Si, minlength=npts)
    f = np.nonzero(~side.is_c)[0]
    order = f[np.lexsort((f, -influence[f]))]
    is_c = side.is_c.copy()
    is_c[order[:need - int(side.is_c.sum())]] = True
    ptr, cols, capped = interp_pattern(Sp, Si, N, is_c, n_t - 1)
    out = Side(is_c, np.nonzero(is_c)[0], ptr, cols, capped)
    out.strength = side.strength
    return out


def identity_side(npts):
    """Every point a C-point: the interpolation is the identity."""
    return Side(np.ones(npts, dtype=bool), np.arange(npts), np.arange(npts + 1), np.arange(npts), 0)


def one_sided_coarsening(su, sv, kind, need):
    """R27: on an SVD level where one side would keep fewer than n_b + n_t C-points while the other
    side coarsens, the first side is not coarsened (identity interpolation) instead of stopping."""
    if kind == SPD:
        return su, sv
    cu, cv = int(su.is_c.sum()), int(sv.is_c.sum())
    if cu < need <= cv:
        su = identity_side(su.is_c.size)
    elif cv < need <= cu:
        sv = identity_side(sv.is_c.size)
    return su, sv


def minimal_presmooth(lev, kind, side_is_u, Vals, omega, square=False):
    """Extra Jacobi step on N z = 0 applied to the F-point values before the LS fit (§3.8, R22).

    N is the operator strength is measured on: A for eigenproblems, A A^t (u) and A^t A (v) for
    SVD levels, and A itself for both sides under square coarsening (§5.1, R28).  Rows whose
    diagonal of N is zero keep their values."""
    A = lev.A
    if kind == SPD or square:
        NZ = A @ Vals; d = _diag(A)
    elif side_is_u:
        NZ = A @ (A.T @ Vals); d = np.asarray(A.multiply(A).sum(axis=1)).ravel()
    else:
        NZ = A.T @ (A @ Vals); d = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    step = np.where(d != 0, 1.0 / np.where(d != 0, d, 1.0), 0.0)
    return Vals - omega * NZ * step[:, None]


def ls_weights(lev, kind, target, U, V, anorm):
    rq = rayleigh(lev, kind, U, V)
    if target == DOMINANT:
        return np.abs(rq)
    return 1.0 / np.maximum(np.abs(rq), 1e-12 * anorm)


def galerkin(lev, kind):
    """(3.4): A_c = P^t A Q, B_c = P^t B P, C_c = Q^t C Q (eigenproblem: P^t A P, P^t B P)."""
    P = lev.su.P
    if kind == SPD:
        return Level(structural_product(P.T.tocsr(), lev.A, P), structural_product(P.T.tocsr(), lev.B, P), None)
    Q = lev.sv.P
    return Level(structural_product(P.T.tocsr(), lev.A, Q), structural_product(P.T.tocsr(), lev.B, P),
                 structural_product(Q.T.tocsr(), lev.C, Q))


def level_size(lev, kind):
    return lev.A.shape[0] if kind == SPD else lev.A.shape[0] + lev.A.shape[1]


# ----------------------------------------------------------------------------------------------
# The solver
# ----------------------------------------------------------------------------------------------
@dataclass
class Result:
    sigma: np.ndarray
    U: np.ndarray
    V: np.ndarray | None
    report: dict


class Solver:
    """Hybrid multiplicative-additive solver (§3, §4, §5) on a prepared (m >= n, no empty rows or
    columns) matrix."""

    def __init__(self, A, kind, target, n_b, params: Params, init=None):
        # R29: the block holds the n_b wanted pairs and n_guard more
        self.kind, self.target, self.n_want, self.p = kind, target, n_b, params
        self.n_b = n_b + params.n_guard
        A = sp.csr_matrix(A, dtype=np.float64)
        A.sort_indices()
        m, n = A.shape
        I_m = sp.identity(m, format="csr"); I_n = sp.identity(n, format="csr")
        self.levels = [Level(A, I_m, None if kind == SPD else I_n)]
        _colourings(self.levels[0], kind, params)
        if init is None:
            self.Ut, self.Vt = initial_test_vectors(kind, m, n, params.n_t, params.seed)
        else:
            self.Ut, self.Vt = init
        self.anorm = norm_estimate(A, params.seed)
        self.sig = None; self.Ub = None; self.Vb = None
        self.report = dict(levels=0, sizes=[], mult_sigma=[], add_sigma=[], rho=[], capped=[],
                           colours=[], mult_cycles=0, add_iters=0, anorm=self.anorm, redo=[])

    # -------------------------------------------------------------- multiplicative cycle (§3.3)
    def mult_cycle(self, c):
        kind, target, p = self.kind, self.target, self.p
        Ut, Vt = self.Ut, self.Vt
        Ub, Vb, sig = self.Ub, self.Vb, self.sig
        tests_u, tests_v = [Ut], [Vt]
        l = 0
        while True:
            lev = self.levels[l]
            if c == 1:
                if self._is_coarsest_size(l):
                    break
                if kind == SVD and p.square_coarsening:
                    # §5.1: strength, C/F split and patterns of both sides from A itself
                    su = build_side(lev.A, p, p.n_t)
                    sv = shared_side(su)
                else:
                    Nu, Nv = strength_operators(lev, kind, p, l == 0)
                    su = build_side(Nu, p, p.n_t)
                    sv = None if kind == SPD else build_side(Nv, p, p.n_t)
                su0, sv0 = su, sv
                su, sv = one_sided_coarsening(su, sv, kind, self.n_b + p.n_t)
                if not self._coarsening_ok(lev, su, sv):
                    if level_size(lev, kind) <= p.coarse_dense_max:
                        break
                    # R30: complete the short sides of Algorithm 1's split instead of stopping
                    su = complete_c_set(su0, self.n_b + p.n_t, p.n_t)
                    if kind == SVD:
                        sv = shared_side(su) if p.square_coarsening else complete_c_set(sv0, self.n_b + p.n_t, p.n_t)
                    if not self._coarsening_ok(lev, su, sv):
                        break
                lev.su, lev.sv = su, sv
                self.report["capped"].append(su.capped + (0 if sv is None else sv.capped))
            elif l == len(self.levels) - 1:
                break
            # relax test vectors (§3.4 / §5.3)
            for _ in range(p.mu_t):
                if target == DOMINANT:
                    Ut, Vt = relax_test_dominant(lev, kind, Ut, Vt, p.omega, p.mu_tJ)
                else:
                    Ut, Vt = relax_test_minimal(lev, kind, Ut, Vt)
            tests_u[l], tests_v[l] = Ut, Vt
            if c >= 2:
                Ub, Vb, sig = relax_boot_with_rq(lev, kind, target, Ub, Vb, sig, p)
            # LS fit of P (and Q) (§3.8)
            if c == 1:
                Uf, Vf = Ut, Vt
            else:
                Uf = np.hstack([Ut, Ub]); Vf = None if kind == SPD else np.hstack([Vt, Vb])
            w = ls_weights(lev, kind, target, Uf, Vf, self.anorm)
            self._fit(lev, lev.su, Uf, w, True)
            if kind == SVD:
                self._fit(lev, lev.sv, Vf, w, False)
            # Galerkin coarse operators (3.4)
            coarse = galerkin(lev, kind)
            if c == 1:
                _colourings(coarse, kind, p)
                self.levels.append(coarse)
            else:
                old = self.levels[l + 1]
                old.A, old.B, old.C = coarse.A, coarse.B, coarse.C
            # injection (§3.3)
            Ut = Ut[lev.su.cpts]
            Vt = None if kind == SPD else Vt[lev.sv.cpts]
            tests_u.append(Ut); tests_v.append(Vt)
            if c >= 2:
                Ub = Ub[lev.su.cpts]
                Vb = None if kind == SPD else Vb[lev.sv.cpts]
            l += 1
        L = l
        if c == 1:
            self.report["levels"] = L + 1
            self.report["sizes"] = [lv.A.shape for lv in self.levels]
        # coarsest generalized SVD (§3.6)
        sig, Ub, Vb = coarsest_gsvd(self.levels[L], kind, target, self.n_b)
        # upward sweep: multiplicative interpolation, boot relaxation with RQ updates (§3.3)
        for l in range(L - 1, -1, -1):
            lev = self.levels[l]
            Ub = lev.su.P @ Ub
            Vb = None if kind == SPD else lev.sv.P @ Vb
            Ub, Vb, sig = relax_boot_with_rq(lev, kind, target, Ub, Vb, sig, p)
            if p.ritz_coarse and l > 0:
                sig, Ub, Vb = ritz_level(lev, kind, target, Ub, Vb)
        self.Ut, self.Vt = tests_u[0], tests_v[0]
        if p.ritz_in_mult:
            sig, Ub, Vb = self._ritz(Ub, Vb)
        self.sig, self.Ub, self.Vb = sig, Ub, Vb
        self.report["mult_sigma"].append(sig.copy())

    def _ritz(self, U, V):
        ufv = bool(self.p.u_from_v) and self.kind == SVD and self.target == MINIMAL
        return ritz(self.levels[0].A, self.kind, self.target, U, V, ufv, self.anorm)

    def _is_coarsest_size(self, l):
        return level_size(self.levels[l], self.kind) <= self.p.coarse_max or l + 1 >= self.p.max_levels

    def _coarsening_ok(self, lev, su, sv):
        kind, p = self.kind, self.p
        nc_u = int(su.is_c.sum())
        nc = nc_u if kind == SPD else nc_u + int(sv.is_c.sum())
        if nc > p.stall_ratio * level_size(lev, kind):
            return False
        need = self.n_b + p.n_t
        if nc_u < need or (kind == SVD and int(sv.is_c.sum()) < need):
            return False
        return True

    def _fit(self, lev, side, Vals, w, is_u):
        bvals = Vals
        if self.target == MINIMAL:
            bvals = minimal_presmooth(lev, self.kind, is_u, Vals, self.p.omega,
                                      square=self.kind == SVD and bool(self.p.square_coarsening))
        side.P = ls_interpolation(side.ptr, side.fine_cols, side.is_c, Vals, bvals, w)

    # -------------------------------------------------------------- additive cycle (§4.1-4.2)
    def _additive_cycle_fns(self):
        """The pieces of the additive cycle with sigma fixed: cycle(l, U, V, kappa, tau) is one
        visit of level l above the coarsest (§4.1-§4.3; cycle_gamma visits of the next level, R34),
        coarsest(kappa, tau) the coarsest solve (§4.2)."""
        kind, target, p, sig = self.kind, self.target, self.p, self.sig
        L = len(self.levels) - 1

        def relax(l, U, V, kap, tau):
            lev = self.levels[l]
            for _ in range(p.mu_b):
                if target == DOMINANT:
                    U, V = relax_boot_dominant(lev, kind, U, V, sig, kap, tau, p.omega, p.mu_bJ)
                else:
                    U, V = relax_boot_minimal(lev, kind, U, V, sig, kap, tau)
            return U, V

        def coarsest(kap, tau):
            X, Y = pencil_matrices(self.levels[L], kind)
            rhs = kap if kind == SPD else np.vstack([kap, tau])
            z = (coarse_pinv_solve if p.coarse_pinv == 0 else coarse_pencil_solve)(X, Y, sig, rhs)
            self.report["coarse_solves"] = self.report.get("coarse_solves", 0) + 1
            if kind == SPD:
                return z, None
            mL = self.levels[L].A.shape[0]
            return z[:mL], z[mL:]

        def cycle(l, U, V, kap, tau):
            lev = self.levels[l]
            U, V = relax(l, U, V, kap, tau)
            # residuals (4.1) and restriction (4.2)
            kc, tc = restrict(l, U, V, kap, tau)
            if l + 1 == L:
                Uc, Vc = coarsest(kc, tc)
            else:
                Uc = np.zeros((lev.su.cpts.size, self.n_b))
                Vc = None if kind == SPD else np.zeros((lev.sv.cpts.size, self.n_b))
                for _ in range(p.cycle_gamma):
                    Uc, Vc = cycle(l + 1, Uc, Vc, kc, tc)
            # correction (4.3) and post-relaxation
            U = U + lev.su.P @ Uc
            V = None if kind == SPD else V + lev.sv.P @ Vc
            return relax(l, U, V, kap, tau)

        def restrict(l, U, V, kap, tau):
            lev = self.levels[l]
            if kind == SPD:
                r = kap - (lev.A @ U - (lev.B @ U) * sig[None, :])
                return lev.su.P.T @ r, None
            r = kap - (lev.A @ V - (lev.B @ U) * sig[None, :])
            t = tau - (lev.A.T @ U - (lev.C @ V) * sig[None, :])
            return lev.su.P.T @ r, lev.sv.P.T @ t

        return cycle, coarsest, restrict

    def additive_vcycle(self):
        """One additive cycle for all n_b columns with sigma fixed: a V-cycle (cycle_gamma 1) or,
        with cycle_gamma 2, a W-cycle (§3.3, R34): every level above the last one before the
        coarsest visits its coarse level twice, the second visit starting from the first one's
        correction; the coarsest level is solved once per visit of the level above it."""
        if len(self.levels) == 1:
            # one level: the multiplicative phase's coarsest generalized SVD is already exact and
            # there is no coarse correction to add
            return
        cycle, _, _ = self._additive_cycle_fns()
        kap0 = np.zeros_like(self.Ub)
        tau0 = None if self.kind == SPD else np.zeros_like(self.Vb)
        self.Ub, self.Vb = cycle(0, self.Ub, self.Vb, kap0, tau0)

    def additive_fmg(self):
        """R37's FMG cycle (§3.3 names FMG): the finest block's residual restricted to every level,
        the coarsest level solved, then from the coarsest upwards every coarse level takes the
        prolonged correction of the level below it and one cycle against its restricted residual;
        the finest block takes the prolonged correction and one cycle."""
        L = len(self.levels) - 1
        if L == 0:
            return
        kind = self.kind
        cycle, coarsest, restrict = self._additive_cycle_fns()
        kap = [None] * (L + 1)
        tau = [None] * (L + 1)
        z0 = np.zeros_like(self.Ub)
        kap[1], tau[1] = restrict(0, self.Ub, self.Vb, z0, None if kind == SPD else np.zeros_like(self.Vb))
        for l in range(1, L):
            lev = self.levels[l]
            kap[l + 1] = lev.su.P.T @ kap[l]
            tau[l + 1] = None if kind == SPD else lev.sv.P.T @ tau[l]
        Uc, Vc = coarsest(kap[L], tau[L])
        for l in range(L - 1, 0, -1):
            lev = self.levels[l]
            U = lev.su.P @ Uc
            V = None if kind == SPD else lev.sv.P @ Vc
            Uc, Vc = cycle(l, U, V, kap[l], tau[l])
        lev = self.levels[0]
        U = self.Ub + lev.su.P @ Uc
        V = None if kind == SPD else self.Vb + lev.sv.P @ Vc
        self.Ub, self.Vb = cycle(0, U, V, z0, None if kind == SPD else np.zeros_like(self.Vb))

    def additive_cycle(self):
        """The additive phase's cycle: FMG (R37) or a V-/W-cycle."""
        if self.p.fmg:
            self.additive_fmg()
        else:
            self.additive_vcycle()

    def lobpcg_iteration(self, P):
        """One iteration of R36's LOBPCG solve phase (§7): W = C(X) - X from the additive cycle
        and the Ritz step on span[X, W, P].  Returns the new search direction."""
        X = (self.Ub.copy(), None if self.Vb is None else self.Vb.copy())
        self.additive_cycle()
        W = (self.Ub - X[0], None if self.Vb is None else self.Vb - X[1])
        sig, (U, V), Pn, kept = lobpcg_ritz(self.levels[0].A, self.kind, self.target, self.n_b, X, W, P)
        self.sig, self.Ub, self.Vb = sig, U, V
        if P is not None and not kept:
            self.report["p_dropped"] = self.report.get("p_dropped", 0) + 1
        return Pn

    # -------------------------------------------------------------- redetermined P (§6.3, R33)
    def redo_interpolation(self, conv):
        """One downward sweep of the multiplicative phase during the additive phase: P, Q and the
        coarse operators are refitted, with the LS weights of the test vectors and of the pairs
        marked in ``conv`` multiplied by REDO_DOWN.  The additive iterates are not changed."""
        kind, target, p = self.kind, self.target, self.p
        Ut, Vt = self.Ut, self.Vt
        Ub = self.Ub.copy()
        Vb = None if self.Vb is None else self.Vb.copy()
        sig = self.sig.copy()
        scale = np.concatenate([np.full(p.n_t, REDO_DOWN), np.where(conv, REDO_DOWN, 1.0)])
        for l in range(len(self.levels) - 1):
            lev = self.levels[l]
            for _ in range(p.mu_t):
                if target == DOMINANT:
                    Ut, Vt = relax_test_dominant(lev, kind, Ut, Vt, p.omega, p.mu_tJ)
                else:
                    Ut, Vt = relax_test_minimal(lev, kind, Ut, Vt)
            if l == 0:
                self.Ut, self.Vt = Ut, Vt
            Ub, Vb, sig = relax_boot_with_rq(lev, kind, target, Ub, Vb, sig, p)
            Uf = np.hstack([Ut, Ub]); Vf = None if kind == SPD else np.hstack([Vt, Vb])
            w = ls_weights(lev, kind, target, Uf, Vf, self.anorm) * scale
            self._fit(lev, lev.su, Uf, w, True)
            if kind == SVD:
                self._fit(lev, lev.sv, Vf, w, False)
            coarse = galerkin(lev, kind)
            old = self.levels[l + 1]
            old.A, old.B, old.C = coarse.A, coarse.B, coarse.C
            Ut = Ut[lev.su.cpts]; Ub = Ub[lev.su.cpts]
            if kind == SVD:
                Vt = Vt[lev.sv.cpts]; Vb = Vb[lev.sv.cpts]

    # -------------------------------------------------------------- solve loop (§3.3, §4)
    def run(self):
        p, A0 = self.p, self.levels[0].A
        for c in range(1, p.n_mult + 1):
            self.mult_cycle(c)
            self.report["mult_cycles"] = c
        if not p.ritz_in_mult:
            self.sig, self.Ub, self.Vb = self._ritz(self.Ub, self.Vb)
        rho = residuals(A0, self.kind, self.Ub, self.Vb, self.sig, self.anorm)
        self.report["rho"].append(rho)
        it = 0
        nw = self.n_want
        conv = np.zeros(self.n_b, dtype=bool)
        prev = self.sig.copy()
        P = None
        while rho[:nw].max() > p.tol and it < p.max_add:
            if p.solve_phase == 1:
                P = self.lobpcg_iteration(P)
            else:
                self.additive_cycle()
                self.sig, self.Ub, self.Vb = self._ritz(self.Ub, self.Vb)
            rho = residuals(A0, self.kind, self.Ub, self.Vb, self.sig, self.anorm)
            it += 1
            self.report["rho"].append(rho)
            self.report["add_sigma"].append(self.sig.copy())
            if p.redo_p:
                now = np.abs(self.sig - prev) <= p.redo_tol * np.abs(self.sig)
                prev = self.sig.copy()
                if (now & ~conv).any() and not now.all() and rho[:nw].max() > p.tol:
                    conv |= now
                    self.redo_interpolation(conv.copy())
                    self.report["redo"].append(it)
        self.report["add_iters"] = it
        self.report["converged"] = bool(rho[:nw].max() <= p.tol)
        return self.sig[:nw], self.Ub[:, :nw], None if self.Vb is None else self.Vb[:, :nw]


def _sign_normalise(U, V):
    """Output convention: the entry of largest magnitude of v_j (x_j) is positive (lowest index on
    ties)."""
    ref = V if V is not None else U
    for j in range(ref.shape[1]):
        k = int(np.argmax(np.abs(ref[:, j])))
        if ref[k, j] < 0:
            U[:, j] *= -1.0
            if V is not None:
                V[:, j] *= -1.0
    return U, V


def solve(A, kind, target, n_b, params: Params | None = None, init=None) -> Result:
    """Entry point: n_b dominant or minimal singular triplets (kind 'svd') or eigenpairs (kind
    'spd') of the sparse matrix A, following §3-§5.

    The matrix is transposed when m < n (§1 assumes m >= n) and empty rows and columns are removed
    (R2).  ``init`` optionally gives the initial test vectors (U_t, V_t) for the prepared matrix.
    Returns sigma (sorted descending for dominant, ascending for minimal), unit-norm U (m x n_b)
    and V (n x n_b; None for eigenproblems), and a report.
    """
    params = params or Params()
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    m0, n0 = A.shape
    transposed = False
    if kind == SVD and m0 < n0:
        A = A.T.tocsr(); transposed = True
    m, n = A.shape
    rows_keep = np.nonzero(np.diff(A.indptr) > 0)[0]
    cols_keep = np.nonzero(np.bincount(A.indices, minlength=n) > 0)[0]
    if kind == SPD:
        keep = np.union1d(rows_keep, cols_keep)
        Ar = A[keep][:, keep]
        rows_keep = cols_keep = keep
    else:
        Ar = A[rows_keep][:, cols_keep]
    Ar = sp.csr_matrix(Ar); Ar.sort_indices()
    if kind == SVD and params.square_coarsening and Ar.shape[0] != Ar.shape[1]:
        raise ValueError("square coarsening needs a square matrix without empty rows or columns")
    s = Solver(Ar, kind, target, n_b, params, init)
    sig, U, V = s.run()
    Ufull = np.zeros((m, n_b)); Ufull[rows_keep] = U
    Vfull = None
    if kind == SVD:
        Vfull = np.zeros((n, n_b)); Vfull[cols_keep] = V
    if transposed:
        Ufull, Vfull = Vfull, Ufull
    Ufull, Vfull = _sign_normalise(Ufull, Vfull)
    s.report["solver"] = s
    return Result(sig, Ufull, Vfull, s.report)
