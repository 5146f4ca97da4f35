"""Seeded synthetic inputs shaped like the paper's model problems, and their closed-form spectra.

This module holds no arithmetic of the method itself: it only builds input matrices (CSR arrays)
and initial vectors, and states the exact spectra that the structured matrices have.  Both the HIP
library's tests and the CPU oracle's tests draw their inputs from here, so that the two sides see
identical data while sharing no code of the method.

Matrix families (the paper's test problems are described in §6; the datasets and discretisations
it does not give are replaced by the synthetic stand-ins below):

* ``laplace2d(k)``      – 5-point Dirichlet finite-difference Laplacian on a k x k interior grid
                          (the FD problem of §6.2 is k=32; the small SPD workload is k=31).
* ``gradient2d(k)``     – discrete gradient (edge-vertex incidence) of the k x k grid graph, a
                          rectangular matrix whose singular values are square roots of the Neumann
                          graph-Laplacian eigenvalues.
* ``termdoc(m, n, ...)``– Zipf-distributed synthetic term-document matrix (log(1 + count) values)
                          standing in for the MEDLINE matrix of §6.4, which is not available here.
* ``termdoc_topics(m, n, ...)`` – a topic-structured variant with raw counts.
* ``aniso3d(k, eps)``   – 7-point anisotropic Dirichlet diffusion on a k^3 grid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Plain CSR triple with shape; int64 row pointer, int32 column indices, float64 values."""
    m: int
    n: int
    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.m, self.n))

    @staticmethod
    def from_scipy(M) -> "CSR":
        M = M.tocsr()
        M.sort_indices()
        return CSR(M.shape[0], M.shape[1], M.indptr.astype(np.int64),
                   M.indices.astype(np.int32), M.data.astype(np.float64))


def _coo_to_csr(m, n, rows, cols, vals) -> CSR:
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    np.cumsum(indptr, out=indptr)
    return CSR(m, n, indptr, cols.astype(np.int32), vals)


# --------------------------------------------------------------------------------------------
# Structured matrices
# --------------------------------------------------------------------------------------------
def laplace2d(k: int) -> CSR:
    """5-point Laplacian, Dirichlet, k x k interior points, id = y*k + x, diagonal 4, neighbours -1."""
    rows, cols, vals = [], [], []
    idx = np.arange(k * k).reshape(k, k)          # [y, x]
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(np.full(k * k, 4.0))
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        ys, xs = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
        ny, nx = ys + dy, xs + dx
        ok = (ny >= 0) & (ny < k) & (nx >= 0) & (nx < k)
        rows.append(idx[ys[ok], xs[ok]]); cols.append(idx[ny[ok], nx[ok]])
        vals.append(np.full(int(ok.sum()), -1.0))
    return _coo_to_csr(k * k, k * k, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def convdiff2d(k: int, c: float = 0.5) -> CSR:
    """Upwind convection-diffusion -Laplace(u) + c (u_x + u_y), Dirichlet, k x k interior points,
    id = y*k + x, in grid units: diagonal 4 + 2c, -(1 + c) to the west and south (upwind)
    neighbours, -1 to the east and north ones.  A square nonsymmetric M-matrix."""
    rows, cols, vals = [], [], []
    idx = np.arange(k * k).reshape(k, k)          # [y, x]
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(np.full(k * k, 4.0 + 2.0 * c))
    for dy, dx, w in ((0, 1, -1.0), (0, -1, -1.0 - c), (1, 0, -1.0), (-1, 0, -1.0 - c)):
        ys, xs = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
        ny, nx = ys + dy, xs + dx
        ok = (ny >= 0) & (ny < k) & (nx >= 0) & (nx < k)
        rows.append(idx[ys[ok], xs[ok]]); cols.append(idx[ny[ok], nx[ok]])
        vals.append(np.full(int(ok.sum()), w))
    return _coo_to_csr(k * k, k * k, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def aniso3d(k: int, eps: float = 0.01) -> CSR:
    """7-point anisotropic Dirichlet diffusion on k^3 points, id = (z*k + y)*k + x.

    Diagonal 4 + 2*eps, -1 to the x and y neighbours, -eps to the z neighbours.
    """
    n = k ** 3
    idx = np.arange(n).reshape(k, k, k)           # [z, y, x]
    zs, ys, xs = np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij")
    rows = [idx.ravel()]; cols = [idx.ravel()]; vals = [np.full(n, 4.0 + 2.0 * eps)]
    for dz, dy, dx, w in ((0, 0, 1, -1.0), (0, 0, -1, -1.0), (0, 1, 0, -1.0), (0, -1, 0, -1.0),
                          (1, 0, 0, -eps), (-1, 0, 0, -eps)):
        nz, ny, nx = zs + dz, ys + dy, xs + dx
        ok = (nz >= 0) & (nz < k) & (ny >= 0) & (ny < k) & (nx >= 0) & (nx < k)
        rows.append(idx[zs[ok], ys[ok], xs[ok]]); cols.append(idx[nz[ok], ny[ok], nx[ok]])
        vals.append(np.full(int(ok.sum()), w))
    return _coo_to_csr(n, n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def gradient2d(k: int) -> CSR:
    """Discrete gradient of the k x k grid graph.

    Vertex id = y*k + x.  Rows 0 .. k(k-1)-1 are the horizontal edges (x,y)-(x+1,y) with row id
    y*(k-1) + x; rows k(k-1) .. 2k(k-1)-1 are the vertical edges (x,y)-(x,y+1) with row id
    k(k-1) + y*k + x.  Each row has -1 at the lower vertex id and +1 at the higher one.
    """
    nh = k * (k - 1)
    ys, xs = np.meshgrid(np.arange(k), np.arange(k - 1), indexing="ij")
    h_rows = (ys * (k - 1) + xs).ravel()
    h_lo = (ys * k + xs).ravel(); h_hi = h_lo + 1
    ys2, xs2 = np.meshgrid(np.arange(k - 1), np.arange(k), indexing="ij")
    v_rows = (nh + ys2 * k + xs2).ravel()
    v_lo = (ys2 * k + xs2).ravel(); v_hi = v_lo + k
    rows = np.concatenate([h_rows, h_rows, v_rows, v_rows])
    cols = np.concatenate([h_lo, h_hi, v_lo, v_hi])
    vals = np.concatenate([-np.ones(nh), np.ones(nh), -np.ones(nh), np.ones(nh)])
    return _coo_to_csr(2 * nh, k * k, rows, cols, vals)


def termdoc_topics(m: int, n: int, per_col: int = 60, n_topics: int = 40, zipf_s: float = 1.1,
                   topic_s: float = 1.5, background: float = 0.15, geom_p: float = 0.3,
                   seed: int = 1102) -> CSR:
    """Synthetic term-document matrix (terms x documents) with topic structure and raw counts.

    Topic k of ``n_topics`` has weight proportional to k^-topic_s; each document belongs to one
    topic drawn from those weights.  A document's ``per_col`` distinct terms are drawn in order:
    with probability ``background`` from a shared background vocabulary, else from its topic's;
    within a vocabulary a term's rank follows a Zipf law with exponent ``zipf_s`` on 1..m (inverse
    CDF of the normalised r^-s) and the rank maps to a term id through that vocabulary's seeded
    permutation.  Entry (term, document) is the term's count, drawn from the geometric law on
    {1, 2, ...} with success probability ``geom_p``.  numpy's PCG64 seeded with ``seed`` drives all
    draws.  The dominant singular values then fall off with gaps like those of real term-document
    data (a common-vocabulary value, then one per topic).
    """
    rng = np.random.default_rng(seed)
    weights = np.arange(1, m + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(weights); cdf /= cdf[-1]
    tw = np.arange(1, n_topics + 1, dtype=np.float64) ** (-topic_s); tw /= tw.sum()
    perms = np.stack([rng.permutation(m) for _ in range(n_topics + 1)])   # row n_topics: background
    topic = rng.choice(n_topics, size=n, p=tw)
    rows = np.empty(n * per_col, dtype=np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), per_col)
    vals = np.empty(n * per_col, dtype=np.float64)
    for j in range(n):
        picked = np.empty(0, dtype=np.int64)
        while picked.size < per_col:
            k = 2 * per_col
            src = np.where(rng.random(k) < background, n_topics, topic[j])
            ranks = np.minimum(np.searchsorted(cdf, rng.random(k), side="right"), m - 1)
            cand = np.concatenate([picked, perms[src, ranks]])
            _, first = np.unique(cand, return_index=True)
            picked = cand[np.sort(first)][:per_col]
        rows[j * per_col:(j + 1) * per_col] = picked
        vals[j * per_col:(j + 1) * per_col] = rng.geometric(geom_p, per_col).astype(np.float64)
    return _coo_to_csr(m, n, rows, cols, vals)


def termdoc(m: int, n: int, per_col: int = 60, zipf_s: float = 1.1, geom_p: float = 0.3,
            seed: int = 1102) -> CSR:
    """Synthetic term-document matrix (terms x documents).

    Each column (document) holds ``per_col`` distinct term ranks, taken in draw order from a Zipf
    law with exponent ``zipf_s`` truncated to ranks 1..m (inverse CDF of the normalised r^-s);
    the term id of a rank comes from one seeded permutation; each value is log(1 + c) with c drawn
    from the geometric law on {1, 2, ...} with success probability ``geom_p``.  numpy's PCG64
    generator seeded with ``seed`` drives all draws.
    """
    rng = np.random.default_rng(seed)
    weights = np.arange(1, m + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(weights); cdf /= cdf[-1]
    perm = rng.permutation(m)
    rows = np.empty(n * per_col, dtype=np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), per_col)
    for j in range(n):
        picked: list[int] = []
        seen: set[int] = set()
        while len(picked) < per_col:
            draws = np.searchsorted(cdf, rng.random(2 * per_col), side="left")
            for r in draws.tolist():
                if r not in seen:
                    seen.add(r); picked.append(r)
                    if len(picked) == per_col:
                        break
        rows[j * per_col:(j + 1) * per_col] = perm[np.array(picked)]
    counts = rng.geometric(geom_p, size=n * per_col)
    vals = np.log1p(counts.astype(np.float64))
    return _coo_to_csr(m, n, rows, cols, vals)


# --------------------------------------------------------------------------------------------
# Initial vectors: SplitMix64 counter generator (Steele, Lea & Flood, OOPSLA 2014)
# --------------------------------------------------------------------------------------------
_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start+1 .. start+count of SplitMix64 started from state ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, count: int, start: int = 0) -> np.ndarray:
    """SplitMix64 outputs mapped to [-1, 1): 2 * (z >> 11) * 2^-53 - 1."""
    z = splitmix64(seed, count, start)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


def initial_tests(rows: int, n_t: int, seed: int) -> np.ndarray:
    """rows x n_t block filled column-major with uniform[-1,1) SplitMix64 values from ``seed``."""
    return uniform_pm1(seed, rows * n_t).reshape(n_t, rows).T.copy()


def seeded_block(rows: int, cols: int, seed: int) -> np.ndarray:
    """Generic seeded dense block for kernel-level tests (numpy PCG64, uniform [-1, 1))."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(rows, cols))


def random_csr(m: int, n: int, seed: int, mean_row: float = 6.0, skew: bool = True,
               empty_rows: bool = True) -> CSR:
    """Random CSR with skewed row lengths (some long rows, some empty), for kernel tests."""
    rng = np.random.default_rng(seed)
    if skew:
        lens = np.minimum(rng.geometric(1.0 / mean_row, size=m), n)
        lens[rng.random(m) < 0.02] = min(n, int(8 * mean_row))
    else:
        lens = np.full(m, min(n, int(mean_row)))
    if empty_rows:
        lens[rng.random(m) < 0.03] = 0
    rows, cols = [], []
    for i in range(m):
        c = rng.choice(n, size=int(lens[i]), replace=False)
        rows.append(np.full(c.size, i)); cols.append(c)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = rng.uniform(-1.0, 1.0, size=rows.size)
    return _coo_to_csr(m, n, rows, cols, vals)


# --------------------------------------------------------------------------------------------
# Closed-form spectra of the structured matrices
# --------------------------------------------------------------------------------------------
def laplace2d_eigs(k: int) -> np.ndarray:
    """All eigenvalues 4 sin^2(i pi/(2(k+1))) + 4 sin^2(j pi/(2(k+1))), i,j = 1..k, ascending."""
    s = 4.0 * np.sin(np.arange(1, k + 1) * math.pi / (2 * (k + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())


def aniso3d_eigs_smallest(k: int, eps: float, count: int) -> np.ndarray:
    """Smallest ``count`` eigenvalues of aniso3d(k, eps), ascending."""
    s = 4.0 * np.sin(np.arange(1, k + 1) * math.pi / (2 * (k + 1))) ** 2
    lim = min(k, count + 2)
    vals = (s[:lim, None, None] + s[None, :lim, None] + eps * s[None, None, :]).ravel()
    return np.sort(vals)[:count]


def aniso3d_eig_max(k: int, eps: float) -> float:
    s = 4.0 * np.sin(k * math.pi / (2 * (k + 1))) ** 2
    return float(s * (2.0 + eps))


def gradient2d_singular_values(k: int) -> np.ndarray:
    """All k^2 singular values sqrt(4 sin^2(i pi/(2k)) + 4 sin^2(j pi/(2k))), i,j = 0..k-1, ascending."""
    s = 4.0 * np.sin(np.arange(k) * math.pi / (2 * k)) ** 2
    return np.sort(np.sqrt(s[:, None] + s[None, :]).ravel())


# --------------------------------------------------------------------------------------------
# The workloads, with the method parameters taken from the nearest experiment of §6
# --------------------------------------------------------------------------------------------
WORKLOADS = {
    # name: (description, builder, kind, target, n_b, parameter overrides)
    "laplace2d_31_min4": dict(desc="2-D Dirichlet 5-point Laplacian 31x31 (n=961), 4 minimal eigenpairs, FP64",
                              kind="spd", target="minimal", n_b=4,
                              params=dict(theta=0.06, n_t=6, mu_t=8, mu_b=4, n_mult=15)),
    "laplace2d_32_min8": dict(desc="2-D FD Laplacian 32x32 (n=1024), 8 minimal eigenpairs (paper §6.2)",
                              kind="spd", target="minimal", n_b=8,
                              params=dict(theta=0.06, n_t=6, mu_t=8, mu_b=4, n_mult=15)),
    "laplace2d_32_dom8": dict(desc="2-D FD Laplacian 32x32 (n=1024), 8 dominant eigenpairs (paper §6.2)",
                              kind="spd", target="dominant", n_b=8,
                              params=dict(theta=0.06, n_t=6, mu_t=8, mu_b=4, n_mult=15)),
    "gradient2d_256_dom8": dict(desc="discrete gradient of the 256x256 grid graph (130560x65536), 8 dominant triplets, FP64",
                                kind="svd", target="dominant", n_b=8,
                                params=dict(theta=0.05, n_t=8, mu_t=4, mu_b=4, n_mult=10)),
    "gradient2d_256_min8": dict(desc="discrete gradient of the 256x256 grid graph (130560x65536), 8 minimal triplets, FP64",
                                kind="svd", target="minimal", n_b=8,
                                params=dict(theta=0.05, n_t=8, mu_t=4, mu_b=4, n_mult=10)),
    # §6.1's square nonsymmetric case (31 x 31 interior points, n_b = 8, n_t = 5, mu_t = mu_b = 4,
    # theta = 0.05, both sides coarsened on A); its FVE operator is not given, an upwind
    # convection-diffusion matrix of the same size stands in.  The minimal run takes n_t = 8: with
    # 5 test vectors it settles on interior triplets of this operator
    "convdiff2d_31_dom8": dict(desc="upwind convection-diffusion 31x31 (n=961, nonsymmetric), 8 dominant triplets, square coarsening",
                               kind="svd", target="dominant", n_b=8,
                               params=dict(theta=0.05, n_t=5, mu_t=4, mu_b=4, n_mult=10, square_coarsening=1)),
    "convdiff2d_31_min8": dict(desc="upwind convection-diffusion 31x31 (n=961, nonsymmetric), 8 minimal triplets, square coarsening",
                               kind="svd", target="minimal", n_b=8,
                               params=dict(theta=0.05, n_t=8, mu_t=4, mu_b=4, n_mult=10, square_coarsening=1)),
    "termdoc_200k_dom10": dict(desc="Zipf(1.1) term-document matrix 200000x50000, 60 distinct terms per document, "
                                    "values log(1+c) with c ~ Geometric(0.3), 10 dominant triplets",
                               kind="svd", target="dominant", n_b=10,
                               # 6 guard pairs (R29): sigma_2 .. sigma_10 of this matrix form one tight
                               # cluster, and the last pair of a 10-wide block stalls next to sigma_11.
                               # mu_b = 1: sigma_1 is ~7 sigma_2, and the Jacobi-type boot relaxation of
                               # pair j (§3.5) multiplies the sigma_1 component by about
                               # ((1 - omega) + omega sigma_1 / sigma_j)^2 ~ 26 per sweep, which with
                               # mu_b = 4 makes a V-cycle's correction 1e12..1e20 times its residual
                               params=dict(strength_rule=2, top_s=4, df_filter=0.01, n_t=14, mu_t=1,
                                           mu_b=1, n_mult=3, coarse_pinv=1, n_guard=6)),
    # §6.4's parameter set (n_t 14, mu_t 1, mu_b 4, 3 multiplicative cycles, 8 dominant triplets) at
    # the MEDLINE submatrix's size: 5735 terms x 1033 documents, 50 distinct Zipf(1.1) terms per
    # document (0.87% dense), log(1+c) values; top-s strength as for configuration 3
    "termdoc_medline_dom8": dict(desc="Zipf(1.1) term-document matrix 5735x1033 (MEDLINE's shape), 50 terms per "
                                      "document, 8 dominant triplets, the parameters of §6.4",
                                 kind="svd", target="dominant", n_b=8,
                                 params=dict(strength_rule=2, top_s=4, df_filter=0.01, n_t=14, mu_t=1, mu_b=4,
                                             n_mult=3, coarse_pinv=1, max_add=300)),
    "termdoc_topics_200k_dom10": dict(desc="topic-structured term-document matrix 200000x50000 (40 topics, raw "
                                           "counts), 60 distinct terms per document, 10 dominant triplets",
                                      kind="svd", target="dominant", n_b=10,
                                      params=dict(strength_rule=2, top_s=4, df_filter=0.01, n_t=14, mu_t=1,
                                                  mu_b=4, n_mult=3, coarse_pinv=1)),
    "aniso3d_128_min8": dict(desc="3-D anisotropic 7-point Dirichlet 128^3 (n=2097152, eps=0.01), 8 minimal eigenpairs",
                             kind="spd", target="minimal", n_b=8,
                             # a diagonally dominant PDE discretisation: the max-based strength rule
                             # of §3.7 with theta 0.25; 8 guard pairs (R29) keep the 8 wanted pairs
                             # clear of the 9th, whose coarse-level representation limits the last
                             # pair of the block
                             params=dict(theta=0.25, strength_rule=1, n_t=8, mu_t=4, mu_b=4, n_mult=10,
                                         coarse_pinv=1, coarse_max=128, n_guard=8)),
}


def build_workload_matrix(name: str, scale: int | None = None) -> CSR:
    """Matrix of a named workload; ``scale`` overrides the grid size (for reduced test sizes)."""
    if name.startswith("laplace2d_31"):
        return laplace2d(scale or 31)
    if name.startswith("laplace2d_32"):
        return laplace2d(scale or 32)
    if name.startswith("gradient2d_256"):
        return gradient2d(scale or 256)
    if name.startswith("convdiff2d_31"):
        return convdiff2d(scale or 31)
    if name.startswith("termdoc_200k"):
        n = scale or 50000
        return termdoc(4 * n, n, 60, seed=1102)
    if name.startswith("termdoc_medline"):
        return termdoc(5735, 1033, 50, seed=1102)
    if name.startswith("termdoc_topics_200k"):
        n = scale or 50000
        return termdoc_topics(4 * n, n, 60, seed=1102)
    if name.startswith("aniso3d_128"):
        return aniso3d(scale or 128, 0.01)
    raise KeyError(name)


# --------------------------------------------------------------------------------------------
# Serving stream: requests drawn from the three matrix families
# --------------------------------------------------------------------------------------------
FAMILY_PARAMS = {
    ("laplace", "minimal"): WORKLOADS["laplace2d_32_min8"]["params"],
    ("laplace", "dominant"): WORKLOADS["laplace2d_32_dom8"]["params"],
    ("gradient", "minimal"): WORKLOADS["gradient2d_256_min8"]["params"],
    ("gradient", "dominant"): WORKLOADS["gradient2d_256_dom8"]["params"],
    ("termdoc", "minimal"): WORKLOADS["termdoc_200k_dom10"]["params"],
    ("termdoc", "dominant"): WORKLOADS["termdoc_200k_dom10"]["params"],
}


def serving_requests(count: int, seed: int = 1102, n_lo: float = 1e3, n_hi: float = 2e5,
                     rate: float = 1.0) -> list[dict]:
    """A seeded request stream: family uniform over {2-D Laplacian with k = round(sqrt(n)), gradient
    of a k x k grid with k = round(sqrt(n)), term-document with n documents, 4n terms and 60
    nonzeros per document}; n log-uniform in [n_lo, n_hi]; n_b uniform in {1, 4, 8, 16}; dominant or
    minimal with probability 1/2; Poisson arrivals at ``rate`` requests per second (arrival times
    in seconds from the start).  Matrices are built on demand by ``serving_matrix``."""
    rng = np.random.default_rng(seed)
    reqs, t = [], 0.0
    for i in range(count):
        fam = ("laplace", "gradient", "termdoc")[int(rng.integers(3))]
        n = float(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))
        nb = int((1, 4, 8, 16)[int(rng.integers(4))])
        target = "dominant" if rng.random() < 0.5 else "minimal"
        t += float(rng.exponential(1.0 / rate))
        reqs.append(dict(id=i, family=fam, n=n, n_b=nb, target=target, arrival=t, seed=seed + 1 + i))
    return reqs


def serving_matrix(req: dict) -> tuple[CSR, str]:
    """Matrix and kind ('spd' or 'svd') of a serving request."""
    if req["family"] == "laplace":
        return laplace2d(max(4, int(round(math.sqrt(req["n"]))))), "spd"
    if req["family"] == "gradient":
        return gradient2d(max(4, int(round(math.sqrt(req["n"]))))), "svd"
    n = max(64, int(round(req["n"])))
    return termdoc(4 * n, n, 60, seed=req["seed"]), "svd"
