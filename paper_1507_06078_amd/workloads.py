"""Seeded synthetic inputs for the eigensolver: sparse symmetric matrices in CSR
form and Gaussian starting blocks.

This module only *generates inputs*. It holds none of the eigensolver's
arithmetic, so both the CPU oracle and the GPU library can be fed from it
without sharing any of the method.

The paper evaluates on matrices from the University of Florida collection,
which are not available here; the generators below stand in for them with
matrices of the shapes and structures named by the benchmark workloads:

* 2D 5-point and 3D 7-point Dirichlet Laplacians (optionally plus a diagonal
  potential drawn uniform on [0, 1)), lexicographic ordering;
* a random sparse symmetric matrix with power-law row lengths
  (Chung-Lu style sampling), N(0,1) off-diagonal values, N(0, var 4) diagonal;
* the normalized Laplacian of a stochastic block model graph;
* small dense random symmetric matrices (for brute-force comparisons).

All matrices are returned as :class:`CSR` with 0-based int64 row pointers,
int32 column indices (sorted within each row, both triangles stored, explicit
diagonal) and float64 values.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    colind: np.ndarray  # int32 [nnz]
    val: np.ndarray     # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def negated(self) -> "CSR":
        return CSR(self.n, self.rowptr, self.colind, -self.val, self.name + "(neg)")


def from_scipy(M, name: str = "") -> CSR:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    return CSR(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32),
               M.data.astype(np.float64), name)


def _tridiag_second_difference(m: int) -> sp.csr_matrix:
    e = np.ones(m)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplacian_2d(m: int) -> CSR:
    """5-point Dirichlet Laplacian on an m x m grid (diag 4, neighbours -1)."""
    T = _tridiag_second_difference(m)
    I = sp.identity(m, format="csr")
    L = sp.kron(I, T) + sp.kron(T, I)
    return from_scipy(L, f"lap2d_m{m}")


def laplacian_3d(m: int, potential_seed: int | None = None) -> CSR:
    """7-point Dirichlet Laplacian on an m^3 grid (diag 6, neighbours -1), plus an
    optional diagonal potential V_i ~ U[0, 1) drawn from ``potential_seed``."""
    T = _tridiag_second_difference(m)
    I = sp.identity(m, format="csr")
    L = sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I))
    L = sp.csr_matrix(L)
    name = f"lap3d_m{m}"
    if potential_seed is not None:
        V = np.random.default_rng(potential_seed).random(m ** 3)
        L = L + sp.diags(V, 0, format="csr")
        name += f"+V(seed{potential_seed})"
    return from_scipy(L, name)


def laplacian_2d_potential(m: int, potential_seed: int) -> CSR:
    """2D 5-point Laplacian plus a diagonal potential V_i ~ U[0, 1)."""
    A = laplacian_2d(m).to_scipy()
    V = np.random.default_rng(potential_seed).random(m * m)
    return from_scipy(A + sp.diags(V, 0, format="csr"), f"lap2d_m{m}+V(seed{potential_seed})")


def laplacian_2d_eigenvalues(m: int) -> np.ndarray:
    """Closed-form spectrum of :func:`laplacian_2d`, ascending:
    4 - 2cos(pi i/(m+1)) - 2cos(pi j/(m+1)), i, j = 1..m."""
    c = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, m + 1) / (m + 1))
    return np.sort((c[:, None] + c[None, :]).ravel())


def laplacian_3d_eigenvalues(m: int) -> np.ndarray:
    """Closed-form spectrum of :func:`laplacian_3d` without potential, ascending."""
    c = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, m + 1) / (m + 1))
    return np.sort((c[:, None, None] + c[None, :, None] + c[None, None, :]).ravel())


def powerlaw_random(n: int, seed: int, alpha: float = 2.1, mean_deg: float = 16.0,
                    cap: int = 2048) -> CSR:
    """Random sparse symmetric matrix with power-law row lengths.

    Target row lengths are drawn from a Pareto(alpha) law truncated at ``cap``
    whose x_min is calibrated so that the truncated mean is ``mean_deg``.
    Edges are sampled Chung-Lu style: both endpoints of each of
    sum(weights)/2 edges are drawn proportionally to the weights; self loops
    are dropped and duplicates merged. Each unordered off-diagonal pair gets an
    N(0,1) value (mirrored), the diagonal is N(0, variance 4).
    """
    rng = np.random.default_rng(seed)
    # truncated Pareto mean: solve for x_min by bisection on the closed form
    def tmean(xm):
        # E[min(X, cap)] for Pareto(alpha, xm)
        if cap <= xm:
            return float(cap)
        return (alpha * xm / (alpha - 1.0)) * (1.0 - (xm / cap) ** (alpha - 1.0)) + cap * (xm / cap) ** alpha
    lo, hi = 1e-3, float(cap)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if tmean(mid) < mean_deg:
            lo = mid
        else:
            hi = mid
    xm = 0.5 * (lo + hi)
    u = rng.random(n)
    wts = np.minimum(xm * (1.0 - u) ** (-1.0 / alpha), float(cap))
    n_edges = int(round(wts.sum() / 2.0))
    p = wts / wts.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    src = np.searchsorted(cdf, rng.random(n_edges), side="right").astype(np.int64)
    dst = np.searchsorted(cdf, rng.random(n_edges), side="right").astype(np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo_i, hi_i = np.minimum(src, dst), np.maximum(src, dst)
    key = np.unique(lo_i * n + hi_i)
    r, c = key // n, key % n
    vals = rng.standard_normal(key.size)
    diag = 2.0 * rng.standard_normal(n)
    rows = np.concatenate([r, c, np.arange(n)])
    cols = np.concatenate([c, r, np.arange(n)])
    data = np.concatenate([vals, vals, diag])
    M = sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    return from_scipy(M, f"powerlaw_n{n}_seed{seed}")


def sbm_normalized_laplacian(n: int, n_blocks: int, seed: int, avg_deg: float = 20.0,
                             ratio: float = 10.0) -> CSR:
    """Normalized Laplacian I - D^-1/2 W D^-1/2 of a stochastic block model graph
    with ``n_blocks`` contiguous equal blocks, p_in/p_out = ``ratio`` and expected
    average degree ``avg_deg``. Isolated vertices keep L_ii = 1."""
    rng = np.random.default_rng(seed)
    s = n // n_blocks
    assert s * n_blocks == n
    # expected degree: (s-1) p_in + (n-s) p_out = avg_deg with p_in = ratio p_out
    p_out = avg_deg / (ratio * (s - 1) + (n - s))
    p_in = ratio * p_out
    pairs_in = n_blocks * s * (s - 1) // 2
    pairs_out = (n * n - n_blocks * s * s) // 2
    m_in = rng.binomial(pairs_in, p_in)
    m_out = rng.binomial(pairs_out, p_out)
    b = rng.integers(0, n_blocks, m_in)
    u = b * s + rng.integers(0, s, m_in)
    v = b * s + rng.integers(0, s, m_in)
    keep = u != v
    u_in, v_in = u[keep], v[keep]
    u = rng.integers(0, n, 2 * m_out + 16)
    v = rng.integers(0, n, 2 * m_out + 16)
    keep = (u // s) != (v // s)
    u_out, v_out = u[keep][:m_out], v[keep][:m_out]
    src = np.concatenate([u_in, u_out]).astype(np.int64)
    dst = np.concatenate([v_in, v_out]).astype(np.int64)
    lo_i, hi_i = np.minimum(src, dst), np.maximum(src, dst)
    key = np.unique(lo_i * n + hi_i)
    r, c = key // n, key % n
    deg = np.bincount(r, minlength=n) + np.bincount(c, minlength=n)
    dinv = np.zeros(n)
    nz = deg > 0
    dinv[nz] = 1.0 / np.sqrt(deg[nz])
    off = -dinv[r] * dinv[c]
    rows = np.concatenate([r, c, np.arange(n)])
    cols = np.concatenate([c, r, np.arange(n)])
    data = np.concatenate([off, off, np.ones(n)])
    M = sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    return from_scipy(M, f"sbm_n{n}_b{n_blocks}_seed{seed}")


def random_symmetric(n: int, seed: int, density: float = 1.0) -> CSR:
    """Random symmetric matrix with N(0,1) entries (symmetrised), optionally
    sparsified; the diagonal is always stored."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    if density < 1.0:
        G = G * (rng.random((n, n)) < density)
    S = np.triu(G, 1)
    S = S + S.T + np.diag(rng.standard_normal(n))
    M = sp.csr_matrix(S)
    # keep explicit diagonal even if zero
    M = M + sp.diags(np.zeros(n), 0)
    M = sp.csr_matrix(M)
    return from_scipy(M, f"randsym_n{n}_seed{seed}")


def gaussian_block(n: int, w: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) block of shape (n, w), C-contiguous (row-major)."""
    return np.random.default_rng(seed).standard_normal((n, w)).astype(dtype, copy=False)


# Named workloads --------------------------------------------------------------

def workload(name: str):
    """Return (CSR, k, which, w, tol) for a named workload.

    ``which`` is 'SA' (smallest algebraic) or 'LA' (largest algebraic).
    """
    if name == "lap2d_40":          # n=1600, k=20 smallest, block 30, tol 1e-10
        return laplacian_2d(40), 20, "SA", 30, 1e-10
    if name == "lap3d_100_V":       # n=1e6, ~6.94e6 nnz, k=200 smallest, block 240
        return laplacian_3d(100, potential_seed=1), 200, "SA", 240, 1e-10
    if name.startswith("lap3d_") and name.endswith("_V"):   # down-scaled versions
        m = int(name.split("_")[1])
        return laplacian_3d(m, potential_seed=1), None, "SA", None, 1e-10
    raise KeyError(name)
