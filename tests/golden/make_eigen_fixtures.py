"""Writes oracle eigenvalue fixtures for the whole-solve parity tests at the
benchmark sizes. Calls only the oracle (oracle/arrabit.py) and the seeded input
generators (paper_1507_06078_amd/workloads.py).

Each case runs the oracle's Algorithm 8 (ARRABIT-MPM) at tol = 1e-12, two
orders tighter than the GPU tests' 1e-10, from the numpy Gaussian starting
block of seed 2 (the GPU solves start from their own device draw, so the two
sides share no iterate), and stores the k eigenvalues with their residuals in
the eq. resi scaling.

Independent checks:
- the 3D stencil (spectrum slicing): by Sylvester's law of inertia the number
  of negative pivots of an LDL^T factorization of A - sigma I equals the
  number of eigenvalues of A below sigma. With sigma halfway between the k-th
  returned eigenvalue and the next Ritz value of the oracle's last iteration,
  that count must be exactly k, so no eigenvalue was skipped. The
  factorization is SuperLU's in symmetric mode with diagonal pivots only (a
  symmetric ordering, so its U has D on the diagonal), in a nested-dissection
  order of the grid;
- the random graphs, whose factorizations fill in almost completely: the
  implicitly restarted Lanczos method (ARPACK through scipy's eigsh, a Krylov
  method sharing nothing with the oracle's block iteration) from a seeded
  start, for the k largest eigenvalues of A (power-law) or of 2I - A (the
  normalized Laplacian, whose spectrum lies in [0, 2]); both value sets must
  agree to 1e-10 max(1, |lambda|).

Run from the repository root, one case at a time (the benchmark case holds
about 40 GB and runs for about an hour on 8 cores):
    python tests/golden/make_eigen_fixtures.py lap3d100|powerlaw1e5|sbm1e5
"""
import os
import platform
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import arrabit as O  # noqa: E402
from paper_1507_06078_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name: (matrix builder, description, k, which, block width)
CASES = {
    "lap3d100": (lambda: W.laplacian_3d(100, potential_seed=1),
                 "3D 7-point Dirichlet Laplacian 100^3 + diagonal U[0,1) potential (seed 1), n = 1e6",
                 200, "SA", 240),
    "powerlaw1e5": (lambda: W.powerlaw_random(100_000, seed=1),
                    "random symmetric, power-law row lengths (Pareto 2.1, mean 16, cap 2048; seed 1), "
                    "N(0,1) off-diagonal, N(0,4) diagonal, n = 1e5",
                    100, "LA", 120),
    "sbm1e5": (lambda: W.sbm_normalized_laplacian(64 * 1563, 64, seed=1),
               "normalized Laplacian of a stochastic block model graph, 64 blocks of 1563, average degree 20, "
               "p_in/p_out = 10 (seed 1), n = 100032",
               100, "SA", 120),
}
TOL = 1e-12
X0_SEED = 2


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        return None


def nested_dissection_3d(m: int) -> np.ndarray:
    """Nested-dissection order of the m^3 lexicographic grid (index z m^2 + y m
    + x): each box is split by the middle plane of its longest side, the two
    halves are ordered first and the plane last. Used only to keep the fill of
    the factorization below small enough for the 100^3 grid."""
    order = []

    def box(lo, hi):
        z, y, x = np.meshgrid(*(np.arange(lo[i], hi[i]) for i in range(3)), indexing="ij")
        return (z * m * m + y * m + x).ravel()

    def rec(lo, hi):
        ext = [hi[i] - lo[i] for i in range(3)]
        if min(ext) <= 0:
            return
        if ext[0] * ext[1] * ext[2] <= 64:
            order.append(box(lo, hi))
            return
        ax = int(np.argmax(ext))
        mid = (lo[ax] + hi[ax]) // 2
        rec(lo, tuple(mid if i == ax else hi[i] for i in range(3)))
        rec(tuple(mid + 1 if i == ax else lo[i] for i in range(3)), hi)
        order.append(box(tuple(mid if i == ax else lo[i] for i in range(3)),
                         tuple(mid + 1 if i == ax else hi[i] for i in range(3))))

    rec((0, 0, 0), (m, m, m))
    p = np.concatenate(order)
    assert p.size == m ** 3 and np.unique(p).size == m ** 3
    return p


def inertia_below(A: sp.csr_matrix, sigma: float, perm=None) -> int:
    """Number of eigenvalues of symmetric A below sigma (Sylvester's law of
    inertia on a symmetric LDL^T-type factorization of A - sigma I). ``perm``
    is a symmetric ordering applied before factorizing (else minimum degree on
    A + A^T)."""
    n = A.shape[0]
    M = A - sigma * sp.identity(n, format="csr")
    if perm is not None:
        M = M[perm][:, perm]
    M = sp.csc_matrix(M)
    lu = spla.splu(M, permc_spec="NATURAL" if perm is not None else "MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    # symmetric ordering (perm_r == perm_c) means U's diagonal is D of L D L^T
    assert np.array_equal(lu.perm_r, lu.perm_c), "factorization used row pivoting"
    return int((lu.U.diagonal() < 0).sum())


def run(name):
    build, desc, k, which, w = CASES[name]
    A = build()
    S = A.to_scipy()
    X0 = W.gaussian_block(A.n, w, seed=X0_SEED)
    t0 = time.perf_counter()
    r = O.arrabit_mpm(S, k, TOL, X0, which)
    wall = time.perf_counter() - t0
    del X0
    # spectrum slicing: sigma between lambda_k and the next Ritz value
    mu = r.history[-1]["mu"]  # the w merged Ritz values of the working operator, descending
    nxt = -mu[k] if which == "SA" else mu[k]
    lam_k = r.evals[k - 1]
    sigma = 0.5 * (lam_k + nxt)
    t1 = time.perf_counter()
    del r.history[:-1]
    if name == "lap3d100":
        below = inertia_below(S, sigma, nested_dissection_3d(100))
        expect_below = k
        check = f"spectrum slicing: {below} eigenvalues below sigma = {sigma:.17g} (expected {expect_below})"
        passed = below == expect_below
    else:
        v0 = np.random.default_rng(X0_SEED).standard_normal(A.n)
        if which == "SA":  # normalized Laplacian: smallest of A = 2 - largest of 2I - A
            M = 2.0 * sp.identity(A.n, format="csr") - S
            th = spla.eigsh(M, k=k, which="LA", tol=1e-14, ncv=3 * k, v0=v0, return_eigenvectors=False)
            ref = np.sort(2.0 - th)
        else:
            th = spla.eigsh(S, k=k, which="LA", tol=1e-14, ncv=3 * k, v0=v0, return_eigenvectors=False)
            ref = np.sort(th)[::-1]
        dev = float(np.max(np.abs(ref - r.evals) / np.maximum(1.0, np.abs(ref))))
        check = f"ARPACK (eigsh, ncv {3 * k}, tol 1e-14) agrees to max |dlambda| / max(1, |lambda|) = {dev:.2e}"
        passed = dev <= 1e-10
    t_inertia = time.perf_counter() - t1
    lines = [
        f"# Oracle eigenvalues: {desc}",
        f"# k = {k} {'smallest' if which == 'SA' else 'largest'}, block {w}, oracle tol {TOL:g}, "
        f"starting block numpy Gaussian seed {X0_SEED}",
        f"# Written by tests/golden/make_eigen_fixtures.py {name} (oracle/arrabit.py, Algorithm 8 with MPM)",
        f"# oracle status {r.status}, outer iterations {r.stats['outer']}, ARR calls {r.stats['arr_calls']}, "
        f"block SpMM degrees {r.stats['spmm_degrees']}, max res (eq. resi) {r.res.max():.3e}",
        f"# oracle wall time {wall:.1f} s on {os.cpu_count()} cores ({cpu_model()}), "
        f"BLAS threads {blas_threads()}, sparse products single-threaded",
        f"# {check}; the check took {t_inertia:.1f} s",
        "# i lambda_i res_i",
    ]
    for i in range(k):
        lines.append(f"{i} {float(r.evals[i])!r} {float(r.res[i]):.3e}")
    path = os.path.join(HERE, f"eig_{name}.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:6]))
    print("wrote", path)
    assert r.status == 0, r.status
    assert passed, check


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["powerlaw1e5", "sbm1e5"]:
        run(nm)
