"""Whole-solve pins for the oracle's ARRABIT-MPM (Algorithm 8): closed-form
Laplacian spectra, brute-force dense diagonalization on small matrices, Weyl
bounds, and the invariants the result must satisfy (orthonormal vectors,
residuals within tolerance)."""
import numpy as np
import pytest

from oracle import arrabit as O
from paper_1507_06078_amd import workloads as W


def _check_invariants(A, r, k, tol):
    X = r.evecs
    np.testing.assert_allclose(X.T @ X, np.eye(k), atol=1e-11)
    rn = np.linalg.norm(A @ X - X * r.evals[None, :], axis=0)
    assert np.all(rn / np.maximum(1.0, np.abs(r.evals)) <= tol)


def test_c1_laplacian_closed_form():
    """2D Laplacian 40x40, k = 20 smallest, block 30, tol 1e-10: eigenvalues
    equal 4 - 2cos(pi i/41) - 2cos(pi j/41) (sorted)."""
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    r = O.arrabit_mpm(A.to_scipy(), k, tol, X0, which)
    assert r.status == 0
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    assert np.abs(r.evals - exact).max() <= 1e-10 * np.maximum(1, np.abs(exact)).max()
    _check_invariants(A.to_scipy(), r, k, tol)
    assert r.stats["arr_calls"] <= 30


@pytest.mark.parametrize("which", ["LA", "SA"])
def test_random_symmetric_vs_dense(which):
    n, k, w = 150, 6, 9
    A = W.random_symmetric(n, seed=31, density=0.2).to_scipy()
    lam = np.linalg.eigvalsh(A.toarray())
    exact = lam[::-1][:k] if which == "LA" else lam[:k]
    X0 = W.gaussian_block(n, w, seed=32)
    r = O.arrabit_mpm(A, k, 1e-10, X0, which)
    assert r.status == 0
    assert np.abs(r.evals - exact).max() <= 1e-9 * np.abs(lam).max()
    _check_invariants(A, r, k, 1e-10)


def test_3d_laplacian_potential_weyl_and_dense():
    """7-point Laplacian 10^3 plus V ~ U[0,1): compare with dense
    diagonalization and with Weyl's bounds lambda_i(L) <= lambda_i(L+V) <= lambda_i(L)+1."""
    A = W.laplacian_3d(10, potential_seed=1).to_scipy()
    k, w = 12, 16
    X0 = W.gaussian_block(1000, w, seed=2)
    r = O.arrabit_mpm(A, k, 1e-10, X0, "SA")
    assert r.status == 0
    lam = np.linalg.eigvalsh(A.toarray())[:k]
    assert np.abs(r.evals - lam).max() <= 1e-10 * max(1.0, np.abs(lam).max())
    L0 = W.laplacian_3d_eigenvalues(10)[:k]
    assert np.all(L0 - 1e-12 <= r.evals) and np.all(r.evals <= L0 + 1.0 + 1e-12)
    _check_invariants(A, r, k, 1e-10)


def test_maxit_one_returns_best_pairs_not_converged():
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    r = O.arrabit_mpm(A.to_scipy(), k, tol, X0, which, O.Options(maxit=1))
    assert r.status == 1
    assert r.evecs.shape == (A.n, k) and np.isfinite(r.res).all()


def test_loose_tolerance_no_continuation():
    """tol > 1e-8: tol_1 = tol (continuation off); the result satisfies tol."""
    A, k, which, w, _ = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    r = O.arrabit_mpm(A.to_scipy(), k, 1e-6, X0, which)
    assert r.status == 0 and r.res.max() <= 1e-6
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    # Kato-Temple-type bound: eigenvalue error ~ residual^2 / gap, far below 1e-6
    assert np.abs(r.evals - exact).max() < 1e-8
