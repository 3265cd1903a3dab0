"""Pins for the oracle's Rayleigh-Ritz (Algorithm 1), augmented RR (Algorithm 5),
rcond (eq. inn-stop), Lanczos interval estimate and residuals (eq. resi).
Checks use closed forms, hand-computed values and theorems (Ky Fan, Cauchy
interlacing, Galerkin orthogonality) rather than the oracle's own formulas."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arrabit as O
from paper_1507_06078_amd import workloads as W


def test_rcond_hand_value():
    # G = [[2,1],[1,2]]: ||G||_1 = 3, G^-1 = [[2,-1],[-1,2]]/3, ||G^-1||_1 = 1
    L = np.linalg.cholesky(np.array([[2.0, 1.0], [1.0, 2.0]]))
    X = np.vstack([L.T, np.zeros((3, 2))])  # X^T X = L L^T = G
    assert abs(O.rcond_gram(X) - 1.0 / 3.0) < 1e-15


def test_rcond_diagonal_and_singular():
    s = np.array([3.0, 0.5, 2.0, 1e-3])
    X = np.vstack([np.diag(s), np.zeros((4, 4))])
    assert abs(O.rcond_gram(X) - (1e-3) ** 2 / 9.0) < 1e-18
    Xs = np.ones((10, 3))  # rank 1: Gram not positive definite
    assert O.rcond_gram(Xs) == 0.0


def test_full_space_rr_gives_exact_spectrum():
    """An RR step on a basis of the whole space returns every eigenvalue:
    compare with the closed form of the 2D Laplacian (m = 6, n = 36)."""
    A = W.laplacian_2d(6).to_scipy()
    Z = W.gaussian_block(36, 36, seed=3)
    Y, sig = O.rayleigh_ritz(A, Z)
    exact = W.laplacian_2d_eigenvalues(6)[::-1]
    np.testing.assert_allclose(sig, exact, atol=1e-12)
    np.testing.assert_allclose(Y.T @ Y, np.eye(36), atol=1e-12)


def test_rr_ky_fan_interlacing_and_galerkin():
    A = W.laplacian_3d(5, potential_seed=4).to_scipy()   # n = 125
    lam = np.sort(np.linalg.eigvalsh(A.toarray()))[::-1]
    Z = W.gaussian_block(125, 12, seed=5)
    Y, sig = O.rayleigh_ritz(A, Z)
    # Cauchy interlacing: mu_i <= lambda_i (descending order), Ky Fan on partial sums
    assert np.all(sig <= lam[:12] + 1e-12)
    assert np.all(np.cumsum(sig) <= np.cumsum(lam[:12]) + 1e-11)
    # Galerkin condition: residuals orthogonal to the trial space
    U, _ = np.linalg.qr(Z)
    R = A @ Y - Y * sig[None, :]
    assert np.abs(U.T @ R).max() < 1e-12
    np.testing.assert_allclose(Y.T @ Y, np.eye(12), atol=1e-12)


def test_arr_p0_is_rr():
    A = W.random_symmetric(60, seed=11).to_scipy()
    X = W.gaussian_block(60, 7, seed=12)
    Y1, s1 = O.augmented_rr(A, X, 0)
    Y2, s2 = O.rayleigh_ritz(A, X)
    np.testing.assert_allclose(s1, s2, atol=1e-13)


def test_arr_krylov_augmentation_captures_two_eigenvectors():
    """A = diag(1..n), x = e_1 + e_2: RR on x alone yields the single Ritz value
    (1+2)/2, while ARR with p = 1 spans {e_1, e_2} and returns 2 and 1 exactly."""
    n = 20
    A = sp.diags(np.arange(1.0, n + 1), 0, format="csr")
    x = np.zeros((n, 1))
    x[0, 0] = x[1, 0] = 1.0
    _, s0 = O.augmented_rr(A, x, 0)
    assert abs(s0[0] - 1.5) < 1e-14
    Y, s1 = O.augmented_rr(A, x, 1)
    np.testing.assert_allclose(np.sort(s1), [1.0, 2.0], atol=1e-13)


def test_arr_projection_keeps_complement():
    """With Qc given, ARR works in R(Qc)^perp: Ritz vectors are orthogonal to Qc
    (Sec. 6, Deflation)."""
    A = W.random_symmetric(80, seed=21).to_scipy()
    lam, Q = np.linalg.eigh(A.toarray())
    Qc = Q[:, -3:]
    X = W.gaussian_block(80, 5, seed=22)
    Y, sig = O.augmented_rr(A, O.project_out(Qc, X), 1, Qc)
    assert np.abs(Qc.T @ Y).max() < 1e-12
    assert sig.max() < lam[-3] + 1e-12  # the locked top-3 cannot reappear


def test_lanczos_bounds_laplacian():
    """Extreme Ritz values of 100 Lanczos steps on the 40x40 Laplacian approach
    the closed-form extremes from inside; a stays below lambda_min."""
    A = W.laplacian_2d(40).to_scipy()
    ex = W.laplacian_2d_eigenvalues(40)
    v0 = W.gaussian_block(1600, 1, seed=2)[:, 0]
    tmin, tmax, r = O.lanczos_extremes(A, v0, 100)
    assert ex[0] - 1e-12 <= tmin and tmax <= ex[-1] + 1e-12
    assert abs(tmax - ex[-1]) < 1e-6  # 7.988263..., the norm
    a, nrm = O.lower_end_estimate(-A, v0, 100)
    assert a <= -ex[-1]
    assert abs(nrm - 7.988263204735) < 1e-6


def test_lanczos_small_invariant_subspace():
    A = sp.diags([1.0, 2.0, 3.0, 4.0], 0, format="csr")
    v0 = np.array([1.0, 1.0, 0.0, 0.0])
    tmin, tmax, r = O.lanczos_extremes(A, v0, 10)
    assert abs(tmin - 1.0) < 1e-14 and abs(tmax - 2.0) < 1e-14 and r < 1e-12


def test_residuals_scaling():
    A = sp.diags([0.5, -3.0, 2.0], 0, format="csr")
    X = np.eye(3)
    mu = np.array([0.5, -3.0, 1.0])  # last pair is off by 1 in value
    res = O.relative_residuals(A, X, mu)
    np.testing.assert_allclose(res, [0.0, 0.0, 1.0 / 1.0], atol=1e-15)
    mu2 = np.array([0.5, -2.0, 2.0])  # second pair off by 1, |mu| = 2
    np.testing.assert_allclose(O.relative_residuals(A, X, mu2), [0.0, 0.5, 0.0], atol=1e-15)
