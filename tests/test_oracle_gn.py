"""Pins of the oracle's Gauss-Newton inner solver (Sec. 2.6, GN branch of
Algorithm 8), each independent of the oracle's own formula:

* the algorithm's update Z - X (Y^T Z - I)/2 equals the closed-form GN step
  with unit step printed in Sec. 2.6, X + (I - X G^{-1} X^T / 2)(M X G^{-1} - X),
  G = X^T X (a different algebraic form of the same map);
* X* = Q_k Lambda_k^{1/2} R (top-k eigenvectors scaled by the square roots of
  the eigenvalues, R orthogonal) is a fixed point, as the minimizer of
  ||X X^T - M||_F over rank-k X;
* a block spanning an invariant subspace keeps spanning it;
* iterating from a random block converges to the dominant subspace;
* Algorithm 8 with the GN inner solver reproduces the closed-form spectrum of
  the 2D Laplacian and the dense eigensolver on a random matrix."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import arrabit as O
from paper_1507_06078_amd import workloads as W


def spd(n, seed, gap_at=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(0.1, 1.0, n))[::-1]
    if gap_at is not None:
        lam[:gap_at] += 2.0
    return Q, lam, (Q * lam) @ Q.T


def test_update_equals_closed_form_of_sec4():
    rng = np.random.default_rng(1)
    _, _, M = spd(40, 2)
    X = rng.standard_normal((40, 6))
    G = X.T @ X
    Gi = np.linalg.inv(G)
    closed = X + (np.eye(40) - 0.5 * X @ Gi @ X.T) @ (M @ X @ Gi - X)
    got = O.gn_update(X, lambda Y: M @ Y)
    assert np.abs(got - closed).max() <= 1e-12 * np.abs(closed).max()


def test_scaled_top_eigenvectors_are_a_fixed_point():
    Q, lam, M = spd(30, 3)
    k = 5
    R, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((k, k)))
    Xs = Q[:, :k] * np.sqrt(lam[:k])[None, :] @ R
    got = O.gn_update(Xs, lambda Y: M @ Y)
    assert np.abs(got - Xs).max() <= 1e-12


def test_invariant_subspace_is_kept():
    Q, lam, M = spd(30, 5)
    rng = np.random.default_rng(6)
    X = Q[:, [2, 7, 11]] @ rng.standard_normal((3, 3))
    got = O.gn_update(X, lambda Y: M @ Y)
    # residual of projecting onto span(Q[:, [2, 7, 11]]) vanishes
    P = Q[:, [2, 7, 11]]
    assert np.abs(got - P @ (P.T @ got)).max() <= 1e-12 * np.abs(got).max()


def test_converges_to_dominant_subspace():
    Q, lam, M = spd(60, 7, gap_at=4)
    X = np.random.default_rng(8).standard_normal((60, 4))
    for _ in range(60):
        X = O.gn_update(X, lambda Y: M @ Y)
    Ux, _ = np.linalg.qr(X)
    s = sla.svdvals(Q[:, :4].T @ Ux)
    assert s.min() > 1 - 1e-10
    # and X X^T approaches the rank-4 part of M
    M4 = (Q[:, :4] * lam[:4]) @ Q[:, :4].T
    assert np.abs(X @ X.T - M4).max() <= 1e-8


def test_whole_solve_gn_c1_closed_form():
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    r = O.arrabit_mpm(A.to_scipy(), k, 1e-12, X0, which, O.Options(inner="gn"))
    assert r.status == 0
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    assert np.all(np.abs(r.evals - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))
    assert np.all(r.res <= 1e-12 * 1.0001)


@pytest.mark.parametrize("which", ["LA", "SA"])
def test_whole_solve_gn_random_vs_dense(which):
    A = W.random_symmetric(300, seed=31, density=0.1)
    lam = np.linalg.eigvalsh(A.to_scipy().toarray())
    k, w = 8, 12
    exact = lam[::-1][:k] if which == "LA" else lam[:k]
    X0 = W.gaussian_block(A.n, w, seed=3)
    r = O.arrabit_mpm(A.to_scipy(), k, 1e-11, X0, which, O.Options(inner="gn"))
    assert r.status == 0
    assert np.abs(r.evals - exact).max() <= 1e-10 * np.abs(lam).max()
