"""Pins for the oracle's classic Chebyshev filter (eq. cheby-poly, the
alternative to psi_d compared in Table comp-cheby). Each check uses something
other than the oracle's recursion: the trigonometric and hyperbolic closed
forms of T_d, numpy's Chebyshev-series evaluation, the spectral identity
rho(A) = Q rho(Lambda) Q^T (eq. poly-A), and closed-form Laplacian spectra for
a whole solve in this mode."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import arrabit as O
from paper_1507_06078_amd import workloads as W


@pytest.mark.parametrize("d", [0, 1, 2, 3, 7, 15])
def test_T_closed_forms(d):
    """T_d(cos th) = cos(d th) on [-1, 1]; T_d(cosh u) = cosh(d u) and
    T_d(-x) = (-1)^d T_d(x) outside it."""
    th = np.linspace(0.0, np.pi, 41)
    np.testing.assert_allclose(O.chebyshev_T(np.cos(th), d), np.cos(d * th), atol=1e-12)
    u = np.linspace(0.0, 2.0, 21)
    x = np.cosh(u)
    np.testing.assert_allclose(O.chebyshev_T(x, d), np.cosh(d * u), rtol=1e-12)
    np.testing.assert_allclose(O.chebyshev_T(-x, d), (-1) ** d * np.cosh(d * u), rtol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 5, 12])
def test_T_matches_numpy_chebval(d):
    x = np.linspace(-1.5, 3.0, 101)
    coef = np.zeros(d + 1)
    coef[d] = 1.0
    np.testing.assert_allclose(O.chebyshev_T(x, d), C.chebval(x, coef), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3, 8, 15])
def test_block_filter_is_T_of_the_mapped_spectrum(d):
    """chebyshev_poly(A - aI, X, 0, b - a, d) = Q T_d(x(Lambda)) Q^T X with
    x(l) = (2(l - a) - (b - a))/(b - a), from a dense eigendecomposition."""
    A = W.random_symmetric(60, seed=5, density=0.3).to_scipy()
    lam, Q = np.linalg.eigh(A.toarray())
    a, b = lam[0] - 0.05, lam[-8]
    X = W.gaussian_block(60, 7, seed=6)
    got = O.chebyshev_poly(O.shifted(A, a), X, 0.0, b - a, d)
    x = (2.0 * (lam - a) - (b - a)) / (b - a)
    coef = np.zeros(d + 1)
    coef[d] = 1.0
    ref = Q @ (C.chebval(x, coef)[:, None] * (Q.T @ X))
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_rho_chebyshev_maps_interval_onto_unit_range():
    """|T_d| <= 1 on the damped interval [a, b]; T_d(1) = 1 at its upper end,
    T_d(-1) = (-1)^d at the lower one."""
    a, b = -3.0, 2.0
    t = np.linspace(a, b, 301)
    for d in (3, 9):
        assert np.all(np.abs(O.rho_chebyshev(t, a, b, d)) <= 1.0 + 1e-12)
        assert abs(O.rho_chebyshev(b, a, b, d) - 1.0) < 1e-12
        assert abs(O.rho_chebyshev(a, a, b, d) - (-1) ** d) < 1e-12


@pytest.mark.parametrize("inner", ["mpm", "gn"])
def test_whole_solve_chebyshev_mode_closed_form(inner):
    """Algorithm 8 with T_d in place of psi_d (and the degree rule evaluated on
    T_d) reaches the closed-form spectrum of the 2D Laplacian."""
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    r = O.arrabit_mpm(A.to_scipy(), k, tol, X0, which, O.Options(poly="chebyshev", inner=inner))
    assert r.status == 0
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    assert np.abs(r.evals - exact).max() <= 1e-10 * np.maximum(1, np.abs(exact)).max()
    X = r.evecs
    np.testing.assert_allclose(X.T @ X, np.eye(k), atol=1e-11)
    rn = np.linalg.norm(A.to_scipy() @ X - X * r.evals[None, :], axis=0)
    assert np.all(rn / np.maximum(1.0, np.abs(r.evals)) <= tol)


def test_degree_rule_in_chebyshev_mode():
    """eq. hat-d on T_d: the smallest d >= 3 with |T_d(x_w)/T_d(x_k)| < 0.9,
    checked against cosh closed forms for points above the interval."""
    a, b = 0.0, 1.0
    mu_k, mu_w = 1.02, 1.01  # x = 1.04 and 1.02
    d = O.degree_update(mu_k, mu_w, a, b, 15, rho_d=lambda t, dd: O.rho_chebyshev(t, a, b, dd))
    xk, xw = 2 * mu_k - 1, 2 * mu_w - 1
    ratio = lambda dd: np.cosh(dd * np.arccosh(xw)) / np.cosh(dd * np.arccosh(xk))
    expect = next((dd for dd in range(3, 16) if ratio(dd) < 0.9), 15)
    assert d == expect
