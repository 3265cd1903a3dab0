"""Pins for the oracle's polynomial accelerator (Sec. 5, eq. def:fN, eq. chebfun-f,
eq. rhod, Algorithm 7). Each check uses something other than the oracle's own
formula: a hand-derived closed form, barycentric Lagrange interpolation (a
different evaluation of the same interpolant), or the spectral identity
rho(A) = Q rho(Lambda) Q^T (eq. poly-A)."""
import numpy as np
import pytest
from scipy.interpolate import BarycentricInterpolator

from oracle import arrabit as O
from paper_1507_06078_amd import workloads as W


def test_nodes_are_second_kind_chebyshev_points():
    t = O.interpolation_nodes(4)
    # -cos(j pi / 4): -1, -1/sqrt2, 0, 1/sqrt2, 1 (written out by hand)
    s = np.sqrt(0.5)
    np.testing.assert_allclose(t, [-1.0, -s, 0.0, s, 1.0], atol=1e-15)


def test_target_function_values():
    # f_d(t) = max(0,t)^(10 d): f_2(0.5) = 2^-20, f_1(-0.3) = 0, f_3(1) = 1
    assert O.target_function(0.5, 2) == 2.0 ** -20
    assert O.target_function(-0.3, 1) == 0.0
    assert O.target_function(1.0, 3) == 1.0


def test_psi3_closed_form():
    """psi_3 interpolates (-1,0), (-1/2,0), (1/2, 2^-30), (1,1). By Lagrange
    (derived by hand): psi_3 = (t+1)(t^2-1/4)/1.5 - 2^-30 (t^2-1)(t+1/2)/0.75,
    i.e. gamma = [2/3, 2/3, -1/6, -1/6] + 2^-30 [-4/3, -2/3, 4/3, 2/3]."""
    e = 2.0 ** -30
    expect = np.array([2 / 3 - 4 * e / 3, 2 / 3 - 2 * e / 3, -1 / 6 + 4 * e / 3, -1 / 6 + 2 * e / 3])
    np.testing.assert_allclose(O.interpolant_coefficients(3), expect, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("d", [3, 4, 5, 8, 11, 15])
def test_interpolant_matches_barycentric_lagrange(d):
    """The monomial coefficients describe the same polynomial as barycentric
    Lagrange interpolation through the nodes (an independent evaluation)."""
    t = O.interpolation_nodes(d)
    bary = BarycentricInterpolator(t, O.target_function(t, d))
    g = O.interpolant_coefficients(d)
    x = np.linspace(-1.1, 1.1, 301)
    ref = bary(x)
    got = O.psi(x, g)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(got - ref).max() <= 2e-10 * scale
    # psi_d(1) = f_d(1) = 1 and psi_d vanishes at the non-positive nodes (Sec. 5)
    assert abs(O.psi(1.0, g) - 1.0) < 1e-11
    assert np.abs(O.psi(t[t <= 0], g)).max() < 1e-11


@pytest.mark.parametrize("d,maxabs,at11,atm105", [
    (3, 0.468, 1.344, -0.028), (5, 0.203, 2.080, -0.036),
    (8, 0.169, 4.96, 0.060), (15, 0.080, 55.7, -0.272)])
def test_interpolant_profile(d, maxabs, at11, atm105):
    """Low profile on [-1, 0.8] (Sec. 5: away from the right end the
    interpolant stays at about 0.2 in magnitude or below); values computed
    independently with barycentric interpolation, 3 significant digits."""
    t = O.interpolation_nodes(d)
    bary = BarycentricInterpolator(t, O.target_function(t, d))
    g = O.interpolant_coefficients(d)
    x = np.linspace(-1.0, 0.8, 4001)
    assert abs(np.abs(O.psi(x, g)).max() - np.abs(bary(x)).max()) < 1e-9
    assert abs(np.abs(O.psi(x, g)).max() - maxabs) < 1.5e-3
    assert abs(float(O.psi(1.1, g)) - at11) < 5e-3 * max(1, abs(at11))
    assert abs(float(O.psi(-1.05, g)) - atm105) < 1.5e-3


@pytest.mark.parametrize("d,q,rtol", [(3, 0.7, 1e-11), (6, 0.7, 1e-11), (10, 0.8, 1e-10),
                                      (15, 0.9, 1e-9), (15, 0.7, 1e-6)])
def test_poly_equals_spectral_definition(d, q, rtol):
    """Algorithm 7 computes rho_d(A) X; compare with Q rho_d(Lambda) Q^T X
    (eq. poly-A) using a dense eigendecomposition and barycentric evaluation of
    psi_d at the mapped eigenvalues (no use of the monomial coefficients)."""
    A = W.random_symmetric(40, seed=5).to_scipy().toarray()
    lam, Q = np.linalg.eigh(A)
    # q sets how far the top eigenvalues map beyond 1 (up to t = 2.1 for q = 0.7),
    # where monomial evaluation of psi_15 (values ~1e7) loses digits
    a, b = lam[0] - 0.05, np.quantile(lam, q)
    X = W.gaussian_block(40, 6, seed=6)
    t = O.interpolation_nodes(d)
    bary = BarycentricInterpolator(t, O.target_function(t, d))
    rho_lam = bary((2 * lam - a - b) / (b - a))
    ref = Q @ (rho_lam[:, None] * (Q.T @ X))
    got = O.poly(lambda Y: A @ Y, X, a, b, O.interpolant_coefficients(d))
    assert np.abs(got - ref).max() <= rtol * np.abs(ref).max()


def test_poly_shifted_operator_is_same_polynomial():
    """Algorithm 8 calls poly(A - aI, X, 0, b - a): the mapped variable
    (2(t-a) - (b-a))/(b-a) equals (2t - a - b)/(b - a), so the result is
    rho_d(A) X on [a, b]."""
    A = W.random_symmetric(30, seed=8).to_scipy()
    lam, Q = np.linalg.eigh(A.toarray())
    a, b = lam[0] - 0.1, lam[15]
    X = W.gaussian_block(30, 4, seed=9)
    g = O.interpolant_coefficients(7)
    direct = O.poly(lambda Y: A @ Y, X, a, b, g)
    via_shift = O.poly(O.shifted(A, a), X, 0.0, b - a, g)
    np.testing.assert_allclose(via_shift, direct, rtol=1e-11, atol=1e-11 * np.abs(direct).max())


def test_degree_update_rule():
    """eq. hat-d: smallest d >= 3 with |rho_d(mu_w)/rho_d(mu_k)| < 0.9, capped.
    Expected d found by scanning barycentric evaluations."""
    a, b = 0.0, 1.0
    for mu_k, mu_w, dmax in [(1.3, 1.0, 15), (1.05, 1.0, 15), (1.001, 1.0, 15), (1.2, 1.1, 6)]:
        expect = dmax
        for d in range(3, dmax + 1):
            t = O.interpolation_nodes(d)
            bary = BarycentricInterpolator(t, O.target_function(t, d))
            if abs(bary(2 * mu_w - 1) / bary(2 * mu_k - 1)) < 0.9:
                expect = d
                break
        assert O.degree_update(mu_k, mu_w, a, b, dmax, O.interpolant_coefficients) == expect
    # large gap: psi_3 at the mapped mu_k is big, so d = 3
    assert O.degree_update(1.5, 1.0, a, b, 15, O.interpolant_coefficients) == 3
