"""Whole-solve parity on the GPU through the C ABI (arr_create / arr_solve /
arr_get_eigpairs) against the FP64 oracle and the closed forms that pin it.

Eigenvalues must agree to |dlambda| <= 1e-10 max(1, |lambda|); residuals are
recomputed on the CPU in FP64 from the returned vectors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import arrabit as O
from paper_1507_06078_amd import arr, workloads as W


def solve(A, k, which, tol, w=None, precision=arr.FP64, X0=None, **kw):
    o = arr.arr_options_default()
    if w:
        o.w = w
    o.precision = precision
    for key, v in kw.items():
        setattr(o, key, v)
    h = arr.arr_create(A, A.n, k, arr.SMALLEST if which == "SA" else arr.LARGEST, tol, o)
    if X0 is not None:
        arr.arr_set_initial_block(h, X0)
    status = arr.arr_solve(h)
    ev, X, res = arr.arr_get_eigpairs(h, k, A.n)
    st = arr.arr_get_stats(h)
    h.close()
    return status, ev, X, res, st


def assert_same_subspaces(ev, X, Y, rel=1e-9):
    i = 0
    k = len(ev)
    while i < k:
        j = i + 1
        while j < k and abs(ev[j] - ev[i]) <= rel * max(1.0, abs(ev[i])):
            j += 1
        s = np.linalg.svd(X[:, i:j].T @ Y[:, i:j], compute_uv=False)
        assert s.min() > 1 - 1e-8, (i, j, s)
        i = j


def check_pairs(A, ev, X, tol):
    S = A.to_scipy()
    k = len(ev)
    r = np.linalg.norm(S @ X - X * ev[None, :], axis=0)
    assert np.all(r / np.maximum(1.0, np.abs(ev)) <= tol * 1.0001), r.max()
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-9
    idx = np.argmax(np.abs(X), axis=0)
    assert np.all(X[idx, np.arange(k)] > 0)  # sign convention


@pytest.mark.parametrize("precision", [arr.FP64, arr.MIXED])
def test_c1_laplacian_matches_oracle_and_closed_form(precision):
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    status, ev, X, res, st = solve(A, k, which, tol, w=w, precision=precision, X0=X0)
    assert status == arr.ARR_OK, st
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    ref = O.arrabit_mpm(A.to_scipy(), k, 1e-12, X0, which)
    assert np.all(np.abs(ev - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))
    assert np.all(np.abs(ev - ref.evals) <= 1e-10 * np.maximum(1, np.abs(ref.evals)))
    check_pairs(A, ev, X, tol)
    assert np.all(res <= tol)
    # eigenvectors are unique only up to rotations inside clusters of equal
    # eigenvalues (the square grid has exact pairs): compare cluster subspaces
    assert_same_subspaces(ev, X, ref.evecs)


@pytest.mark.parametrize("precision", [arr.FP64, arr.MIXED])
def test_c1_gn_inner_solver_matches_oracle_and_closed_form(precision):
    """ARRABIT-GN (the GN branch of Algorithm 8)."""
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    status, ev, X, res, st = solve(A, k, which, tol, w=w, precision=precision, X0=X0, inner_solver=arr.INNER_GN)
    assert status == arr.ARR_OK, st
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    ref = O.arrabit_mpm(A.to_scipy(), k, 1e-12, X0, which, O.Options(inner="gn"))
    assert np.all(np.abs(ev - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))
    assert np.all(np.abs(ev - ref.evals) <= 1e-10 * np.maximum(1, np.abs(ref.evals)))
    check_pairs(A, ev, X, tol)
    assert_same_subspaces(ev, X, ref.evecs)


@pytest.mark.parametrize("precision,inner", [(arr.FP64, arr.INNER_MPM), (arr.MIXED, arr.INNER_MPM),
                                             (arr.FP64, arr.INNER_GN)])
def test_c1_chebyshev_mode_matches_oracle_and_closed_form(precision, inner):
    """Algorithm 8 with the classic Chebyshev filter T_d in place of psi_d
    (Table comp-cheby's alternative), MPM and GN inner solvers."""
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    status, ev, X, res, st = solve(A, k, which, tol, w=w, precision=precision, X0=X0, inner_solver=inner,
                                   poly_form=arr.POLY_CHEBYSHEV)
    assert status == arr.ARR_OK, st
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    ref = O.arrabit_mpm(A.to_scipy(), k, 1e-12, X0, which,
                        O.Options(poly="chebyshev", inner="gn" if inner == arr.INNER_GN else "mpm"))
    assert np.all(np.abs(ev - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))
    assert np.all(np.abs(ev - ref.evals) <= 1e-10 * np.maximum(1, np.abs(ref.evals)))
    check_pairs(A, ev, X, tol)
    assert_same_subspaces(ev, X, ref.evecs)


@pytest.mark.parametrize("precision", [arr.FP64, arr.MIXED])
def test_c1_horner_form_matches_oracle_and_closed_form(precision):
    """Algorithm 8 with psi_d applied by Algorithm 7's recurrence (the Horner
    form, whose last launch also carries the deferred column normalization)."""
    A, k, which, w, tol = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    status, ev, X, res, st = solve(A, k, which, tol, w=w, precision=precision, X0=X0,
                                   poly_form=arr.POLY_HORNER)
    assert status == arr.ARR_OK, st
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    ref = O.arrabit_mpm(A.to_scipy(), k, 1e-12, X0, which)
    assert np.all(np.abs(ev - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))
    assert np.all(np.abs(ev - ref.evals) <= 1e-10 * np.maximum(1, np.abs(ref.evals)))
    check_pairs(A, ev, X, tol)
    assert_same_subspaces(ev, X, ref.evecs)


@pytest.mark.parametrize("which", ["LA", "SA"])
def test_gn_random_symmetric_vs_dense(which):
    n, k, w = 300, 8, 12
    A = W.random_symmetric(n, seed=31, density=0.1)
    lam = np.linalg.eigvalsh(A.to_scipy().toarray())
    exact = lam[::-1][:k] if which == "LA" else lam[:k]
    status, ev, X, res, st = solve(A, k, which, 1e-10, w=w, inner_solver=arr.INNER_GN)
    assert status == arr.ARR_OK, st
    assert np.abs(ev - exact).max() <= 1e-10 * np.abs(lam).max()
    check_pairs(A, ev, X, 1e-10)


def test_c1_device_gaussian_start():
    A, k, which, w, tol = W.workload("lap2d_40")
    status, ev, X, res, st = solve(A, k, which, tol, w=w)
    assert status == arr.ARR_OK
    exact = W.laplacian_2d_eigenvalues(40)[:k]
    assert np.all(np.abs(ev - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))


@pytest.mark.parametrize("which", ["LA", "SA"])
def test_random_symmetric_vs_dense(which):
    n, k, w = 300, 8, 12
    A = W.random_symmetric(n, seed=31, density=0.1)
    lam = np.linalg.eigvalsh(A.to_scipy().toarray())
    exact = lam[::-1][:k] if which == "LA" else lam[:k]
    status, ev, X, res, st = solve(A, k, which, 1e-10, w=w)
    assert status == arr.ARR_OK, st
    assert np.abs(ev - exact).max() <= 1e-10 * np.abs(lam).max()
    check_pairs(A, ev, X, 1e-10)


def test_3d_laplacian_potential_vs_dense_and_weyl():
    A = W.laplacian_3d(12, potential_seed=1)
    k, w = 24, 30
    status, ev, X, res, st = solve(A, k, "SA", 1e-10, w=w, precision=arr.MIXED)
    assert status == arr.ARR_OK, st
    lam = np.linalg.eigvalsh(A.to_scipy().toarray())[:k]
    assert np.abs(ev - lam).max() <= 1e-10 * max(1, np.abs(lam).max())
    L0 = W.laplacian_3d_eigenvalues(12)[:k]
    assert np.all(L0 - 1e-12 <= ev) and np.all(ev <= L0 + 1 + 1e-12)
    check_pairs(A, ev, X, 1e-10)


@pytest.mark.parametrize("precision", [arr.FP64, arr.MIXED])
def test_row_forms_agree_in_solve(precision):
    """The 3D 7-point operator runs in the paired row form (P = 20) unless
    the plain form is asked for; both solves reach the closed-form spectrum
    and the timed SpMM variant reports the form it ran."""
    A = W.laplacian_3d(20)
    k, w, tol = 24, 30, 1e-10
    exact = W.laplacian_3d_eigenvalues(20)[:k]
    assert arr.arr_row_form(A) == (20, 3, 0)
    for form, paired in ((arr.ROW_AUTO, 8), (arr.ROW_PLAIN, 0)):
        status, ev, X, res, st = solve(A, k, "SA", tol, w=w, precision=precision, row_form=form, timing=1)
        assert status == arr.ARR_OK, st
        assert np.all(np.abs(ev - exact) <= 1e-10 * np.maximum(1, np.abs(exact)))
        check_pairs(A, ev, X, tol)
        assert st["spmm_flags"] & 8 == paired
        if precision == arr.MIXED:
            assert st["spmm32_flags"] & 8 == paired


def test_powerlaw_largest():
    A = W.powerlaw_random(3000, seed=3, cap=200)
    k, w = 16, 20
    status, ev, X, res, st = solve(A, k, "LA", 1e-10, w=w)
    assert status in (arr.ARR_OK,), st
    lam = np.sort(np.linalg.eigvalsh(A.to_scipy().toarray()))[::-1][:k]
    assert np.abs(ev - lam).max() <= 1e-10 * max(1, np.abs(lam).max())
    check_pairs(A, ev, X, 1e-10)


def test_powerlaw_largest_mixed():
    """The power-law family (FP32 filter stage, FP64 closing iterations)."""
    A = W.powerlaw_random(3000, seed=3, cap=200)
    k, w = 16, 20
    status, ev, X, res, st = solve(A, k, "LA", 1e-10, w=w, precision=arr.MIXED)
    assert status == arr.ARR_OK, st
    lam = np.sort(np.linalg.eigvalsh(A.to_scipy().toarray()))[::-1][:k]
    assert np.abs(ev - lam).max() <= 1e-10 * max(1, np.abs(lam).max())
    check_pairs(A, ev, X, 1e-10)


@pytest.mark.parametrize("precision", [arr.FP64, arr.MIXED])
def test_sbm_normalized_laplacian_smallest(precision):
    """The SBM normalized-Laplacian family: with 16 blocks the 16 smallest
    eigenvalues (0 and a cluster near 0.5) lie below the bulk; k = 24 takes
    them and the start of the bulk. Spectrum in [0, 2] (checked); eigenvalues
    against a dense eigensolve."""
    A = W.sbm_normalized_laplacian(3008, 16, seed=5)
    lam = np.linalg.eigvalsh(A.to_scipy().toarray())
    assert lam[0] > -1e-12 and lam[-1] < 2 + 1e-12
    k, w = 24, 36
    status, ev, X, res, st = solve(A, k, "SA", 1e-10, w=w, precision=precision)
    assert status == arr.ARR_OK, st
    assert np.abs(ev - lam[:k]).max() <= 1e-10 * max(1, np.abs(lam[:k]).max())
    check_pairs(A, ev, X, 1e-10)


def test_deterministic_repeat():
    A, k, which, w, tol = W.workload("lap2d_40")
    a = solve(A, k, which, tol, w=w)
    b = solve(A, k, which, tol, w=w)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_maxit_one_not_converged_but_pairs_available():
    A, k, which, w, tol = W.workload("lap2d_40")
    status, ev, X, res, st = solve(A, k, which, tol, w=w, maxit=1)
    assert status == arr.ARR_NOT_CONVERGED
    assert np.isfinite(ev).all() and np.isfinite(res).all() and X.shape == (A.n, k)


def test_results_before_solve_is_state_error():
    A, k, which, w, tol = W.workload("lap2d_40")
    h = arr.arr_create(A, A.n, k, arr.SMALLEST, tol)
    with pytest.raises(arr.ArrError) as e:
        arr.arr_get_eigpairs(h, k, A.n)
    assert e.value.code == arr.ARR_ESTATE
    h.close()
