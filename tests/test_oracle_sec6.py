"""Pins for the oracle's Sec. 6 bookkeeping inside Algorithm 8: the first
continuation tolerance (reading R8), the continuation rule (eq. contin), the
deflation threshold (eq. defl), and the outer stop rules (ii) (no reduction of
maxres in three consecutive outer iterations) and (iii) (maxres below
(1 + 9h/k) tol, with h the pairs below 0.1 tol; on with paper_faithful).

These rules only steer the trajectory and the returned status, so the
converged-eigenpair pins of test_oracle_solve.py cannot see them. Each test
here drives the oracle into the branch and checks the recorded history
against the rule as the paper states it, on the 2D Laplacian 40 x 40
(k = 20 smallest, block 30, starting block seed 2). Where a threshold is
checked, the test also asserts that the run had pairs or iterations on both
sides of it, so that a wrong constant changes the outcome."""
import numpy as np
import pytest

from oracle import arrabit as O
from paper_1507_06078_amd import workloads as W


def _run(tol, **kw):
    A, k, which, w, _ = W.workload("lap2d_40")
    X0 = W.gaussian_block(A.n, w, seed=2)
    return O.arrabit_mpm(A.to_scipy(), k, tol, X0, which, O.Options(**kw)), k, w


def test_first_tolerance_reading():
    """Reading R8: tol_1 = 1e-6 when tol <= 1e-8 (continuation on), tol_1 = tol
    otherwise; an explicit tol1 is used but never below tol."""
    opts = O.Options()
    assert O.first_tolerance(1e-10, opts) == 1e-6
    assert O.first_tolerance(1e-8, opts) == 1e-6
    assert O.first_tolerance(1e-7, opts) == 1e-7
    assert O.first_tolerance(1e-10, O.Options(tol1=1e-4)) == 1e-4
    assert O.first_tolerance(1e-3, O.Options(tol1=1e-4)) == 1e-3


def test_continuation_sequence_follows_eq_contin():
    """tol = 1e-10: the sequence starts at tol_1 = 1e-6 and every continuation
    step divides it by exactly 100 down to tol (eq. contin), so the only values
    it can take are 1e-6, 1e-8 and 1e-10. A step happens exactly when maxres
    <= tol_t, and b moves to mu_{k+q} then (Algorithm 8, continuation)."""
    r, k, w = _run(1e-10)
    assert r.status == 0
    hist = r.history
    assert hist[0]["tol_t"] == 1e-6
    seen = {h["tol_t"] for h in hist}
    assert seen <= {1e-6, 1e-8, 1e-10}
    steps = 0
    for h, nxt in zip(hist[:-1], hist[1:]):
        if h["maxres"] <= h["tol_t"]:
            assert h["tol_t_next"] == max(1e-2 * h["tol_t"], 1e-10)
            assert h["b_next"] == h["mu"][w - 1]
            steps += 1
        else:
            assert h["tol_t_next"] == h["tol_t"] and h["b_next"] == h["b"]
        assert nxt["tol_t"] == h["tol_t_next"] and nxt["b"] == h["b_next"]
    assert steps >= 2  # both 1e-6 -> 1e-8 and 1e-8 -> 1e-10 were taken


def test_no_continuation_for_loose_tolerance():
    """tol > 1e-8: tol_t stays at tol for the whole solve (R8, eq. contin)."""
    r, _, _ = _run(1e-7)
    assert r.status == 0
    assert all(h["tol_t"] == 1e-7 for h in r.history)


def test_deflation_locks_exactly_below_max_1e14_tol_t_squared():
    """eq. defl: after each ARR step a merged pair is locked iff its residual
    is <= max(1e-14, tol_t^2), with tol_t the value after that iteration's
    continuation step (reading R9). The run must contain unlocked pairs whose
    residual is below tol_t itself (so a threshold of tol_t instead of
    tol_t^2 would lock them) and locked pairs."""
    r, k, w = _run(1e-10)
    below_tol_t_but_unlocked = 0
    locked_total = 0
    for h, nxt in zip(r.history[:-1], r.history[1:]):
        thr = max(1e-14, h["tol_t_next"] ** 2)
        np.testing.assert_array_equal(h["locked"], h["res"] <= thr)
        assert nxt["n_conv"] == int(h["locked"].sum())
        assert nxt["width"] == w - nxt["n_conv"]
        below_tol_t_but_unlocked += int(((h["res"] <= h["tol_t_next"]) & ~h["locked"]).sum())
        locked_total += int(h["locked"].sum())
    assert below_tol_t_but_unlocked > 0
    assert locked_total > 0


def test_stop_rule_ii_stagnation():
    """tol = 1e-16 lies below what FP64 residuals can reach (about 1e-15 here),
    so maxres stops improving; rule (ii) must end the solve with status 2 at
    the third consecutive outer iteration without a new smallest maxres, and
    not earlier."""
    r, k, w = _run(1e-16)
    assert r.status == 2
    m = [h["maxres"] for h in r.history]
    assert len(m) >= 4 and len(m) < 30
    best_before = min(m[:-3])
    assert all(x >= best_before for x in m[-3:])
    # no earlier window of three iterations without improvement
    for j in range(3, len(m) - 1):
        assert min(m[j - 2:j + 1]) < min(m[:j - 2]), j
    assert r.history[-1]["since_best"] == 3
    assert all(h["since_best"] < 3 for h in r.history[:-1])
    # the best pairs are still returned, with finite residuals near the FP64 floor
    assert np.isfinite(r.res).all() and r.res.max() < 1e-12


def test_stop_rule_iii_accepts_slightly_larger_residuals():
    """paper_faithful, tol = 6e-11: in the fourth outer iteration maxres is
    about 3.5 tol while most pairs are below 0.1 tol (h >= 15 of k = 20), so
    rule (iii) stops there: status 0 with tol < maxres < (1 + 9h/k) tol. The
    same solve without rule (iii) goes on and ends at maxres <= tol."""
    tol = 6e-11
    r, k, w = _run(tol, paper_faithful=True)
    assert r.status == 0
    last = r.history[-1]
    h = int((last["res"][:k] < 0.1 * tol).sum())
    assert tol < last["maxres"] < (1.0 + 9.0 * h / k) * tol
    assert last["maxres"] < 10 * tol
    r2, _, _ = _run(tol)
    assert r2.status == 0 and r2.history[-1]["maxres"] <= tol
    assert len(r2.history) > len(r.history)


def test_stop_rule_iii_weighting_by_h():
    """paper_faithful, tol = 2e-11: in the fourth outer iteration maxres is
    above 10 tol, which rule (iii) can never accept since 1 + 9h/k <= 10; the
    solve must go on to maxres <= tol. (A rule with a larger weight on h would
    have stopped there: h >= 10 pairs were below 0.1 tol.)"""
    tol = 2e-11
    r, k, w = _run(tol, paper_faithful=True)
    assert r.status == 0
    fourth = r.history[3]
    assert fourth["maxres"] > 10 * tol
    assert int((fourth["res"][:k] < 0.1 * tol).sum()) >= 10
    assert len(r.history) > 4
    for hh in r.history[:-1]:
        h = int((hh["res"][:k] < 0.1 * tol).sum())
        assert not hh["maxres"] < (1.0 + 9.0 * h / k) * tol
    assert r.history[-1]["maxres"] < 10 * tol


@pytest.mark.parametrize("tol", [3e-11, 6e-11, 1.5e-10])
def test_paper_faithful_result_within_ten_tol(tol):
    """Whatever rule stops a paper_faithful solve, its maxres is < 10 tol
    (Sec. 6, rule (iii): (1 + 9h/k) tol < 10 tol)."""
    r, k, w = _run(tol, paper_faithful=True)
    assert r.status == 0
    assert r.history[-1]["maxres"] < 10 * tol
    assert r.res.max() < 10 * tol


def _gapped_matrix():
    """Dense symmetric 120 x 120 matrix Q diag(lam) Q^T with the 6 largest
    eigenvalues near 10 and the rest in [0, 1]: the shifted Ritz-value ratio
    (mu_{k+q} - a)/(mu_k - a) of eq. block is about 0.1."""
    n, k = 120, 6
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([10 - 0.01 * np.arange(k), np.linspace(1.0, 0.0, n - k)])
    M = (Q * lam) @ Q.T
    return W.from_scipy(0.5 * (M + M.T)), k


def _check_block_rule(hist, k, w, p_max=3):
    """eq. block with reading R5 (shifted values mu - a) and R17 (no update in
    the first outer iteration): p grows by one, up to p_max, iff the ratio of
    shifted Ritz values exceeds 0.95 and maxres/maxresp exceeds 0.1."""
    grew = held_by_ratio = held_by_decay = 0
    for j in range(len(hist) - 1):
        h, nxt = hist[j], hist[j + 1]
        ratio = (h["mu"][w - 1] - h["a"]) / (h["mu"][k - 1] - h["a"])
        up = j > 0 and ratio > 0.95 and h["maxres"] / hist[j - 1]["maxres"] > 0.1
        assert nxt["p"] == (min(h["p"] + 1, p_max) if up else h["p"]), j
        grew += up
        if j > 0 and not up:
            held_by_ratio += ratio <= 0.95
            held_by_decay += h["maxres"] / hist[j - 1]["maxres"] <= 0.1
    return grew, held_by_ratio, held_by_decay


def test_augmentation_block_rule():
    """eq. block on two runs that take both branches: the Laplacian solve that
    stagnates at tol = 1e-16 (ratio 0.99; p grows once maxres stops falling,
    and is held while maxres falls by more than 10x per iteration), and a
    matrix with a wide gap after the k wanted eigenvalues (ratio about 0.1;
    p is held although maxres stops falling)."""
    r, k, w = _run(1e-16)
    grew, _, held_by_decay = _check_block_rule(r.history, k, w)
    assert grew >= 1 and held_by_decay >= 1
    A, k2 = _gapped_matrix()
    w2 = k2 + 2
    r2 = O.arrabit_mpm(A.to_scipy(), k2, 1e-16, W.gaussian_block(A.n, w2, seed=2), "LA")
    grew2, held_by_ratio, _ = _check_block_rule(r2.history, k2, w2)
    assert grew2 == 0 and held_by_ratio >= 1
    assert all(h["p"] == 1 for h in r2.history)


def test_degree_from_most_accurate_iteration():
    """eq. hat-d / eq. degree: after each outer iteration d is the rule applied
    to mu_k and mu_{k+q} of the iteration with the smallest maxres so far
    (the first of equal ones), on the interval [a, b] in force after it."""
    r, k, w = _run(1e-16)
    hist = r.history
    for j in range(len(hist) - 1):
        best = min(range(j + 1), key=lambda i: (hist[i]["maxres"], i))
        mu = hist[best]["mu"]
        expect = O.degree_update(mu[k - 1], mu[w - 1], hist[j]["a"], hist[j]["b_next"], 15,
                                 O.interpolant_coefficients)
        assert hist[j + 1]["d"] == expect, j
    assert len({h["d"] for h in hist}) >= 2  # the degree moved at least once
