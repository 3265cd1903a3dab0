"""Plain FP64 CPU oracle for the ARRABIT-MPM block eigensolver.

TEST INFRASTRUCTURE ONLY. This module is the slow, obviously-correct reference
that the GPU library is checked against. Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the GPU library never
does, and the two share no code (the only shared module is the seeded input
generator, which holds none of the method's arithmetic).

Source: Wen & Zhang, "Block algorithms with augmented Rayleigh-Ritz projections
for large-scale eigenpair computation" (arXiv 1507.06078). Each function names
the passage it follows. Library primitives used as single steps: sparse and
dense matrix products (scipy/numpy), Householder QR (numpy.linalg.qr),
the dense symmetric eigensolver (numpy.linalg.eigh), a dense linear solve
(numpy.linalg.solve), Cholesky and inverse for the condition number.

Readings of the paper where it is silent or ambiguous are marked "Reading:".
Pins (what each function is checked against, independently of itself) live in
tests/test_oracle_*.py.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# Section 5 (Polynomial Accelerators): the interpolant psi_d
# --------------------------------------------------------------------------


def interpolation_nodes(d: int) -> np.ndarray:
    """Chebyshev points of the second kind t_j = -cos(j*pi/d), j = 0..d (Sec. 5)."""
    j = np.arange(d + 1, dtype=np.float64)
    return -np.cos(j * np.pi / d)


def target_function(t, d: int):
    """f_d(t) = (max(0,t)^10)^d (eq. def:fN)."""
    t = np.asarray(t, dtype=np.float64)
    return np.maximum(0.0, t) ** (10 * d)


def interpolant_coefficients(d: int) -> np.ndarray:
    """Monomial coefficients Gamma_d = (gamma_1, ..., gamma_{d+1}) of the degree-d
    polynomial psi_d that interpolates f_d at the d+1 nodes, leading coefficient
    first (eq. chebfun-f). Computed from the definition: the Vandermonde system
    sum_i gamma_i t_j^(d+1-i) = f_d(t_j), j = 0..d."""
    t = interpolation_nodes(d)
    V = np.vander(t, d + 1, increasing=False)  # columns t^d, ..., t, 1
    return np.linalg.solve(V, target_function(t, d))


def psi(t, gam: np.ndarray):
    """psi_d(t) = sum_i gamma_i t^(d+1-i), evaluated as a plain power sum."""
    t = np.asarray(t, dtype=np.float64)
    d = len(gam) - 1
    return sum(gam[i] * t ** (d - i) for i in range(d + 1))


def rho(t, a: float, b: float, gam: np.ndarray):
    """rho_d(t) = psi_d((2t - a - b)/(b - a)): [a,b] mapped onto [-1,1] (eq. rhod)."""
    return psi((2.0 * np.asarray(t, dtype=np.float64) - a - b) / (b - a), gam)


# --------------------------------------------------------------------------
# Algorithm 7: Y = poly(A, X, a, b, Gamma_d)
# --------------------------------------------------------------------------


def poly(Aop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, a: float, b: float,
         gam: np.ndarray) -> np.ndarray:
    """Algorithm 7 (Horner in the mapped variable): c0 = (a+b)/(a-b),
    c1 = 2/(b-a); Y = gamma_1 X; for j = 1..d: Y = c0 Y + c1 A Y + gamma_{j+1} X.
    ``Aop`` applies the (possibly shifted) matrix to a block."""
    c0 = (a + b) / (a - b)
    c1 = 2.0 / (b - a)
    Y = gam[0] * X
    for j in range(1, len(gam)):
        Y = c0 * Y + c1 * Aop(Y) + gam[j] * X
    return Y


def chebyshev_T(x, d: int):
    """T_d(x) by the three-term recursion of eq. cheby-poly: T_0 = 1, T_1 = x,
    T_{j+1} = 2 x T_j - T_{j-1}."""
    x = np.asarray(x, dtype=np.float64)
    t_prev, t = np.ones_like(x), x
    if d == 0:
        return t_prev
    for _ in range(1, d):
        t_prev, t = t, 2.0 * x * t - t_prev
    return t


def rho_chebyshev(t, a: float, b: float, d: int):
    """The classic Chebyshev filter: T_d((2t - a - b)/(b - a)), [a,b] mapped
    onto [-1,1] as in eq. rhod, with T_d of eq. cheby-poly in place of psi_d
    (the alternative compared in Table comp-cheby)."""
    return chebyshev_T((2.0 * np.asarray(t, dtype=np.float64) - a - b) / (b - a), d)


def chebyshev_poly(Aop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, a: float, b: float,
                   d: int) -> np.ndarray:
    """Y = T_d(t(A)) X with t(A) = (2A - (a+b)I)/(b-a), by the block form of eq.
    cheby-poly: Y_0 = X, Y_1 = t(A) X, Y_{j+1} = 2 t(A) Y_j - Y_{j-1}."""
    assert d >= 1
    c0 = (a + b) / (a - b)
    c1 = 2.0 / (b - a)

    def t(Y):
        return c1 * Aop(Y) + c0 * Y

    Y_prev, Y = X, t(X)
    for _ in range(1, d):
        Y_prev, Y = Y, 2.0 * t(Y) - Y_prev
    return Y


def shifted(A: sp.spmatrix, a: float) -> Callable[[np.ndarray], np.ndarray]:
    """The operator Y -> (A - aI) Y used by the inner solvers (Sec. 6, inner loop)."""
    return lambda Y: A @ Y - a * Y


# --------------------------------------------------------------------------
# Section 2.6 (A Gauss-Newton Algorithm) and the GN branch of Algorithm 8
# --------------------------------------------------------------------------


def gn_update(X: np.ndarray, rho_op: Callable[[np.ndarray], np.ndarray]) -> np.ndarray:
    """One Gauss-Newton iteration with unit step for the least-squares fit of
    X X^T to rho(A) (the GN algorithm of Sec. 2.6, as Algorithm 8 calls it):
    Y = X (X^T X)^{-1}, Z = rho(A) Y, X+ = Z - X (Y^T Z - I) / 2.
    ``rho_op`` applies rho(A) to a block."""
    G = X.T @ X
    Y = np.linalg.solve(G, X.T).T  # X G^{-1}; G is symmetric
    Z = rho_op(Y)
    C = Y.T @ Z
    return Z - X @ (C - np.eye(C.shape[0])) / 2.0


def gn_step(Aop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, a: float, b: float,
            gam: np.ndarray) -> np.ndarray:
    """The GN inner iteration of Algorithm 8: rho is Algorithm 7's poly on the
    shifted operator over [a, b] with coefficients gam."""
    return gn_update(X, lambda Y: poly(Aop, Y, a, b, gam))


# --------------------------------------------------------------------------
# Section 6: inner-loop quantities
# --------------------------------------------------------------------------


def normalize_columns(X: np.ndarray) -> np.ndarray:
    """x_i = x_i / ||x_i||_2 for each column (Sec. 3, multi-power method)."""
    return X / np.linalg.norm(X, axis=0)[None, :]


def project_out(Qc: np.ndarray | None, X: np.ndarray) -> np.ndarray:
    """X - Qc (Qc^T X) (Sec. 6, Deflation; Algorithm 8 projection step)."""
    if Qc is None or Qc.shape[1] == 0:
        return X
    return X - Qc @ (Qc.T @ X)


def rcond_gram(X: np.ndarray) -> float:
    """rc = rcond(X^T X), the reciprocal 1-norm condition number (eq. inn-stop).
    Reading: the exact value 1/(||G||_1 ||G^-1||_1) rather than LAPACK's
    estimate; rc = 0 when G = X^T X is not numerically positive definite."""
    G = X.T @ X
    G = 0.5 * (G + G.T)
    try:
        np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        return 0.0
    Ginv = np.linalg.inv(G)
    return 1.0 / (np.abs(G).sum(axis=0).max() * np.abs(Ginv).sum(axis=0).max())


# --------------------------------------------------------------------------
# Section 6: interval estimation
# --------------------------------------------------------------------------


def lanczos_extremes(A: sp.spmatrix, v0: np.ndarray, steps: int = 100):
    """Lanczos with full reorthogonalization from v0 (Sec. 2.1 background; used
    in place of the paper's call to eigs for lambda_n, Sec. 6 'Estimation').
    Returns (theta_min, theta_max, r_min): the extreme Ritz values of the
    tridiagonal matrix and the residual bound |beta_m s_m| of the smallest."""
    n = v0.shape[0]
    steps = min(steps, n)
    V = np.zeros((n, steps))
    alpha, beta = [], []
    v = v0 / np.linalg.norm(v0)
    for j in range(steps):
        V[:, j] = v
        wv = A @ v
        alpha.append(float(v @ wv))
        wv = wv - alpha[-1] * v
        if j > 0:
            wv = wv - beta[-1] * V[:, j - 1]
        for _ in range(2):  # full reorthogonalization, twice
            wv = wv - V[:, : j + 1] @ (V[:, : j + 1].T @ wv)
        beta.append(float(np.linalg.norm(wv)))
        if beta[-1] <= 1e-14 * max(1.0, abs(alpha[-1])) or j == steps - 1:
            break
        v = wv / beta[-1]
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
    theta, S = np.linalg.eigh(T)
    r = np.abs(beta[m - 1] * S[m - 1, :])
    return float(theta[0]), float(theta[-1]), float(r[0])


def lower_end_estimate(A: sp.spmatrix, v0: np.ndarray, steps: int = 100):
    """a <= lambda_n estimate. Reading: Lanczos smallest Ritz value minus the
    larger of its residual bound and 1e-3 of the Ritz spread. Also returns the
    spectral-norm estimate max(|theta_min|, |theta_max|)."""
    tmin, tmax, r = lanczos_extremes(A, v0, steps)
    a = tmin - max(r, 1e-3 * (tmax - tmin))
    return a, max(abs(tmin), abs(tmax))


# --------------------------------------------------------------------------
# Algorithm 1 (RR) and Algorithm 5 (ARR)
# --------------------------------------------------------------------------


def rayleigh_ritz(A: sp.spmatrix, Z: np.ndarray):
    """Algorithm 1: U in orth(Z); H = U^T A U; H = V Sigma V^T; Y = U V.
    Reading: orth(Z) by Householder QR keeping every column (a valid
    orthonormal basis containing R(Z) even when Z is numerically rank
    deficient); the eigendecomposition is written H = V Sigma V^T.
    Ritz pairs are returned sorted by value, largest first."""
    U, _ = np.linalg.qr(Z, mode="reduced")
    H = U.T @ (A @ U)
    H = 0.5 * (H + H.T)
    sig, V = np.linalg.eigh(H)
    order = np.argsort(-sig, kind="stable")
    return U @ V[:, order], sig[order]


def krylov_block(A: sp.spmatrix, X: np.ndarray, p: int) -> np.ndarray:
    """[X, AX, A^2 X, ..., A^p X] (eq. S:ARR)."""
    blocks = [X]
    for _ in range(p):
        blocks.append(A @ blocks[-1])
    return np.hstack(blocks)


def augmented_rr(A: sp.spmatrix, X: np.ndarray, p: int, Qc: np.ndarray | None = None):
    """Algorithm 5 with the deflation projection of Sec. 6: RR on
    Z = [X, AX, ..., A^p X] - Qc(Qc^T [..]). Returns all Ritz pairs (largest
    first); the caller extracts the leading ones."""
    Z = project_out(Qc, krylov_block(A, X, p))
    return rayleigh_ritz(A, Z)


def residual_norms(A: sp.spmatrix, X: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """||A x_i - mu_i x_i||_2 for each column."""
    return np.linalg.norm(A @ X - X * mu[None, :], axis=0)


def relative_residuals(A: sp.spmatrix, X: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """res_i = ||A x_i - mu_i x_i||_2 / max(1, |mu_i|) (eq. resi)."""
    return residual_norms(A, X, mu) / np.maximum(1.0, np.abs(mu))


# --------------------------------------------------------------------------
# Section 6 heuristics
# --------------------------------------------------------------------------


def degree_update(mu_k: float, mu_w: float, a: float, b: float, d_max: int,
                  coeffs: Callable[[int], np.ndarray] | None = None,
                  rho_d: Callable[[float, int], float] | None = None) -> int:
    """d = min(d_hat, d_max), d_hat = min{d >= 3 : rho_d(mu*_{k+q})/rho_d(mu*_k) < 0.9}
    (eq. hat-d, eq. degree). Reading: the ratio is taken in absolute value and
    d = d_max when no d in [3, d_max] satisfies it. rho_d is eq. rhod with
    psi_d (from ``coeffs``) unless ``rho_d(t, d)`` is given (Chebyshev mode)."""
    if rho_d is None:
        rho_d = lambda t, dd: rho(t, a, b, coeffs(dd))
    for d in range(3, d_max + 1):
        num = abs(float(rho_d(mu_w, d)))
        den = abs(float(rho_d(mu_k, d)))
        if den > 0.0 and num / den < 0.9:
            return d
    return d_max


@dataclasses.dataclass
class Options:
    """Parameters of Algorithm 8 with the defaults of Sec. 6."""
    d0: int = 3            # initial degree
    d_max: int = 15        # maximal degree
    p0: int = 1            # initial number of augmentation blocks
    p_max: int = 3
    maxit: int = 30        # outer iterations, stop rule (i)
    maxit1: int = 10       # inner checks
    maxit2: int = 5        # inner iterations between checks
    tol1: float | None = None   # first continuation tolerance (Reading below)
    lanczos_steps: int = 100
    stagnation: int = 3    # stop rule (ii)
    paper_faithful: bool = False  # stop rule (iii)
    inner: str = "mpm"     # inner solver of Algorithm 8: "mpm" or "gn"
    poly: str = "interp"   # filter: "interp" (psi_d, Sec. 5) or "chebyshev" (T_d, eq. cheby-poly)


@dataclasses.dataclass
class Result:
    evals: np.ndarray      # k eigenvalues of A (descending for LA, ascending for SA)
    evecs: np.ndarray      # n x k, unit columns
    res: np.ndarray        # eq. resi scaling, k entries
    rnorm: np.ndarray      # ||A x - lambda x||_2, k entries
    status: int            # 0 converged, 1 maxit reached, 2 stagnated
    history: list
    stats: dict


def first_tolerance(tol: float, opts: Options) -> float:
    """Reading of Sec. 6 'Continuation': tol_1 is 'considerably larger' than tol
    when tol <= 1e-8 (continuation on); 1e-6 is taken. Otherwise tol_1 = tol."""
    if opts.tol1 is not None:
        return max(opts.tol1, tol)
    return 1e-6 if tol <= 1e-8 else tol


def arrabit_mpm(A: sp.spmatrix, k: int, tol: float, X0: np.ndarray, which: str = "LA",
                opts: Options | None = None) -> Result:
    """Algorithm 8 (ARRABIT, detailed version) with the MPM inner solver, or
    with the GN inner solver when ``opts.inner == "gn"``.

    Computes the k algebraically largest ('LA') or smallest ('SA') eigenpairs of
    symmetric A. Reading: 'SA' is solved as 'LA' of -A. ``X0`` (n x (k+q)) is
    the i.i.d. Gaussian starting block; its first column also starts Lanczos.
    """
    opts = opts or Options()
    assert opts.poly in ("interp", "chebyshev") and opts.inner in ("mpm", "gn")
    A = sp.csr_matrix(A, dtype=np.float64)
    B = -A if which == "SA" else A
    n = B.shape[0]
    w = X0.shape[1]
    assert 0 < k <= w and (opts.p_max + 1) * w < n, "needs (p_max+1)(k+q) < n"
    coeff_cache: dict[int, np.ndarray] = {}

    def coeffs(dd):
        if dd not in coeff_cache:
            coeff_cache[dd] = interpolant_coefficients(dd)
        return coeff_cache[dd]

    d, p = opts.d0, opts.p0
    tol_t = first_tolerance(tol, opts)
    stats = dict(poly_calls=0, spmm_degrees=0, block_spmm_cols=0, arr_calls=0, outer=0)

    # interval [a, b] (Sec. 6, 'Estimation of lambda_n and lambda_{k+q}')
    a, normA = lower_end_estimate(B, X0[:, 0], opts.lanczos_steps)
    U, _ = np.linalg.qr(X0, mode="reduced")
    H = U.T @ (B @ U)
    b = float(np.linalg.eigvalsh(0.5 * (H + H.T))[0])

    X = X0.copy()
    Qc = np.zeros((n, 0))
    sig_c = np.zeros(0)
    res_c = np.zeros(0)
    history = []
    best_maxres = math.inf
    best_mu = None
    since_best = 0
    maxresp = None
    status = 1
    Xw = mu = res = None
    for j in range(1, opts.maxit + 1):
        stats["outer"] = j
        opB = shifted(B, a)

        def filt(Y, dd):
            """rho_d(A - aI) Y over [0, b - a]: Algorithm 7's psi_d, or T_d."""
            if opts.poly == "chebyshev":
                return chebyshev_poly(opB, Y, 0.0, b - a, dd)
            return poly(opB, Y, 0.0, b - a, coeffs(dd))

        rc = math.inf
        Qp = Qc if Qc.shape[1] else None
        for _i1 in range(opts.maxit1):
            for _i2 in range(opts.maxit2):
                if opts.inner == "gn":
                    # GN branch: no normalization; X X^T tracks rho(A - aI)
                    X = gn_update(X, lambda Y: filt(Y, d))
                else:
                    X = normalize_columns(filt(X, d))
                stats["poly_calls"] += 1
                stats["spmm_degrees"] += d
                stats["block_spmm_cols"] += d * X.shape[1]
                X = project_out(Qp, X)
            rcp = rc
            rc = rcond_gram(X)
            if rc <= tol_t or rc / rcp > 0.99:
                break
        # augmentation + ARR in the complement of R(Qc)
        Y, sig = augmented_rr(B, X, p, Qp)
        stats["arr_calls"] += 1
        # merge with converged pairs, keep the k+q leading ones
        allv = np.hstack([Qc, Y])
        alls = np.concatenate([sig_c, sig])
        order = np.argsort(-alls, kind="stable")[:w]
        Xw = allv[:, order]
        mu = alls[order]
        rnorm = residual_norms(B, Xw, mu)
        res = rnorm / np.maximum(1.0, np.abs(mu))
        maxres = float(res[:k].max())
        if maxres < best_maxres:
            best_maxres, best_mu, since_best = maxres, (mu[k - 1], mu[w - 1]), 0
        else:
            since_best += 1
        history.append(dict(outer=j, maxres=maxres, d=d, p=p, n_conv=int(Qc.shape[1]),
                            tol_t=tol_t, a=a, b=b, width=int(X.shape[1]), res=res.copy(),
                            mu=mu.copy(), since_best=since_best))
        if maxres <= tol:
            status = 0
            break
        if opts.paper_faithful:
            h = int((res[:k] < 0.1 * tol).sum())
            if maxres < (1.0 + 9.0 * h / k) * tol:
                status = 0
                break
        if since_best >= opts.stagnation:
            status = 2
            break
        if j == opts.maxit:
            break
        if maxres <= tol_t:  # continuation (eq. contin)
            tol_t = max(1e-2 * tol_t, tol)
            b = float(mu[w - 1])
        # deflation (eq. defl): converged pairs are re-collected from the merged set
        tol_d = max(1e-14, tol_t ** 2)
        conv = res <= tol_d
        history[-1].update(locked=conv.copy(), tol_t_next=tol_t, b_next=b)
        Qc, sig_c, res_c = Xw[:, conv], mu[conv], res[conv]
        X = Xw[:, ~conv]
        # augmentation blocks (eq. block). Reading: ratio of shifted values
        # mu - a; no update before a previous maxres exists.
        if maxresp is not None:
            ratio = (mu[w - 1] - a) / (mu[k - 1] - a)
            if ratio > 0.95 and maxres / maxresp > 0.1:
                p = min(p + 1, opts.p_max)
        maxresp = maxres
        # degree (eq. hat-d, eq. degree) from the best iterate so far
        if opts.poly == "chebyshev":
            d = degree_update(best_mu[0], best_mu[1], a, b, opts.d_max,
                              rho_d=lambda t, dd: rho_chebyshev(t, a, b, dd))
        else:
            d = degree_update(best_mu[0], best_mu[1], a, b, opts.d_max, coeffs)
        if X.shape[1] == 0:  # every pair locked; nothing left to iterate
            break

    stats.update(final_p=p, final_d=d, a=a, b=b, normA_est=normA, tol_final=tol_t)
    evecs = Xw[:, :k].copy()
    lam = mu[:k].copy()
    rn = residual_norms(B, evecs, lam)
    if which == "SA":
        lam = -lam
    # sign convention: largest-magnitude entry positive
    idx = np.argmax(np.abs(evecs), axis=0)
    sgn = np.sign(evecs[idx, np.arange(k)])
    sgn[sgn == 0] = 1.0
    evecs *= sgn[None, :]
    return Result(lam, evecs, rn / np.maximum(1.0, np.abs(lam)), rn, status, history, stats)
