"""GPU parity of each step of the path, called through the C ABI, against the
FP64 oracle (or the definition the oracle pins). Sizes span several tiles and
ragged tails; edge cases: width 1, widths one past a tile, empty rows, ld > w."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import arrabit as O
from paper_1507_06078_amd import arr, workloads as W


def dev(x, dtype=None):
    dtype = dtype or torch.float64
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def with_empty_rows(n=700, seed=3):
    """Symmetric matrix with fully empty rows (no diagonal either)."""
    rng = np.random.default_rng(seed)
    S = sp.random(n, n, density=0.01, random_state=seed, format="csr")
    S = S + S.T
    keep = np.ones(n)
    keep[rng.choice(n, 60, replace=False)] = 0.0
    D = sp.diags(keep)
    S = sp.csr_matrix(D @ S @ D)
    S.eliminate_zeros()
    return W.from_scipy(S, "empty_rows")


def tridiagonal(n=1001, seed=5):
    """Only the band the kernels keep in registers: the far CSR is empty."""
    rng = np.random.default_rng(seed)
    off = rng.standard_normal(n - 1)
    S = sp.diags([off, rng.standard_normal(n), off], [-1, 0, 1], format="csr")
    return W.from_scipy(S, "tridiagonal")


def lap2d_holes(m=41, seed=4):
    """2D 5-point Laplacian (two entries off the band per row, so no row
    overflows the four far slots) with 50 rows and columns removed: empty
    rows inside full runs of the pipelined path. n = 1681 is not a multiple
    of the run length."""
    rng = np.random.default_rng(seed)
    S = W.laplacian_2d(m).to_scipy()
    keep = np.ones(m * m)
    keep[rng.choice(m * m, 50, replace=False)] = 0.0
    D = sp.diags(keep)
    S = sp.csr_matrix(D @ S @ D)
    S.eliminate_zeros()
    return W.from_scipy(S, "lap2d_holes")


def band_p40(n=1070, seed=6):
    """Diagonals 0, +-1, +-3, +-40: the paired row form with P = 40 and three
    far entries a row; n = 13 * 80 + 30 leaves a tail of upper and lower
    rows past the last whole block of 80."""
    rng = np.random.default_rng(seed)
    diags, offs = [rng.standard_normal(n) + 8.0], [0]
    for k in (1, 3, 40):
        v = rng.standard_normal(n - k)
        diags += [v, v]
        offs += [k, -k]
    return W.from_scipy(sp.diags(diags, offs, shape=(n, n), format="csr"), "band_p40")


def lap2d_holes60(m=60, seed=8):
    """Paired form with one far entry a row (P = 60), 40 rows and columns
    removed: empty rows and rows without their partner inside full runs."""
    rng = np.random.default_rng(seed)
    S = W.laplacian_2d(m).to_scipy()
    keep = np.ones(m * m)
    keep[rng.choice(m * m, 40, replace=False)] = 0.0
    S = sp.csr_matrix(sp.diags(keep) @ S @ sp.diags(keep))
    S.eliminate_zeros()
    return W.from_scipy(S, "lap2d_holes60")


def grid3d(nx, ny, nz, seed=11, drop=0):
    """7-point operator with random values on an nx x ny x nz grid (x
    fastest), optionally with `drop` rows and columns removed (holes)."""
    rng = np.random.default_rng(seed)
    def d1(m):
        return sp.diags([np.ones(m - 1), np.ones(m - 1)], [-1, 1])
    I = lambda m: sp.identity(m)
    P = (sp.kron(I(nz), sp.kron(I(ny), d1(nx))) + sp.kron(I(nz), sp.kron(d1(ny), I(nx)))
         + (sp.kron(d1(nz), sp.kron(I(ny), I(nx))) if nz > 1 else 0))
    P = sp.csr_matrix(P)
    U = sp.triu(P, 1).tocoo()
    v = rng.standard_normal(U.nnz)
    S = sp.coo_matrix((v, (U.row, U.col)), shape=P.shape)
    S = sp.csr_matrix(S + S.T + sp.diags(rng.standard_normal(P.shape[0]) + 6.0))
    if drop:
        keep = np.ones(P.shape[0])
        keep[rng.choice(P.shape[0], drop, replace=False)] = 0.0
        S = sp.csr_matrix(sp.diags(keep) @ S @ sp.diags(keep))
        S.eliminate_zeros()
    return W.from_scipy(S, f"grid{nx}x{ny}x{nz}")


# Row forms: lap3d_12V paired (P = 144; the last run of each half block
# starts 16 rows early), lap3d_11V plain with four far entries a row,
# lap3d_23V paired (P = 529, 11 rows recomputed, a tail of 529 rows),
# band_p40 and lap2d_holes60 paired; the grid operators named "grid" and
# "*:grid" take the grid form (8 x 8 tiles in 3D, 64 x 1 in 2D; ragged tiles,
# holes, a single tile, segments of one plane); the others plain.
MATS = {
    "lap3d_12V": lambda: W.laplacian_3d(12, potential_seed=1),
    "lap3d_11V": lambda: W.laplacian_3d(11, potential_seed=3),
    "lap3d_23V": lambda: W.laplacian_3d(23, potential_seed=5),
    "band_p40": band_p40,
    "lap2d_holes60": lap2d_holes60,
    "lap2d_holes": lap2d_holes,
    "powerlaw_4000": lambda: W.powerlaw_random(4000, seed=7, cap=300),
    "empty_rows": with_empty_rows,
    "tridiagonal": tridiagonal,
    "lap3d_23V:grid": lambda: W.laplacian_3d(23, potential_seed=5),
    "grid_13x11x9": lambda: grid3d(13, 11, 9),
    "grid_8x8x40_holes": lambda: grid3d(8, 8, 40, seed=12, drop=30),
    "grid_3x17x5": lambda: grid3d(3, 17, 5, seed=13),
    "lap2d_holes:grid": lap2d_holes,
    "grid_130x37_2d": lambda: grid3d(130, 1, 37, seed=14),
}
# row form each matrix is tested in (default: automatic)
FORMS = {"lap3d_12V": arr.ROW_PAIRED, "lap3d_11V": arr.ROW_PAIRED, "lap3d_23V": arr.ROW_PAIRED,
         "lap2d_holes60": arr.ROW_PAIRED, "lap2d_holes": arr.ROW_PAIRED, "lap3d_23V:grid": arr.ROW_GRID,
         "grid_13x11x9": arr.ROW_GRID, "grid_8x8x40_holes": arr.ROW_GRID, "grid_3x17x5": arr.ROW_GRID}


def dcsr(mat, A, dtype=None):
    return arr.DeviceCSR(A, dtype=dtype, row_form=FORMS.get(mat, arr.ROW_AUTO))


def test_matrix_forms_are_the_intended_ones():
    """Host check that each test matrix takes the row form it stands for."""
    for mat, make in MATS.items():
        A = make()
        grid = arr.arr_row_grid(A, FORMS.get(mat, arr.ROW_AUTO))
        assert (grid[0] > 0) == (mat.startswith("grid") or mat.endswith(":grid")), (mat, grid)


@pytest.mark.parametrize("mat", list(MATS))
@pytest.mark.parametrize("w", [1, 30, 64, 65, 240, 300])
def test_filter_step_fp64(mat, w):
    A = MATS[mat]()
    S = A.to_scipy()
    Ad = dcsr(mat, A)
    rng = np.random.default_rng(w)
    ld = w + 3
    Yin = rng.standard_normal((A.n, ld))
    Z = rng.standard_normal((A.n, ld))
    out = np.full((A.n, ld + 1), 7.0)
    Yd, Zd, Od = dev(Yin), dev(Z), dev(out)
    ss = torch.zeros(w, dtype=torch.float64, device="cuda")
    al, be, ga = 0.37, -1.25, 0.5
    arr.arr_filter_step(Ad, Yd[:, :w], Zd[:, :w], Od[:, :w], al, be, ga, colsumsq=ss)
    torch.cuda.synchronize()
    got = Od.cpu().numpy()
    ref = al * (S @ Yin[:, :w]) + be * Yin[:, :w] + ga * Z[:, :w]
    bound = abs(al) * (abs(S) @ np.abs(Yin[:, :w])) + abs(be) * np.abs(Yin[:, :w]) + abs(ga) * np.abs(Z[:, :w])
    assert np.all(np.abs(got[:, :w] - ref) <= 64 * 1.2e-16 * bound + 1e-300)
    assert np.all(got[:, w:] == 7.0)  # columns beyond w untouched
    np.testing.assert_allclose(ss.cpu().numpy(), (ref ** 2).sum(axis=0), rtol=1e-12)


@pytest.mark.parametrize("mat", list(MATS))
@pytest.mark.parametrize("w,ld", [(1, 1), (33, 36), (240, 240), (240, 243), (600, 604), (1000, 1000), (1100, 1104)])
def test_filter_step_fp32(mat, w, ld):
    """FP32 blocks: 16-byte loads when rows are 16-byte aligned (ld and w
    multiples of 4), one column per lane otherwise; several column chunks."""
    A = MATS[mat]()
    Ad = dcsr(mat, A, dtype=torch.float32)
    S32 = sp.csr_matrix((A.val.astype(np.float32).astype(np.float64), A.colind, A.rowptr), shape=(A.n, A.n))
    rng = np.random.default_rng(w + ld)
    Yin = rng.standard_normal((A.n, ld)).astype(np.float32).astype(np.float64)
    Z = rng.standard_normal((A.n, ld)).astype(np.float32).astype(np.float64)
    Yd, Zd = dev(Yin, torch.float32), dev(Z, torch.float32)
    Od = torch.full((A.n, ld), 7.0, dtype=torch.float32, device="cuda")
    ss = torch.zeros(w, dtype=torch.float64, device="cuda")
    al, be, ga = 0.37, -1.25, 0.5
    arr.arr_filter_step(Ad, Yd[:, :w], Zd[:, :w], Od[:, :w], al, be, ga, colsumsq=ss)
    got = Od.double().cpu().numpy()
    ref = np.float32(al) * (S32 @ Yin[:, :w]) + np.float32(be) * Yin[:, :w] + np.float32(ga) * Z[:, :w]
    bound = abs(al) * (abs(S32) @ np.abs(Yin[:, :w])) + abs(be) * np.abs(Yin[:, :w]) + abs(ga) * np.abs(Z[:, :w])
    kmax = int(np.diff(A.rowptr).max()) + 4
    assert np.all(np.abs(got[:, :w] - ref) <= kmax * 6e-8 * bound + 1e-30)
    assert np.all(got[:, w:] == 7.0)
    # column norms of the stored FP32 output, summed in FP64
    np.testing.assert_allclose(ss.cpu().numpy(), (got[:, :w] ** 2).sum(axis=0), rtol=1e-12)


def _small_matrix(kind, n):
    if kind == "band5":  # tridiagonal plus the diagonals at +-5: two far entries a row, no overflow
        rng = np.random.default_rng(n)
        diags, offs = [rng.standard_normal(n) + 4.0], [0]
        for k in (1, 5):
            if k < n:
                v = rng.standard_normal(n - k)
                diags += [v, v]
                offs += [k, -k]
        return W.from_scipy(sp.diags(diags, offs, shape=(n, n), format="csr"), "band5")
    return W.random_symmetric(n, seed=n, density=0.08 if kind == "sparse" else 0.5)


@pytest.mark.parametrize("n", [1, 2, 3, 33, 34, 35, 66, 97])
@pytest.mark.parametrize("kind", ["band5", "sparse", "dense"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_filter_step_small_n(n, kind, dtype):
    """Matrices shorter than one or two 32-row runs: the guarded row path, a
    single full run, and full runs next to ragged ones; without overflow rows
    (band5) and with them (random sparse and dense rows)."""
    A = _small_matrix(kind, n)
    tdt, u = (torch.float32, 6e-8) if dtype == "f32" else (torch.float64, 1.2e-16)
    vals = A.val.astype(np.float32).astype(np.float64) if dtype == "f32" else A.val
    Sx = sp.csr_matrix((vals, A.colind, A.rowptr), shape=(A.n, A.n))
    Ad = arr.DeviceCSR(A, dtype=tdt)
    for w in (1, 5, 65):
        rng = np.random.default_rng(w)
        Yin = rng.standard_normal((n, w))
        Z = rng.standard_normal((n, w))
        if dtype == "f32":
            Yin = Yin.astype(np.float32).astype(np.float64)
            Z = Z.astype(np.float32).astype(np.float64)
        Yd, Zd = dev(Yin, tdt), dev(Z, tdt)
        Od = torch.zeros_like(Yd)
        ss = torch.zeros(w, dtype=torch.float64, device="cuda")
        arr.arr_filter_step(Ad, Yd, Zd, Od, 0.5, -0.25, 2.0, colsumsq=ss)
        got = Od.double().cpu().numpy()
        ref = 0.5 * (Sx @ Yin) - 0.25 * Yin + 2.0 * Z
        bound = 0.5 * (abs(Sx) @ np.abs(Yin)) + 0.25 * np.abs(Yin) + 2.0 * np.abs(Z)
        kmax = int(np.diff(A.rowptr).max()) + 4
        assert np.all(np.abs(got - ref) <= kmax * u * bound + 1e-30), (n, w)
        np.testing.assert_allclose(ss.cpu().numpy(), (got ** 2).sum(axis=0), rtol=1e-12)


NO_Z_MATS = {"powerlaw_3000": lambda: W.powerlaw_random(3000, seed=9, cap=500), **MATS}


@pytest.mark.parametrize("mat", list(NO_Z_MATS))
@pytest.mark.parametrize("w", [1, 33, 240])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("sums", [False, True])
def test_filter_step_no_z(mat, w, dtype, sums):
    """Y = alpha A X + beta X with no Z operand (the product form's factors),
    with and without the column sums: every kernel variant on matrices with
    and without rows past four far entries."""
    A = NO_Z_MATS[mat]()
    tdt, u = (torch.float32, 6e-8) if dtype == "f32" else (torch.float64, 1.2e-16)
    Ad = dcsr(mat, A, dtype=tdt)
    vals = A.val.astype(np.float32).astype(np.float64) if dtype == "f32" else A.val
    Sx = sp.csr_matrix((vals, A.colind, A.rowptr), shape=(A.n, A.n))
    rng = np.random.default_rng(1 + w)
    Yin = rng.standard_normal((A.n, w))
    if dtype == "f32":
        Yin = Yin.astype(np.float32).astype(np.float64)
    Yd = dev(Yin, tdt)
    Od = torch.zeros_like(Yd)
    ss = torch.zeros(w, dtype=torch.float64, device="cuda") if sums else None
    arr.arr_filter_step(Ad, Yd, None, Od, 2.0, 0.25, 0.0, colsumsq=ss)
    torch.cuda.synchronize()
    got = Od.double().cpu().numpy()
    ref = 2.0 * (Sx @ Yin) + 0.25 * Yin
    bound = 2.0 * (abs(Sx) @ np.abs(Yin)) + 0.25 * np.abs(Yin)
    kmax = int(np.diff(A.rowptr).max()) + 4
    assert np.all(np.abs(got - ref) <= kmax * u * bound + 1e-30)
    if sums:
        np.testing.assert_allclose(ss.cpu().numpy(), (got ** 2).sum(axis=0), rtol=1e-12)


PAIRED = {"lap3d_20": lambda: W.laplacian_3d(20, potential_seed=2), "lap2d_107": lambda: W.laplacian_2d(107),
          "lap3d_23V": MATS["lap3d_23V"], "band_p40": band_p40, "grid_13x11x9": MATS["grid_13x11x9"],
          "grid_130x37_2d": MATS["grid_130x37_2d"]}


@pytest.mark.parametrize("mat", list(PAIRED))
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("w", [1, 65, 240, 520])
@pytest.mark.parametrize("zs", [(False, False), (True, False), (False, True), (True, True)])
def test_filter_step_row_forms(mat, dtype, w, zs):
    """The grid, paired and plain row forms against the definition, every
    variant (Z operand, column sums, FP32 16-byte / 8-byte and FP64 column
    chunks): one run per half block (lap3d_20), one far slot with recomputed
    rows and an upper-row tail (lap2d_107), three far slots with a tail
    (lap3d_23V), a tail holding lower rows too (band_p40); grid form (forced,
    and automatic for the 2D grids) on the grids (3D 8 x 8 tiles and 2D
    64 x 1 tiles, ragged), paired form on all but the two whose grid strides
    are below the run length."""
    A = PAIRED[mat]()
    pair, _, _ = arr.arr_row_form(A, arr.ROW_PAIRED)
    assert pair > 0 or mat.startswith("grid")
    has_z, sums = zs
    tdt, u = (torch.float32, 6e-8) if dtype == "f32" else (torch.float64, 1.2e-16)
    vals = A.val.astype(np.float32).astype(np.float64) if dtype == "f32" else A.val
    Sx = sp.csr_matrix((vals, A.colind, A.rowptr), shape=(A.n, A.n))
    rng = np.random.default_rng(w)
    Yin = rng.standard_normal((A.n, w))
    Z = rng.standard_normal((A.n, w))
    if dtype == "f32":
        Yin = Yin.astype(np.float32).astype(np.float64)
        Z = Z.astype(np.float32).astype(np.float64)
    al, be, ga = 0.75, -0.5, (1.5 if has_z else 0.0)
    ref = al * (Sx @ Yin) + be * Yin + ga * Z
    bound = abs(al) * (abs(Sx) @ np.abs(Yin)) + abs(be) * np.abs(Yin) + abs(ga) * np.abs(Z)
    kmax = int(np.diff(A.rowptr).max()) + 4
    outs = []
    for form in (arr.ROW_GRID, arr.ROW_AUTO, arr.ROW_PAIRED, arr.ROW_PLAIN):
        Ad = arr.DeviceCSR(A, dtype=tdt, row_form=form)
        Yd, Zd = dev(Yin, tdt), dev(Z, tdt)
        Od = torch.zeros_like(Yd)
        ss = torch.zeros(w, dtype=torch.float64, device="cuda") if sums else None
        arr.arr_filter_step(Ad, Yd, Zd if has_z else None, Od, al, be, ga, colsumsq=ss)
        torch.cuda.synchronize()
        got = Od.double().cpu().numpy()
        assert np.all(np.abs(got - ref) <= kmax * u * bound + 1e-30), form
        if sums:
            np.testing.assert_allclose(ss.cpu().numpy(), (got ** 2).sum(axis=0), rtol=1e-12)
        outs.append(got)
    for o in outs[1:]:
        assert np.all(np.abs(outs[0] - o) <= 2 * kmax * u * bound + 1e-30)


@pytest.mark.parametrize("d", [3, 8, 15])
def test_poly_matches_oracle_fp64(d):
    """Algorithm 7 on the shifted operator, as Algorithm 8 calls it."""
    A = W.laplacian_3d(12, potential_seed=1)
    S = -A.to_scipy()  # the working operator of a smallest-eigenvalue solve
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-40]
    X = W.gaussian_block(A.n, 37, seed=4)
    g = O.interpolant_coefficients(d)
    ref = O.poly(O.shifted(S, a), X, 0.0, b - a, g)
    Ad = arr.DeviceCSR(A.negated())
    Xd = dev(X)
    arr.arr_poly(Ad, Xd, a, 0.0, b - a, arr.arr_filter_coefficients(d))
    got = Xd.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("d", [1, 2, 3, 8, 15])
@pytest.mark.parametrize("form", ["product", "horner"])
def test_filter_forms_match_oracle_fp64(d, form):
    """psi_d applied as the product over its roots, or by Algorithm 7's
    recurrence, against the oracle's Algorithm 7."""
    A = W.laplacian_3d(12, potential_seed=1)
    S = -A.to_scipy()
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-40]
    X = W.gaussian_block(A.n, 37, seed=4)
    g = O.interpolant_coefficients(d) if d > 1 else np.array([0.5, 0.5])
    ref = O.poly(O.shifted(S, a), X, 0.0, b - a, g)
    Xd = dev(X)
    arr.arr_filter(arr.DeviceCSR(A.negated()), Xd, a, 0.0, b - a, d,
                   arr.POLY_PRODUCT if form == "product" else arr.POLY_HORNER)
    got = Xd.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("d", [1, 2, 3, 4, 8, 15])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_chebyshev_filter_matches_oracle(d, dtype):
    """The classic Chebyshev filter T_d (eq. cheby-poly) on the mapped operator,
    against the oracle's recursion; d mod 3 covers every buffer rotation."""
    A = W.laplacian_3d(12, potential_seed=1)
    S = -A.to_scipy()
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-40]
    X = W.gaussian_block(A.n, 37, seed=4)
    ref = O.chebyshev_poly(O.shifted(S, a), X, 0.0, b - a, d)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Xd = dev(X, tdt)
    arr.arr_filter(arr.DeviceCSR(A.negated(), dtype=tdt), Xd, a, 0.0, b - a, d, arr.POLY_CHEBYSHEV)
    err = np.abs(Xd.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= (1e-12 if dtype == "f64" else 2e-6 * d), err


def test_filter_product_fp32_more_accurate_than_horner():
    """In FP32 the product form keeps psi_15's accuracy (no cancellation of
    large monomial terms); Algorithm 7's monomial recurrence loses about
    three digits more (the FP32 reading of Algorithm 7)."""
    A = W.laplacian_3d(12, potential_seed=1).negated()
    S = A.to_scipy()
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-40]
    X = W.gaussian_block(A.n, 16, seed=4)
    g = O.interpolant_coefficients(15)
    ref = O.poly(O.shifted(S, a), X, 0.0, b - a, g)
    errs = {}
    for form in (arr.POLY_PRODUCT, arr.POLY_HORNER):
        Xd = dev(X, torch.float32)
        arr.arr_filter(arr.DeviceCSR(A, dtype=torch.float32), Xd, a, 0.0, b - a, 15, form)
        errs[form] = np.abs(Xd.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert errs[arr.POLY_PRODUCT] < 1e-5, errs
    assert errs[arr.POLY_PRODUCT] < errs[arr.POLY_HORNER], errs


@pytest.mark.parametrize("d", [3, 8, 15])
def test_gn_step_matches_oracle_fp64(d):
    """The GN inner iteration of Algorithm 8 (Sec. 2.6) against the oracle."""
    A = W.laplacian_3d(12, potential_seed=1)
    S = -A.to_scipy()
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-40]
    X = W.gaussian_block(A.n, 37, seed=5)
    g = O.interpolant_coefficients(d)
    ref = O.gn_step(O.shifted(S, a), X, 0.0, b - a, g)
    Xd = dev(X)
    arr.arr_gn_step(arr.DeviceCSR(A.negated()), Xd, a, 0.0, b - a, arr.arr_filter_coefficients(d))
    got = Xd.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_gn_step_fp32_and_repeated_steps_track_oracle():
    """FP32 blocks against the oracle; and 40 GN steps in FP64 follow the
    oracle's trajectory to the same X X^T (GN contracts towards the rank-w
    part of rho(A), so the two agree to rounding)."""
    A = W.laplacian_2d_potential(20, potential_seed=3)
    S = -A.to_scipy()
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-30]
    g = O.interpolant_coefficients(5)
    X = W.gaussian_block(A.n, 12, seed=6)
    ref = O.gn_step(O.shifted(S, a), X, 0.0, b - a, g)
    Xf = dev(X, torch.float32)
    arr.arr_gn_step(arr.DeviceCSR(A.negated(), dtype=torch.float32), Xf, a, 0.0, b - a, arr.arr_filter_coefficients(5))
    assert np.abs(Xf.double().cpu().numpy() - ref).max() <= 1e-4 * np.abs(ref).max()
    Xd = dev(X)
    Ad = arr.DeviceCSR(A.negated())
    Xo = X.copy()
    for _ in range(40):
        arr.arr_gn_step(Ad, Xd, a, 0.0, b - a, arr.arr_filter_coefficients(5))
        Xo = O.gn_step(O.shifted(S, a), Xo, 0.0, b - a, g)
    Xg = Xd.cpu().numpy()
    Pg, Po = Xg @ Xg.T, Xo @ Xo.T
    assert np.abs(Pg - Po).max() <= 1e-8 * np.abs(Po).max()


def test_poly_fp32_error_is_small():
    A = W.laplacian_3d(12, potential_seed=1).negated()
    S = A.to_scipy()
    lam = np.linalg.eigvalsh(S.toarray())
    a, b = lam[0] - 0.01, lam[-40]
    X = W.gaussian_block(A.n, 16, seed=4)
    g = O.interpolant_coefficients(8)
    ref = O.poly(O.shifted(S, a), X, 0.0, b - a, g)
    Xd = dev(X, torch.float32)
    arr.arr_poly(arr.DeviceCSR(A, dtype=torch.float32), Xd, a, 0.0, b - a, arr.arr_filter_coefficients(8))
    err = np.abs(Xd.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-4, err


@pytest.mark.parametrize("n,mx,my", [(5003, 1, 1), (5003, 17, 65), (777, 64, 64), (20011, 130, 200), (33, 5, 3),
                                     (4099, 300, 300), (3001, 257, 128), (100, 128, 129)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32cores"])
def test_gram(n, mx, my, dtype):
    rng = np.random.default_rng(n + mx)
    fast = dtype == "f32cores"
    dtype = "f32" if fast else dtype
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X = rng.standard_normal((n, mx + 2))
    Y = rng.standard_normal((n, my + 1))
    if dtype == "f32":
        X, Y = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    Xd, Yd = dev(X, tdt), dev(Y, tdt)
    G = torch.zeros((mx, my), dtype=torch.float64, device="cuda")
    arr.arr_gram(Xd[:, :mx], Yd[:, :my], G, fp32_cores=fast)
    ref = X[:, :mx].T @ Y[:, :my]
    bound = np.abs(X[:, :mx]).T @ np.abs(Y[:, :my])
    # FP64 products and sums, except on the FP32 matrix cores: each 32-row
    # slice summed in FP32 (error at most gamma_32 of the slice's |x||y|), the
    # slices added in FP64.
    rel = 1e-14 * np.sqrt(n) + (32 * 2.0**-24 if fast else 0.0)
    assert np.all(np.abs(G.cpu().numpy() - ref) <= rel * bound + 1e-300)
    # symmetric product (same buffer): exactly symmetric
    Gs = torch.zeros((mx, mx), dtype=torch.float64, device="cuda")
    arr.arr_gram(Xd[:, :mx], Xd[:, :mx], Gs, fp32_cores=fast)
    gs = Gs.cpu().numpy()
    assert np.array_equal(gs, gs.T)
    ref_s = X[:, :mx].T @ X[:, :mx]
    assert np.all(np.abs(gs - ref_s) <= rel * (np.abs(X[:, :mx]).T @ np.abs(X[:, :mx])))


@pytest.mark.parametrize("n,m,c", [(5003, 1, 1), (5003, 16, 65), (4097, 17, 64), (20011, 480, 240), (70, 100, 3)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32cores"])
def test_block_update(n, m, c, dtype):
    rng = np.random.default_rng(m * c)
    fast = dtype == "f32cores"
    dtype = "f32" if fast else dtype
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X = rng.standard_normal((n, m))
    Wm = rng.standard_normal((m, c + 2))
    Y0 = rng.standard_normal((n, c + 1))
    if dtype == "f32":
        X, Y0 = X.astype(np.float32).astype(np.float64), Y0.astype(np.float32).astype(np.float64)
    Xd, Wd, Yd = dev(X, tdt), dev(Wm), dev(Y0, tdt)
    arr.arr_block_update(Xd, Wd[:, :c], Yd[:, :c], alpha=-0.5, beta=2.0, fp32_cores=fast)
    torch.cuda.synchronize()
    ref = 2.0 * Y0[:, :c] - 0.5 * X @ Wm[:, :c]
    bound = 2.0 * np.abs(Y0[:, :c]) + 0.5 * np.abs(X) @ np.abs(Wm[:, :c])
    got = Yd.double().cpu().numpy()
    if dtype == "f32" and not fast:
        # FP64 products and sums: only the final rounding to FP32
        assert np.all(np.abs(got[:, :c] - ref) <= (2.0**-24 + 4 * m * 1.2e-16) * bound + 1e-300)
    else:
        eps = 1.2e-16 if dtype == "f64" else 6e-8
        assert np.all(np.abs(got[:, :c] - ref) <= 4 * m * eps * bound + 1e-300)
    assert np.array_equal(got[:, c:], Y0[:, c:])


def test_rcond_matches_oracle():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3001, 40))
    assert abs(arr.arr_rcond_gram(dev(X)) / O.rcond_gram(X) - 1) < 1e-10
    Xw = rng.standard_normal((4001, 200)) * np.logspace(0, 3, 200)[None, :]
    assert abs(arr.arr_rcond_gram(dev(Xw)) / O.rcond_gram(Xw) - 1) < 1e-8
    # ill conditioned: two nearly parallel columns
    Xi = X.copy()
    Xi[:, 1] = Xi[:, 0] + 1e-5 * Xi[:, 1]
    r_or, r_gpu = O.rcond_gram(Xi), arr.arr_rcond_gram(dev(Xi))
    assert abs(r_gpu / r_or - 1) < 1e-4
    # exactly dependent: not positive definite numerically (both tiny or zero)
    Xs = X.copy()
    Xs[:, 3] = Xs[:, 2]
    assert arr.arr_rcond_gram(dev(Xs)) < 1e-14 and O.rcond_gram(Xs) < 1e-14


@pytest.mark.parametrize("kind", ["random", "ill", "krylov", "wide"])
def test_orthonormalize(kind):
    rng = np.random.default_rng(11)
    n, m = 6007, (300 if kind == "wide" else 96)
    Z = rng.standard_normal((n, m))
    if kind == "ill":
        Z[:, m // 2:] = Z[:, : m // 2] + 1e-7 * rng.standard_normal((n, m // 2))
    if kind == "krylov":
        A = W.laplacian_3d(18, potential_seed=2).to_scipy()  # n = 5832
        n = A.shape[0]
        X = rng.standard_normal((n, 32))
        for _ in range(20):  # nearly dependent columns, like the MPM iterate
            X = A @ X
            X /= np.linalg.norm(X, axis=0)
        Z = np.hstack([X, A @ X, A @ (A @ X)])
        m = Z.shape[1]
    Zd = dev(Z)
    arr.arr_orthonormalize(Zd)
    U = Zd.cpu().numpy()
    assert np.abs(U.T @ U - np.eye(m)).max() < 1e-12
    # R(Z) is contained in R(U)
    assert np.linalg.norm(Z - U @ (U.T @ Z)) <= 1e-9 * np.linalg.norm(Z)


@pytest.mark.parametrize("m", [1, 2, 3, 31, 64, 100, 257])
def test_syev_random(m):
    rng = np.random.default_rng(m)
    Hm = rng.standard_normal((m, m))
    Hm = Hm + Hm.T
    _check_syev(Hm)


@pytest.mark.parametrize("m", [720, 960])
def test_syev_rayleigh_ritz_sized_clustered(m):
    """Orders the solver reaches on the 1e6-row benchmark (m = (p + 1) w' up
    to 960), with a spectrum shaped like a Rayleigh-Ritz matrix near
    convergence: a clustered wanted part (200 values within 1e-3, some
    repeated to 1e-12), a gap, and a spread tail."""
    rng = np.random.default_rng(m + 1)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    lam = np.concatenate([12.5 - 1e-3 * rng.random(180), np.repeat(12.49, 20) + 1e-12 * rng.random(20),
                          6.0 + 5.0 * rng.random(m - 200)])
    _check_syev(Q @ np.diag(lam) @ Q.T)


def test_syev_degenerate_and_zero():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.array([3.0] * 5 + [1.0] * 10 + [0.0] * 20 + [-2.0] * 5)
    _check_syev(Q @ np.diag(lam) @ Q.T)
    _check_syev(np.zeros((12, 12)))
    _check_syev(np.diag(np.arange(9.0)))


def _check_syev(Hm):
    m = Hm.shape[0]
    Hd = dev(Hm)
    ev = torch.zeros(m, dtype=torch.float64, device="cuda")
    V = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    arr.arr_syev(Hd, ev, V)
    e, Vh = ev.cpu().numpy(), V.cpu().numpy()
    nrm = max(1.0, np.abs(Hm).max())
    ref = np.sort(np.linalg.eigvalsh(Hm))[::-1]
    assert np.all(np.diff(e) <= 0)
    assert np.abs(e - ref).max() <= 1e-13 * m * nrm
    assert np.abs(Hm @ Vh - Vh * e[None, :]).max() <= 1e-12 * m * nrm
    assert np.abs(Vh.T @ Vh - np.eye(m)).max() <= 1e-13 * m


@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("deflate", [False, True])
def test_augmented_rr_matches_oracle(p, deflate):
    A = W.laplacian_3d(12, potential_seed=1).negated()
    S = A.to_scipy()
    w = 24
    X = W.gaussian_block(A.n, w, seed=8)
    Qc = None
    if deflate:
        lam, Qf = np.linalg.eigh(S.toarray())
        Qc = Qf[:, -4:].copy()
        X = O.project_out(Qc, X)
    Yo, so = O.augmented_rr(S, X, p, Qc)
    Yd = torch.zeros((A.n, w), dtype=torch.float64, device="cuda")
    vals = arr.arr_augmented_rr(arr.DeviceCSR(A), dev(X), p, None if Qc is None else dev(Qc), Yd)
    assert np.abs(vals - so[:w]).max() <= 1e-10 * max(1.0, np.abs(so).max())
    Y = Yd.cpu().numpy()
    # Ritz pairs: orthonormal, Galerkin residuals match the oracle's in size
    assert np.abs(Y.T @ Y - np.eye(w)).max() < 1e-11
    r_gpu = np.linalg.norm(S @ Y - Y * vals[None, :], axis=0)
    r_or = np.linalg.norm(S @ Yo[:, :w] - Yo[:, :w] * so[None, :w], axis=0)
    assert np.all(r_gpu <= r_or * (1 + 1e-6) + 1e-10)
    if deflate:
        assert np.abs(Qc.T @ Y).max() < 1e-10


# Items of one multi-request batch: (matrix, row form, dtype, w, Z operand,
# column sums). Paired and plain forms in both precisions, with and without
# overflow rows, Z and column sums, widths with one and several column
# chunks, and a grid-form item (its own launch) among them.
BATCH = [
    ("lap3d_20", arr.ROW_PAIRED, torch.float64, 240, False, False),
    ("lap3d_20", arr.ROW_PAIRED, torch.float32, 240, False, True),
    ("lap3d_23V", arr.ROW_PAIRED, torch.float64, 520, True, True),
    ("powerlaw_4000", arr.ROW_AUTO, torch.float64, 65, True, False),
    ("powerlaw_4000", arr.ROW_AUTO, torch.float32, 300, False, True),
    ("lap3d_11V", arr.ROW_PLAIN, torch.float64, 1, False, True),
    ("band_p40", arr.ROW_AUTO, torch.float32, 131, True, True),
    ("grid_130x37_2d", arr.ROW_AUTO, torch.float64, 240, False, True),
]


@pytest.mark.parametrize("subset", [list(range(len(BATCH))), [0], [3, 4], [1, 2, 5, 6]])
def test_filter_step_batch_equals_single_launches(subset):
    """arr_filter_step_batch (the multi-request kernel: the items' workgroups
    from one task table per kernel variant) gives each item bitwise the
    output and column sums of its own arr_filter_step, and writes nothing
    else (canaries around every output)."""
    mats = {"lap3d_20": PAIRED["lap3d_20"], **MATS}
    items, singles = [], []
    for q, i in enumerate(subset):
        mat, form, tdt, w, has_z, sums = BATCH[i]
        A = mats[mat]()
        Ad = arr.DeviceCSR(A, dtype=tdt, row_form=form)
        rng = np.random.default_rng(100 + i)
        Yd = dev(rng.standard_normal((A.n, w)), tdt)
        Zd = dev(rng.standard_normal((A.n, w)), tdt) if has_z else None
        al, be, ga = 0.75 + 0.01 * i, -0.5, (1.25 if has_z else 0.0)
        # output block with a canary column on the right and canary rows around
        big = torch.full((A.n + 2, w + 1), 7.0, dtype=tdt, device="cuda")
        Od = big[1:A.n + 1, :w]
        ss = torch.full((w,), -1.0, dtype=torch.float64, device="cuda") if sums else None
        items.append((Ad, Yd, Zd, Od, al, be, ga, ss))
        O1 = torch.zeros((A.n + 2, w + 1), dtype=tdt, device="cuda")[1:A.n + 1, :w]  # the same layout
        s1 = torch.zeros(w, dtype=torch.float64, device="cuda") if sums else None
        arr.arr_filter_step(Ad, Yd, Zd, O1, al, be, ga, colsumsq=s1)
        singles.append((O1, s1, big))
    arr.arr_filter_step_batch(items)
    torch.cuda.synchronize()
    for (Ad, Yd, Zd, Od, al, be, ga, ss), (O1, s1, big) in zip(items, singles):
        assert torch.equal(Od, O1)
        if ss is not None:
            assert torch.equal(ss, s1)
        assert bool((big[0] == 7.0).all()) and bool((big[-1] == 7.0).all()) and bool((big[:, -1] == 7.0).all())


def test_filter_step_batch_rejects_bad_items():
    A = W.laplacian_2d(30)
    Ad = arr.DeviceCSR(A)
    Y = torch.zeros((A.n, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(arr.ArrError):
        arr.arr_filter_step_batch([])
    with pytest.raises(arr.ArrError):
        arr.arr_filter_step_batch([(Ad, Y, None, Y, 1.0, 0.0, 0.0, None)])  # Yout aliases Yin
