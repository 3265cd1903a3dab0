"""Host choice of the SpMM row form (no GPU): the grid form for 7-point (3D)
and 5-point (2D) operators on a lexicographic grid with no entry wrapping
from one grid line to the next; otherwise the paired form for operators with
a frequent far column offset P whose rows keep at most three other far
entries, the plain form otherwise. The pairing offset follows from the
grid's strides, the run length of 20 rows and the at-most-P/8 recomputed
rows per half block."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1507_06078_amd import arr, workloads as W


def banded(n, offsets, seed=0):
    rng = np.random.default_rng(seed)
    diags, offs = [rng.standard_normal(n) + 8.0], [0]
    for k in offsets:
        v = rng.standard_normal(n - k)
        diags += [v, v]
        offs += [k, -k]
    return W.from_scipy(sp.diags(diags, offs, shape=(n, n), format="csr"), "banded")


def lap2d_9pt(m):
    T = sp.diags([np.ones(m - 1), np.ones(m), np.ones(m - 1)], [-1, 0, 1])
    S = sp.kron(T, T, format="csr")
    return W.from_scipy(S, "lap2d_9pt")


@pytest.mark.parametrize("make,expect", [
    (lambda: W.laplacian_3d(20), (20, 3, 0)),         # y stride: 20 rows, one run per half block
    (lambda: W.laplacian_3d(12), (144, 3, 0)),        # y stride 12 < 20: the z stride, 8 runs, 16 rows again
    (lambda: W.laplacian_3d(11), (0, 4, 0)),          # 121: 7 runs would recompute 19 > 121/8 rows
    (lambda: W.laplacian_3d(30, potential_seed=2), (900, 3, 0)),  # 30: 2 runs recompute 10 > 30/8
    (lambda: W.laplacian_3d(23), (529, 3, 0)),        # 27 runs, 11 rows recomputed, tail of 529 rows
    (lambda: W.laplacian_2d(100), (100, 1, 0)),       # 2D: one far entry besides the partner
    (lambda: W.laplacian_2d(107), (107, 1, 0)),       # 6 runs, 13 <= 107/8 recomputed
    (lambda: W.laplacian_2d(41), (0, 4, 0)),          # 3 runs recompute 19 > 41/8
    (lambda: banded(1070, (1, 3, 40)), (40, 3, 0)),   # lower rows in the tail
    (lambda: banded(1000, (1, 2, 3, 4, 40)), None),  # partner plus seven far entries: plain, overflow
    (lambda: banded(100, (1, 40)), (40, 1, 0)),       # a single block of 80 rows and a tail of 20
    (lambda: lap2d_9pt(40), None),                    # +-40 pairs, but five far entries remain: plain
])
def test_row_form_choice(make, expect):
    A = make()
    plain = (0, 4, plain_overflow(A))
    assert arr.arr_row_form(A, arr.ROW_PAIRED) == (expect or plain)
    assert arr.arr_row_form(A, arr.ROW_PLAIN) == plain
    assert arr.arr_row_grid(A, arr.ROW_PAIRED) == (0, 0, 0)
    assert arr.arr_row_grid(A, arr.ROW_PLAIN) == (0, 0, 0)


def grid_operator(nx, ny, nz, wrap=False):
    """Pattern of a 7-point (5-point if ny == 1 or nz == 1) operator on an
    nx x ny x nz grid, x fastest; `wrap` adds one entry joining the end of an
    x line to the start of the next (not a grid operator)."""
    n = nx * ny * nz
    idx = np.arange(n)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    rows, cols = [idx], [idx]
    for ok, d in ((x + 1 < nx, 1), (y + 1 < ny, nx), (z + 1 < nz, nx * ny)):
        r = idx[ok]
        rows += [r, r + d]
        cols += [r + d, r]
    if wrap:
        rows += [np.array([nx - 1, nx])]
        cols += [np.array([nx, nx - 1])]
    r, c = np.concatenate(rows), np.concatenate(cols)
    return W.from_scipy(sp.csr_matrix((np.ones(r.size), (r, c)), shape=(n, n)), "grid")


@pytest.mark.parametrize("dims", [(20, 20, 20), (13, 11, 9), (3, 17, 5), (100, 1, 100), (130, 1, 37), (2, 2, 2),
                                  (64, 64, 2)])
def test_grid_form_detected_with_its_dimensions(dims):
    """ARR_ROW_GRID takes the grid form, with the grid's dimensions (gy = 1
    for a 2D grid), no pairing and no gathered far entries; the automatic
    choice does so for 2D grids and leaves 3D grids to the paired form."""
    nx, ny, nz = dims
    A = grid_operator(nx, ny, nz)
    assert arr.arr_row_grid(A, arr.ROW_GRID) == (nx, ny, nz)
    assert arr.arr_row_form(A, arr.ROW_GRID) == (0, 0, 0)
    if ny == 1:
        assert arr.arr_row_grid(A, arr.ROW_AUTO) == (nx, ny, nz)
    else:
        assert arr.arr_row_grid(A, arr.ROW_AUTO) == (0, 0, 0)
        assert arr.arr_row_form(A, arr.ROW_AUTO) == arr.arr_row_form(A, arr.ROW_PAIRED)


def test_grid_form_of_the_workload_generators():
    assert arr.arr_row_grid(W.laplacian_3d(30, potential_seed=2), arr.ROW_GRID) == (30, 30, 30)
    assert arr.arr_row_grid(W.laplacian_3d(30, potential_seed=2)) == (0, 0, 0)
    assert arr.arr_row_grid(W.laplacian_2d(41)) == (41, 1, 41)
    assert arr.arr_row_grid(W.laplacian_2d_potential(50, potential_seed=3)) == (50, 1, 50)


@pytest.mark.parametrize("make", [
    lambda: grid_operator(12, 10, 6, wrap=True),      # an entry wrapping from one x line to the next
    lambda: grid_operator(40, 1, 30, wrap=True),
    lambda: lap2d_9pt(20),                            # diagonal neighbours: four strides
    lambda: banded(1070, (1, 3, 40)),                 # strides 3 and 40: 40 is not a multiple of 3
    lambda: banded(1000, (1, 40)),                    # 40 x 25 grid strides, but the +-1 entries wrap
    lambda: banded(1001, (1, 40)),                    # 1001 is no multiple of the stride 40
    lambda: W.powerlaw_random(3000, seed=9, cap=500),
])
def test_grid_form_rejected(make):
    A = make()
    grid = arr.arr_row_grid(A, arr.ROW_GRID)
    if grid != (0, 0, 0):
        # a banded matrix whose strides happen to describe a grid is one:
        # every entry must then be a neighbour inside it
        nx, ny, nz = grid
        assert nx * ny * nz == A.n
        rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
        d = np.asarray(A.colind, dtype=np.int64) - rows
        x = rows % nx
        ok = (d == 0) | ((d == 1) & (x + 1 < nx)) | ((d == -1) & (x > 0)) | (np.abs(d) == nx) | (np.abs(d) == nx * ny)
        assert ok.all()
    else:
        assert arr.arr_row_form(A, arr.ROW_GRID) == arr.arr_row_form(A, arr.ROW_PAIRED)


def plain_overflow(A):
    """Entries of the plain form's overflow CSR: far entries (|j - i| > 1)
    past the fourth of each row."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    far = np.abs(np.asarray(A.colind, dtype=np.int64) - rows) > 1
    per_row = np.bincount(rows[far], minlength=A.n)
    return int(np.maximum(per_row - 4, 0).sum())


def test_row_form_irregular_matrix_is_plain():
    A = W.powerlaw_random(3000, seed=9, cap=500)
    pair, far, ovf = arr.arr_row_form(A)
    assert (pair, far) == (0, 4) and ovf > 0
    assert arr.arr_row_grid(A) == (0, 0, 0)


def test_row_form_rejects_bad_input():
    A = W.laplacian_2d(10)
    with pytest.raises(arr.ArrError):
        arr.arr_row_form(A, 7)
    bad = W.from_scipy(sp.csr_matrix(np.eye(3)), "eye")
    bad.colind = np.array([0, 5, 2], dtype=np.int32)  # column out of range
    with pytest.raises(arr.ArrError):
        arr.arr_row_form(bad)
