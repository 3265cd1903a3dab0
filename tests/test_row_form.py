"""Host choice of the SpMM row form (no GPU): the paired form for operators
with a frequent far column offset P whose rows keep at most three other far
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
    assert arr.arr_row_form(A, arr.ROW_AUTO) == (expect or plain)
    assert arr.arr_row_form(A, arr.ROW_PLAIN) == plain


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


def test_row_form_rejects_bad_input():
    A = W.laplacian_2d(10)
    with pytest.raises(arr.ArrError):
        arr.arr_row_form(A, 7)
    bad = W.from_scipy(sp.csr_matrix(np.eye(3)), "eye")
    bad.colind = np.array([0, 5, 2], dtype=np.int32)  # column out of range
    with pytest.raises(arr.ArrError):
        arr.arr_row_form(bad)
