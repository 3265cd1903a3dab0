"""Stored oracle values (tests/golden/, written by tests/golden/make_golden.py
from the oracle only): the filter coefficients Gamma_d of Sec. 5 (eq. def:fN,
eq. chebfun-f). The oracle must keep reproducing them, and the library's own
derivation (discrete Chebyshev transform) must agree with them."""
import os

import numpy as np
import pytest

from oracle import arrabit as O
from paper_1507_06078_amd import arr

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load():
    out = {}
    for line in open(os.path.join(HERE, "psi_coefficients.txt")):
        if line.startswith("#") or not line.strip():
            continue
        vals = line.split()
        out[int(vals[0])] = np.array([float(v) for v in vals[1:]])
    return out


GOLD = _load()


def test_fixture_covers_degrees_1_to_15():
    assert sorted(GOLD) == list(range(1, 16))
    for d, g in GOLD.items():
        assert g.shape == (d + 1,)


@pytest.mark.parametrize("d", range(1, 16))
def test_oracle_reproduces_stored_coefficients(d):
    np.testing.assert_allclose(O.interpolant_coefficients(d), GOLD[d], rtol=1e-12, atol=1e-12 * np.abs(GOLD[d]).max())


@pytest.mark.parametrize("d", range(1, 16))
def test_library_coefficients_match_stored(d):
    g = GOLD[d]
    np.testing.assert_allclose(arr.arr_filter_coefficients(d), g, rtol=1e-9, atol=1e-9 * np.abs(g).max())
